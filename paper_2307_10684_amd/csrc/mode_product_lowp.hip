// Reduced-precision mu-mode products for the Tucker operators of the step
// (the state, the stage combinations and the small matrix functions stay
// FP64; only the bulk products run in lower precision):
//
//   FP32      v_mfma_f32_16x16x4_f32 on FP32 data;
//   BF16X3    each FP32 operand x is split into three bf16 parts,
//             x = hi + mid + lo (each part the bf16 rounding of what the
//             previous ones leave; for an FP32 x the three carry all 24 bits,
//             so the split is exact), and a*b is taken as the six products
//             hi_a hi_b + hi_a mid_b + mid_a hi_b + hi_a lo_b + mid_a mid_b +
//             lo_a hi_b on v_mfma_f32_16x16x32_bf16 with FP32 accumulation;
//             the dropped terms are below 2^-22 of |a b|.  The instruction
//             itself adds each group of eight k-products after aligning them
//             to the largest and drops the bits below its 24-bit precision
//             (probed on gfx950; its addition of the accumulator rounds to
//             nearest), so a group sum can lose up to about seven units of
//             2^-24 of its largest product: the accuracy ends near 2^-21 of
//             the largest product, not at the FP32 rounding;
//   BF16X2    two parts, x ~ hi + lo, three products hi hi + hi lo + lo hi
//             (about 2^-16 relative: a faster, less accurate variant).
//
// All use one "transposing" product form,
//
//   out[x + X*i] = alpha * sum_k M[i,k] W[k + n*x]  (+ beta * Y[x + X*i]),
//
// i.e. the input fibres are contiguous and the output is written with the
// fibre index fastest.  Chaining d of these rotates the tensor layout
// (n1,n2,n3) -> (n2,n3,n1) -> (n3,n1,n2) -> (n1,n2,n3): every product of the
// Tucker operator reads contiguous fibres and the last one writes the
// natural layout again.  The host drives the chain (run_tucker in adr_api).
//
// Fragment layouts (wave64, probed on gfx950): f32 16x16x4 takes A[l%16][l/16],
// B[l/16][l%16]; bf16 16x16x32 takes A[l%16][8(l/16)+j], B[8(l/16)+j][l%16],
// j = 0..7; both return D[4(l/16)+v][l%16], v = 0..3.
#include <algorithm>

#include "common.h"

namespace adr {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));

typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

// float -> bf16 bits, round to nearest even (the conversion instruction; on
// gfx950 it gives the same bits as rounding the FP32 bit pattern to nearest
// even, denormals included, checked over 2^24 finite values)
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  return __builtin_bit_cast(unsigned short, static_cast<__bf16>(x));
}
__device__ __forceinline__ float bf16_float(unsigned short b) {
  return __uint_as_float((unsigned)b << 16);
}

struct LowpArgs {
  const float* W[kMaxGroup];     // inputs, n x X column-major (fibres contiguous)
  const float* M[kMaxGroup];     // FP32: n x n column-major
  // split BF16: the parts of M (hi, mid, lo) as transposed planes, k fastest
  const unsigned short* Mp[kMaxGroup][3];
  void* out[kMaxGroup];          // FP32 (rotated) or FP64 (last product)
  const double* Y[kMaxGroup];    // FP64 addend for the last product, may alias out
  const float* Z[kMaxGroup];     // FP32 second addend of the last product, or null
  double alpha, beta;
  int n;
  unsigned X;
  int group;
};

constexpr int kThreads = 256;
constexpr int kOutF32 = 0, kOutF64 = 1;   // output of the wide kernel

// the product g of a single launch as a job
__device__ __forceinline__ LowpJob job_of(const LowpArgs& a, int g) {
  LowpJob j;
  j.W = a.W[g];
  j.M = a.M[g];
  j.out = a.out[g];
  j.Y = a.Y[g];
  j.Z = a.Z[g];
  j.alpha = a.alpha;
  j.beta = a.beta;
  j.n = a.n;
  j.X = a.X;
  j.out_f64 = 0;
  j.n_itiles = 0;
  j.tile_begin = 0;
  return j;
}

// Epilogue of a wave's TI x TX block of D[i][x] (lane: rows 4*krow + v of each
// 16x16 block, column col).
//
// FP64 output (the last product of a chain): out = alpha*acc + beta*Y, or with
// a second addend Z, (beta*Y + Z) + alpha*acc -- the last product of
// reduced-precision ETD2RKds writes C_{n+1} = (C_n + D1) + D2 in place of C_n
// without storing D2.  Y may alias out (each element is read, then written, by
// the same lane), so the addends of strip fx + 1 are loaded, in program order,
// before the results of strip fx are stored: one memory wait per strip, with
// the next strip's loads in flight.  Loads use clamped indices (no branches);
// only stores outside the tensor are masked, and a wave tile that lies wholly
// inside it skips the masks.
// NBUF = 1 loads each strip's addends just before its stores (fewer registers).
template <int FI, int FX, bool HASY, bool HASZ, bool GUARD, int NBUF = 2>
__device__ __forceinline__ void tgemm_epilogue64(const LowpJob& a, const f4 (&acc)[FI][FX], int ib,
                                                 unsigned xb, int col, int krow) {
  const int n = a.n;
  const unsigned X = (unsigned)a.X;
  const double alpha = a.alpha, beta = a.beta;
  const double* Y = a.Y;
  const float* Z = a.Z;
  double* out = static_cast<double*>(a.out);
  double y[NBUF][FI][4];
  float z[NBUF][FI][4];
  // outside the tensor the loads read a clamped (valid, lane-varying) element
  auto index = [&](int fx, int fi, int v, bool& ok) {
    unsigned x = xb + fx * 16 + col;
    int i = ib + fi * 16 + 4 * krow + v;
    ok = !GUARD || (x < X && i < n);
    if (GUARD) {
      x = min(x, X - 1);
      i = min(i, n - 1);
    }
    return x + X * (unsigned)i;
  };
  auto load_strip = [&](int fx) {
#pragma unroll
    for (int fi = 0; fi < FI; ++fi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        bool ok;
        const unsigned o = index(fx, fi, v, ok);
        if (HASY) y[fx % NBUF][fi][v] = Y[o];
        if (HASZ) z[fx % NBUF][fi][v] = Z[o];
      }
  };
  if (NBUF == 2) load_strip(0);
#pragma unroll
  for (int fx = 0; fx < FX; ++fx) {
    if (NBUF == 1) load_strip(fx);
    else if (fx + 1 < FX) load_strip(fx + 1);
#pragma unroll
    for (int fi = 0; fi < FI; ++fi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        bool ok;
        const unsigned o = index(fx, fi, v, ok);
        const double p = alpha * (double)acc[fi][fx][v];
        double val = p;
        if (HASZ) val = ((HASY ? beta * y[fx % NBUF][fi][v] : 0.0) + (double)z[fx % NBUF][fi][v]) + p;
        else if (HASY) val = p + beta * y[fx % NBUF][fi][v];
        if (ok) out[o] = val;
      }
  }
}

template <int FI, int FX, int TI, int TX, bool OUT64, int NBUF = 2>
__device__ __forceinline__ void tgemm_epilogue(const LowpJob& a, const f4 (&acc)[FI][FX],
                                               int ib, unsigned xb, int col, int krow) {
  const int n = a.n;
  const unsigned X = (unsigned)a.X;
  if (OUT64) {
    // ib and xb are the same in every lane of the wave: a scalar branch
    const bool inside = __builtin_amdgcn_readfirstlane((int)(ib + TI <= n && xb + TX <= X)) != 0;
    const bool hy = a.Y != nullptr, hz = a.Z != nullptr;
    if (inside) {
      if (hz) {
        if (hy) tgemm_epilogue64<FI, FX, true, true, false, NBUF>(a, acc, ib, xb, col, krow);
        else tgemm_epilogue64<FI, FX, false, true, false, NBUF>(a, acc, ib, xb, col, krow);
      } else if (hy) {
        tgemm_epilogue64<FI, FX, true, false, false, NBUF>(a, acc, ib, xb, col, krow);
      } else {
        tgemm_epilogue64<FI, FX, false, false, false, NBUF>(a, acc, ib, xb, col, krow);
      }
    } else {
      if (hz) {
        if (hy) tgemm_epilogue64<FI, FX, true, true, true, NBUF>(a, acc, ib, xb, col, krow);
        else tgemm_epilogue64<FI, FX, false, true, true, NBUF>(a, acc, ib, xb, col, krow);
      } else if (hy) {
        tgemm_epilogue64<FI, FX, true, false, true, NBUF>(a, acc, ib, xb, col, krow);
      } else {
        tgemm_epilogue64<FI, FX, false, false, true, NBUF>(a, acc, ib, xb, col, krow);
      }
    }
    return;
  }
  const double alpha = a.alpha;
  float* out = static_cast<float*>(a.out);
#pragma unroll
  for (int fx = 0; fx < FX; ++fx) {
    const unsigned x = xb + fx * 16 + col;
    const bool xok = x < X;
#pragma unroll
    for (int fi = 0; fi < FI; ++fi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = ib + fi * 16 + 4 * krow + v;
        if (xok && i < n) out[x + X * (unsigned)i] = (float)(alpha * (double)acc[fi][fx][v]);
      }
  }
}

// ------------------------------------------------------------------ FP32
// Tile: BI rows i x BX fibres x, BK = 16 per chunk, four waves in a 2x2 grid.
// The single-launch kernel and the grouped kernel (one LowpJob per product)
// both call this.  VEC (n % 4 == 0, 16-byte aligned operands): every lane
// moves four consecutive floats per load and per LDS store.
// LDS row pads (PADI, PADK, PADB below) are the fastest of a sweep at 256^3.
template <int BI, int BX, bool OUT64, bool VEC, int PADI = 4, int PADK = 4, int WI = 2, int WX = 2>
__device__ __forceinline__ void tgemm_f32_tile(const LowpJob& job, int itile, int xtile) {
  constexpr int BK = 16;
  constexpr int kThreads = 64 * WI * WX;
  constexpr int TI = BI / WI, TX = BX / WX, FI = TI / 16, FX = TX / 16;
  constexpr int LDI = BI + PADI;             // [k][i] rows
  constexpr int LDK = VEC ? BK + PADK : BK + 1;  // [x][k] rows: 16-byte aligned or odd pitch
  // scalar mapping
  constexpr int MROWS = kThreads / BI, MLOADS = BK / MROWS;
  constexpr int XSTEP = kThreads / BK, WLOADS = BX / XSTEP;
  static_assert(MROWS * BI == kThreads && XSTEP * BK == kThreads, "mapping");
  // vector mapping: M rows of BI/4 lanes, W fibres of BK/4 lanes
  constexpr int MV = BI / 4, MVROWS = kThreads / MV, MVLOADS = BK / MVROWS;
  constexpr int WV = BK / 4, WVSTEP = kThreads / WV, WVLOADS = BX / WVSTEP;
  static_assert(MVROWS * MV == kThreads && MVLOADS * MVROWS == BK, "M vector mapping");
  static_assert(WVSTEP * WV == kThreads && WVLOADS * WVSTEP == BX, "W vector mapping");
  __shared__ float sM[2][BK * LDI];
  __shared__ float sW[2][BX * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave / WX, wx = wave % WX;
  const int n = job.n;
  const unsigned X = (unsigned)job.X;
  const int i0 = itile * BI;
  const unsigned x0 = (unsigned)xtile * BX;
  const float* __restrict__ W = job.W;
  const float* __restrict__ M = job.M;

  const int m_i = tid % BI, m_k0 = tid / BI;
  const int w_k = tid % BK, w_x0 = tid / BK;
  const int mv_i = 4 * (tid % MV), mv_k0 = tid / MV;
  const int wv_k = 4 * (tid % WV), wv_x0 = tid / WV;
  float rm[MLOADS], rw[WLOADS];
  f4 vm[MVLOADS], vw[WVLOADS];
  auto load = [&](int k0) {
    if (VEC) {
#pragma unroll
      for (int p = 0; p < MVLOADS; ++p) {
        const int i = i0 + mv_i, k = k0 + mv_k0 + p * MVROWS;
        const bool ok = i < n && k < n;
        vm[p] = *reinterpret_cast<const f4*>(M + (ok ? (unsigned)i + (unsigned)n * (unsigned)k : 0u));
      }
#pragma unroll
      for (int p = 0; p < WVLOADS; ++p) {
        const unsigned x = x0 + wv_x0 + p * WVSTEP;
        const int k = k0 + wv_k;
        const bool ok = x < X && k < n;
        vw[p] = *reinterpret_cast<const f4*>(W + (ok ? x * (unsigned)n + (unsigned)k : 0u));
      }
      return;
    }
#pragma unroll
    for (int p = 0; p < MLOADS; ++p) {
      const int i = i0 + m_i, k = k0 + m_k0 + p * MROWS;
      const bool ok = i < n && k < n;
      rm[p] = M[ok ? (unsigned)i + (unsigned)n * (unsigned)k : 0u];
    }
#pragma unroll
    for (int p = 0; p < WLOADS; ++p) {
      const unsigned x = x0 + w_x0 + p * XSTEP;
      const int k = k0 + w_k;
      const bool ok = x < X && k < n;
      rw[p] = W[ok ? x * (unsigned)n + (unsigned)k : 0u];
    }
  };
  auto store = [&](int buf, int k0) {
    if (VEC) {
      const f4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int p = 0; p < MVLOADS; ++p) {
        const bool ok = (i0 + mv_i) < n && (k0 + mv_k0 + p * MVROWS) < n;
        *reinterpret_cast<f4*>(&sM[buf][(mv_k0 + p * MVROWS) * LDI + mv_i]) = ok ? vm[p] : z;
      }
#pragma unroll
      for (int p = 0; p < WVLOADS; ++p) {
        const bool ok = (x0 + wv_x0 + p * WVSTEP) < X && (k0 + wv_k) < n;
        *reinterpret_cast<f4*>(&sW[buf][(wv_x0 + p * WVSTEP) * LDK + wv_k]) = ok ? vw[p] : z;
      }
      return;
    }
#pragma unroll
    for (int p = 0; p < MLOADS; ++p) {
      const bool ok = (i0 + m_i) < n && (k0 + m_k0 + p * MROWS) < n;
      sM[buf][(m_k0 + p * MROWS) * LDI + m_i] = ok ? rm[p] : 0.0f;
    }
#pragma unroll
    for (int p = 0; p < WLOADS; ++p) {
      const bool ok = (x0 + w_x0 + p * XSTEP) < X && (k0 + w_k) < n;
      sW[buf][(w_x0 + p * XSTEP) * LDK + w_k] = ok ? rw[p] : 0.0f;
    }
  };

  f4 acc[FI][FX];
#pragma unroll
  for (int fi = 0; fi < FI; ++fi)
#pragma unroll
    for (int fx = 0; fx < FX; ++fx) acc[fi][fx] = f4{0.f, 0.f, 0.f, 0.f};
  const int nchunks = (n + BK - 1) / BK;
  load(0);
  store(0, 0);
  __syncthreads();
  const int col = lane & 15, krow = lane >> 4;
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunks) load((c + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + krow;
      float af[FI], bfr[FX];
#pragma unroll
      for (int fi = 0; fi < FI; ++fi) af[fi] = sM[buf][kr * LDI + wi * TI + fi * 16 + col];
#pragma unroll
      for (int fx = 0; fx < FX; ++fx) bfr[fx] = sW[buf][(wx * TX + fx * 16 + col) * LDK + kr];
#pragma unroll
      for (int fi = 0; fi < FI; ++fi)
#pragma unroll
        for (int fx = 0; fx < FX; ++fx)
          acc[fi][fx] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[fi], bfr[fx], acc[fi][fx], 0, 0, 0);
    }
    if (c + 1 < nchunks) store(buf ^ 1, (c + 1) * BK);
    __syncthreads();
  }
  // D[i][x]: lane holds rows i = 4*krow + v, column x = col
  tgemm_epilogue<FI, FX, TI, TX, OUT64>(job, acc, i0 + wi * TI, x0 + wx * TX, col, krow);
}

template <int BI, int BX, bool OUT64, bool VEC, int PADI = 4, int PADK = 4, int WI = 2, int WX = 2>
__global__ __launch_bounds__(64 * WI * WX, 2) void k_tgemm_f32(LowpArgs a, int n_itiles,
                                                              int n_xtiles) {
  const int G = gridDim.x, b = blockIdx.x;
  int t = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const int itile = t % n_itiles;
  t /= n_itiles;
  const int xtile = t % n_xtiles;
  const int g = t / n_xtiles;
  tgemm_f32_tile<BI, BX, OUT64, VEC, PADI, PADK, WI, WX>(job_of(a, g), itile, xtile);
}

// Grouped FP32 products with FP32 outputs (one LowpJob per product, binary
// search over the sorted tile offsets).
template <int BI, int BX, bool VEC>
__global__ __launch_bounds__(kThreads, 2) void k_tgemm_f32_grouped(const LowpJob* __restrict__ jobs,
                                                                  int njobs) {
  const long long t = xcd_tile(blockIdx.x, gridDim.x);
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
  }
  const LowpJob job = jobs[lo];
  const long long local = t - job.tile_begin;
  tgemm_f32_tile<BI, BX, false, VEC>(job, (int)(local % job.n_itiles), (int)(local / job.n_itiles));
}

// ------------------------------------------------------------------ split BF16
// Split of FP32 values into PARTS bf16 parts: each part is the bf16 rounding
// (to nearest even) of what the previous parts leave.  The remainders are
// exact FP32 differences; with three parts the last one is exactly
// representable, so hi + mid + lo == x.  Two values at a time through the
// packed conversion: part[p] holds the p-th parts of x0 (low half) and x1
// (high half).
template <int PARTS>
__device__ __forceinline__ void split_bf16_pair(float x0, float x1, unsigned (&part)[PARTS]) {
  float r0 = x0, r1 = x1;
#pragma unroll
  for (int p = 0; p < PARTS; ++p) {
    const unsigned b = __builtin_bit_cast(unsigned, __builtin_convertvector(f2{r0, r1}, bf2));
    part[p] = b;
    if (p + 1 < PARTS) {
      r0 = r0 - __uint_as_float(b << 16);
      r1 = r1 - __uint_as_float(b & 0xffff0000u);
    }
  }
}

// Split eight consecutive FP32 values into PARTS vectors of eight bf16.
template <int PARTS>
__device__ __forceinline__ void split_bf16_8(const float (&x)[8], s8 (&v)[PARTS]) {
  u4 w[PARTS];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    unsigned part[PARTS];
    split_bf16_pair<PARTS>(x[2 * j], x[2 * j + 1], part);
#pragma unroll
    for (int pp = 0; pp < PARTS; ++pp) w[pp][j] = part[pp];
  }
#pragma unroll
  for (int pp = 0; pp < PARTS; ++pp) v[pp] = __builtin_bit_cast(s8, w[pp]);
}

// One 16x16 block of the split product over a 32-deep chunk: the products of
// parts (pa, pb) with pa + pb < PARTS, the smallest first.
template <int PARTS>
__device__ __forceinline__ f4 split_mfma(const s8 (&a)[PARTS], const s8 (&b)[PARTS], f4 acc) {
  if constexpr (PARTS == 3) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], acc, 0, 0, 0);
  }
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], acc, 0, 0, 0);
}

// Generic tiles: BI rows i x BX fibres, BK = 32 (one bf16 MFMA depth) per
// chunk, one tile per workgroup, bounds-checked unless FULL.  The W chunk is
// loaded as FP32 (eight consecutive k per lane), split and stored k-fastest;
// M arrives pre-split and transposed (k fastest).  Each LDS row holds 32 bf16
// (four 16-byte quads) and quad q of row r sits in slot q ^ ((r >> 1) & 3),
// so the rows of a fragment read spread over the banks.  NBUF = 2: two chunk
// buffers, one barrier per chunk; NBUF = 1: one buffer (the chunk after next
// waits in registers), two barriers per chunk, and half the LDS, so that more
// workgroups share a CU and overlap each other's phases.
template <int BI, int BX, bool OUT64, bool FULL, int PARTS, int NBUF = 2, int WI = 2, int WX = 2>
__global__ __launch_bounds__(64 * WI * WX, 2) void k_tgemm_bf16s(LowpArgs a, int n_itiles,
                                                                int n_xtiles) {
  constexpr int BK = 32;
  constexpr int kThreads = 64 * WI * WX;
  constexpr int TI = BI / WI, TX = BX / WX, FI = TI / 16, FX = TX / 16;
  constexpr int LDK = BK;                    // bf16 elements per row
  constexpr int MSEG = BI * (BK / 8);        // 8-element segments of the M chunk
  constexpr int WSEG = BX * (BK / 8);
  constexpr int MLOADS = MSEG / kThreads, WLOADS = WSEG / kThreads;
  static_assert(MLOADS * kThreads == MSEG && WLOADS * kThreads == WSEG, "mapping");
  static_assert(TI % 16 == 0 && TX % 16 == 0, "fragment rows keep their low four bits");
  __shared__ unsigned short sM[NBUF][PARTS][BI * LDK];
  __shared__ unsigned short sW[NBUF][PARTS][BX * LDK];
  auto slot = [](int r, int q) { return 8 * (q ^ ((r >> 1) & 3)); };

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave / WX, wx = wave % WX;
  const int G = gridDim.x, b = blockIdx.x;
  int t = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const int itile = t % n_itiles;
  t /= n_itiles;
  const int xtile = t % n_xtiles;
  const int g = t / n_xtiles;
  const int n = a.n;
  const unsigned X = a.X;
  const int i0 = itile * BI;
  const unsigned x0 = (unsigned)xtile * BX;
  const float* __restrict__ W = a.W[g];

  // segment s of a chunk: row r = s / 4 (i or x), k-group q = s % 4 (8 k-values)
  s8 rm[MLOADS][PARTS];
  float rw[WLOADS][8];
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < MLOADS; ++p) {
      const int s = tid + p * kThreads, r = s >> 2, q = s & 3;
      const int i = i0 + r, k = k0 + 8 * q;
#pragma unroll
      for (int pp = 0; pp < PARTS; ++pp) {
        const unsigned short* __restrict__ Mp = a.Mp[g][pp];
        if (FULL) {  // whole tile in range, 16-byte aligned rows
          rm[p][pp] = *reinterpret_cast<const s8*>(Mp + (unsigned)i * (unsigned)n + (unsigned)k);
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const bool ok = i < n && (k + j) < n;
            const unsigned idx = ok ? (unsigned)i * (unsigned)n + (unsigned)(k + j) : 0u;
            rm[p][pp][j] = ok ? (short)Mp[idx] : (short)0;
          }
        }
      }
    }
#pragma unroll
    for (int p = 0; p < WLOADS; ++p) {
      const int s = tid + p * kThreads, r = s >> 2, q = s & 3;
      const unsigned x = x0 + r;
      const int k = k0 + 8 * q;
      if (FULL) {
        const f4* src = reinterpret_cast<const f4*>(W + x * (unsigned)n + (unsigned)k);
        const f4 lo4 = src[0], hi4 = src[1];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          rw[p][j] = lo4[j];
          rw[p][4 + j] = hi4[j];
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const bool ok = x < X && (k + j) < n;
          rw[p][j] = ok ? W[x * (unsigned)n + (unsigned)(k + j)] : 0.0f;
        }
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < MLOADS; ++p) {
      const int s = tid + p * kThreads, r = s >> 2, q = s & 3;
#pragma unroll
      for (int pp = 0; pp < PARTS; ++pp)
        *reinterpret_cast<s8*>(&sM[buf][pp][r * LDK + slot(r, q)]) = rm[p][pp];
    }
#pragma unroll
    for (int p = 0; p < WLOADS; ++p) {
      const int s = tid + p * kThreads, r = s >> 2, q = s & 3;
      s8 v[PARTS];
      split_bf16_8<PARTS>(rw[p], v);
#pragma unroll
      for (int pp = 0; pp < PARTS; ++pp)
        *reinterpret_cast<s8*>(&sW[buf][pp][r * LDK + slot(r, q)]) = v[pp];
    }
  };

  f4 acc[FI][FX];
#pragma unroll
  for (int fi = 0; fi < FI; ++fi)
#pragma unroll
    for (int fx = 0; fx < FX; ++fx) acc[fi][fx] = f4{0.f, 0.f, 0.f, 0.f};
  const int nchunks = (n + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  const int col = lane & 15, kq = lane >> 4;
  const int frag = slot(col, kq);   // the rows read below keep col as their low four bits
  for (int c = 0; c < nchunks; ++c) {
    const int buf = NBUF == 2 ? (c & 1) : 0;
    if (c + 1 < nchunks) load((c + 1) * BK);
    s8 af[FI][PARTS];
#pragma unroll
    for (int fi = 0; fi < FI; ++fi) {
      const int r = wi * TI + fi * 16 + col;
#pragma unroll
      for (int pp = 0; pp < PARTS; ++pp)
        af[fi][pp] = *reinterpret_cast<const s8*>(&sM[buf][pp][r * LDK + frag]);
    }
#pragma unroll
    for (int fx = 0; fx < FX; ++fx) {
      const int r = wx * TX + fx * 16 + col;
      s8 bf[PARTS];
#pragma unroll
      for (int pp = 0; pp < PARTS; ++pp)
        bf[pp] = *reinterpret_cast<const s8*>(&sW[buf][pp][r * LDK + frag]);
#pragma unroll
      for (int fi = 0; fi < FI; ++fi) acc[fi][fx] = split_mfma<PARTS>(af[fi], bf, acc[fi][fx]);
    }
    if (NBUF == 1) __syncthreads();   // every wave is done with the buffer
    if (c + 1 < nchunks) store(NBUF == 2 ? (buf ^ 1) : 0);
    __syncthreads();
  }
  tgemm_epilogue<FI, FX, TI, TX, OUT64>(job_of(a, g), acc, i0 + wi * TI, x0 + wx * TX, col, kq);
}

// The split product with the operands' roles exchanged: A is the W fragment
// (its rows are fibres x), B the M fragment (its columns are rows i), so the
// block holds out^T and a lane ends with four consecutive fibres of one row.
// The parts are multiplied in split_mfma's order (pm, pw) = (2,0), (1,1), (0,2),
// (1,0), (0,1), (0,0): each of the 16 x 16 sums adds the same products in the
// same order as split_mfma(M, W) does.
template <int PARTS>
__device__ __forceinline__ f4 split_mfma_t(const s8 (&w)[PARTS], const s8 (&m)[PARTS], f4 acc) {
  if constexpr (PARTS == 3) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[0], m[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[1], m[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[2], m[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[0], m[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[1], m[0], acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[0], m[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[1], m[0], acc, 0, 0, 0);
  }
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[0], m[0], acc, 0, 0, 0);
}

// Epilogue of a wave's 64 x 64 block in the exchanged layout: acc[fx][fi][v] is
// out[x + X i] with x = xb + 16 fx + 4 krow + v, i = ib + 16 fi + col, so each
// lane writes four consecutive elements of a row: 16 bytes of FP32 or 32 bytes
// of FP64.  The FP64 form reads its addends the same way (Y may alias out:
// every element is read and then written by one lane), the loads of the next
// 16 x 16 block issued before the stores of this one.
template <int OUTK, int PARTS, bool HASY, bool HASZ>
__device__ __forceinline__ void wide_epilogue(const LowpArgs& a, int g, const f4 (&acc)[4][4],
                                              int ib, unsigned xb, int col, int krow) {
  constexpr int FX = 4, FI = 4;
  const unsigned X = a.X;
  const double alpha = a.alpha;
  auto index = [&](int fx, int fi) {
    return xb + (unsigned)(fx * 16 + 4 * krow) + X * (unsigned)(ib + fi * 16 + col);
  };
  if constexpr (OUTK == kOutF32) {
    float* out = static_cast<float*>(a.out[g]);
#pragma unroll
    for (int fx = 0; fx < FX; ++fx)
#pragma unroll
      for (int fi = 0; fi < FI; ++fi) {
        f4 o;
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] = (float)(alpha * (double)acc[fx][fi][v]);
        *reinterpret_cast<f4*>(out + index(fx, fi)) = o;
      }
  } else {
    typedef double d2 __attribute__((ext_vector_type(2)));
    double* out = static_cast<double*>(a.out[g]);
    const double* Y = a.Y[g];
    const float* Z = a.Z[g];
    const double beta = a.beta;
    // the addends of kDepth blocks ahead are in flight while a block is
    // combined and stored
    constexpr int kDepth = 4, kRing = kDepth + 1;
    d2 y[kRing][2];
    f4 z[kRing];
    // block b = (fx, fi) = (b / FI, b % FI)
    auto load = [&](int b) {
      const unsigned o = index(b / FI, b % FI);
      if (HASY) {
        y[b % kRing][0] = *reinterpret_cast<const d2*>(Y + o);
        y[b % kRing][1] = *reinterpret_cast<const d2*>(Y + o + 2);
      }
      if (HASZ) z[b % kRing] = *reinterpret_cast<const f4*>(Z + o);
    };
#pragma unroll
    for (int b = 0; b < kDepth && b < FX * FI; ++b) load(b);
#pragma unroll
    for (int b = 0; b < FX * FI; ++b) {
      if (b + kDepth < FX * FI) load(b + kDepth);
      const int fx = b / FI, fi = b % FI;
      double val[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double p = alpha * (double)acc[fx][fi][v];
        const double yv = HASY ? y[b % kRing][v / 2][v % 2] : 0.0;
        if (HASZ) val[v] = ((HASY ? beta * yv : 0.0) + (double)z[b % kRing][v]) + p;
        else if (HASY) val[v] = p + beta * yv;
        else val[v] = p;
      }
      const unsigned o = index(fx, fi);
      *reinterpret_cast<d2*>(out + o) = d2{val[0], val[1]};
      *reinterpret_cast<d2*>(out + o + 2) = d2{val[2], val[3]};
    }
  }
}

// LDS-direct copy of SPANS x 16 rows of a 32-deep chunk of PARTS bf16 planes:
// rows row0 + R0 + (0 .. 16 SPANS - 1) (row stride n, elements k0 .. k0 + 31)
// into LDS rows R0 onward (64 bytes each, quad q of row r in slot
// q ^ ((r >> 1) & 3)).  Lane l fills row R0 + 16 h + l / 4, slot l % 4, with the
// quad that slot holds; one wave instruction fills one 1 KB span.
template <int PARTS, int PLANE, int SPANS>
__device__ __forceinline__ void dma_split_rows(unsigned short* dst,
                                               const unsigned short* const* planes,
                                               unsigned row0, int n, int k0, int R0) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int h = 0; h < SPANS; ++h) {
    const int Rh = R0 + 16 * h;
    const int r = Rh + (lane >> 2);
    const int q = (lane & 3) ^ ((r >> 1) & 3);
    const unsigned src = (row0 + (unsigned)r) * (unsigned)n + (unsigned)(k0 + 8 * q);
#pragma unroll
    for (int pp = 0; pp < PARTS; ++pp)
      __builtin_amdgcn_global_load_lds(planes[pp] + src, dst + pp * PLANE + Rh * 32, 16, 0, 0);
  }
}

// Wide tiles for evenly tiled shapes (n % 256 == 0, X % 128 == 0): 256 rows x
// 128 fibres per workgroup, eight waves in a 4 x 2 grid of 64 x 64 wave
// tiles, one workgroup per CU walking the tiles of the launch (persistent:
// tile b, b + G, ...).  Two chunk buffers of PARTS bf16 planes each (three
// parts: 96 KB of M, 48 KB of W).  The M planes arrive pre-split and go from
// global memory straight into LDS (global_load_lds, lane l writing bytes
// 16 l onward of the wave's 1 KB span); W arrives as FP32, is split in
// registers and stored.  Each LDS row
// holds 32 bf16 (four 16-byte quads), and quad q of row r sits in slot
// q ^ ((r >> 1) & 3): the eight rows a fragment read puts in one 128-byte bank
// window then use all eight 16-byte slots.  The next chunk (of this tile, or
// the first of the next) is in flight while the current one is multiplied;
// the two buffers are distinct LDS objects and the chunk loop is unrolled by
// two, so the loads into one buffer are waited for only at the barrier.  The
// output is FP32 or FP64 with the addends (OUTK).
template <int PARTS, int OUTK>
__global__ __launch_bounds__(512, 1) void k_tgemm_bf16s_wide(LowpArgs a, int n_itiles,
                                                            int n_xtiles, int ntiles) {
  constexpr int BI = 256, BX = 128, BK = 32, WX = 2;
  constexpr int TI = 64, TX = 64, FI = TI / 16, FX = TX / 16;
  constexpr int PLANE_M = BI * BK, PLANE_W = BX * BK;   // bf16 elements per plane
  __shared__ __attribute__((aligned(16))) unsigned short sM0[PARTS * PLANE_M];
  __shared__ __attribute__((aligned(16))) unsigned short sM1[PARTS * PLANE_M];
  __shared__ __attribute__((aligned(16))) unsigned short sW0[PARTS * PLANE_W];
  __shared__ __attribute__((aligned(16))) unsigned short sW1[PARTS * PLANE_W];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave / WX, wx = wave % WX;
  const int n = a.n;
  const int nchunks = n / BK;              // even: n % 256 == 0
  const int G = gridDim.x;

  struct Tile {
    int g, i0;
    unsigned x0;
  };
  auto tile_of = [&](int t) {
    Tile T;
    T.i0 = (t % n_itiles) * BI;
    t /= n_itiles;
    T.x0 = (unsigned)(t % n_xtiles) * BX;
    T.g = t / n_xtiles;
    return T;
  };

  // M chunk: per part 256 rows x 64 bytes = 16 spans of 1 KB (16 rows each);
  // wave w fills rows 32 w .. 32 w + 31.
  auto dma_m = [&](unsigned short* dst, const Tile& T, int k0) {
    const unsigned short* planes[PARTS];
#pragma unroll
    for (int pp = 0; pp < PARTS; ++pp) planes[pp] = a.Mp[T.g][pp];
    dma_split_rows<PARTS, PLANE_M, 2>(dst, planes, (unsigned)T.i0, n, k0, 32 * wave);
  };
  // half h (16 rows) of the wave's share of an M chunk
  auto dma_m_half = [&](unsigned short* dst, const Tile& T, int k0, int h) {
    const unsigned short* planes[PARTS];
#pragma unroll
    for (int pp = 0; pp < PARTS; ++pp) planes[pp] = a.Mp[T.g][pp];
    dma_split_rows<PARTS, PLANE_M, 1>(dst, planes, (unsigned)T.i0, n, k0, 32 * wave + 16 * h);
  };
  // FP32 W chunk: 128 fibres x 32 k; thread t takes fibre t / 4, k-quad t % 4
  const int w_x = tid >> 2, w_q = tid & 3;
  const int w_slot = w_q ^ ((w_x >> 1) & 3);
  f4 rw0, rw1;
  auto load_w = [&](const Tile& T, int k0) {
    const f4* src = reinterpret_cast<const f4*>(a.W[T.g] + (T.x0 + (unsigned)w_x) * (unsigned)n +
                                                (unsigned)(k0 + 8 * w_q));
    rw0 = src[0];
    rw1 = src[1];
  };
  auto store_w = [&](unsigned short* dst) {
    const float x[8] = {rw0[0], rw0[1], rw0[2], rw0[3], rw1[0], rw1[1], rw1[2], rw1[3]};
    s8 v[PARTS];
    split_bf16_8<PARTS>(x, v);
#pragma unroll
    for (int pp = 0; pp < PARTS; ++pp)
      *reinterpret_cast<s8*>(dst + pp * PLANE_W + w_x * BK + 8 * w_slot) = v[pp];
  };

  // fragment reads: row r (low four bits = lane % 16), quad lane / 16
  const int col = lane & 15, kq = lane >> 4;
  const int frag_off = 8 * (kq ^ ((col >> 1) & 3));
  f4 acc[FX][FI];
  s8 mf[FI][PARTS];
  auto read_mf = [&](const unsigned short* cm) {
#pragma unroll
    for (int fi = 0; fi < FI; ++fi)
#pragma unroll
      for (int pp = 0; pp < PARTS; ++pp)
        mf[fi][pp] = *reinterpret_cast<const s8*>(cm + pp * PLANE_M +
                                                  (wi * TI + fi * 16 + col) * BK + frag_off);
  };
  // the products of block column fx (with the M fragments of read_mf)
  auto compute_fx = [&](const unsigned short* cw, int fx) {
    s8 wf[PARTS];
#pragma unroll
    for (int pp = 0; pp < PARTS; ++pp)
      wf[pp] = *reinterpret_cast<const s8*>(cw + pp * PLANE_W +
                                            (wx * TX + fx * 16 + col) * BK + frag_off);
#pragma unroll
    for (int fi = 0; fi < FI; ++fi) acc[fx][fi] = split_mfma_t<PARTS>(wf, mf[fi], acc[fx][fi]);
  };
  auto epilogue = [&](const Tile& T) {
    const int ib = T.i0 + wi * TI;
    const unsigned xb = T.x0 + wx * TX;
    if constexpr (OUTK == kOutF64) {
      const bool hy = a.Y[T.g] != nullptr, hz = a.Z[T.g] != nullptr;
      if (hz) {
        if (hy) wide_epilogue<OUTK, PARTS, true, true>(a, T.g, acc, ib, xb, col, kq);
        else wide_epilogue<OUTK, PARTS, false, true>(a, T.g, acc, ib, xb, col, kq);
      } else if (hy) {
        wide_epilogue<OUTK, PARTS, true, false>(a, T.g, acc, ib, xb, col, kq);
      } else {
        wide_epilogue<OUTK, PARTS, false, false>(a, T.g, acc, ib, xb, col, kq);
      }
    } else {
      wide_epilogue<OUTK, PARTS, false, false>(a, T.g, acc, ib, xb, col, kq);
    }
  };

  int t = blockIdx.x;
  if (t >= ntiles) return;
  Tile cur = tile_of(t);
  dma_m(sM0, cur, 0);
  load_w(cur, 0);
  store_w(sW0);
  __syncthreads();
  while (true) {
    const int tn = t + G;
    const bool next_tile = tn < ntiles;
    const Tile nxt = tile_of(next_tile ? tn : t);
#pragma unroll
    for (int fx = 0; fx < FX; ++fx)
#pragma unroll
      for (int fi = 0; fi < FI; ++fi) acc[fx][fi] = f4{0.f, 0.f, 0.f, 0.f};
    // Chunk c from (cm, cw); the next chunk goes into (nm, nw).  Its loads
    // are spread over this chunk's products: issued
    // together after the barrier, every wave's would queue behind the others'
    // and hold back its first product.  W goes first (from HBM), the M copy
    // in two halves after the first and second block columns, and W is split
    // and stored before the last column.  Past the last chunk of the last
    // tile they reload this tile's first chunk into the free buffers, so the
    // step has no branches.
    auto step = [&](int c, const unsigned short* cm, const unsigned short* cw, unsigned short* nm,
                    unsigned short* nw) {
      const bool in_tile = c + 1 < nchunks;
      const Tile& T = (!in_tile && next_tile) ? nxt : cur;
      const int k0 = in_tile ? (c + 1) * BK : 0;
      load_w(T, k0);
      read_mf(cm);
      __builtin_amdgcn_sched_barrier(0);
      compute_fx(cw, 0);
      __builtin_amdgcn_sched_barrier(0);
      dma_m_half(nm, T, k0, 0);
      __builtin_amdgcn_sched_barrier(0);
      compute_fx(cw, 1);
      __builtin_amdgcn_sched_barrier(0);
      dma_m_half(nm, T, k0, 1);
      __builtin_amdgcn_sched_barrier(0);
      compute_fx(cw, 2);
      __builtin_amdgcn_sched_barrier(0);
      store_w(nw);
      __builtin_amdgcn_sched_barrier(0);
      compute_fx(cw, 3);
      __syncthreads();   // the next chunk has landed and nobody reads (cm, cw) any more
    };
    for (int c = 0; c < nchunks; c += 2) {
      step(c, sM0, sW0, sM1, sW1);
      step(c + 1, sM1, sW1, sM0, sW0);
    }
    epilogue(cur);
    if (!next_tile) break;
    t = tn;
    cur = nxt;
  }
}

// Split an FP64 n x n column-major matrix into PARTS transposed bf16 planes,
// P[p][i*n + k], with sum_p P[p][i*n + k] ~ M[i + n*k]: each part is the bf16
// rounding of the FP64 remainder the previous parts leave.
__global__ __launch_bounds__(256) void k_split_bf16(int n, int parts, const double* __restrict__ M,
                                                    unsigned short* __restrict__ P0,
                                                    unsigned short* __restrict__ P1,
                                                    unsigned short* __restrict__ P2) {
  const long long nn = (long long)n * n;
  unsigned short* const P[3] = {P0, P1, P2};
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nn;
       q += (long long)gridDim.x * blockDim.x) {
    const long long i = q / n, k = q % n;   // q = i*n + k
    double r = M[i + (long long)n * k];
    for (int p = 0; p < parts; ++p) {
      const unsigned short h = bf16_bits((float)r);
      P[p][q] = h;
      r -= (double)bf16_float(h);
    }
  }
}

int lowp_cu_count() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
  }
  return cus;
}

template <class K>
hipError_t launch_tiles(K kern, const LowpArgs& a, int BI, int BX, hipStream_t s) {
  const int n_itiles = (a.n + BI - 1) / BI;
  const long long n_xtiles = ((long long)a.X + BX - 1) / BX;
  const long long grid = (long long)a.group * n_itiles * n_xtiles;
  if (grid <= 0 || grid > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kThreads), 0, s, a, n_itiles, (int)n_xtiles);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tgemm_lowp(int precision, const void* const* W, const void* const* Mf32,
                             const SplitPlanes* Mp, void* const* out, const double* const* Y,
                             int group, int n, long long X, double alpha, double beta, int out_f64,
                             hipStream_t s, const float* const* Z) {
  if (group < 1 || group > kMaxGroup || X <= 0 || X >= (1LL << 31) ||
      (long long)n * X >= (1LL << 31) || (Z && !out_f64))
    return hipErrorInvalidValue;
  const int parts = precision == kLowpBF16X3 ? 3 : precision == kLowpBF16X2 ? 2 : 0;
  if (precision != kLowpF32 && parts == 0) return hipErrorInvalidValue;
  if (parts && !Mp) return hipErrorInvalidValue;
  LowpArgs a{};
  for (int g = 0; g < group; ++g) {
    a.W[g] = static_cast<const float*>(W[g]);
    a.M[g] = Mf32 ? static_cast<const float*>(Mf32[g]) : nullptr;
    for (int p = 0; p < 3; ++p) a.Mp[g][p] = (parts && p < parts) ? Mp[g].p[p] : nullptr;
    a.out[g] = out[g];
    a.Y[g] = Y ? Y[g] : nullptr;
    a.Z[g] = Z ? Z[g] : nullptr;
  }
  a.alpha = alpha;
  a.beta = beta;
  a.n = n;
  a.X = (unsigned)X;
  a.group = group;
  // 64-row tiles where 128-row ones would be ragged (n <= 64, or a multiple of
  // 64 but not of 128), or fewer than two per CU (measured, FP32 / split BF16:
  // 1024^2 59 / 31 us against 94 / 39; 128^3 18 / 11 against 19 / 12; at 256^3,
  // 2048 tiles, 128 rows stay ahead: 185 / 82 against 197 / 89)
  const long long tiles128 = (long long)group * ((n + 127) / 128) * ((X + 127) / 128);
  const bool rows64 = n <= 64 || (n % 128 != 0 && n % 64 == 0) || tiles128 < 2LL * lowp_cu_count();
  if (precision == kLowpF32) {
    // n % 4 == 0 with 16-byte aligned operands: four floats per lane per load
    bool vec = n % 4 == 0;
    for (int g = 0; g < group; ++g)
      vec = vec && (reinterpret_cast<uintptr_t>(W[g]) % 16 == 0) &&
            (reinterpret_cast<uintptr_t>(Mf32[g]) % 16 == 0);
    if (rows64) {
      if (vec)
        return out_f64 ? launch_tiles(k_tgemm_f32<64, 128, true, true>, a, 64, 128, s)
                       : launch_tiles(k_tgemm_f32<64, 128, false, true>, a, 64, 128, s);
      return out_f64 ? launch_tiles(k_tgemm_f32<64, 128, true, false>, a, 64, 128, s)
                     : launch_tiles(k_tgemm_f32<64, 128, false, false>, a, 64, 128, s);
    }
    if (vec)
      return out_f64 ? launch_tiles(k_tgemm_f32<128, 128, true, true>, a, 128, 128, s)
                     : launch_tiles(k_tgemm_f32<128, 128, false, true>, a, 128, 128, s);
    return out_f64 ? launch_tiles(k_tgemm_f32<128, 128, true, false>, a, 128, 128, s)
                   : launch_tiles(k_tgemm_f32<128, 128, false, false>, a, 128, 128, s);
  }
  // evenly tiled shapes with 16-byte aligned fibres and planes take the vectorised loads
  bool aligned = true;
  for (int g = 0; g < group; ++g) {
    aligned = aligned && (reinterpret_cast<uintptr_t>(W[g]) % 16 == 0);
    for (int p = 0; p < parts; ++p)
      aligned = aligned && (reinterpret_cast<uintptr_t>(Mp[g].p[p]) % 16 == 0);
  }
  // evenly tiled by 256 rows, two or three parts: the wide persistent tiles,
  // one workgroup per CU (measured at 256^3: three parts 109 us against 116 us
  // for the single-buffered 128 x 128 tiles below; two parts, with the loads
  // spread over the products, 79 against 82 us, bitwise equal); their epilogue
  // stores 16-byte pieces of out (and reads Y, Z so), which must then be
  // 16-byte aligned too
  bool wide = parts >= 2 && aligned && n % 256 == 0 && X % 128 == 0;
  for (int g = 0; wide && g < group; ++g)
    wide = reinterpret_cast<uintptr_t>(out[g]) % 16 == 0 &&
           !(Y && Y[g] && reinterpret_cast<uintptr_t>(Y[g]) % 16) &&
           !(Z && Z[g] && reinterpret_cast<uintptr_t>(Z[g]) % 16);
  if (wide) {
    const long long ntiles = (long long)group * (n / 256) * (X / 128);
    if (ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
    const int grid = (int)std::min<long long>(ntiles, lowp_cu_count());
    const int n_itiles = n / 256, n_xtiles = (int)(X / 128);
    if (parts == 2) {
      if (out_f64)
        hipLaunchKernelGGL((k_tgemm_bf16s_wide<2, kOutF64>), dim3(grid), dim3(512), 0, s, a,
                           n_itiles, n_xtiles, (int)ntiles);
      else
        hipLaunchKernelGGL((k_tgemm_bf16s_wide<2, kOutF32>), dim3(grid), dim3(512), 0, s, a,
                           n_itiles, n_xtiles, (int)ntiles);
    } else if (out_f64)
      hipLaunchKernelGGL((k_tgemm_bf16s_wide<3, kOutF64>), dim3(grid), dim3(512), 0, s, a,
                         n_itiles, n_xtiles, (int)ntiles);
    else
      hipLaunchKernelGGL((k_tgemm_bf16s_wide<3, kOutF32>), dim3(grid), dim3(512), 0, s, a,
                         n_itiles, n_xtiles, (int)ntiles);
    return hipGetLastError();
  }
  // evenly tiled by 128 (n not a multiple of 256) with enough tiles: 128 x 128
  // tiles with one LDS buffer, two workgroups per CU
  if (aligned && n % 128 == 0 && X % 128 == 0 && !rows64) {
    if (parts == 3)
      return out_f64 ? launch_tiles(k_tgemm_bf16s<128, 128, true, true, 3, 1>, a, 128, 128, s)
                     : launch_tiles(k_tgemm_bf16s<128, 128, false, true, 3, 1>, a, 128, 128, s);
    return out_f64 ? launch_tiles(k_tgemm_bf16s<128, 128, true, true, 2, 1>, a, 128, 128, s)
                   : launch_tiles(k_tgemm_bf16s<128, 128, false, true, 2, 1>, a, 128, 128, s);
  }
  // three parts take 64-row tiles (two workgroups per CU fit in LDS)
  if (rows64 || parts == 3) {
    const bool full = aligned && n % 64 == 0 && X % 128 == 0;
#define ADR_BF16S_64(P)                                                                          \
  (full ? (out_f64 ? launch_tiles(k_tgemm_bf16s<64, 128, true, true, P>, a, 64, 128, s)          \
                   : launch_tiles(k_tgemm_bf16s<64, 128, false, true, P>, a, 64, 128, s))        \
        : (out_f64 ? launch_tiles(k_tgemm_bf16s<64, 128, true, false, P>, a, 64, 128, s)         \
                   : launch_tiles(k_tgemm_bf16s<64, 128, false, false, P>, a, 64, 128, s)))
    return parts == 3 ? ADR_BF16S_64(3) : ADR_BF16S_64(2);
#undef ADR_BF16S_64
  }
  // ragged 128-row tiles (two parts), bounds-checked
  return out_f64 ? launch_tiles(k_tgemm_bf16s<128, 128, true, false, 2>, a, 128, 128, s)
                 : launch_tiles(k_tgemm_bf16s<128, 128, false, false, 2>, a, 128, 128, s);
}

hipError_t launch_tgemm_lowp_grouped(int precision, const LowpJob* jobs, int njobs,
                                     long long ntiles, bool vec, hipStream_t s) {
  if (precision != 1 || njobs <= 0 || ntiles <= 0 || ntiles > 0x7fffffffLL)
    return hipErrorInvalidValue;
  if (vec)
    hipLaunchKernelGGL((k_tgemm_f32_grouped<128, 128, true>), dim3((unsigned)ntiles),
                       dim3(kThreads), 0, s, jobs, njobs);
  else
    hipLaunchKernelGGL((k_tgemm_f32_grouped<128, 128, false>), dim3((unsigned)ntiles),
                       dim3(kThreads), 0, s, jobs, njobs);
  return hipGetLastError();
}

hipError_t launch_split_bf16(int n, int parts, const double* M, unsigned short* const* P,
                             hipStream_t s) {
  if (parts < 2 || parts > 3) return hipErrorInvalidValue;
  long long blocks = ((long long)n * n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)blocks), dim3(256), 0, s, n, parts, M, P[0], P[1],
                     parts == 3 ? P[2] : nullptr);
  return hipGetLastError();
}

}  // namespace adr
