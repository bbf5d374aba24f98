// Reduced-precision mu-mode products for the Tucker operators of the step
// (the state, the stage combinations and the small matrix functions stay
// FP64; only the bulk products run in lower precision):
//
//   FP32      v_mfma_f32_16x16x4_f32 on FP32 data;
//   BF16X3    each FP32 operand x is split as x = hi + lo with hi = bf16(x),
//             lo = bf16(x - hi), and a*b is taken as hi_a hi_b + hi_a lo_b +
//             lo_a hi_b on v_mfma_f32_16x16x32_bf16 with FP32 accumulation (the
//             lo_a lo_b term, ~2^-16 relative, is dropped).
//
// Both use one "transposing" product form,
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
#include "common.h"

namespace adr {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));

// float -> bf16 bits, round to nearest even (inputs are finite)
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  const unsigned u = __float_as_uint(x);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short b) {
  return __uint_as_float((unsigned)b << 16);
}

struct LowpArgs {
  const float* W[kMaxGroup];     // inputs, n x X column-major (fibres contiguous)
  const float* M[kMaxGroup];     // FP32: n x n column-major
  const unsigned short* Mh[kMaxGroup];  // BF16X3: transposed hi/lo parts, k fastest
  const unsigned short* Ml[kMaxGroup];
  void* out[kMaxGroup];          // FP32 (rotated) or FP64 (last product)
  const double* Y[kMaxGroup];    // FP64 addend for the last product, may alias out
  const float* Z[kMaxGroup];     // FP32 second addend of the last product, or null
  double alpha, beta;
  int n;
  unsigned X;
  int group;
};

constexpr int kThreads = 256;

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
template <int FI, int FX, bool HASY, bool HASZ, bool GUARD>
__device__ __forceinline__ void tgemm_epilogue64(const LowpJob& a, const f4 (&acc)[FI][FX], int ib,
                                                 unsigned xb, int col, int krow) {
  const int n = a.n;
  const unsigned X = (unsigned)a.X;
  const double alpha = a.alpha, beta = a.beta;
  const double* Y = a.Y;
  const float* Z = a.Z;
  double* out = static_cast<double*>(a.out);
  double y[2][FI][4];
  float z[2][FI][4];
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
        if (HASY) y[fx & 1][fi][v] = Y[o];
        if (HASZ) z[fx & 1][fi][v] = Z[o];
      }
  };
  load_strip(0);
#pragma unroll
  for (int fx = 0; fx < FX; ++fx) {
    if (fx + 1 < FX) load_strip(fx + 1);
#pragma unroll
    for (int fi = 0; fi < FI; ++fi)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        bool ok;
        const unsigned o = index(fx, fi, v, ok);
        const double p = alpha * (double)acc[fi][fx][v];
        double val = p;
        if (HASZ) val = ((HASY ? beta * y[fx & 1][fi][v] : 0.0) + (double)z[fx & 1][fi][v]) + p;
        else if (HASY) val = p + beta * y[fx & 1][fi][v];
        if (ok) out[o] = val;
      }
  }
}

template <int FI, int FX, int TI, int TX, bool OUT64>
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
        if (hy) tgemm_epilogue64<FI, FX, true, true, false>(a, acc, ib, xb, col, krow);
        else tgemm_epilogue64<FI, FX, false, true, false>(a, acc, ib, xb, col, krow);
      } else if (hy) {
        tgemm_epilogue64<FI, FX, true, false, false>(a, acc, ib, xb, col, krow);
      } else {
        tgemm_epilogue64<FI, FX, false, false, false>(a, acc, ib, xb, col, krow);
      }
    } else {
      if (hz) {
        if (hy) tgemm_epilogue64<FI, FX, true, true, true>(a, acc, ib, xb, col, krow);
        else tgemm_epilogue64<FI, FX, false, true, true>(a, acc, ib, xb, col, krow);
      } else if (hy) {
        tgemm_epilogue64<FI, FX, true, false, true>(a, acc, ib, xb, col, krow);
      } else {
        tgemm_epilogue64<FI, FX, false, false, true>(a, acc, ib, xb, col, krow);
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
// Tile: BI rows i x BX fibres, BK = 32 (one bf16 MFMA depth) per chunk.  The W
// chunk is loaded as FP32 (eight consecutive k per lane), split into hi/lo and
// stored k-fastest; M arrives pre-split and transposed (k fastest).
template <int BI, int BX, bool OUT64, bool FULL, int PADB = 0, int WI = 2, int WX = 2>
__global__ __launch_bounds__(64 * WI * WX, 2) void k_tgemm_bf16x3(LowpArgs a, int n_itiles,
                                                                 int n_xtiles) {
  constexpr int BK = 32;
  constexpr int kThreads = 64 * WI * WX;
  constexpr int TI = BI / WI, TX = BX / WX, FI = TI / 16, FX = TX / 16;
  constexpr int LDK = BK + PADB;            // bf16 elements per row (16-byte aligned pitch)
  constexpr int MSEG = BI * (BK / 8);        // 8-element segments of the M chunk
  constexpr int WSEG = BX * (BK / 8);
  constexpr int MLOADS = MSEG / kThreads, WLOADS = WSEG / kThreads;
  static_assert(MLOADS * kThreads == MSEG && WLOADS * kThreads == WSEG, "mapping");
  __shared__ unsigned short sMh[2][BI * LDK], sMl[2][BI * LDK];
  __shared__ unsigned short sWh[2][BX * LDK], sWl[2][BX * LDK];

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
  const unsigned short* __restrict__ Mh = a.Mh[g];
  const unsigned short* __restrict__ Ml = a.Ml[g];

  // segment s of a chunk: row r = s / 4 (i or x), k-group q = s % 4 (8 k-values)
  s8 rmh[MLOADS], rml[MLOADS];
  float rw[WLOADS][8];
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < MLOADS; ++p) {
      const int s = tid + p * kThreads, r = s >> 2, q = s & 3;
      const int i = i0 + r, k = k0 + 8 * q;
      if (FULL) {  // whole tile in range, 16-byte aligned rows
        const unsigned idx = (unsigned)i * (unsigned)n + (unsigned)k;
        rmh[p] = *reinterpret_cast<const s8*>(Mh + idx);
        rml[p] = *reinterpret_cast<const s8*>(Ml + idx);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const bool ok = i < n && (k + j) < n;
          const unsigned idx = ok ? (unsigned)i * (unsigned)n + (unsigned)(k + j) : 0u;
          rmh[p][j] = ok ? (short)Mh[idx] : (short)0;
          rml[p][j] = ok ? (short)Ml[idx] : (short)0;
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
      *reinterpret_cast<s8*>(&sMh[buf][r * LDK + 8 * q]) = rmh[p];
      *reinterpret_cast<s8*>(&sMl[buf][r * LDK + 8 * q]) = rml[p];
    }
#pragma unroll
    for (int p = 0; p < WLOADS; ++p) {
      const int s = tid + p * kThreads, r = s >> 2, q = s & 3;
      s8 h, l;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const unsigned short hb = bf16_bits(rw[p][j]);
        h[j] = (short)hb;
        l[j] = (short)bf16_bits(rw[p][j] - bf16_float(hb));
      }
      *reinterpret_cast<s8*>(&sWh[buf][r * LDK + 8 * q]) = h;
      *reinterpret_cast<s8*>(&sWl[buf][r * LDK + 8 * q]) = l;
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
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunks) load((c + 1) * BK);
    s8 ah[FI], al[FI], bh[FX], bl[FX];
#pragma unroll
    for (int fi = 0; fi < FI; ++fi) {
      const int r = wi * TI + fi * 16 + col;
      ah[fi] = *reinterpret_cast<const s8*>(&sMh[buf][r * LDK + 8 * kq]);
      al[fi] = *reinterpret_cast<const s8*>(&sMl[buf][r * LDK + 8 * kq]);
    }
#pragma unroll
    for (int fx = 0; fx < FX; ++fx) {
      const int r = wx * TX + fx * 16 + col;
      bh[fx] = *reinterpret_cast<const s8*>(&sWh[buf][r * LDK + 8 * kq]);
      bl[fx] = *reinterpret_cast<const s8*>(&sWl[buf][r * LDK + 8 * kq]);
    }
#pragma unroll
    for (int fi = 0; fi < FI; ++fi)
#pragma unroll
      for (int fx = 0; fx < FX; ++fx) {
        // small terms first, the dominant product last
        acc[fi][fx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[fi], bh[fx], acc[fi][fx], 0, 0, 0);
        acc[fi][fx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[fi], bl[fx], acc[fi][fx], 0, 0, 0);
        acc[fi][fx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[fi], bh[fx], acc[fi][fx], 0, 0, 0);
      }
    if (c + 1 < nchunks) store(buf ^ 1);
    __syncthreads();
  }
  tgemm_epilogue<FI, FX, TI, TX, OUT64>(job_of(a, g), acc, i0 + wi * TI, x0 + wx * TX, col, kq);
}

// Split an FP64 n x n column-major matrix into transposed bf16 hi/lo parts:
// Mh[i*n + k] + Ml[i*n + k] ~ M[i + n*k] (via FP32).
__global__ __launch_bounds__(256) void k_split_bf16(int n, const double* __restrict__ M,
                                                    unsigned short* __restrict__ Mh,
                                                    unsigned short* __restrict__ Ml) {
  const long long nn = (long long)n * n;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nn;
       q += (long long)gridDim.x * blockDim.x) {
    const long long i = q / n, k = q % n;   // q = i*n + k
    const float x = (float)M[i + (long long)n * k];
    const unsigned short h = bf16_bits(x);
    Mh[q] = h;
    Ml[q] = bf16_bits(x - bf16_float(h));
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
                             const void* const* Mh, const void* const* Ml, void* const* out,
                             const double* const* Y, int group, int n, long long X, double alpha,
                             double beta, int out_f64, hipStream_t s, const float* const* Z) {
  if (group < 1 || group > kMaxGroup || X <= 0 || X >= (1LL << 31) ||
      (long long)n * X >= (1LL << 31) || (Z && !out_f64))
    return hipErrorInvalidValue;
  LowpArgs a{};
  for (int g = 0; g < group; ++g) {
    a.W[g] = static_cast<const float*>(W[g]);
    a.M[g] = Mf32 ? static_cast<const float*>(Mf32[g]) : nullptr;
    a.Mh[g] = Mh ? static_cast<const unsigned short*>(Mh[g]) : nullptr;
    a.Ml[g] = Ml ? static_cast<const unsigned short*>(Ml[g]) : nullptr;
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
  if (precision == 1) {
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
  // evenly tiled shapes with 16-byte aligned fibres take the vectorised loads
  bool aligned = true;
  for (int g = 0; g < group; ++g)
    aligned = aligned && (reinterpret_cast<uintptr_t>(W[g]) % 16 == 0) &&
              (reinterpret_cast<uintptr_t>(Mh[g]) % 16 == 0) &&
              (reinterpret_cast<uintptr_t>(Ml[g]) % 16 == 0);
  if (rows64) {
    const bool full = aligned && n % 64 == 0 && X % 128 == 0;
    if (full)
      return out_f64 ? launch_tiles(k_tgemm_bf16x3<64, 128, true, true>, a, 64, 128, s)
                     : launch_tiles(k_tgemm_bf16x3<64, 128, false, true>, a, 64, 128, s);
    return out_f64 ? launch_tiles(k_tgemm_bf16x3<64, 128, true, false>, a, 64, 128, s)
                   : launch_tiles(k_tgemm_bf16x3<64, 128, false, false>, a, 64, 128, s);
  }
  const bool full = aligned && n % 128 == 0 && X % 128 == 0;
  if (full)
    return out_f64 ? launch_tiles(k_tgemm_bf16x3<128, 128, true, true>, a, 128, 128, s)
                   : launch_tiles(k_tgemm_bf16x3<128, 128, false, true>, a, 128, 128, s);
  return out_f64 ? launch_tiles(k_tgemm_bf16x3<128, 128, true, false>, a, 128, 128, s)
                 : launch_tiles(k_tgemm_bf16x3<128, 128, false, false>, a, 128, 128, s);
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

hipError_t launch_split_bf16(int n, const double* M, unsigned short* Mh, unsigned short* Ml,
                             hipStream_t s) {
  long long blocks = ((long long)n * n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)blocks), dim3(256), 0, s, n, M, Mh, Ml);
  return hipGetLastError();
}

}  // namespace adr
