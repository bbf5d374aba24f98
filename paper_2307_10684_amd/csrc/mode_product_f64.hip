// FP64 mu-mode product on CDNA4 matrix cores (v_mfma_f64_16x16x4_f64).
//
// out = alpha * (W x_mu M) + beta * Y + gamma * Z,
//   (W x_mu M)[.., i, ..] = sum_k M[i, k] W[.., k, ..]           (Sec. 2)
//
// The tensor is viewed as (L, n, R) (see ModeArgs).  Each workgroup computes a
// BI x BX output tile: BI rows i of the n x n matrix against BX fibres x, with
// the contraction over k staged through LDS in chunks of BK.  This is a GEMM
// whose small operand M is shared by every workgroup (it stays in L2) and
// whose large operand W is streamed from HBM once per i-tile.
//
// Two memory orientations:
//  * L > 1 ("x-contiguous"): consecutive fibres are consecutive in memory, so
//    the W tile is loaded along x and the MFMA computes D[i][x] so that the 16
//    lanes of an output row write 16 consecutive doubles.
//  * L = 1 (mu = 1, "k-contiguous"): each fibre is contiguous, so the W tile is
//    loaded along k, kept k-fastest in LDS, and the MFMA computes D[x][i] so the
//    16 lanes of an output row again write consecutive doubles (along i).
//
// Fragment layout of v_mfma_f64_16x16x4f64 (wave64): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; it receives D[l/16 + 4v][l%16], v = 0..3
// (the row interleave differs from the FP32 16x16x4 instruction).
//
// Element indices fit in 32 bits (the host rejects tensors of 2^31 or more
// elements), so loads use a 32-bit offset from a scalar base pointer.
#include "common.h"
#include "reaction.h"

namespace adr {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int kPad = 16;  // row padding (doubles): the next k-row lands 32 banks away

// One output tile of a mu-mode product (see ModeArgs for the geometry).  The
// single-product kernel and the grouped kernel (many products of different
// shapes in one launch, one TileJob each) both call this.
//
// FULL: every tile is complete (n % BI == 0, n % BK == 0, X % BX == 0), so the
// loads need no bounds predicates and stay in flight across the MFMAs.
template <int BI, int BX, int WI, int WX, int BK, bool KFAST, bool FULL>
__device__ __forceinline__ void mode_tile_f64(const TileJob& job, int itile, int xtile,
                                              double* __restrict__ sMbase,
                                              double* __restrict__ sWbase) {
  constexpr int NT = 64 * WI * WX;
  constexpr int TI = BI / WI, TX = BX / WX;  // wave tile
  constexpr int FI = TI / 16, FX = TX / 16;  // 16x16 blocks per wave
  static_assert(FI * 16 == TI && FX * 16 == TX, "wave tile must be a multiple of 16");
  static_assert(BK % 4 == 0, "k chunk must be a multiple of the MFMA depth");
  constexpr int LDI = BI + kPad;
  constexpr int LDX = BX + kPad;
  constexpr int LDK = BK + 2;                          // k-fastest rows: conflict-free fragments
  constexpr int SW = KFAST ? BX * LDK : BK * LDX;      // W tile size in LDS
  constexpr int SM = BK * LDI;
  constexpr int MROWS = NT / BI;                       // k-rows of M loaded per pass
  constexpr int MLOADS = BK / MROWS;                   // doubles per thread
  static_assert(MROWS * BI == NT && MLOADS * MROWS == BK, "M tile mapping");
  constexpr int WROWS = NT / BX;                       // x-contiguous: k-rows per pass
  constexpr int XSTEP = NT / BK;                       // k-contiguous: fibres per pass
  constexpr int WLOADS = BX * BK / NT;                 // W doubles per thread
  static_assert(KFAST ? (XSTEP * BK == NT && WLOADS * XSTEP == BX)
                      : (WROWS * BX == NT && WLOADS * WROWS == BK), "W tile mapping");
  // double buffers: buffer b of M at sMbase + b*SM, of W at sWbase + b*SW

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wi = wave / WX, wx = wave % WX;

  const int n = job.n;
  const unsigned L = (unsigned)job.L;
  const unsigned X = (unsigned)job.X;
  const unsigned Ln = L * (unsigned)n;
  const int i0 = itile * BI;
  const unsigned x0 = (unsigned)xtile * BX;
  const double* __restrict__ W = job.W;
  const double* __restrict__ M = job.M;

  // ---- per-thread load descriptors ------------------------------------------
  const int m_i = tid % BI;  // M: row i0 + m_i, k-rows m_k0 + p*MROWS
  const int m_k0 = tid / BI;
  const bool m_iok = (i0 + m_i) < n;
  const unsigned m_base = (unsigned)(i0 + m_i) + (unsigned)n * (unsigned)m_k0;

  int w_a, w_b;
  unsigned w_base = 0;
  bool w_ok = true;
  if (!KFAST) {
    w_a = tid % BX;  // x within tile
    w_b = tid / BX;  // first k-row
    const unsigned x = x0 + w_a;
    w_ok = x < X;
    if (w_ok) w_base = (x % L) + Ln * (x / L) + L * (unsigned)w_b;
  } else {
    w_a = tid % BK;  // k within chunk
    w_b = tid / BK;  // first fibre within tile
    w_base = (x0 + w_b) * (unsigned)n + (unsigned)w_a;
  }

  double rm[MLOADS], rw[WLOADS];

  // Loads read raw values (out-of-range elements read index 0); the zeroing of
  // out-of-range elements happens when the chunk is written to LDS, after the
  // MFMAs of the current chunk, so the loads stay in flight during the compute.
  auto m_ok = [&](int k0, int p) { return FULL || (m_iok && (k0 + m_k0 + p * MROWS) < n); };
  auto w_okp = [&](int k0, int p) {
    return FULL || (KFAST ? ((k0 + w_a) < n && (x0 + w_b + p * XSTEP) < X)
                          : (w_ok && (k0 + w_b + p * WROWS) < n));
  };
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int p = 0; p < MLOADS; ++p)
      rm[p] = M[m_ok(k0, p) ? m_base + (unsigned)n * (unsigned)(k0 + p * MROWS) : 0u];
#pragma unroll
    for (int p = 0; p < WLOADS; ++p) {
      const unsigned off = KFAST ? (unsigned)n * (unsigned)(p * XSTEP) + (unsigned)k0
                                 : L * (unsigned)(k0 + p * WROWS);
      rw[p] = W[w_okp(k0, p) ? w_base + off : 0u];
    }
  };
  auto store_chunk = [&](int buf, int k0) {
#pragma unroll
    for (int p = 0; p < MLOADS; ++p)
      sMbase[buf * SM + (m_k0 + p * MROWS) * LDI + m_i] = m_ok(k0, p) ? rm[p] : 0.0;
#pragma unroll
    for (int p = 0; p < WLOADS; ++p) {
      const double v = w_okp(k0, p) ? rw[p] : 0.0;
      if (!KFAST)
        sWbase[buf * SW + (w_b + p * WROWS) * LDX + w_a] = v;
      else
        sWbase[buf * SW + (w_b + p * XSTEP) * LDK + w_a] = v;
    }
  };

  d4 acc[FI][FX];
#pragma unroll
  for (int fi = 0; fi < FI; ++fi)
#pragma unroll
    for (int fx = 0; fx < FX; ++fx) acc[fi][fx] = d4{0.0, 0.0, 0.0, 0.0};

  const int nchunks = (n + BK - 1) / BK;
  load_chunk(0);
  store_chunk(0, 0);
  __syncthreads();

  const int col = lane & 15;
  const int krow = lane >> 4;
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunks) load_chunk((c + 1) * BK);
    const double* sm = sMbase + buf * SM;
    const double* sw = sWbase + buf * SW;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + krow;
      double af[FI], bf[FX];
#pragma unroll
      for (int fi = 0; fi < FI; ++fi) af[fi] = sm[kr * LDI + wi * TI + fi * 16 + col];
#pragma unroll
      for (int fx = 0; fx < FX; ++fx) {
        const int xl = wx * TX + fx * 16 + col;
        bf[fx] = KFAST ? sw[xl * LDK + kr] : sw[kr * LDX + xl];
      }
#pragma unroll
      for (int fi = 0; fi < FI; ++fi)
#pragma unroll
        for (int fx = 0; fx < FX; ++fx)
          acc[fi][fx] = KFAST ? __builtin_amdgcn_mfma_f64_16x16x4f64(bf[fx], af[fi], acc[fi][fx], 0, 0, 0)
                              : __builtin_amdgcn_mfma_f64_16x16x4f64(af[fi], bf[fx], acc[fi][fx], 0, 0, 0);
    }
    if (c + 1 < nchunks) store_chunk(buf ^ 1, (c + 1) * BK);
    __syncthreads();
  }

  // ---- epilogue: out = alpha*acc + beta*Y + gamma*Z --------------------------
  // Y may alias out (each element is read, then written, by the same lane)
  double* out = job.out;
  const double* Y = job.Y;
  const double* Z = job.Z;
  const double alpha = job.alpha, beta = job.beta, gamma = job.gamma;
  if (!KFAST) {
#pragma unroll
    for (int fx = 0; fx < FX; ++fx) {
      const unsigned x = x0 + wx * TX + fx * 16 + col;
      if (x >= X) continue;
      const unsigned xo = (x % L) + Ln * (x / L);
#pragma unroll
      for (int fi = 0; fi < FI; ++fi) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + wi * TI + fi * 16 + krow + 4 * v;
          if (i < n) {
            const unsigned o = xo + L * (unsigned)i;
            double val = alpha * acc[fi][fx][v];
            if (Y) val += beta * Y[o];
            if (Z) val += gamma * Z[o];
            out[o] = val;
          }
        }
      }
    }
  } else {
#pragma unroll
    for (int fi = 0; fi < FI; ++fi) {
      const int i = i0 + wi * TI + fi * 16 + col;
      if (i >= n) continue;
#pragma unroll
      for (int fx = 0; fx < FX; ++fx) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const unsigned x = x0 + wx * TX + fx * 16 + krow + 4 * v;
          if (x < X) {
            const unsigned o = x * (unsigned)n + (unsigned)i;
            double val = alpha * acc[fi][fx][v];
            if (Y) val += beta * Y[o];
            if (Z) val += gamma * Z[o];
            out[o] = val;
          }
        }
      }
    }
  }
}


template <int BI, int BX, int WI, int WX, int BK, bool KFAST, bool FULL, int MINB = 2>
__global__ __launch_bounds__(64 * WI * WX, MINB) void k_mode_f64(ModeArgs a, int n_itiles,
                                                                int n_xtiles) {
  constexpr int SW = KFAST ? BX * (BK + 2) : BK * (BX + kPad);
  __shared__ double sM[2 * BK * (BI + kPad)];
  __shared__ double sW[2 * SW];
  // Tile index.  The hardware deals workgroups to the 8 XCDs round-robin; give
  // each XCD a contiguous range of tiles so the i-tiles that re-read the same
  // W fibres run on the same L2.
  const int G = gridDim.x;
  const int b = blockIdx.x;
  int t = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const int itile = t % n_itiles;
  t /= n_itiles;
  const int xtile = t % n_xtiles;
  const int g = t / n_xtiles;
  TileJob job;
  job.W = static_cast<const double*>(a.W[g]);
  job.M = static_cast<const double*>(a.M[g]);
  job.out = static_cast<double*>(a.out[g]);
  job.Y = a.Y[g];
  job.Z = a.Z[g];
  job.alpha = a.alpha;
  job.beta = a.beta;
  job.gamma = a.gamma;
  job.L = a.L;
  job.X = a.X;
  job.n = a.n;
  mode_tile_f64<BI, BX, WI, WX, BK, KFAST, FULL>(job, itile, xtile, sM, sW);
}

// Grouped products: job j covers tiles [jobs[j].tile_begin, jobs[j+1].tile_begin)
// with its own shape, matrix, addend and scalars; a workgroup finds its job by
// binary search over the sorted tile offsets.
template <int BI, int BX, int WI, int WX, int BK, bool KFAST>
__global__ __launch_bounds__(64 * WI * WX, 2) void k_mode_f64_grouped(const TileJob* __restrict__ jobs,
                                                                     int njobs) {
  constexpr int SW = KFAST ? BX * (BK + 2) : BK * (BX + kPad);
  __shared__ double sM[2 * BK * (BI + kPad)];
  __shared__ double sW[2 * SW];
  const long long t = xcd_tile(blockIdx.x, gridDim.x);
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
  }
  const TileJob job = jobs[lo];
  const long long local = t - job.tile_begin;
  const int itile = (int)(local % job.n_itiles);
  const int xtile = (int)(local / job.n_itiles);
  mode_tile_f64<BI, BX, WI, WX, BK, KFAST, false>(job, itile, xtile, sM, sW);
}

// Persistent grouped products: about MINB workgroups per CU walk the grouped tile
// sequence (jobs sorted by tile offset) in rounds of one tile each, with the
// first k-chunk of the next tile -- possibly of another job, with its own shape
// -- loaded while the last chunk of the current tile is multiplied.  Loads and
// stores are bounds-checked as in mode_tile_f64 (any shape), and every output
// element is summed in the same order as there.
template <int BI, int BX, int WI, int WX, int BK, bool KFAST, int MINB>
__global__ __launch_bounds__(64 * WI * WX, MINB) void k_mode_f64_grouped_persist(
    const TileJob* __restrict__ jobs, int njobs, long long ntiles) {
  constexpr int NT = 64 * WI * WX;
  constexpr int TI = BI / WI, TX = BX / WX;
  constexpr int FI = TI / 16, FX = TX / 16;
  static_assert(FI * 16 == TI && FX * 16 == TX, "wave tile must be a multiple of 16");
  constexpr int LDI = BI + kPad;
  constexpr int LDX = BX + kPad;
  constexpr int LDK = BK + 2;
  constexpr int SW = KFAST ? BX * LDK : BK * LDX;
  constexpr int SM = BK * LDI;
  constexpr int MROWS = NT / BI;
  constexpr int MLOADS = BK / MROWS;
  static_assert(MROWS * BI == NT && MLOADS * MROWS == BK, "M tile mapping");
  constexpr int WROWS = NT / BX;
  constexpr int XSTEP = NT / BK;
  constexpr int WLOADS = BX * BK / NT;
  static_assert(KFAST ? (XSTEP * BK == NT && WLOADS * XSTEP == BX)
                      : (WROWS * BX == NT && WLOADS * WROWS == BK), "W tile mapping");
  __shared__ double sM[2 * SM];
  __shared__ double sW[2 * SW];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wi = wave / WX, wx = wave % WX;
  const int col = lane & 15;
  const int krow = lane >> 4;

  // round k: the grid takes tiles [k*G, (k+1)*G), dealt as the one-tile-per-
  // workgroup launch deals them (xcd_tile), so every workgroup sees the same mix
  // of long and short contractions
  const long long G = gridDim.x;
  const long long b = blockIdx.x;
  const long long off = xcd_tile(b, G);
  auto tile_index = [&](long long k) -> long long {
    const long long t = k * G + off;
    return t < ntiles ? t : -1;
  };

  // per-tile state: the job's geometry and this thread's load descriptors
  struct Tile {
    TileJob job;
    int i0;
    unsigned x0, L, X, Ln;
    bool m_iok, w_ok;
    unsigned m_base, w_base;
  };
  const int m_i = tid % BI, m_k0 = tid / BI;
  const int w_a = KFAST ? tid % BK : tid % BX;
  const int w_b = KFAST ? tid / BK : tid / BX;
  auto tile_of = [&](long long t) {
    Tile d;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    d.job = jobs[lo];
    const long long local = t - d.job.tile_begin;
    d.i0 = (int)(local % d.job.n_itiles) * BI;
    d.x0 = (unsigned)(local / d.job.n_itiles) * BX;
    d.L = (unsigned)d.job.L;
    d.X = (unsigned)d.job.X;
    d.Ln = d.L * (unsigned)d.job.n;
    d.m_iok = (d.i0 + m_i) < d.job.n;
    d.m_base = (unsigned)(d.i0 + m_i) + (unsigned)d.job.n * (unsigned)m_k0;
    if (!KFAST) {
      const unsigned x = d.x0 + w_a;
      d.w_ok = x < d.X;
      d.w_base = d.w_ok ? (x % d.L) + d.Ln * (x / d.L) + d.L * (unsigned)w_b : 0u;
    } else {
      d.w_ok = true;
      d.w_base = (d.x0 + w_b) * (unsigned)d.job.n + (unsigned)w_a;
    }
    return d;
  };

  double rm[MLOADS], rw[WLOADS];
  auto m_ok = [&](const Tile& d, int k0, int p) {
    return d.m_iok && (k0 + m_k0 + p * MROWS) < d.job.n;
  };
  auto w_okp = [&](const Tile& d, int k0, int p) {
    return KFAST ? ((k0 + w_a) < d.job.n && (d.x0 + w_b + p * XSTEP) < d.X)
                 : (d.w_ok && (k0 + w_b + p * WROWS) < d.job.n);
  };
  auto load_chunk = [&](const Tile& d, int k0) {
    const unsigned n = (unsigned)d.job.n;
#pragma unroll
    for (int p = 0; p < MLOADS; ++p)
      rm[p] = d.job.M[m_ok(d, k0, p) ? d.m_base + n * (unsigned)(k0 + p * MROWS) : 0u];
#pragma unroll
    for (int p = 0; p < WLOADS; ++p) {
      const unsigned off = KFAST ? n * (unsigned)(p * XSTEP) + (unsigned)k0
                                 : d.L * (unsigned)(k0 + p * WROWS);
      rw[p] = d.job.W[w_okp(d, k0, p) ? d.w_base + off : 0u];
    }
  };
  auto store_chunk = [&](const Tile& d, int buf, int k0) {
#pragma unroll
    for (int p = 0; p < MLOADS; ++p)
      sM[buf * SM + (m_k0 + p * MROWS) * LDI + m_i] = m_ok(d, k0, p) ? rm[p] : 0.0;
#pragma unroll
    for (int p = 0; p < WLOADS; ++p) {
      const double v = w_okp(d, k0, p) ? rw[p] : 0.0;
      if (!KFAST)
        sW[buf * SW + (w_b + p * WROWS) * LDX + w_a] = v;
      else
        sW[buf * SW + (w_b + p * XSTEP) * LDK + w_a] = v;
    }
  };

  long long k = 0;
  const long long t0 = tile_index(0);
  if (t0 < 0) return;
  Tile cur = tile_of(t0);
  load_chunk(cur, 0);
  store_chunk(cur, 0, 0);
  __syncthreads();
  int buf = 0;
  while (true) {
    const long long tn = tile_index(k + 1);
    const Tile nxt = tile_of(tn < 0 ? t0 : tn);
    d4 acc[FI][FX];
#pragma unroll
    for (int fi = 0; fi < FI; ++fi)
#pragma unroll
      for (int fx = 0; fx < FX; ++fx) acc[fi][fx] = d4{0.0, 0.0, 0.0, 0.0};
    const int nchunks = (cur.job.n + BK - 1) / BK;
    for (int c = 0; c < nchunks; ++c) {
      const bool in_tile = c + 1 < nchunks;
      const bool more = in_tile || tn >= 0;
      if (more) load_chunk(in_tile ? cur : nxt, in_tile ? (c + 1) * BK : 0);
      const double* sm = sM + buf * SM;
      const double* sw = sW + buf * SW;
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const int kr = kk + krow;
        double af[FI], bf[FX];
#pragma unroll
        for (int fi = 0; fi < FI; ++fi) af[fi] = sm[kr * LDI + wi * TI + fi * 16 + col];
#pragma unroll
        for (int fx = 0; fx < FX; ++fx) {
          const int xl = wx * TX + fx * 16 + col;
          bf[fx] = KFAST ? sw[xl * LDK + kr] : sw[kr * LDX + xl];
        }
#pragma unroll
        for (int fi = 0; fi < FI; ++fi)
#pragma unroll
          for (int fx = 0; fx < FX; ++fx)
            acc[fi][fx] = KFAST ? __builtin_amdgcn_mfma_f64_16x16x4f64(bf[fx], af[fi], acc[fi][fx], 0, 0, 0)
                                : __builtin_amdgcn_mfma_f64_16x16x4f64(af[fi], bf[fx], acc[fi][fx], 0, 0, 0);
      }
      if (more) store_chunk(in_tile ? cur : nxt, buf ^ 1, in_tile ? (c + 1) * BK : 0);
      __syncthreads();
      buf ^= 1;
    }
    // epilogue (as mode_tile_f64): out = alpha*acc + beta*Y + gamma*Z
    const TileJob& j = cur.job;
    const int n = j.n;
    if (!KFAST) {
#pragma unroll
      for (int fx = 0; fx < FX; ++fx) {
        const unsigned x = cur.x0 + wx * TX + fx * 16 + col;
        if (x >= cur.X) continue;
        const unsigned xo = (x % cur.L) + cur.Ln * (x / cur.L);
#pragma unroll
        for (int fi = 0; fi < FI; ++fi)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = cur.i0 + wi * TI + fi * 16 + krow + 4 * v;
            if (i < n) {
              const unsigned o = xo + cur.L * (unsigned)i;
              double val = j.alpha * acc[fi][fx][v];
              if (j.Y) val += j.beta * j.Y[o];
              if (j.Z) val += j.gamma * j.Z[o];
              j.out[o] = val;
            }
          }
      }
    } else {
#pragma unroll
      for (int fi = 0; fi < FI; ++fi) {
        const int i = cur.i0 + wi * TI + fi * 16 + col;
        if (i >= n) continue;
#pragma unroll
        for (int fx = 0; fx < FX; ++fx)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const unsigned x = cur.x0 + wx * TX + fx * 16 + krow + 4 * v;
            if (x < cur.X) {
              const unsigned o = x * (unsigned)n + (unsigned)i;
              double val = j.alpha * acc[fi][fx][v];
              if (j.Y) val += j.beta * j.Y[o];
              if (j.Z) val += j.gamma * j.Z[o];
              j.out[o] = val;
            }
          }
      }
    }
    if (tn < 0) break;
    cur = nxt;
    ++k;
  }
}

// Epilogue of a V tile that carries ETD2RKds stage 2 (see k_mode_f64_persist),
// for reaction model MODEL.  The six tensors are distinct buffers: the
// restrict-qualified parameters let the loads of a batch of elements be issued
// together, and ahead of the stores of the previous batch, so the epilogue
// waits for memory about once per batch rather than once per element (a batch
// of 4 keeps the kernel within 256 VGPRs; 8 spilled).
template <int MODEL, int FI, int FX, typename Index>
__device__ __forceinline__ void stage2_epilogue_m(const d4 (&acc)[FI][FX], double alpha,
                                                  double beta, Index idx,
                                                  const Reaction& r, double* __restrict__ V2,
                                                  const double* __restrict__ U2,
                                                  const double* __restrict__ Un,
                                                  const double* __restrict__ Vn,
                                                  double* __restrict__ Ru, double* __restrict__ Rv) {
  constexpr int NE = FI * FX * 4;
  constexpr int B = 4;  // elements per batch
  static_assert(NE % B == 0, "batch size");
#pragma unroll
  for (int b0 = 0; b0 < NE; b0 += B) {
    unsigned o[B];
    double un[B], vn[B], u2[B];
#pragma unroll
    for (int e = 0; e < B; ++e) {
      const int q = b0 + e;
      o[e] = idx(q / (FX * 4), (q / 4) % FX, q % 4);
      un[e] = Un[o[e]];
      vn[e] = Vn[o[e]];
      u2[e] = U2[o[e]];
    }
#pragma unroll
    for (int e = 0; e < B; ++e) {
      const int q = b0 + e;
      const double v2 = alpha * acc[q / (FX * 4)][(q / 4) % FX][q % 4] + beta * vn[e];
      double gu, gv, gu2, gv2;
      react_model<MODEL>(r, un[e], vn[e], gu, gv);
      react_model<MODEL>(r, u2[e], v2, gu2, gv2);
      V2[o[e]] = v2;
      Ru[o[e]] = gu2 - gu;
      Rv[o[e]] = gv2 - gv;
    }
  }
}

template <int FI, int FX, typename Index>
__device__ __forceinline__ void stage2_epilogue(const d4 (&acc)[FI][FX], double alpha, double beta,
                                                Index idx,
                                                const Reaction& r, double* V2, const double* U2,
                                                const double* Un, const double* Vn, double* Ru,
                                                double* Rv) {
  switch (r.model) {
    case 0: stage2_epilogue_m<0>(acc, alpha, beta, idx, r, V2, U2, Un, Vn, Ru, Rv); break;
    case 1: stage2_epilogue_m<1>(acc, alpha, beta, idx, r, V2, U2, Un, Vn, Ru, Rv); break;
    case 2: stage2_epilogue_m<2>(acc, alpha, beta, idx, r, V2, U2, Un, Vn, Ru, Rv); break;
    case 4: stage2_epilogue_m<4>(acc, alpha, beta, idx, r, V2, U2, Un, Vn, Ru, Rv); break;
    default: stage2_epilogue_m<3>(acc, alpha, beta, idx, r, V2, U2, Un, Vn, Ru, Rv);
  }
}

// Persistent variant for evenly tiled shapes (n % BI == 0, X % BX == 0,
// 16-byte aligned rows): a grid of about two workgroups per CU walks the tiles,
// loads move two doubles per lane, and the first k-chunk of the next tile is
// fetched while the last chunk of the current one is multiplied, so tile
// boundaries (epilogue stores, first loads) overlap with MFMA work.
//
// S2 (ETD2RKds stage 2 in the epilogue, a.Rout set): the two tensors' tiles
// alternate (U tile, then the V tile of the same rows and fibres) within each
// workgroup's sequence, so when a V tile ends the same lanes have already
// stored the U values of the same elements.  The V epilogue reads them back
// (same-lane read after write), adds V_n (not folded into its accumulators),
// evaluates the reaction at the new and the old states and stores
// R^c = G^c(C_{n2}) - G^c(C_n) for both components, which saves the separate
// pass over four FP64 tensors.
//
// DMA: the chunks go from global memory straight to LDS (global_load_lds,
// 16 bytes per lane, lane l writing bytes 16 l onward of the wave's LDS row):
// no staging registers and no LDS store instructions.  Each wave then loads
// whole 128-double rows, so only x-contiguous 128x128 tiles of four waves take
// it.  The two chunk buffers are distinct LDS objects and the chunk loop is
// unrolled by two, so that the compiler sees that the loads into one buffer do
// not alias the reads of the other and waits for them only at the barrier.
template <int BI, int BX, int WI, int WX, int BK, bool KFAST, int MINB = 2, bool S2 = false,
          bool DMA = false>
__global__ __launch_bounds__(64 * WI * WX, MINB) void k_mode_f64_persist(ModeArgs a, int n_itiles,
                                                                        int n_xtiles, int ntiles,
                                                                        int stream_out) {
  static_assert(!(S2 && KFAST), "stage 2 is carried by x-contiguous products only");
  static_assert(!DMA || (!KFAST && BI == 128 && BX == 128 && WI * WX == 4),
                "LDS-direct loads need one 128-double LDS row per wave and load");
  constexpr int NT = 64 * WI * WX;
  constexpr int TI = BI / WI, TX = BX / WX;
  constexpr int FI = TI / 16, FX = TX / 16;
  static_assert(FI * 16 == TI && FX * 16 == TX, "wave tile must be a multiple of 16");
  constexpr int LDI = BI + kPad;
  constexpr int LDX = BX + kPad;
  constexpr int LDK = BK + 2;
  constexpr int SW = KFAST ? BX * LDK : BK * LDX;
  // pair-granular load mappings (each lane moves two consecutive doubles)
  constexpr int MPR = BI / 2;            // lanes per M k-row
  constexpr int MROWS = NT / MPR;        // k-rows per pass
  constexpr int MLOADS = BK / MROWS;     // passes
  static_assert(MROWS * MPR == NT && MLOADS * MROWS == BK, "M mapping");
  constexpr int WPR = BX / 2;            // x-contiguous: lanes per k-row
  constexpr int WROWS = NT / WPR;
  constexpr int KPR = BK / 2;            // k-contiguous: lanes per fibre
  constexpr int XSTEP = NT / KPR;        // fibres per pass
  constexpr int WLOADS = KFAST ? BX / XSTEP : BK / WROWS;
  static_assert(KFAST ? (XSTEP * KPR == NT && WLOADS * XSTEP == BX)
                      : (WROWS * WPR == NT && WLOADS * WROWS == BK), "W mapping");

  __shared__ double sM[2][BK * LDI];
  __shared__ double sW[2][SW];
  __shared__ double dM0[BK * LDI], dM1[BK * LDI];   // DMA: distinct buffers
  __shared__ double dW0[SW], dW1[SW];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wi = wave / WX, wx = wave % WX;
  const int col = lane & 15;
  const int krow = lane >> 4;

  const int n = a.n;
  const unsigned L = (unsigned)a.L;
  const unsigned Ln = L * (unsigned)n;
  const int nchunks = n / BK;   // even: n is a multiple of 64 here

  // tile sequence of this workgroup: XCD-contiguous ranges (see k_mode_f64)
  const int G = gridDim.x;
  const int b = blockIdx.x;
  int per = (ntiles + G - 1) / G;           // tiles per workgroup (upper bound)
  if (S2) per += per & 1;                   // U/V tile pairs never split
  // workgroup b handles logical tiles base, base+1, ... within its XCD's range
  const int xcd = b % 8, slot = b / 8;

  // per-tile state; the group member's pointers are picked with explicit selects
  // (a dynamic index into the kernel-argument arrays would spill them to scratch)
  struct TileDesc {
    int g, i0;
    unsigned x0;
    const double* W;
    const double* M;
  };
  auto pick = [](const void* const* arr, int g) {
    const void* p = arr[0];
    p = g == 1 ? arr[1] : p;
    p = g == 2 ? arr[2] : p;
    p = g == 3 ? arr[3] : p;
    return p;
  };
  // logical tile k of this workgroup (k = 0, 1, ...); -1 when done.
  // When the workgroups of an XCD can be grouped n_itiles at a time, the group
  // members take the n_itiles row tiles of the same fibre blocks in lockstep:
  // they read the same W chunks at about the same time, so the XCD's L2 serves
  // the repeats and W is fetched from HBM about once.  (Measured at 256^3: a
  // little faster for mu < d and 3-4 % slower for the last direction of a
  // multi-dimensional tensor (R = 1), which keeps contiguous per-workgroup ranges;
  // the product that carries stage 2 reads more and pairs.)
  const int slots = G / 8;
  const bool paired = (G % 8 == 0) && n_itiles > 1 && slots % n_itiles == 0 &&
                      ntiles % n_itiles == 0 && (S2 || a.R > 1 || a.L == 1);
  const int nu = ntiles / n_itiles;                        // fibre blocks (all tensors)
  const int groups = 8 * (slots / n_itiles);
  int per_u = (nu + groups - 1) / groups;                  // fibre blocks per group
  if (S2) per_u += per_u & 1;                              // U/V block pairs never split
  auto tile_of = [&](int t) {
    TileDesc d;
    if (S2) {
      // paired: fibre block u = g + 2 * xtile, so a group member's blocks alternate
      // U, V of the same fibres; otherwise tensor fastest: U tile, V tile, next
      // row tile, ...
      int itile, u;
      if (paired) {
        itile = t % n_itiles;
        u = t / n_itiles;
        d.g = u & 1;
      } else {
        d.g = t & 1;
        itile = (t >> 1) % n_itiles;
        u = (t >> 1) / n_itiles * 2;
      }
      d.i0 = itile * BI;
      d.x0 = (unsigned)(u >> 1) * BX;
      d.W = static_cast<const double*>(pick(a.W, d.g));
      d.M = static_cast<const double*>(pick(a.M, d.g));
      return d;
    }
    const int itile = t % n_itiles;
    const int rest = t / n_itiles;
    d.i0 = itile * BI;
    d.x0 = (unsigned)(rest % n_xtiles) * BX;
    d.g = rest / n_xtiles;
    d.W = static_cast<const double*>(pick(a.W, d.g));
    d.M = static_cast<const double*>(pick(a.M, d.g));
    return d;
  };
  auto tile_index = [&](int k) {
    if (paired) {
      const int u = (xcd * (slots / n_itiles) + slot / n_itiles) * per_u + k;
      return (k < per_u && u < nu) ? slot % n_itiles + n_itiles * u : -1;
    }
    const int t = (G % 8 == 0) ? xcd * (G / 8) * per + slot * per + k : b * per + k;
    return (k < per && t < ntiles) ? t : -1;
  };

  // output element of accumulator (fi, fx, v) of this lane: a tile base (uniform)
  // + a lane offset + a constant, since a tile's fibres never straddle a batch
  // (L % BX == 0 is a launch condition of this kernel)
  const unsigned lane_off = !KFAST ? (unsigned)(wx * TX + col) + L * (unsigned)(wi * TI + krow)
                                   : (unsigned)(wx * TX + krow) * (unsigned)n + (unsigned)(wi * TI + col);
  auto out_index = [&](const TileDesc& d, int fi, int fx, int v) -> unsigned {
    if (!KFAST) {
      const unsigned base = (d.x0 % L) + Ln * (d.x0 / L) + L * (unsigned)d.i0;
      return base + lane_off + (unsigned)(fx * 16) + L * (unsigned)(fi * 16 + 4 * v);
    }
    const unsigned base = d.x0 * (unsigned)n + (unsigned)d.i0;
    return base + lane_off + (unsigned)((fx * 16 + 4 * v) * n) + (unsigned)(fi * 16);
  };
  // (only for x-contiguous products: in the FP64 Tucker chain the last product,
  // which carries the addend, is x-contiguous whenever d > 1)
  const bool y_in_acc = !KFAST && a.alpha != 0.0;

  const int m_j = tid % MPR, m_k0 = tid / MPR;
  const int w_j = KFAST ? tid % KPR : tid % WPR;
  const int w_b = KFAST ? tid / KPR : tid / WPR;

  d2 rm[MLOADS], rw[WLOADS];
  auto load_chunk = [&](const double* __restrict__ M, const double* __restrict__ W, int i0,
                        unsigned x0, int k0) {
#pragma unroll
    for (int p = 0; p < MLOADS; ++p) {
      const unsigned idx = (unsigned)(i0 + 2 * m_j) + (unsigned)n * (unsigned)(k0 + m_k0 + p * MROWS);
      rm[p] = *reinterpret_cast<const d2*>(M + idx);
    }
    if (!KFAST) {
      const unsigned x = x0 + 2 * w_j;
      const unsigned base = (x % L) + Ln * (x / L);
#pragma unroll
      for (int p = 0; p < WLOADS; ++p)
        rw[p] = *reinterpret_cast<const d2*>(W + base + L * (unsigned)(k0 + w_b + p * WROWS));
    } else {
#pragma unroll
      for (int p = 0; p < WLOADS; ++p) {
        const unsigned x = x0 + w_b + p * XSTEP;
        rw[p] = *reinterpret_cast<const d2*>(W + x * (unsigned)n + (unsigned)(k0 + 2 * w_j));
      }
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int p = 0; p < MLOADS; ++p)
      *reinterpret_cast<d2*>(&sM[buf][(m_k0 + p * MROWS) * LDI + 2 * m_j]) = rm[p];
#pragma unroll
    for (int p = 0; p < WLOADS; ++p) {
      if (!KFAST)
        *reinterpret_cast<d2*>(&sW[buf][(w_b + p * WROWS) * LDX + 2 * w_j]) = rw[p];
      else
        *reinterpret_cast<d2*>(&sW[buf][(w_b + p * XSTEP) * LDK + 2 * w_j]) = rw[p];
    }
  };

  // DMA: one instruction per LDS row; the row (m_k0 + p * MROWS, w_b + p * WROWS)
  // is the wave's own, so the LDS address is uniform across the wave
  auto dma_chunk = [&](double* dm, double* dw, const double* __restrict__ M,
                       const double* __restrict__ W, int i0, unsigned x0, int k0) {
#pragma unroll
    for (int p = 0; p < MLOADS; ++p) {
      const unsigned idx = (unsigned)(i0 + 2 * m_j) + (unsigned)n * (unsigned)(k0 + m_k0 + p * MROWS);
      __builtin_amdgcn_global_load_lds(M + idx, dm + (m_k0 + p * MROWS) * LDI, 16, 0, 0);
    }
    const unsigned x = x0 + 2 * w_j;
    const unsigned base = (x % L) + Ln * (x / L);
#pragma unroll
    for (int p = 0; p < WLOADS; ++p)
      __builtin_amdgcn_global_load_lds(W + base + L * (unsigned)(k0 + w_b + p * WROWS),
                                       dw + (w_b + p * WROWS) * LDX, 16, 0, 0);
  };

  int k = 0;
  int t = tile_index(0);
  if (t < 0) return;
  TileDesc cur = tile_of(t);
  if constexpr (DMA) {
    dma_chunk(dM0, dW0, cur.M, cur.W, cur.i0, cur.x0, 0);
  } else {
    load_chunk(cur.M, cur.W, cur.i0, cur.x0, 0);
    store_chunk(0);
  }
  __syncthreads();
  int buf = 0;

  const double alpha = a.alpha, beta = a.beta, gamma = a.gamma;
  while (true) {
    const int tn = tile_index(k + 1);
    const TileDesc nxt = tile_of(tn < 0 ? 0 : tn);
    // With an addend, the accumulators start from (beta/alpha) * Y: the loads
    // are issued together at the start of the tile (one memory latency, hidden
    // behind the first chunk) instead of in the epilogue, and the epilogue is a
    // pure store of alpha * acc.
    double* out = static_cast<double*>(const_cast<void*>(pick(a.out, cur.g)));
    const double* Y = y_in_acc ? static_cast<const double*>(pick(reinterpret_cast<const void* const*>(a.Y), cur.g)) : nullptr;
    const double* Z = static_cast<const double*>(pick(reinterpret_cast<const void* const*>(a.Z), cur.g));
    d4 acc[FI][FX];
    // (a V tile that carries stage 2 reads V_n in its epilogue anyway and adds it there)
    if (!KFAST && Y && !(S2 && cur.g == 1)) {
      const double ys = beta / alpha;
#pragma unroll
      for (int fi = 0; fi < FI; ++fi)
#pragma unroll
        for (int fx = 0; fx < FX; ++fx)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[fi][fx][v] = ys * Y[out_index(cur, fi, fx, v)];
    } else {
#pragma unroll
      for (int fi = 0; fi < FI; ++fi)
#pragma unroll
        for (int fx = 0; fx < FX; ++fx) acc[fi][fx] = d4{0.0, 0.0, 0.0, 0.0};
    }

    if constexpr (DMA) {
      // chunk c from (sm, sw); the next chunk (of this tile, or the first of the
      // next tile) goes straight into (nm, nw)
      auto chunk = [&](int c, const double* sm, const double* sw, double* nm, double* nw) {
        const bool in_tile = c + 1 < nchunks;
        if (in_tile || tn >= 0)
          dma_chunk(nm, nw, in_tile ? cur.M : nxt.M, in_tile ? cur.W : nxt.W,
                    in_tile ? cur.i0 : nxt.i0, in_tile ? cur.x0 : nxt.x0,
                    in_tile ? (c + 1) * BK : 0);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
          const int kr = kk + krow;
          double af[FI], bf[FX];
#pragma unroll
          for (int fi = 0; fi < FI; ++fi) af[fi] = sm[kr * LDI + wi * TI + fi * 16 + col];
#pragma unroll
          for (int fx = 0; fx < FX; ++fx) bf[fx] = sw[kr * LDX + wx * TX + fx * 16 + col];
#pragma unroll
          for (int fi = 0; fi < FI; ++fi)
#pragma unroll
            for (int fx = 0; fx < FX; ++fx)
              acc[fi][fx] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[fi], bf[fx], acc[fi][fx], 0, 0, 0);
        }
        __syncthreads();   // the next chunk has landed and nobody reads (sm, sw) any more
      };
      for (int c = 0; c < nchunks; c += 2) {
        chunk(c, dM0, dW0, dM1, dW1);
        chunk(c + 1, dM1, dW1, dM0, dW0);
      }
    } else {
      for (int c = 0; c < nchunks; ++c) {
        // next chunk: the following one of this tile, or the first of the next tile
        const bool in_tile = c + 1 < nchunks;
        const bool more = in_tile || tn >= 0;
        if (more) {
          const double* Mn = in_tile ? cur.M : nxt.M;
          const double* Wn = in_tile ? cur.W : nxt.W;
          const int i0n = in_tile ? cur.i0 : nxt.i0;
          const unsigned x0n = in_tile ? cur.x0 : nxt.x0;
          load_chunk(Mn, Wn, i0n, x0n, in_tile ? (c + 1) * BK : 0);
        }
        const double* sm = sM[buf];
        const double* sw = sW[buf];
  #pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
          const int kr = kk + krow;
          double af[FI], bf[FX];
  #pragma unroll
          for (int fi = 0; fi < FI; ++fi) af[fi] = sm[kr * LDI + wi * TI + fi * 16 + col];
  #pragma unroll
          for (int fx = 0; fx < FX; ++fx) {
            const int xl = wx * TX + fx * 16 + col;
            bf[fx] = KFAST ? sw[xl * LDK + kr] : sw[kr * LDX + xl];
          }
  #pragma unroll
          for (int fi = 0; fi < FI; ++fi)
  #pragma unroll
            for (int fx = 0; fx < FX; ++fx)
              acc[fi][fx] = KFAST ? __builtin_amdgcn_mfma_f64_16x16x4f64(bf[fx], af[fi], acc[fi][fx], 0, 0, 0)
                                  : __builtin_amdgcn_mfma_f64_16x16x4f64(af[fi], bf[fx], acc[fi][fx], 0, 0, 0);
        }
        if (more) store_chunk(buf ^ 1);
        __syncthreads();
        buf ^= 1;
      }
    }

    // epilogue of the current tile (the next tile's first chunk is already in LDS)
    if (S2 && cur.g == 1) {
      // V tile: V_{n2} = alpha*acc + beta*V_n; U_{n2} was stored by these lanes
      // when they finished the U tile of the same rows and fibres
      stage2_epilogue<FI, FX>(acc, alpha, beta, [&](int fi, int fx, int v) { return out_index(cur, fi, fx, v); },
                              a.react, out, static_cast<const double*>(a.out[0]), a.Y[0], a.Y[1],
                              static_cast<double*>(a.Rout[0]), static_cast<double*>(a.Rout[1]));
      if (tn < 0) break;
      cur = nxt;
      ++k;
      continue;
    }
    const double* Ye = y_in_acc ? nullptr : static_cast<const double*>(pick(reinterpret_cast<const void* const*>(a.Y), cur.g));
    auto epilogue = [&](auto store) {
#pragma unroll
      for (int fi = 0; fi < FI; ++fi)
#pragma unroll
        for (int fx = 0; fx < FX; ++fx)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const unsigned o = out_index(cur, fi, fx, v);
            double val = alpha * acc[fi][fx][v];
            if (Ye) val += beta * Ye[o];
            if (Z) val += gamma * Z[o];
            store(out + o, val);
          }
    };
    // Large outputs (stream_out, set by the launcher) go out with streaming
    // (non-temporal) stores; the U tiles of a stage-2 launch keep ordinary ones,
    // since their V tiles read U_{n2} straight back.
    if (!S2 && stream_out)
      epilogue([](double* p, double x) { __builtin_nontemporal_store(x, p); });
    else
      epilogue([](double* p, double x) { *p = x; });
    if (tn < 0) break;
    cur = nxt;
    ++k;
  }
}

int device_cu_count() {
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

template <int BI, int BX, int BK>
bool persist_fits(const ModeArgs& a) {
  // evenly tiled, pair-aligned shapes only; a tile's fibres stay within one batch
  if (a.n % BI != 0 || a.n % BK != 0 || a.X % BX != 0) return false;
  if (a.L != 1 && a.L % BX != 0) return false;
  if (a.n % 2 != 0) return false;
  for (int g = 0; g < a.group; ++g)
    if ((reinterpret_cast<uintptr_t>(a.W[g]) | reinterpret_cast<uintptr_t>(a.M[g])) % 16 != 0)
      return false;
  return true;
}

template <int BI, int BX, int WI, int WX, int BK>
bool launch_persist(const ModeArgs& a, hipStream_t s, hipError_t& err) {
  if (!persist_fits<BI, BX, BK>(a)) return false;
  const int n_itiles = a.n / BI;
  const long long n_xtiles = a.X / BX;
  const long long ntiles = (long long)a.group * n_itiles * n_xtiles;
  if (ntiles <= 0 || ntiles > 0x7fffffffLL || a.X >= (1LL << 31)) return false;
  long long grid = 2LL * device_cu_count();
  if (grid > ntiles) grid = ntiles;
  constexpr int NT = 64 * WI * WX;
  // x-contiguous 128x128 tiles of four waves load their chunks straight into
  // LDS (measured at 256^3: 1.4-3.5 % faster, results bitwise equal)
  constexpr bool kDma = BI == 128 && BX == 128 && WI * WX == 4;
  // streaming stores for outputs of 128 MiB or more, half the last-level cache
  // (measured, FP64 256^3 step: 1.89 against 1.915 ms, results bitwise the
  // same); smaller outputs keep ordinary stores, so that the next launch can
  // find them in that cache
  const int stream_out = (long long)a.group * a.X * a.n * 8 >= (128LL << 20) ? 1 : 0;
  if (a.Rout[0])
    hipLaunchKernelGGL((k_mode_f64_persist<BI, BX, WI, WX, BK, false, 2, true, kDma>),
                       dim3((unsigned)grid), dim3(NT), 0, s, a, n_itiles, (int)n_xtiles, (int)ntiles,
                       stream_out);
  else if (a.L == 1)
    hipLaunchKernelGGL((k_mode_f64_persist<BI, BX, WI, WX, BK, true>), dim3((unsigned)grid),
                       dim3(NT), 0, s, a, n_itiles, (int)n_xtiles, (int)ntiles,
                       stream_out);
  else
    hipLaunchKernelGGL((k_mode_f64_persist<BI, BX, WI, WX, BK, false, 2, false, kDma>),
                       dim3((unsigned)grid), dim3(NT), 0, s, a, n_itiles, (int)n_xtiles, (int)ntiles,
                       stream_out);
  err = hipGetLastError();
  return true;
}

template <int BI, int BX, int WI, int WX, int BK, int MINB = 2>
hipError_t launch_cfg(const ModeArgs& a, hipStream_t s) {
  const int n_itiles = (a.n + BI - 1) / BI;
  const long long n_xtiles = (a.X + BX - 1) / BX;
  const long long grid = (long long)a.group * n_itiles * n_xtiles;
  if (grid <= 0 || grid > 0x7fffffffLL || a.X >= (1LL << 31)) return hipErrorInvalidValue;
  constexpr int NT = 64 * WI * WX;
  const bool full = (a.n % BI == 0) && (a.n % BK == 0) && (a.X % BX == 0);
  const dim3 gd((unsigned)grid), bd(NT);
  const int nx = (int)n_xtiles;
  if (a.L == 1) {
    if (full) hipLaunchKernelGGL((k_mode_f64<BI, BX, WI, WX, BK, true, true, MINB>), gd, bd, 0, s, a, n_itiles, nx);
    else hipLaunchKernelGGL((k_mode_f64<BI, BX, WI, WX, BK, true, false, MINB>), gd, bd, 0, s, a, n_itiles, nx);
  } else {
    if (full) hipLaunchKernelGGL((k_mode_f64<BI, BX, WI, WX, BK, false, true, MINB>), gd, bd, 0, s, a, n_itiles, nx);
    else hipLaunchKernelGGL((k_mode_f64<BI, BX, WI, WX, BK, false, false, MINB>), gd, bd, 0, s, a, n_itiles, nx);
  }
  return hipGetLastError();
}

template <int BI, int BX, int WI, int WX>
hipError_t launch_grouped(bool kfast, const TileJob* jobs, int njobs, long long ntiles,
                          hipStream_t s) {
  if (njobs <= 0 || ntiles <= 0 || ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
  constexpr int NT = 64 * WI * WX;
  if (kfast)
    hipLaunchKernelGGL((k_mode_f64_grouped<BI, BX, WI, WX, 16, true>), dim3((unsigned)ntiles),
                       dim3(NT), 0, s, jobs, njobs);
  else
    hipLaunchKernelGGL((k_mode_f64_grouped<BI, BX, WI, WX, 16, false>), dim3((unsigned)ntiles),
                       dim3(NT), 0, s, jobs, njobs);
  return hipGetLastError();
}

}  // namespace

void tile_cfg_dims(TileCfg c, int& BI, int& BX) {
  switch (c) {
    case TileCfg::I64X64:
    case TileCfg::P64X64: BI = 64; BX = 64; break;
    case TileCfg::I64X128: BI = 64; BX = 128; break;
    case TileCfg::I128X64: BI = 128; BX = 64; break;
    default: BI = 128; BX = 128; break;
  }
}

hipError_t launch_mode_grouped_f64(TileCfg cfg, bool kfast, const TileJob* jobs, int njobs,
                                   long long ntiles, hipStream_t s) {
  switch (cfg) {
    case TileCfg::I64X64: return launch_grouped<64, 64, 2, 2>(kfast, jobs, njobs, ntiles, s);
    case TileCfg::I64X128: return launch_grouped<64, 128, 1, 4>(kfast, jobs, njobs, ntiles, s);
    case TileCfg::I128X64: return launch_grouped<128, 64, 2, 2>(kfast, jobs, njobs, ntiles, s);
    case TileCfg::P64X64: {
      if (njobs <= 0 || ntiles <= 0 || ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
      long long grid = 4LL * device_cu_count();
      if (grid > ntiles) grid = ntiles;
      if (kfast)
        hipLaunchKernelGGL((k_mode_f64_grouped_persist<64, 64, 2, 2, 16, true, 4>), dim3((unsigned)grid),
                           dim3(256), 0, s, jobs, njobs, ntiles);
      else
        hipLaunchKernelGGL((k_mode_f64_grouped_persist<64, 64, 2, 2, 16, false, 4>), dim3((unsigned)grid),
                           dim3(256), 0, s, jobs, njobs, ntiles);
      return hipGetLastError();
    }
    default: return launch_grouped<128, 128, 2, 2>(kfast, jobs, njobs, ntiles, s);
  }
}

bool mode_f64_stage2_fusable(const ModeArgs& a) {
  if (a.group != 2 || a.L == 1 || !a.Y[0] || !a.Y[1] || !a.out[0] || !a.out[1]) return false;
  if (a.alpha == 0.0) return false;
  return a.n % 128 != 0 ? persist_fits<64, 128, 16>(a) : persist_fits<128, 128, 16>(a);
}

// Whether `units` work items, dealt to `slots` persistent workgroups in
// contiguous ranges, keep them busy: at least one whole round, and the last
// round at least a quarter full (at 256^3: 2048 tiles of 128x128 for 512 slots).
static bool fills_rounds(long long units, long long slots) {
  if (units < slots) return false;
  const long long rounds = (units + slots - 1) / slots;
  return 4 * units >= 3 * rounds * slots;
}

// Workgroups that receive work when `units` are dealt in ranges of ceil(units / slots).
static long long active_workgroups(long long units, long long slots) {
  const long long per = (units + slots - 1) / slots;
  return (units + per - 1) / per;
}

hipError_t launch_mode_product_f64(const ModeArgs& a, hipStream_t s) {
  hipError_t e = hipSuccess;
  const long long slots = 2LL * device_cu_count();   // persistent grid (two workgroups per CU)
  if (a.Rout[0] || a.Rout[1]) {
    // stage 2 in the epilogue: only the persistent x-contiguous kernels carry it.
    // A workgroup takes U/V tile pairs; of the tile shapes that fit, the largest
    // one that puts the most workgroups to work (measured: 128^3 47 us with
    // 64x64 tiles against 72 with 128x128, 1024^2 184 against 319, 256^3 keeps
    // 128x128).
    if (!a.Rout[0] || !a.Rout[1] || !mode_f64_stage2_fusable(a)) return hipErrorInvalidValue;
    const long long u128 = persist_fits<128, 128, 16>(a) ? (a.n / 128) * (a.X / 128) : 0;
    const long long u64x128 = persist_fits<64, 128, 16>(a) ? (a.n / 64) * (a.X / 128) : 0;
    const long long u64 = persist_fits<64, 64, 16>(a) ? (a.n / 64) * (a.X / 64) : 0;
    long long best = 0;
    int pick = 0;
    if (u128 && active_workgroups(u128, slots) > best) { best = active_workgroups(u128, slots); pick = 1; }
    if (u64x128 && active_workgroups(u64x128, slots) > best) { best = active_workgroups(u64x128, slots); pick = 2; }
    if (u64 && active_workgroups(u64, slots) > best) pick = 3;
    bool launched = false;
    if (pick == 1) launched = launch_persist<128, 128, 2, 2, 16>(a, s, e);
    else if (pick == 2) launched = launch_persist<64, 128, 1, 4, 16>(a, s, e);
    else if (pick == 3) launched = launch_persist<64, 64, 2, 2, 16>(a, s, e);
    return launched ? e : hipErrorInvalidValue;
  }
  // short contractions (n < 128): 64x64 tiles, one per workgroup, four
  // workgroups per CU (measured at 64^3: 8 us per direction against 10-19 with
  // 64-row persistent tiles; 80^3: 13 against 22)
  if (a.n < 128) return launch_cfg<64, 64, 2, 2, 16, 4>(a, s);
  // 128x128 persistent tiles where they fill whole rounds of the grid;
  // fibre-contiguous products (L = 1) run best with a 2 x 4 wave grid (64 x 32
  // per wave), the others with 2 x 2 (64 x 64 per wave), measured at 256^3
  if (persist_fits<128, 128, 16>(a) &&
      fills_rounds((long long)a.group * (a.n / 128) * (a.X / 128), slots)) {
    if (a.L == 1 && launch_persist<128, 128, 2, 4, 16>(a, s, e)) return e;
    if (a.L != 1 && launch_persist<128, 128, 2, 2, 16>(a, s, e)) return e;
  }
  // long contractions that 128-row tiles would leave ragged (n % 128 != 0):
  // 64x128 persistent tiles (320x192x64, mu = 1: 111 us against 116 for 64x64)
  if (a.n % 128 != 0 && a.n >= 256 && persist_fits<64, 128, 16>(a) &&
      fills_rounds((long long)a.group * (a.n / 64) * (a.X / 128), slots) &&
      launch_persist<64, 128, 1, 4, 16>(a, s, e))
    return e;
  // otherwise 64x64 tiles: persistent when they fit in one round, else one per
  // workgroup at four workgroups per CU (measured: 192^3 128 us against 140 for
  // 64x128 tiles; 192x192x128, mu = 3: 59 against 91 for 128x128; 1024^2 93
  // against 152; 1536^2 324 against 405)
  if (persist_fits<64, 64, 16>(a)) {
    if ((long long)a.group * (a.n / 64) * (a.X / 64) <= slots && launch_persist<64, 64, 2, 2, 16>(a, s, e))
      return e;
    return launch_cfg<64, 64, 2, 2, 16, 4>(a, s);
  }
  // ragged shapes: 64-row tiles waste fewer rows while n is short
  if (a.n < 256) return launch_cfg<64, 64, 2, 2, 16, 4>(a, s);
  return launch_cfg<128, 128, 2, 2, 16>(a, s);
}

}  // namespace adr
