// FP64 mu-mode product on CDNA4 matrix cores (v_mfma_f64_16x16x4_f64).
//
// out = alpha * (W x_mu M) + beta * Y + gamma * Z,
//   (W x_mu M)[.., i, ..] = sum_k M[i, k] W[.., k, ..]           (Sec. 2)
//
// The tensor is viewed as (L, n, R) (see ModeArgs).  Each workgroup computes a
// BI x BX output tile: BI rows i of the n x n matrix against BX fibres x, with
// the contraction over k staged through LDS in chunks of BK = 16.  This is a
// GEMM whose small operand M is shared by every workgroup (it stays in L2)
// and whose large operand W is streamed from HBM once per i-tile.
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
#include "common.h"

namespace adr {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;  // 4 waves
constexpr int kBK = 16;        // contraction chunk
constexpr int kPad = 16;       // row padding (doubles): next k-row lands 32 banks away
constexpr int kLdK = kBK + 2;  // k-fastest W tile row length: conflict-free fragment reads

template <int BI, int BX, int WI, int WX, bool KFAST>
__global__ __launch_bounds__(kThreads, 2) void k_mode_f64(ModeArgs a, int n_itiles,
                                                         int n_xtiles) {
  static_assert(WI * WX == kThreads / 64, "four waves per workgroup");
  constexpr int TI = BI / WI, TX = BX / WX;  // wave tile
  constexpr int FI = TI / 16, FX = TX / 16;  // 16x16 blocks per wave
  static_assert(FI * 16 == TI && FX * 16 == TX, "wave tile must be a multiple of 16");
  constexpr int LDI = BI + kPad;
  constexpr int LDX = BX + kPad;
  constexpr int SW = KFAST ? BX * kLdK : kBK * LDX;   // W tile size in LDS
  constexpr int MROWS = kThreads / BI;                // k-rows of M loaded per pass
  constexpr int MLOADS = kBK / MROWS;                 // passes (doubles per thread)
  constexpr int WLOADS = BX * kBK / kThreads;         // W doubles per thread
  static_assert(MROWS * BI == kThreads && MLOADS * MROWS == kBK, "M tile mapping");

  __shared__ double sM[2][kBK * LDI];
  __shared__ double sW[2][SW];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wi = wave / WX, wx = wave % WX;

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

  const int n = a.n;
  const long long L = a.L, X = a.X;
  const long long Ln = L * (long long)n;
  const int i0 = itile * BI;
  const long long x0 = (long long)xtile * BX;
  const double* __restrict__ W = static_cast<const double*>(a.W[g]);
  const double* __restrict__ M = static_cast<const double*>(a.M[g]);

  // ---- per-thread load descriptors ------------------------------------------
  const int m_i = tid % BI;          // M: row i0 + m_i, k-rows m_k0 + p*MROWS
  const int m_k0 = tid / BI;
  const bool m_iok = (i0 + m_i) < n;

  // x-contiguous W: fibre x0 + w_x, k-rows w_k0 + p*(kThreads/BX)
  // k-contiguous W: k-row w_k, fibres w_x0 + p*(kThreads/kBK)
  long long w_off = -1;
  int w_a = 0, w_b = 0;
  if (!KFAST) {
    w_a = tid % BX;          // x within tile
    w_b = tid / BX;          // first k-row
    const long long x = x0 + w_a;
    if (x < X) {
      const long long l = x % L, r = x / L;
      w_off = l + Ln * r;
    }
  } else {
    w_a = tid % kBK;         // k within chunk
    w_b = tid / kBK;         // first fibre within tile
  }

  double rm[MLOADS], rw[WLOADS];

  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int p = 0; p < MLOADS; ++p) {
      const int k = k0 + m_k0 + p * MROWS;
      rm[p] = (m_iok && k < n) ? M[(i0 + m_i) + (long long)n * k] : 0.0;
    }
    if (!KFAST) {
      constexpr int WROWS = kThreads / BX;
#pragma unroll
      for (int p = 0; p < WLOADS; ++p) {
        const int k = k0 + w_b + p * WROWS;
        rw[p] = (w_off >= 0 && k < n) ? W[w_off + L * k] : 0.0;
      }
    } else {
      constexpr int XSTEP = kThreads / kBK;
      const int k = k0 + w_a;
#pragma unroll
      for (int p = 0; p < WLOADS; ++p) {
        const long long x = x0 + w_b + p * XSTEP;
        rw[p] = (x < X && k < n) ? W[x * n + k] : 0.0;
      }
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int p = 0; p < MLOADS; ++p) sM[buf][(m_k0 + p * MROWS) * LDI + m_i] = rm[p];
    if (!KFAST) {
      constexpr int WROWS = kThreads / BX;
#pragma unroll
      for (int p = 0; p < WLOADS; ++p) sW[buf][(w_b + p * WROWS) * LDX + w_a] = rw[p];
    } else {
      constexpr int XSTEP = kThreads / kBK;
#pragma unroll
      for (int p = 0; p < WLOADS; ++p) sW[buf][(w_b + p * XSTEP) * kLdK + w_a] = rw[p];
    }
  };

  d4 acc[FI][FX];
#pragma unroll
  for (int fi = 0; fi < FI; ++fi)
#pragma unroll
    for (int fx = 0; fx < FX; ++fx) acc[fi][fx] = d4{0.0, 0.0, 0.0, 0.0};

  const int nchunks = (n + kBK - 1) / kBK;
  load_chunk(0);
  store_chunk(0);
  __syncthreads();

  const int col = lane & 15;
  const int krow = lane >> 4;
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunks) load_chunk((c + 1) * kBK);
    const double* sm = sM[buf];
    const double* sw = sW[buf];
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      const int kr = kk + krow;
      double af[FI], bf[FX];
#pragma unroll
      for (int fi = 0; fi < FI; ++fi) af[fi] = sm[kr * LDI + wi * TI + fi * 16 + col];
#pragma unroll
      for (int fx = 0; fx < FX; ++fx) {
        const int xl = wx * TX + fx * 16 + col;
        bf[fx] = KFAST ? sw[xl * kLdK + kr] : sw[kr * LDX + xl];
      }
#pragma unroll
      for (int fi = 0; fi < FI; ++fi)
#pragma unroll
        for (int fx = 0; fx < FX; ++fx)
          acc[fi][fx] = KFAST ? __builtin_amdgcn_mfma_f64_16x16x4f64(bf[fx], af[fi], acc[fi][fx], 0, 0, 0)
                              : __builtin_amdgcn_mfma_f64_16x16x4f64(af[fi], bf[fx], acc[fi][fx], 0, 0, 0);
    }
    if (c + 1 < nchunks) store_chunk(buf ^ 1);
    __syncthreads();
  }

  // ---- epilogue: out = alpha*acc + beta*Y + gamma*Z --------------------------
  // Y may alias out (each element is read, then written, by the same lane)
  double* out = static_cast<double*>(a.out[g]);
  const double* Y = a.Y[g];
  const double* Z = a.Z[g];
  const double alpha = a.alpha, beta = a.beta, gamma = a.gamma;
  if (!KFAST) {
#pragma unroll
    for (int fx = 0; fx < FX; ++fx) {
      const long long x = x0 + wx * TX + fx * 16 + col;
      if (x >= X) continue;
      const long long xo = (x % L) + Ln * (x / L);
#pragma unroll
      for (int fi = 0; fi < FI; ++fi) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + wi * TI + fi * 16 + krow + 4 * v;
          if (i < n) {
            const long long o = xo + L * i;
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
          const long long x = x0 + wx * TX + fx * 16 + krow + 4 * v;
          if (x < X) {
            const long long o = x * n + i;
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

template <int BI, int BX, int WI, int WX>
hipError_t launch_cfg(const ModeArgs& a, hipStream_t s) {
  const int n_itiles = (a.n + BI - 1) / BI;
  const long long n_xtiles = (a.X + BX - 1) / BX;
  const long long grid = (long long)a.group * n_itiles * n_xtiles;
  if (grid <= 0 || grid > 0x7fffffffLL || n_xtiles > 0x7fffffffLL) return hipErrorInvalidValue;
  if (a.L == 1)
    hipLaunchKernelGGL((k_mode_f64<BI, BX, WI, WX, true>), dim3((unsigned)grid), dim3(kThreads), 0,
                       s, a, n_itiles, (int)n_xtiles);
  else
    hipLaunchKernelGGL((k_mode_f64<BI, BX, WI, WX, false>), dim3((unsigned)grid), dim3(kThreads), 0,
                       s, a, n_itiles, (int)n_xtiles);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mode_product_f64(const ModeArgs& a, hipStream_t s) {
  if (a.n <= 64) return launch_cfg<64, 128, 1, 4>(a, s);
  return launch_cfg<128, 128, 2, 2>(a, s);
}

}  // namespace adr
