// The first two mu-mode products of a Tucker operator (Sec. 2, eq. (5)) in
// one pass, for tensors whose (i1, i2) planes fit in LDS:
//
//   out[:, :, p] = alpha * M1 W[:, :, p] M2^T  (+ beta * Y[:, :, p]),
//
// i.e. (W x_1 M1 x_2 M2) plane by plane: the products along directions 1 and 2
// act within each i3 plane.  One workgroup takes one plane of one tensor: the
// plane (N x N FP64, N = 64 or 128) goes from HBM straight into LDS, the first
// product Y = M1 W reads it there, Y replaces it in LDS, the second product
// Z = Y M2^T reads Y there, and Z goes back through LDS so that the stores
// are whole 16-byte pieces of contiguous columns.  The plane is read from and
// written to HBM once for both products.  M1 and M2 stream through LDS in
// chunks of 16 columns (they are small and stay in L2).
//
// LDS layout of the plane: column c (the i2 index) holds rows r (i1) at
// c * N + (r ^ (c % 16)); the permutation sends the 16 consecutive columns of
// a fragment read (fixed r) to 16 different double slots of a 128-byte bank
// window, so those reads and the stores of the products' results are free of
// bank conflicts.  (Keeping row pairs together for 16-byte LDS-direct loads
// allows only even masks, 8 distinct slots and two-way conflicts; the plane
// is therefore copied with 4-byte LDS-direct loads, each lane choosing the
// half of the double its LDS word holds.)
//
// FP64 MFMA fragments (v_mfma_f64_16x16x4f64): A[l%16][l/16], B[l/16][l%16],
// D[4v + l/16][l%16], v = 0..3.
#include "common.h"

namespace adr {
namespace {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));

struct PlaneArgs {
  const double* W[kMaxGroup];
  const double* M1[kMaxGroup];
  const double* M2[kMaxGroup];
  double* out[kMaxGroup];
  const double* Y[kMaxGroup];   // optional addend (may alias out)
  double alpha, beta;
  int planes;                   // planes per tensor (n3; 1 for d = 2)
};

template <int N>
__device__ __forceinline__ int pidx(int r, int c) {
  return c * N + (r ^ (c & 15));
}

// 16 KB (N = 128) or 8 KB (N = 64) of a chunk: 16 whole columns of M, contiguous
// in global memory and in LDS; each wave copies 1 KB spans.
template <int N, int NW>
__device__ __forceinline__ void dma_chunk(double* dst, const double* __restrict__ M, int k0, int wave) {
  constexpr int SPANS = 16 * N / 128;          // 1 KB spans (128 doubles) per chunk
  static_assert(SPANS % NW == 0, "spans per wave");
#pragma unroll
  for (int s = 0; s < SPANS / NW; ++s) {
    const int span = wave + s * NW;
    const int lane = threadIdx.x & 63;
    __builtin_amdgcn_global_load_lds(M + (size_t)k0 * N + span * 128 + 2 * lane, dst + span * 128, 16, 0, 0);
  }
}

// The plane: each wave instruction fills 32 consecutive LDS doubles (256
// bytes, 4 per lane); lane l fills the low (l even) or high (l odd) word of
// position l / 2 of them with the same word of row (q ^ (c % 16)), q the
// position in column c.  The 32 rows of one instruction are a permutation of
// an aligned block of 32 rows, so each instruction reads 256 contiguous bytes.
template <int N, int NW>
__device__ __forceinline__ void dma_plane(double* P, const double* __restrict__ W, int wave) {
  constexpr int PSPANS = N * N / 32;
  const int lane = threadIdx.x & 63;
#pragma unroll 8
  for (int s = wave; s < PSPANS; s += NW) {
    const int e = s * 32 + (lane >> 1);
    const int c = e / N, q = e % N;
    const char* src = reinterpret_cast<const char*>(W + (size_t)c * N + (q ^ (c & 15))) + 4 * (lane & 1);
    __builtin_amdgcn_global_load_lds(src, P + s * 32, 4, 0, 0);
  }
}

template <int N, int WI, int WX>
__global__ __launch_bounds__(64 * WI * WX, 1) void k_mode12_plane(PlaneArgs a) {
  constexpr int NW = WI * WX;
  constexpr int TI = N / WI, TX = N / WX, FI = TI / 16, FX = TX / 16;
  constexpr int BK = 16, NCH = N / BK;
  static_assert(FI * 16 == TI && FX * 16 == TX && NCH % 2 == 0, "tiling");
  __shared__ double P[N * N];
  __shared__ double C0[BK * N], C1[BK * N];   // chunks of M1, then of M2: [k][row]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave / WX, wx = wave % WX;
  const int col = lane & 15, krow = lane >> 4;
  const int g = blockIdx.x / a.planes, p = blockIdx.x % a.planes;
  const size_t plane_off = (size_t)p * N * N;
  const double* __restrict__ W = a.W[g] + plane_off;
  const double* __restrict__ M1 = a.M1[g];
  const double* __restrict__ M2 = a.M2[g];

  dma_plane<N, NW>(P, W, wave);
  dma_chunk<N, NW>(C0, M1, 0, wave);
  __syncthreads();

  d4 acc[FI][FX];
#pragma unroll
  for (int fi = 0; fi < FI; ++fi)
#pragma unroll
    for (int fx = 0; fx < FX; ++fx) acc[fi][fx] = d4{0.0, 0.0, 0.0, 0.0};

  // ---- Y = M1 W: A from the M1 chunk [k][i], B from the plane (rows k, columns j)
  auto gemm1 = [&](int c, const double* cm, double* nm) {
    if (c + 1 < NCH) dma_chunk<N, NW>(nm, M1, (c + 1) * BK, wave);
    else dma_chunk<N, NW>(nm, M2, 0, wave);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int k = c * BK + kk + krow;
      double af[FI], bf[FX];
#pragma unroll
      for (int fi = 0; fi < FI; ++fi) af[fi] = cm[(kk + krow) * N + wi * TI + fi * 16 + col];
#pragma unroll
      for (int fx = 0; fx < FX; ++fx) bf[fx] = P[pidx<N>(k, wx * TX + fx * 16 + col)];
#pragma unroll
      for (int fi = 0; fi < FI; ++fi)
#pragma unroll
        for (int fx = 0; fx < FX; ++fx)
          acc[fi][fx] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[fi], bf[fx], acc[fi][fx], 0, 0, 0);
    }
    __syncthreads();
  };
  for (int c = 0; c < NCH; c += 2) {
    gemm1(c, C0, C1);
    gemm1(c + 1, C1, C0);
  }
  // the last barrier also ended every read of the plane: Y replaces W
#pragma unroll
  for (int fi = 0; fi < FI; ++fi)
#pragma unroll
    for (int fx = 0; fx < FX; ++fx)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        P[pidx<N>(wi * TI + fi * 16 + 4 * v + krow, wx * TX + fx * 16 + col)] = acc[fi][fx][v];
        acc[fi][fx][v] = 0.0;
      }
  __syncthreads();

  // ---- Z = Y M2^T: A from the plane (Y[i][k]), B[k][j] = M2[j][k] from the M2 chunk [k][j]
  auto gemm2 = [&](int c, const double* cm, double* nm) {
    if (c + 1 < NCH) dma_chunk<N, NW>(nm, M2, (c + 1) * BK, wave);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int k = c * BK + kk + krow;
      double af[FI], bf[FX];
#pragma unroll
      for (int fi = 0; fi < FI; ++fi) af[fi] = P[pidx<N>(wi * TI + fi * 16 + col, k)];
#pragma unroll
      for (int fx = 0; fx < FX; ++fx) bf[fx] = cm[(kk + krow) * N + wx * TX + fx * 16 + col];
#pragma unroll
      for (int fi = 0; fi < FI; ++fi)
#pragma unroll
        for (int fx = 0; fx < FX; ++fx)
          acc[fi][fx] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[fi], bf[fx], acc[fi][fx], 0, 0, 0);
    }
    __syncthreads();
  };
  for (int c = 0; c < NCH; c += 2) {
    gemm2(c, C0, C1);
    gemm2(c + 1, C1, C0);
  }
  // Z replaces Y in LDS (the last barrier ended every read of Y) ...
#pragma unroll
  for (int fi = 0; fi < FI; ++fi)
#pragma unroll
    for (int fx = 0; fx < FX; ++fx)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        P[pidx<N>(wi * TI + fi * 16 + 4 * v + krow, wx * TX + fx * 16 + col)] = acc[fi][fx][v];
  __syncthreads();
  // ... and leaves it column by column, two consecutive rows per lane
  double* out = a.out[g] + plane_off;   // may alias Yp (same element, same lane)
  const double* Yp = a.Y[g] ? a.Y[g] + plane_off : nullptr;
  const double alpha = a.alpha, beta = a.beta;
  constexpr int NT = 64 * NW;
#pragma unroll 4
  for (int e = 2 * tid; e < N * N; e += 2 * NT) {
    const int c = e / N, r = e % N;
    const d2 z = {P[pidx<N>(r, c)], P[pidx<N>(r + 1, c)]};
    d2 o = {alpha * z[0], alpha * z[1]};
    if (Yp) {
      const d2 y = *reinterpret_cast<const d2*>(Yp + e);
      o[0] += beta * y[0];
      o[1] += beta * y[1];
    }
    *reinterpret_cast<d2*>(out + e) = o;
  }
}

}  // namespace

bool mode12_plane_fits(int n1, int n2) { return n1 == n2 && (n1 == 64 || n1 == 128); }

hipError_t launch_mode12_plane(int group, const double* const* W, const double* const* M1,
                               const double* const* M2, double* const* out,
                               const double* const* Y, double alpha, double beta, int n,
                               int planes, hipStream_t s) {
  if (group < 1 || group > kMaxGroup || planes < 1 || !mode12_plane_fits(n, n))
    return hipErrorInvalidValue;
  PlaneArgs a{};
  for (int g = 0; g < group; ++g) {
    if (!W[g] || !M1[g] || !M2[g] || !out[g] || W[g] == out[g]) return hipErrorInvalidValue;
    if (reinterpret_cast<uintptr_t>(W[g]) % 16 || reinterpret_cast<uintptr_t>(out[g]) % 16 ||
        reinterpret_cast<uintptr_t>(M1[g]) % 16 || reinterpret_cast<uintptr_t>(M2[g]) % 16 ||
        (Y && Y[g] && reinterpret_cast<uintptr_t>(Y[g]) % 16))
      return hipErrorInvalidValue;
    a.W[g] = W[g];
    a.M1[g] = M1[g];
    a.M2[g] = M2[g];
    a.out[g] = out[g];
    a.Y[g] = Y ? Y[g] : nullptr;
  }
  a.alpha = alpha;
  a.beta = beta;
  a.planes = planes;
  const long long grid = (long long)group * planes;
  if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
  if (n == 128)
    hipLaunchKernelGGL((k_mode12_plane<128, 4, 2>), dim3((unsigned)grid), dim3(512), 0, s, a);
  else
    hipLaunchKernelGGL((k_mode12_plane<64, 2, 2>), dim3((unsigned)grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace adr
