// Dynamics indicators of Sec. 4 as one fused, deterministic reduction:
// trapezoidal spatial means of U and V on the node-centred grid, Frobenius
// norms of the increments U - Uprev, V - Vprev, and a count of grid points
// holding a non-finite value.  HBM-bound: one pass over up to four tensors.
//
// Pass 1: block b reduces the contiguous index range [b*chunk, (b+1)*chunk)
// into five partial sums; pass 2: one block adds the partials in a fixed
// order and forms the record.  No atomics, so the result does not depend on
// scheduling.
#include "common.h"

namespace adr {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Sum five per-thread values over the block; thread 0 gets the totals.
__device__ __forceinline__ void block_sum5(double (&v)[5]) {
  __shared__ double part[kThreads / 64][5];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 5; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 5; ++k) part[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      double s = 0.0;
      for (int w = 0; w < kThreads / 64; ++w) s += part[w][k];
      v[k] = s;
    }
}

// trapezoidal weight of node i of n (a direction of length 1 is not a grid
// direction: weight 1)
__device__ __forceinline__ double edge_weight(unsigned i, unsigned n) {
  return (n > 1u && (i == 0u || i + 1u == n)) ? 0.5 : 1.0;
}

__global__ __launch_bounds__(kThreads) void k_ind_partial(unsigned N, unsigned n1, unsigned n2,
                                                          unsigned n3, unsigned chunk,
                                                          const double* __restrict__ U,
                                                          const double* __restrict__ V,
                                                          const double* __restrict__ Up,
                                                          const double* __restrict__ Vp,
                                                          double* __restrict__ partial) {
  const unsigned q0 = blockIdx.x * chunk;
  const unsigned q1 = min(q0 + chunk, N);
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const bool inc = Up != nullptr;
  for (unsigned q = q0 + threadIdx.x; q < q1; q += kThreads) {
    const unsigned i1 = q % n1, r = q / n1;
    const unsigned i2 = r % n2, i3 = r / n2;
    const double w = edge_weight(i1, n1) * edge_weight(i2, n2) * edge_weight(i3, n3);
    const double u = U[q], v = V[q];
    acc[0] += w * u;
    acc[1] += w * v;
    bool bad = !isfinite(u) || !isfinite(v);
    if (inc) {
      const double pu = Up[q], pv = Vp[q];
      const double du = u - pu, dv = v - pv;
      acc[2] += du * du;
      acc[3] += dv * dv;
      bad = bad || !isfinite(pu) || !isfinite(pv);
    }
    acc[4] += bad ? 1.0 : 0.0;
  }
  block_sum5(acc);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 5; ++k) partial[blockIdx.x * 5 + k] = acc[k];
}

__global__ __launch_bounds__(kThreads) void k_ind_final(int nblocks, double wsum,
                                                        const double* __restrict__ partial,
                                                        double* __restrict__ rec) {
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kThreads)
#pragma unroll
    for (int k = 0; k < 5; ++k) acc[k] += partial[b * 5 + k];
  block_sum5(acc);
  if (threadIdx.x == 0) {
    rec[0] = acc[0] / wsum;
    rec[1] = acc[1] / wsum;
    rec[2] = sqrt(acc[2]);
    rec[3] = sqrt(acc[3]);
    rec[4] = acc[4];
  }
}

}  // namespace

int indicator_blocks(long long N) {
  const long long per = 8LL * kThreads;  // at least 8 points per thread
  long long nb = (N + per - 1) / per;
  if (nb > kMaxIndicatorBlocks) nb = kMaxIndicatorBlocks;
  return (int)(nb < 1 ? 1 : nb);
}

hipError_t launch_indicators(int d, const int* n, const double* U, const double* V,
                             const double* Up, const double* Vp, double* partial, double* rec,
                             hipStream_t s) {
  unsigned nn[3] = {1u, 1u, 1u};
  long long N = 1;
  double wsum = 1.0;
  for (int mu = 0; mu < d; ++mu) {
    nn[mu] = (unsigned)n[mu];
    N *= n[mu];
    wsum *= (double)(n[mu] - 1);
  }
  if (N <= 0 || N >= (1LL << 31) || (Up == nullptr) != (Vp == nullptr)) return hipErrorInvalidValue;
  const int nb = indicator_blocks(N);
  const unsigned chunk = (unsigned)((N + nb - 1) / nb);
  hipLaunchKernelGGL(k_ind_partial, dim3(nb), dim3(kThreads), 0, s, (unsigned)N, nn[0], nn[1],
                     nn[2], chunk, U, V, Up, Vp, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ind_final, dim3(1), dim3(kThreads), 0, s, nb, wsum, partial, rec);
  return hipGetLastError();
}

}  // namespace adr
