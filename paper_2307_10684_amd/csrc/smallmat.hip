// Small dense n x n helpers for the matrix-function precompute (FP64,
// column-major): the 1-norm that sets the scaling power, scaled copies, and
// linear combinations of matrix powers for the Taylor polynomial.  Products
// of two n x n matrices go through the mode-product kernel (a GEMM is the
// mode-1 product of a 2-tensor).
#include "common.h"

namespace adr {
namespace {

// ||scale * X||_1 = max_j sum_i |scale X[i,j]|; NaN if any entry is not finite.
__global__ __launch_bounds__(256) void k_norm1(int n, const double* __restrict__ X, double scale,
                                               double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  bool bad = false;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      const double x = scale * X[i + (long long)n * j];
      bad |= !isfinite(x);
      s += fabs(x);
    }
    m = fmax(m, s);
  }
  red[threadIdx.x] = bad ? __builtin_nan("") : m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double a = red[threadIdx.x], b = red[threadIdx.x + w];
      red[threadIdx.x] = (isnan(a) || isnan(b)) ? __builtin_nan("") : fmax(a, b);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ __launch_bounds__(256) void k_scale_copy(long long count, const double* __restrict__ in,
                                                    double scale, double* __restrict__ out) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < count;
       q += (long long)gridDim.x * blockDim.x)
    out[q] = scale * in[q];
}

struct Comb {
  const double* P[8];
  double c[8];
  int count;
  double c0;
};

__global__ __launch_bounds__(256) void k_lincomb(int n, Comb cb, double* __restrict__ out) {
  const long long nn = (long long)n * n;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nn;
       q += (long long)gridDim.x * blockDim.x) {
    const long long i = q % n, j = q / n;
    double acc = (i == j) ? cb.c0 : 0.0;
    for (int t = 0; t < cb.count; ++t) acc += cb.c[t] * cb.P[t][q];
    out[q] = acc;
  }
}

unsigned small_grid(long long count) {
  long long b = (count + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_norm1(int n, const double* X, double scale, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_norm1, dim3(1), dim3(256), 0, s, n, X, scale, out);
  return hipGetLastError();
}

hipError_t launch_scale_copy(long long count, const double* in, double scale, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(small_grid(count)), dim3(256), 0, s, count, in, scale, out);
  return hipGetLastError();
}

hipError_t launch_lincomb(int n, int count, const double* const* P, const double* c, double c0,
                          double* out, hipStream_t s) {
  if (count < 0 || count > 8) return hipErrorInvalidValue;
  Comb cb{};
  for (int t = 0; t < count; ++t) {
    cb.P[t] = P[t];
    cb.c[t] = c[t];
  }
  cb.count = count;
  cb.c0 = c0;
  hipLaunchKernelGGL(k_lincomb, dim3(small_grid((long long)n * n)), dim3(256), 0, s, n, cb, out);
  return hipGetLastError();
}

}  // namespace adr
