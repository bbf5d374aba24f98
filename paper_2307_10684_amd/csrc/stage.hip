// Pointwise stage kernels of ETD2RKds (Sec. 3, eq. (11)) and Lawson2b (Sec. 2,
// eq. (7)): reaction terms G^u, G^v, the Kronecker-sum action K C as a stencil
// when A_mu is tridiagonal, and the combinations that feed the Tucker operators.
// All are HBM-bound streaming kernels; the state U, V is FP64 throughout.
#include "common.h"

namespace adr {
namespace {

// Reaction terms (the constants' order is documented in include/adr.h).
__device__ __forceinline__ void react(const Reaction& r, double u, double v, double& gu,
                                      double& gv) {
  switch (r.model) {
    case 0: {  // Schnakenberg: gamma(a - u + u^2 v), gamma(b - u^2 v)
      const double u2v = u * u * v;
      gu = r.p[0] * (r.p[1] - u + u2v);
      gv = r.p[0] * (r.p[2] - u2v);
      break;
    }
    case 1: {  // FitzHugh-Nagumo: rho(u - u^3 - v), rho eps(u - a1 v - a0)
      gu = r.p[0] * (u - u * u * u - v);
      gv = r.p[0] * r.p[1] * (u - r.p[2] * v - r.p[3]);
      break;
    }
    case 2: {  // Brusselator: A - (B+1) u + u^2 v,  B u - u^2 v
      const double u2v = u * u * v;
      gu = r.p[0] - (r.p[1] + 1.0) * u + u2v;
      gv = r.p[1] * u - u2v;
      break;
    }
    default:
      gu = 0.0;
      gv = 0.0;
  }
}

template <typename T>
__device__ __forceinline__ void put(void* p, long long q, double x) {
  static_cast<T*>(p)[q] = static_cast<T>(x);
}

// Stage 1: R^c = sum_mu (C x_mu A_mu^c) + G^c(U, V) for the directions with a
// band; directions without one are added afterwards by dense mode products.
// Block = (64, 4): each wave covers 64 consecutive i_1 of one grid row, so the
// i_1 +- 1 neighbours come from lane shuffles; i_2, i_3 neighbours are plain
// loads that hit in cache (the rows were just streamed by nearby waves).
template <typename TR>
__global__ __launch_bounds__(256) void k_etd_stage1(StageGeom g, Reaction r,
                                                    const double* __restrict__ U,
                                                    const double* __restrict__ V, void* Ru,
                                                    void* Rv, long long rows) {
  const int n1 = g.n[0];
  const int i1 = blockIdx.x * 64 + threadIdx.x;
  for (long long row = (long long)blockIdx.y * 4 + threadIdx.y; row < rows;
       row += (long long)gridDim.y * 4) {
    const bool live = i1 < n1;
    const long long q = row * n1 + i1;
    const double u = live ? U[q] : 0.0;
    const double v = live ? V[q] : 0.0;
    // i_1 neighbours from the adjacent lanes; the wave edges load directly
    double um = __shfl_up(u, 1, 64), up = __shfl_down(u, 1, 64);
    double vm = __shfl_up(v, 1, 64), vp = __shfl_down(v, 1, 64);
    const int lane = threadIdx.x;
    if (lane == 0) {
      um = (live && i1 > 0) ? U[q - 1] : 0.0;
      vm = (live && i1 > 0) ? V[q - 1] : 0.0;
    }
    if (lane == 63 || i1 + 1 >= n1) {
      up = (live && i1 + 1 < n1) ? U[q + 1] : 0.0;
      vp = (live && i1 + 1 < n1) ? V[q + 1] : 0.0;
    }
    if (!live) continue;
    if (i1 == 0) { um = 0.0; vm = 0.0; }
    double gu, gv;
    react(r, u, v, gu, gv);
    double ku = 0.0, kv = 0.0;
    // direction 1
    if (g.band[0][0]) {
      const double* b = g.band[0][0];
      ku += b[i1] * um + b[n1 + i1] * u + b[2 * n1 + i1] * up;
    }
    if (g.band[1][0]) {
      const double* b = g.band[1][0];
      kv += b[i1] * vm + b[n1 + i1] * v + b[2 * n1 + i1] * vp;
    }
    // directions 2 and 3
    long long stride = n1;
    long long rem = row;
#pragma unroll
    for (int mu = 1; mu < 3; ++mu) {
      if (mu >= g.d) break;
      const int nm = g.n[mu];
      const int im = (int)(rem % nm);
      rem /= nm;
      const bool has_m = im > 0, has_p = im + 1 < nm;
      if (g.band[0][mu]) {
        const double* b = g.band[0][mu];
        const double cm = has_m ? U[q - stride] : 0.0;
        const double cp = has_p ? U[q + stride] : 0.0;
        ku += b[im] * cm + b[nm + im] * u + b[2 * nm + im] * cp;
      }
      if (g.band[1][mu]) {
        const double* b = g.band[1][mu];
        const double cm = has_m ? V[q - stride] : 0.0;
        const double cp = has_p ? V[q + stride] : 0.0;
        kv += b[im] * cm + b[nm + im] * v + b[2 * nm + im] * cp;
      }
      stride *= nm;
    }
    put<TR>(Ru, q, ku + gu);
    put<TR>(Rv, q, kv + gv);
  }
}

// Stage 2: R^c = G^c(U2, V2) - G^c(U, V).
template <typename TR>
__global__ __launch_bounds__(256) void k_etd_stage2(long long N, Reaction r,
                                                    const double* __restrict__ U,
                                                    const double* __restrict__ V,
                                                    const double* __restrict__ U2,
                                                    const double* __restrict__ V2, void* Ru,
                                                    void* Rv) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
       q += (long long)gridDim.x * blockDim.x) {
    double gu, gv, gu2, gv2;
    react(r, U[q], V[q], gu, gv);
    react(r, U2[q], V2[q], gu2, gv2);
    put<TR>(Ru, q, gu2 - gu);
    put<TR>(Rv, q, gv2 - gv);
  }
}

// Lawson2b stage 1: A^c = C + tau G^c,  B^c = C + tau/2 G^c.
template <typename TR>
__global__ __launch_bounds__(256) void k_law_stage1(long long N, Reaction r, double tau,
                                                    const double* __restrict__ U,
                                                    const double* __restrict__ V, void* Au,
                                                    void* Av, void* Bu, void* Bv) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
       q += (long long)gridDim.x * blockDim.x) {
    const double u = U[q], v = V[q];
    double gu, gv;
    react(r, u, v, gu, gv);
    put<TR>(Au, q, u + tau * gu);
    put<TR>(Av, q, v + tau * gv);
    put<TR>(Bu, q, u + 0.5 * tau * gu);
    put<TR>(Bv, q, v + 0.5 * tau * gv);
  }
}

// Lawson2b stage 2: C += tau/2 G^c(U2, V2).
__global__ __launch_bounds__(256) void k_law_stage2(long long N, Reaction r, double tau,
                                                    double* __restrict__ U,
                                                    double* __restrict__ V,
                                                    const double* __restrict__ U2,
                                                    const double* __restrict__ V2) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
       q += (long long)gridDim.x * blockDim.x) {
    double gu, gv;
    react(r, U2[q], V2[q], gu, gv);
    U[q] += 0.5 * tau * gu;
    V[q] += 0.5 * tau * gv;
  }
}

__global__ __launch_bounds__(256) void k_copy(const double* __restrict__ in,
                                              double* __restrict__ out, size_t count) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < count;
       q += (size_t)gridDim.x * blockDim.x)
    out[q] = in[q];
}

__global__ __launch_bounds__(256) void k_f64_to_f32(const double* __restrict__ in,
                                                    float* __restrict__ out, size_t count) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < count;
       q += (size_t)gridDim.x * blockDim.x)
    out[q] = (float)in[q];
}

unsigned stream_grid(long long N) {
  // enough workgroups to cover the 256 CUs many times over, capped for grid-stride loops
  long long b = (N + 255) / 256;
  if (b > 256 * 64) b = 256 * 64;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_etd_stage1(const StageGeom& g, const Reaction& r, const double* U,
                             const double* V, void* Ru, void* Rv, int r_f32, hipStream_t s) {
  long long rows = 1;
  for (int mu = 1; mu < g.d; ++mu) rows *= g.n[mu];
  const unsigned gx = (unsigned)((g.n[0] + 63) / 64);
  long long gy = (rows + 3) / 4;
  if (gy > 65535) gy = 65535;
  dim3 grid(gx, (unsigned)gy), block(64, 4);
  if (r_f32)
    hipLaunchKernelGGL(k_etd_stage1<float>, grid, block, 0, s, g, r, U, V, Ru, Rv, rows);
  else
    hipLaunchKernelGGL(k_etd_stage1<double>, grid, block, 0, s, g, r, U, V, Ru, Rv, rows);
  return hipGetLastError();
}

hipError_t launch_etd_stage2(long long N, const Reaction& r, const double* U, const double* V,
                             const double* U2, const double* V2, void* Ru, void* Rv, int r_f32,
                             hipStream_t s) {
  if (r_f32)
    hipLaunchKernelGGL(k_etd_stage2<float>, dim3(stream_grid(N)), dim3(256), 0, s, N, r, U, V, U2,
                       V2, Ru, Rv);
  else
    hipLaunchKernelGGL(k_etd_stage2<double>, dim3(stream_grid(N)), dim3(256), 0, s, N, r, U, V, U2,
                       V2, Ru, Rv);
  return hipGetLastError();
}

hipError_t launch_lawson_stage1(long long N, const Reaction& r, double tau, const double* U,
                                const double* V, void* Au, void* Av, void* Bu, void* Bv, int f32,
                                hipStream_t s) {
  if (f32)
    hipLaunchKernelGGL(k_law_stage1<float>, dim3(stream_grid(N)), dim3(256), 0, s, N, r, tau, U, V,
                       Au, Av, Bu, Bv);
  else
    hipLaunchKernelGGL(k_law_stage1<double>, dim3(stream_grid(N)), dim3(256), 0, s, N, r, tau, U,
                       V, Au, Av, Bu, Bv);
  return hipGetLastError();
}

hipError_t launch_lawson_stage2(long long N, const Reaction& r, double tau, double* U, double* V,
                                const double* U2, const double* V2, hipStream_t s) {
  hipLaunchKernelGGL(k_law_stage2, dim3(stream_grid(N)), dim3(256), 0, s, N, r, tau, U, V, U2, V2);
  return hipGetLastError();
}

hipError_t launch_copy_f64(const double* in, double* out, size_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(stream_grid((long long)count)), dim3(256), 0, s, in, out, count);
  return hipGetLastError();
}

hipError_t launch_convert_f64_f32(const double* in, float* out, size_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_f64_to_f32, dim3(stream_grid((long long)count)), dim3(256), 0, s, in, out,
                     count);
  return hipGetLastError();
}

}  // namespace adr
