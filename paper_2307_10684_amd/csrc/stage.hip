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
// Block = (64, 4) threads over (i_1, i_2); each block marches through ZB planes
// of i_3.  The loop is software-pipelined: while plane z is computed, the
// values of plane z+1 that a thread needs (its own point, its i_2 +- 1
// neighbours and, on the wave edges, its i_1 +- 1 neighbours) are already in
// flight, and the i_3 neighbours are the previous / next planes held in
// registers.  Inside a wave the i_1 +- 1 neighbours come from lane shuffles.
constexpr int kZB = 16;  // planes per block

struct Plane {
  double c, ym, yp, xm, xp;  // centre, i_2 -+ 1, i_1 -+ 1 (wave-edge lanes only)
};

template <typename TR>
__global__ __launch_bounds__(256) void k_etd_stage1(StageGeom g, Reaction r,
                                                    const double* __restrict__ U,
                                                    const double* __restrict__ V, void* Ru,
                                                    void* Rv) {
  const int n1 = g.n[0], n2 = g.d >= 2 ? g.n[1] : 1, n3 = g.d >= 3 ? g.n[2] : 1;
  const int i1 = blockIdx.x * 64 + threadIdx.x;
  const int i2 = blockIdx.y * 4 + threadIdx.y;
  const int z0 = blockIdx.z * kZB;
  const int z1 = min(z0 + kZB, n3);
  const bool live = i1 < n1 && i2 < n2;
  const unsigned P = (unsigned)n1 * (unsigned)n2;  // plane stride
  const int lane = threadIdx.x;
  // per-thread band coefficients of directions 1 and 2 (zero where there is no
  // neighbour and where the direction has no band)
  double a1u[3] = {0, 0, 0}, a1v[3] = {0, 0, 0}, a2u[3] = {0, 0, 0}, a2v[3] = {0, 0, 0};
  if (live) {
    if (g.band[0][0]) for (int j = 0; j < 3; ++j) a1u[j] = g.band[0][0][j * n1 + i1];
    if (g.band[1][0]) for (int j = 0; j < 3; ++j) a1v[j] = g.band[1][0][j * n1 + i1];
    if (g.d >= 2) {
      if (g.band[0][1]) for (int j = 0; j < 3; ++j) a2u[j] = g.band[0][1][j * n2 + i2];
      if (g.band[1][1]) for (int j = 0; j < 3; ++j) a2v[j] = g.band[1][1][j * n2 + i2];
    }
  }
  const double* b3u = g.d >= 3 ? g.band[0][2] : nullptr;
  const double* b3v = g.d >= 3 ? g.band[1][2] : nullptr;
  const bool has_m2 = live && i2 > 0, has_p2 = live && i2 + 1 < n2;
  const bool edge_m = live && lane == 0 && i1 > 0;
  const bool edge_p = live && lane == 63 && i1 + 1 < n1;
  const unsigned q0 = (unsigned)i2 * (unsigned)n1 + (unsigned)i1;

  auto fetch = [&](const double* __restrict__ C, int z, Plane& o) {
    const unsigned q = q0 + (unsigned)z * P;
    o.c = live ? C[q] : 0.0;
    o.ym = has_m2 ? C[q - n1] : 0.0;
    o.yp = has_p2 ? C[q + n1] : 0.0;
    o.xm = edge_m ? C[q - 1] : 0.0;
    o.xp = edge_p ? C[q + 1] : 0.0;
  };

  Plane cu, cv, nu, nv;
  double pu = 0.0, pv = 0.0;  // plane z-1 centre values
  if (live && z0 > 0) {
    pu = U[q0 + (unsigned)(z0 - 1) * P];
    pv = V[q0 + (unsigned)(z0 - 1) * P];
  }
  fetch(U, z0, cu);
  fetch(V, z0, cv);
  for (int z = z0; z < z1; ++z) {
    const bool has_n3 = z + 1 < n3;
    if (has_n3) {
      fetch(U, z + 1, nu);
      fetch(V, z + 1, nv);
    } else {
      nu = Plane{0, 0, 0, 0, 0};
      nv = Plane{0, 0, 0, 0, 0};
    }
    // i_1 neighbours from the adjacent lanes (the edge lanes use their loads)
    double um = __shfl_up(cu.c, 1, 64), uq = __shfl_down(cu.c, 1, 64);
    double vm = __shfl_up(cv.c, 1, 64), vq = __shfl_down(cv.c, 1, 64);
    if (lane == 0) { um = cu.xm; vm = cv.xm; }
    if (lane == 63) { uq = cu.xp; vq = cv.xp; }
    if (live) {
      double gu, gv;
      react(r, cu.c, cv.c, gu, gv);
      double ku = a1u[0] * um + a1u[1] * cu.c + a1u[2] * uq;
      double kv = a1v[0] * vm + a1v[1] * cv.c + a1v[2] * vq;
      ku += a2u[0] * cu.ym + a2u[1] * cu.c + a2u[2] * cu.yp;
      kv += a2v[0] * cv.ym + a2v[1] * cv.c + a2v[2] * cv.yp;
      if (b3u) ku += b3u[z] * pu + b3u[n3 + z] * cu.c + b3u[2 * n3 + z] * nu.c;
      if (b3v) kv += b3v[z] * pv + b3v[n3 + z] * cv.c + b3v[2 * n3 + z] * nv.c;
      const unsigned q = q0 + (unsigned)z * P;
      put<TR>(Ru, q, ku + gu);
      put<TR>(Rv, q, kv + gv);
    }
    pu = cu.c;
    pv = cv.c;
    cu = nu;
    cv = nv;
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
  const int n2 = g.d >= 2 ? g.n[1] : 1, n3 = g.d >= 3 ? g.n[2] : 1;
  const dim3 grid((unsigned)((g.n[0] + 63) / 64), (unsigned)((n2 + 3) / 4),
                  (unsigned)((n3 + kZB - 1) / kZB));
  if (grid.y > 65535 || grid.z > 65535) return hipErrorInvalidValue;
  const dim3 block(64, 4);
  if (r_f32)
    hipLaunchKernelGGL(k_etd_stage1<float>, grid, block, 0, s, g, r, U, V, Ru, Rv);
  else
    hipLaunchKernelGGL(k_etd_stage1<double>, grid, block, 0, s, g, r, U, V, Ru, Rv);
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
