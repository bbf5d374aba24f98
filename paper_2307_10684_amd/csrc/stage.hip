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
    case 4: {  // DIB: rho(a1u(1-v)u - a2u u^3 - a3u(v-a4u)),
               //      rho(a1v(1+a2v u)(1-v)(1-a3v(1-v)) - a4v v(1+a5v u)(1+a3v v))
      const double w = 1.0 - v;
      gu = r.p[0] * (r.p[1] * w * u - r.p[2] * u * u * u - r.p[3] * (v - r.p[4]));
      gv = r.p[0] * (r.p[5] * (1.0 + r.p[6] * u) * w * (1.0 - r.p[7] * w) -
                     r.p[8] * v * (1.0 + r.p[9] * u) * (1.0 + r.p[7] * v));
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
// Block = (64, 4) threads over (i_1, i_2); each block marches through kZB planes
// of i_3.  A plane's centre value is loaded once: it serves as the i_3 + 1
// neighbour of the plane before, then as the centre, then as the i_3 - 1
// neighbour.  Inside a wave the i_1 +- 1 neighbours come from lane shuffles
// (the wave-edge lanes load theirs); the i_2 +- 1 neighbours are loads that
// the neighbouring rows of the block have just brought into the L1 cache.
// Loads are branch-free (clamped index, then masked).  Latency is hidden by
// occupancy: the kernel keeps few registers so that many waves share a SIMD.
constexpr int kZB = 16;  // planes per block

template <typename TR>
__device__ __forceinline__ void etd_stage1_block(const StageGeom& g, const Reaction& r,
                                                 const double* __restrict__ U,
                                                 const double* __restrict__ V, void* Ru,
                                                 void* Rv, int bx, int by, int bz) {
  const int n1 = g.n[0], n2 = g.d >= 2 ? g.n[1] : 1, n3 = g.d >= 3 ? g.n[2] : 1;
  const int i1 = bx * 64 + threadIdx.x;
  // i_2 is the same on the whole wave (blockDim.x = 64): keep it in a scalar
  // register so its band coefficients are scalar loads
  const int i2 = __builtin_amdgcn_readfirstlane(by * 4 + threadIdx.y);
  const int z0 = bz * kZB;
  const int z1 = min(z0 + kZB, n3);
  const bool live = i1 < n1 && i2 < n2;
  const unsigned P = (unsigned)n1 * (unsigned)n2;  // plane stride
  const int lane = threadIdx.x;
  const int tid = threadIdx.y * 64 + threadIdx.x;

  // i_3 band coefficients of this block's planes (zero without a band)
  __shared__ double sb3[2][3][kZB];
  if (tid < 2 * 3 * kZB) {
    const int c = tid / (3 * kZB), j = (tid / kZB) % 3, zz = tid % kZB, z = z0 + zz;
    const double* b = g.d >= 3 ? g.band[c][2] : nullptr;
    sb3[c][j][zz] = (b && z < n3) ? b[j * n3 + z] : 0.0;
  }
  // per-thread band coefficients of directions 1 and 2
  double a1u[3] = {0, 0, 0}, a1v[3] = {0, 0, 0}, a2u[3] = {0, 0, 0}, a2v[3] = {0, 0, 0};
  if (live) {
    if (g.band[0][0]) for (int j = 0; j < 3; ++j) a1u[j] = g.band[0][0][j * n1 + i1];
    if (g.band[1][0]) for (int j = 0; j < 3; ++j) a1v[j] = g.band[1][0][j * n1 + i1];
  }
  if (g.d >= 2 && i2 < n2) {
    if (g.band[0][1]) for (int j = 0; j < 3; ++j) a2u[j] = g.band[0][1][j * n2 + i2];
    if (g.band[1][1]) for (int j = 0; j < 3; ++j) a2v[j] = g.band[1][1][j * n2 + i2];
  }
  __syncthreads();
  const bool has_m2 = live && i2 > 0, has_p2 = live && i2 + 1 < n2;
  const bool edge_m = live && lane == 0 && i1 > 0;
  const bool edge_p = live && lane == 63 && i1 + 1 < n1;
  const unsigned q0 = (unsigned)i2 * (unsigned)n1 + (unsigned)i1;

  double pu, pv, uc, vc;  // centres of planes z-1 and z
  {
    const bool okp = live && z0 > 0;
    const unsigned qp = okp ? q0 + (unsigned)(z0 - 1) * P : 0u;
    const unsigned qc = live ? q0 + (unsigned)z0 * P : 0u;
    const double a = U[qp], b = V[qp], c = U[qc], d = V[qc];
    pu = okp ? a : 0.0;
    pv = okp ? b : 0.0;
    uc = live ? c : 0.0;
    vc = live ? d : 0.0;
  }
  for (int z = z0; z < z1; ++z) {
    const unsigned q = q0 + (unsigned)z * P;
    const bool has_n3 = z + 1 < n3;
    const bool okn = live && has_n3;
    const unsigned qn = okn ? q + P : 0u;
    const unsigned qym = has_m2 ? q - n1 : 0u, qyp = has_p2 ? q + n1 : 0u;
    const unsigned qxm = edge_m ? q - 1 : 0u, qxp = edge_p ? q + 1 : 0u;
    const double l_un = U[qn], l_vn = V[qn];
    const double l_uym = U[qym], l_uyp = U[qyp], l_vym = V[qym], l_vyp = V[qyp];
    const double l_uxm = U[qxm], l_uxp = U[qxp], l_vxm = V[qxm], l_vxp = V[qxp];
    const double un = okn ? l_un : 0.0, vn = okn ? l_vn : 0.0;
    // i_1 neighbours from the adjacent lanes (the edge lanes use their loads)
    double um = __shfl_up(uc, 1, 64), uq = __shfl_down(uc, 1, 64);
    double vm = __shfl_up(vc, 1, 64), vq = __shfl_down(vc, 1, 64);
    if (lane == 0) {
      um = edge_m ? l_uxm : 0.0;
      vm = edge_m ? l_vxm : 0.0;
    }
    if (lane == 63) {
      uq = edge_p ? l_uxp : 0.0;
      vq = edge_p ? l_vxp : 0.0;
    }
    const double uym = has_m2 ? l_uym : 0.0, uyp = has_p2 ? l_uyp : 0.0;
    const double vym = has_m2 ? l_vym : 0.0, vyp = has_p2 ? l_vyp : 0.0;
    if (live) {
      const int zz = z - z0;
      double gu, gv;
      react(r, uc, vc, gu, gv);
      double ku = a1u[0] * um + a1u[1] * uc + a1u[2] * uq;
      double kv = a1v[0] * vm + a1v[1] * vc + a1v[2] * vq;
      ku += a2u[0] * uym + a2u[1] * uc + a2u[2] * uyp;
      kv += a2v[0] * vym + a2v[1] * vc + a2v[2] * vyp;
      ku += sb3[0][0][zz] * pu + sb3[0][1][zz] * uc + sb3[0][2][zz] * un;
      kv += sb3[1][0][zz] * pv + sb3[1][1][zz] * vc + sb3[1][2][zz] * vn;
      put<TR>(Ru, q, ku + gu);
      put<TR>(Rv, q, kv + gv);
    }
    pu = uc;
    pv = vc;
    uc = un;
    vc = vn;
  }
}

template <typename TR>
__global__ __launch_bounds__(256) void k_etd_stage1(StageGeom g, Reaction r,
                                                    const double* __restrict__ U,
                                                    const double* __restrict__ V, void* Ru,
                                                    void* Rv) {
  etd_stage1_block<TR>(g, r, U, V, Ru, Rv, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Grouped stage 1 over several problems: job j owns blocks
// [jobs[j].block_begin, jobs[j+1].block_begin), laid out as gx * gy * gz.
template <typename TR>
__global__ __launch_bounds__(256) void k_etd_stage1_grouped(const StageJob* __restrict__ jobs,
                                                            int njobs) {
  const long long b = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block_begin <= b) lo = mid; else hi = mid - 1;
  }
  const StageJob& j = jobs[lo];
  const int local = (int)(b - j.block_begin);
  const int bx = local % j.gx, rest = local / j.gx;
  etd_stage1_block<TR>(j.g, j.r, j.U, j.V, j.R[0], j.R[1], bx, rest % j.gy, rest / j.gy);
}

// Grouped pointwise stages: job j owns blocks [block_begin, next block_begin) of
// 256 points each over its N points; kind 0 = ETD2RKds stage 2 (FP64 states
// A = U2, B = V2), kind 1 = stage 2 from FP32 increments (A = D1u, B = D1v),
// kind 2 = final C += D1 + D2 (A, B = D1, C2, D2 = D2).
template <typename TR>
__global__ __launch_bounds__(256) void k_pointwise_grouped(const PointJob* __restrict__ jobs,
                                                           int njobs) {
  const long long b = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block_begin <= b) lo = mid; else hi = mid - 1;
  }
  const PointJob& j = jobs[lo];
  const long long q = (b - j.block_begin) * 256 + threadIdx.x;
  if (q >= j.N) return;
  if (j.kind == 0) {
    double gu, gv, gu2, gv2;
    react(j.r, j.U[q], j.V[q], gu, gv);
    react(j.r, static_cast<const double*>(j.A)[q], static_cast<const double*>(j.B)[q], gu2, gv2);
    put<TR>(j.R[0], q, gu2 - gu);
    put<TR>(j.R[1], q, gv2 - gv);
  } else if (j.kind == 1) {
    const double u = j.U[q], v = j.V[q];
    double gu, gv, gu2, gv2;
    react(j.r, u, v, gu, gv);
    react(j.r, u + (double)static_cast<const float*>(j.A)[q],
          v + (double)static_cast<const float*>(j.B)[q], gu2, gv2);
    put<TR>(j.R[0], q, gu2 - gu);
    put<TR>(j.R[1], q, gv2 - gv);
  } else {
    double* U = const_cast<double*>(j.U);
    double* V = const_cast<double*>(j.V);
    U[q] = (U[q] + (double)static_cast<const float*>(j.A)[q]) + (double)static_cast<const float*>(j.C2)[q];
    V[q] = (V[q] + (double)static_cast<const float*>(j.B)[q]) + (double)static_cast<const float*>(j.D2)[q];
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

// Reduced-precision ETD2RKds keeps the Tucker results as FP32 increments
// D1 = tau T1, D2 = 2^(d-1) tau T2 and forms the FP64 states pointwise:
// stage 2: R^c = G^c(U + D1u, V + D1v) - G^c(U, V);
// final:   C <- C + D1^c + D2^c   (i.e. C_{n+1} = C_{n2} + D2 with C_{n2} = C_n + D1).
__global__ __launch_bounds__(256) void k_etd_stage2_inc(long long N, Reaction r,
                                                        const double* __restrict__ U,
                                                        const double* __restrict__ V,
                                                        const float* __restrict__ Du,
                                                        const float* __restrict__ Dv,
                                                        float* __restrict__ Ru,
                                                        float* __restrict__ Rv) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
       q += (long long)gridDim.x * blockDim.x) {
    const double u = U[q], v = V[q];
    double gu, gv, gu2, gv2;
    react(r, u, v, gu, gv);
    react(r, u + (double)Du[q], v + (double)Dv[q], gu2, gv2);
    Ru[q] = (float)(gu2 - gu);
    Rv[q] = (float)(gv2 - gv);
  }
}

__global__ __launch_bounds__(256) void k_etd_final_inc(long long N, double* __restrict__ U,
                                                       double* __restrict__ V,
                                                       const float* __restrict__ D1u,
                                                       const float* __restrict__ D1v,
                                                       const float* __restrict__ D2u,
                                                       const float* __restrict__ D2v) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < N;
       q += (long long)gridDim.x * blockDim.x) {
    U[q] = (U[q] + (double)D1u[q]) + (double)D2u[q];
    V[q] = (V[q] + (double)D1v[q]) + (double)D2v[q];
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

hipError_t launch_etd_stage2_inc(long long N, const Reaction& r, const double* U, const double* V,
                                 const float* Du, const float* Dv, float* Ru, float* Rv,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_etd_stage2_inc, dim3(stream_grid(N)), dim3(256), 0, s, N, r, U, V, Du, Dv,
                     Ru, Rv);
  return hipGetLastError();
}

hipError_t launch_etd_final_inc(long long N, double* U, double* V, const float* D1u,
                                const float* D1v, const float* D2u, const float* D2v,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_etd_final_inc, dim3(stream_grid(N)), dim3(256), 0, s, N, U, V, D1u, D1v,
                     D2u, D2v);
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

hipError_t launch_stage1_grouped(const StageJob* jobs, int njobs, long long nblocks, int r_f32,
                                 hipStream_t s) {
  if (njobs <= 0 || nblocks <= 0 || nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 block(64, 4);
  if (r_f32)
    hipLaunchKernelGGL(k_etd_stage1_grouped<float>, dim3((unsigned)nblocks), block, 0, s, jobs, njobs);
  else
    hipLaunchKernelGGL(k_etd_stage1_grouped<double>, dim3((unsigned)nblocks), block, 0, s, jobs, njobs);
  return hipGetLastError();
}

hipError_t launch_pointwise_grouped(const PointJob* jobs, int njobs, long long nblocks, int r_f32,
                                    hipStream_t s) {
  if (njobs <= 0 || nblocks <= 0 || nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (r_f32)
    hipLaunchKernelGGL(k_pointwise_grouped<float>, dim3((unsigned)nblocks), dim3(256), 0, s, jobs, njobs);
  else
    hipLaunchKernelGGL(k_pointwise_grouped<double>, dim3((unsigned)nblocks), dim3(256), 0, s, jobs, njobs);
  return hipGetLastError();
}

int stage1_blocks(const StageGeom& g, int& gx, int& gy, int& gz) {
  const int n2 = g.d >= 2 ? g.n[1] : 1, n3 = g.d >= 3 ? g.n[2] : 1;
  gx = (g.n[0] + 63) / 64;
  gy = (n2 + 3) / 4;
  gz = (n3 + kZB - 1) / kZB;
  return gx * gy * gz;
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
