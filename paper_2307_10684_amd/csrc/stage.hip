// Pointwise stage kernels of ETD2RKds (Sec. 3, eq. (11)) and Lawson2b (Sec. 2,
// eq. (7)): reaction terms G^u, G^v, the Kronecker-sum action K C as a stencil
// when A_mu is tridiagonal, and the combinations that feed the Tucker operators.
// All are HBM-bound streaming kernels; the state U, V is FP64 throughout.
#include <algorithm>

#include "common.h"
#include "reaction.h"

namespace adr {
namespace {

template <typename T>
__device__ __forceinline__ void put(void* p, long long q, double x) {
  static_cast<T*>(p)[q] = static_cast<T>(x);
}

// Stage 1: R^c = sum_mu (C x_mu A_mu^c) + G^c(U, V) for the directions with a
// band; directions without one are added afterwards by dense mode products.
// Two kernels: an LDS-tiled plane march for large grids and a one-plane-per-
// block kernel for small ones (stage1_plan picks by the problem's own size).
// Loads are branch-free (clamped index, then masked); outside the grid the
// neighbour is taken as 0, where the band coefficient is 0 as well.

// Workgroups are dealt to the 8 XCDs round-robin by linear dispatch index, and
// each XCD has its own L2.  Remapping linear index b to (b % 8) * (G / 8) + b / 8
// gives each XCD a contiguous range of tiles, so the halo rows and planes that
// neighbouring tiles share are mostly fetched once into one L2.
__device__ __forceinline__ void xcd_block(int& bx, int& by, int& bz) {
  const unsigned gx = gridDim.x, gy = gridDim.y, G = gx * gy * gridDim.z;
  unsigned b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  if (G % 8u == 0u) b = (b % 8u) * (G / 8u) + b / 8u;
  bx = (int)(b % gx);
  b /= gx;
  by = (int)(b % gy);
  bz = (int)(b / gy);
}

// Stage 1 on LDS tiles.  A block of 64 x 4 threads owns a tile of kTX = 64
// values of i_1 by kTY = 16 rows of i_2 and marches through planes z0..z1-1 of
// i_3 (at most ZB of them).
// The plane being computed sits in LDS with a one-point halo in i_1 and i_2
// (zero outside the grid, where the band coefficient is zero too); two LDS
// buffers let the next plane be written while this one is read, with one
// barrier per plane.  Its i_3 neighbours are the previous and next planes'
// values of the thread's own points, held in registers.  The loads of the plane after next are issued
// before the current plane is computed, so the compute of one plane covers
// the memory latency of the loads for a later one.  Every value of the tile is
// read from HBM once per plane; halos come from neighbouring tiles (L2).
constexpr int kTX = 64, kTY = 16, kRows = kTY / 4;
constexpr int kZB = 8;      // planes per block of the tiled kernel in grouped launches
constexpr int kZBmax = 32;  // most planes one block marches in single-problem launches

template <typename TR, int ZB>
__device__ __forceinline__ void etd_stage1_tile(const StageGeom& g, const Reaction& r,
                                                const double* __restrict__ U,
                                                const double* __restrict__ V, void* Ru, void* Rv,
                                                int bx, int by, int z0, int z1) {
  const int n1 = g.n[0], n2 = g.d >= 2 ? g.n[1] : 1, n3 = g.d >= 3 ? g.n[2] : 1;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 64 + tx;
  const int x0 = bx * kTX, y0 = by * kTY;
  const unsigned P = (unsigned)n1 * (unsigned)n2;

  __shared__ double sU[2][kTY + 2][kTX + 2];   // double-buffered planes
  __shared__ double sV[2][kTY + 2][kTX + 2];
  __shared__ double sb2[2][3][kTY];
  __shared__ double sb3[2][3][ZB];

  // band coefficients of directions 2 and 3 for this tile (zero without a band)
  if (tid < 2 * 3 * kTY) {
    const int c = tid / (3 * kTY), j = (tid / kTY) % 3, yy = tid % kTY, y = y0 + yy;
    const double* b = g.d >= 2 ? g.band[c][1] : nullptr;
    sb2[c][j][yy] = (b && y < n2) ? b[j * n2 + y] : 0.0;
  }
  if (tid < 2 * 3 * ZB) {
    const int c = tid / (3 * ZB), j = (tid / ZB) % 3, zz = tid % ZB, z = z0 + zz;
    const double* b = g.d >= 3 ? g.band[c][2] : nullptr;
    sb3[c][j][zz] = (b && z < n3) ? b[j * n3 + z] : 0.0;
  }
  const int i1 = x0 + tx;
  const bool col_ok = i1 < n1;
  double a1u[3] = {0, 0, 0}, a1v[3] = {0, 0, 0};
  if (col_ok) {
    if (g.band[0][0]) for (int j = 0; j < 3; ++j) a1u[j] = g.band[0][0][j * n1 + i1];
    if (g.band[1][0]) for (int j = 0; j < 3; ++j) a1v[j] = g.band[1][0][j * n1 + i1];
  }

  // this thread's points: column i1, rows y0 + ty + 4k; in-plane offsets
  bool pt_ok[kRows];
  unsigned pt_off[kRows];
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int i2 = y0 + ty + 4 * k;
    pt_ok[k] = col_ok && i2 < n2;
    pt_off[k] = pt_ok[k] ? (unsigned)i2 * (unsigned)n1 + (unsigned)i1 : 0u;
  }
  // halo point of this thread (threads 0..159): rows above/below, columns left/right
  int h_r = 0, h_c = 0;
  bool h_ok = false;
  unsigned h_off = 0;
  if (tid < 2 * kTX + 2 * kTY) {
    int hx, hy;
    if (tid < kTX) { hx = x0 + tid; hy = y0 - 1; h_r = 0; h_c = tid + 1; }
    else if (tid < 2 * kTX) { hx = x0 + tid - kTX; hy = y0 + kTY; h_r = kTY + 1; h_c = tid - kTX + 1; }
    else if (tid < 2 * kTX + kTY) { hx = x0 - 1; hy = y0 + tid - 2 * kTX; h_r = tid - 2 * kTX + 1; h_c = 0; }
    else { hx = x0 + kTX; hy = y0 + tid - 2 * kTX - kTY; h_r = tid - 2 * kTX - kTY + 1; h_c = kTX + 1; }
    h_ok = hx >= 0 && hx < n1 && hy >= 0 && hy < n2;
    h_off = h_ok ? (unsigned)hy * (unsigned)n1 + (unsigned)hx : 0u;
  }
  const bool has_halo = tid < 2 * kTX + 2 * kTY;

  // plane loads (clamped index, masked afterwards)
  auto load_plane = [&](int z, double (&iu)[kRows], double (&iv)[kRows], double& hu, double& hv) {
    const bool zok = z >= 0 && z < n3;
    const unsigned base = zok ? (unsigned)z * P : 0u;
    double lu[kRows], lv[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      lu[k] = U[base + pt_off[k]];
      lv[k] = V[base + pt_off[k]];
    }
    const double a = U[base + h_off], b = V[base + h_off];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      iu[k] = (zok && pt_ok[k]) ? lu[k] : 0.0;
      iv[k] = (zok && pt_ok[k]) ? lv[k] : 0.0;
    }
    hu = (zok && h_ok) ? a : 0.0;
    hv = (zok && h_ok) ? b : 0.0;
  };
  auto to_lds = [&](int buf, const double (&iu)[kRows], const double (&iv)[kRows], double hu,
                    double hv) {
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      sU[buf][ty + 4 * k + 1][tx + 1] = iu[k];
      sV[buf][ty + 4 * k + 1][tx + 1] = iv[k];
    }
    if (has_halo) {
      sU[buf][h_r][h_c] = hu;
      sV[buf][h_r][h_c] = hv;
    }
  };

  double pu[kRows], pv[kRows], cu[kRows], cv[kRows], nu[kRows], nv[kRows];
  double hcu, hcv, hnu, hnv, dummy_u, dummy_v;
  load_plane(z0 - 1, pu, pv, dummy_u, dummy_v);
  load_plane(z0, cu, cv, hcu, hcv);
  load_plane(z0 + 1, nu, nv, hnu, hnv);
  to_lds(0, cu, cv, hcu, hcv);
  __syncthreads();

  int buf = 0;
  for (int z = z0; z < z1; ++z) {
    // loads of plane z + 2, in flight during this plane's compute; plane z + 1
    // goes to the other LDS buffer (its readers finished before the last barrier)
    double lu[kRows], lv[kRows], lhu, lhv;
    const bool more = z + 1 < z1;
    if (more) {
      load_plane(z + 2, lu, lv, lhu, lhv);
      to_lds(buf ^ 1, nu, nv, hnu, hnv);
    }
    const int zz = z - z0;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int ly = ty + 4 * k + 1, lx = tx + 1;
      const double uc = cu[k], vc = cv[k];
      const double um = sU[buf][ly][lx - 1], uq = sU[buf][ly][lx + 1];
      const double vm = sV[buf][ly][lx - 1], vq = sV[buf][ly][lx + 1];
      const double uym = sU[buf][ly - 1][lx], uyp = sU[buf][ly + 1][lx];
      const double vym = sV[buf][ly - 1][lx], vyp = sV[buf][ly + 1][lx];
      const int yy = ty + 4 * k;
      double gu, gv;
      react(r, uc, vc, gu, gv);
      double ku = a1u[0] * um + a1u[1] * uc + a1u[2] * uq;
      double kv = a1v[0] * vm + a1v[1] * vc + a1v[2] * vq;
      ku += sb2[0][0][yy] * uym + sb2[0][1][yy] * uc + sb2[0][2][yy] * uyp;
      kv += sb2[1][0][yy] * vym + sb2[1][1][yy] * vc + sb2[1][2][yy] * vyp;
      ku += sb3[0][0][zz] * pu[k] + sb3[0][1][zz] * uc + sb3[0][2][zz] * nu[k];
      kv += sb3[1][0][zz] * pv[k] + sb3[1][1][zz] * vc + sb3[1][2][zz] * nv[k];
      if (pt_ok[k]) {
        const unsigned q = (unsigned)z * P + pt_off[k];
        put<TR>(Ru, q, ku + gu);
        put<TR>(Rv, q, kv + gv);
      }
    }
    if (!more) break;
    __syncthreads();  // plane z + 1 is in LDS and everyone is done with plane z
    buf ^= 1;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      pu[k] = cu[k];
      pv[k] = cv[k];
      cu[k] = nu[k];
      cv[k] = nv[k];
      nu[k] = lu[k];
      nv[k] = lv[k];
    }
    hnu = lhu;
    hnv = lhv;
  }
}

// Stage 1, one plane per block: every load of a thread is independent and
// issued at once (no marching), so latency is hidden by the many waves a CU
// holds at this kernel's small register footprint.  i_1 neighbours come from
// lane shuffles; i_2 and i_3 neighbours are loads that mostly hit L1/L2 (the
// neighbouring rows and planes are loaded by neighbouring blocks of the same
// XCD at about the same time).
template <typename TR>
__device__ __forceinline__ void etd_stage1_point(const StageGeom& g, const Reaction& r,
                                                 const double* __restrict__ U,
                                                 const double* __restrict__ V, void* Ru, void* Rv,
                                                 int bx, int by, int z) {
  const int n1 = g.n[0], n2 = g.d >= 2 ? g.n[1] : 1, n3 = g.d >= 3 ? g.n[2] : 1;
  const int lane = threadIdx.x;
  const int i1 = bx * 64 + lane;
  const int i2 = __builtin_amdgcn_readfirstlane(by * 4 + threadIdx.y);
  const bool live = i1 < n1 && i2 < n2;
  const unsigned P = (unsigned)n1 * (unsigned)n2;
  const unsigned q = live ? (unsigned)z * P + (unsigned)i2 * (unsigned)n1 + (unsigned)i1 : 0u;
  const bool okm2 = live && i2 > 0, okp2 = live && i2 + 1 < n2;
  const bool okm3 = live && z > 0, okp3 = live && z + 1 < n3;
  const bool edm = live && lane == 0 && i1 > 0, edp = live && lane == 63 && i1 + 1 < n1;
  const unsigned qym = okm2 ? q - n1 : 0u, qyp = okp2 ? q + n1 : 0u;
  const unsigned qzm = okm3 ? q - P : 0u, qzp = okp3 ? q + P : 0u;
  const unsigned qxm = edm ? q - 1 : 0u, qxp = edp ? q + 1 : 0u;
  const double l_u = U[q], l_v = V[q];
  const double l_uym = U[qym], l_uyp = U[qyp], l_vym = V[qym], l_vyp = V[qyp];
  const double l_uzm = U[qzm], l_uzp = U[qzp], l_vzm = V[qzm], l_vzp = V[qzp];
  const double l_uxm = U[qxm], l_uxp = U[qxp], l_vxm = V[qxm], l_vxp = V[qxp];
  double a1u[3] = {0, 0, 0}, a1v[3] = {0, 0, 0}, a2u[3] = {0, 0, 0}, a2v[3] = {0, 0, 0};
  double a3u[3] = {0, 0, 0}, a3v[3] = {0, 0, 0};
  if (live) {
    if (g.band[0][0]) for (int j = 0; j < 3; ++j) a1u[j] = g.band[0][0][j * n1 + i1];
    if (g.band[1][0]) for (int j = 0; j < 3; ++j) a1v[j] = g.band[1][0][j * n1 + i1];
  }
  if (g.d >= 2 && i2 < n2) {
    if (g.band[0][1]) for (int j = 0; j < 3; ++j) a2u[j] = g.band[0][1][j * n2 + i2];
    if (g.band[1][1]) for (int j = 0; j < 3; ++j) a2v[j] = g.band[1][1][j * n2 + i2];
  }
  if (g.d >= 3) {
    if (g.band[0][2]) for (int j = 0; j < 3; ++j) a3u[j] = g.band[0][2][j * n3 + z];
    if (g.band[1][2]) for (int j = 0; j < 3; ++j) a3v[j] = g.band[1][2][j * n3 + z];
  }
  const double uc = live ? l_u : 0.0, vc = live ? l_v : 0.0;
  double um = __shfl_up(uc, 1, 64), uq = __shfl_down(uc, 1, 64);
  double vm = __shfl_up(vc, 1, 64), vq = __shfl_down(vc, 1, 64);
  if (lane == 0) {
    um = edm ? l_uxm : 0.0;
    vm = edm ? l_vxm : 0.0;
  }
  if (lane == 63) {
    uq = edp ? l_uxp : 0.0;
    vq = edp ? l_vxp : 0.0;
  }
  if (!live) return;
  const double uym = okm2 ? l_uym : 0.0, uyp = okp2 ? l_uyp : 0.0;
  const double vym = okm2 ? l_vym : 0.0, vyp = okp2 ? l_vyp : 0.0;
  const double uzm = okm3 ? l_uzm : 0.0, uzp = okp3 ? l_uzp : 0.0;
  const double vzm = okm3 ? l_vzm : 0.0, vzp = okp3 ? l_vzp : 0.0;
  double gu, gv;
  react(r, uc, vc, gu, gv);
  double ku = a1u[0] * um + a1u[1] * uc + a1u[2] * uq;
  double kv = a1v[0] * vm + a1v[1] * vc + a1v[2] * vq;
  ku += a2u[0] * uym + a2u[1] * uc + a2u[2] * uyp;
  kv += a2v[0] * vym + a2v[1] * vc + a2v[2] * vyp;
  ku += a3u[0] * uzm + a3u[1] * uc + a3u[2] * uzp;
  kv += a3v[0] * vzm + a3v[1] * vc + a3v[2] * vzp;
  put<TR>(Ru, q, ku + gu);
  put<TR>(Rv, q, kv + gv);
}

template <typename TR>
__global__ __launch_bounds__(256) void k_etd_stage1_point(StageGeom g, Reaction r,
                                                          const double* __restrict__ U,
                                                          const double* __restrict__ V, void* Ru,
                                                          void* Rv) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  etd_stage1_point<TR>(g, r, U, V, Ru, Rv, bx, by, bz);
}

template <typename TR, int ZB>
__global__ __launch_bounds__(256) void k_etd_stage1_tile(StageGeom g, Reaction r,
                                                         const double* __restrict__ U,
                                                         const double* __restrict__ V, void* Ru,
                                                         void* Rv) {
  int bx, by, bz;
  xcd_block(bx, by, bz);
  // block bz marches planes [bz n3 / gz, (bz + 1) n3 / gz): every block gets
  // floor or ceil of n3 / gz planes (the launcher keeps that at most ZB)
  const int n3 = g.d >= 3 ? g.n[2] : 1;
  const int z0 = (int)((long long)bz * n3 / gridDim.z);
  const int z1 = (int)((long long)(bz + 1) * n3 / gridDim.z);
  etd_stage1_tile<TR, ZB>(g, r, U, V, Ru, Rv, bx, by, z0, z1);
}

// Grouped stage 1 over several problems of one kernel variant (KIND): job j
// owns blocks [jobs[j].block_begin, jobs[j+1].block_begin), laid out as
// gx * gy * gz.  The variant follows from each problem's own size
// (stage1_plan), so a problem computes the same values alone and in any mix;
// the two variants are separate launches so that the small-grid kernel keeps
// its small register footprint (and occupancy).
template <typename TR, int KIND>
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
  if (KIND == kStage1Tile) {
    const int z0 = (rest / j.gy) * kZB, n3 = j.g.d >= 3 ? j.g.n[2] : 1;
    etd_stage1_tile<TR, kZB>(j.g, j.r, j.U, j.V, j.R[0], j.R[1], bx, rest % j.gy, z0,
                             min(z0 + kZB, n3));
  } else
    etd_stage1_point<TR>(j.g, j.r, j.U, j.V, j.R[0], j.R[1], bx, rest % j.gy, rest / j.gy);
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
// the final C_{n+1} = (C_n + D1) + D2 is formed by the last product of the
// phi_2 operator (its FP32 second addend) or, in grouped plans, pointwise.
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

// Compute units of the current device (cached; 256 if the query fails).
static int stage_cu_count() {
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

int stage1_plan(const StageGeom& g, int& kind, int& gx, int& gy, int& gz) {
  const int n2 = g.d >= 2 ? g.n[1] : 1, n3 = g.d >= 3 ? g.n[2] : 1;
  // measured crossovers: the LDS-tiled kernel wins from 2^20 points in 3D and
  // from 2^16 in 2D; below, the one-plane kernel's independent loads win
  kind = ((g.d == 3 && g.N >= (1LL << 20)) || (g.d == 2 && g.N >= (1LL << 16))) ? kStage1Tile
                                                                               : kStage1Point;
  gx = (g.n[0] + 63) / 64;
  gy = kind == kStage1Tile ? (n2 + kTY - 1) / kTY : (n2 + 3) / 4;
  // tile kernel: kZB planes per block, the layout of grouped launches
  // (launch_etd_stage1 re-splits the planes of a single problem)
  gz = kind == kStage1Tile ? (n3 + kZB - 1) / kZB : n3;
  return gx * gy * gz;
}

// Resident workgroups per CU of a tile-kernel variant (cached; 3 if the query fails).
template <typename TR>
static int stage1_tile_occupancy() {
  static int occ = 0;
  if (occ == 0 &&
      (hipOccupancyMaxActiveBlocksPerMultiprocessor(
           &occ, reinterpret_cast<const void*>(&k_etd_stage1_tile<TR, kZBmax>), 256, 0) !=
           hipSuccess ||
       occ <= 0))
    occ = 3;
  return occ;
}

hipError_t launch_etd_stage1(const StageGeom& g, const Reaction& r, const double* U,
                             const double* V, void* Ru, void* Rv, int r_f32, hipStream_t s) {
  int kind, gx, gy, gz;
  stage1_plan(g, kind, gx, gy, gz);
  if (kind == kStage1Tile) {
    // One round of resident workgroups: the planes are split evenly over
    // gz = (workgroups the chip holds at once) / (tiles per plane) blocks per
    // column of tiles, at most kZBmax planes each.  A grid of several rounds
    // leaves part of the chip idle in its last one and pays a three-plane
    // start-up per block more often (measured, FP64, same values: 256^3 121 against
    // 134 us with 8-plane blocks, 128^3 20.7 against 22.0, 200x150x101 27.7
    // against 33.0).
    const int n3 = g.d >= 3 ? g.n[2] : 1;
    const long long slots =
        (long long)(r_f32 ? stage1_tile_occupancy<float>() : stage1_tile_occupancy<double>()) *
        stage_cu_count();
    long long z = slots / ((long long)gx * gy);
    z = std::max<long long>(z, (n3 + kZBmax - 1) / kZBmax);
    gz = (int)std::min<long long>(std::max<long long>(z, 1), n3);
  }
  if (gy > 65535 || gz > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)gx, (unsigned)gy, (unsigned)gz), block(64, 4);
  if (kind == kStage1Tile) {
    if (r_f32)
      hipLaunchKernelGGL((k_etd_stage1_tile<float, kZBmax>), grid, block, 0, s, g, r, U, V, Ru,
                         Rv);
    else
      hipLaunchKernelGGL((k_etd_stage1_tile<double, kZBmax>), grid, block, 0, s, g, r, U, V, Ru,
                         Rv);
  } else {
    if (r_f32)
      hipLaunchKernelGGL(k_etd_stage1_point<float>, grid, block, 0, s, g, r, U, V, Ru, Rv);
    else
      hipLaunchKernelGGL(k_etd_stage1_point<double>, grid, block, 0, s, g, r, U, V, Ru, Rv);
  }
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

hipError_t launch_stage1_grouped(const StageJob* jobs, int njobs, long long nblocks, int kind,
                                 int r_f32, hipStream_t s) {
  if (njobs <= 0 || nblocks <= 0 || nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 block(64, 4), grid((unsigned)nblocks);
  if (kind == kStage1Tile) {
    if (r_f32)
      hipLaunchKernelGGL((k_etd_stage1_grouped<float, kStage1Tile>), grid, block, 0, s, jobs, njobs);
    else
      hipLaunchKernelGGL((k_etd_stage1_grouped<double, kStage1Tile>), grid, block, 0, s, jobs, njobs);
  } else {
    if (r_f32)
      hipLaunchKernelGGL((k_etd_stage1_grouped<float, kStage1Point>), grid, block, 0, s, jobs, njobs);
    else
      hipLaunchKernelGGL((k_etd_stage1_grouped<double, kStage1Point>), grid, block, 0, s, jobs, njobs);
  }
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
