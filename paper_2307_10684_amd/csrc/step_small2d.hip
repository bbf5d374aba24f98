// Whole ETD2RKds steps (Sec. 3, eq. (11)) of a small 2D problem in one
// cooperative launch.  At 64 x 64 a step's kernels each finish in a few
// microseconds, so a step launched kernel by kernel is bound by launch and
// drain latency.  Here one launch runs every step, and the workgroups meet at
// two grid barriers per step.
//
// Work split.  The grid is n1 = 64 rows (i1, one row per lane) by n2 columns
// (i2).  Workgroup b owns the kCB = 4 columns j0 = 4b .. 4b + 3 of both
// components and also keeps the state on the halo columns j0 - 1 and j0 + 4
// (the extended columns, je = 0 .. 5 for j = j0 - 1 + je).  For each
// component c, one step is:
//
//   S1  R = K C + G(C) on the own columns (the stencil needs the halo
//       columns, held locally);
//   P1  Y = M1 R on the own columns (direction 1 acts within a column),
//       where M1 is phi_1(tau A_1); Y goes to global memory;
//       grid barrier A: every column of Y is written;
//   P2  C2 = C + tau (Y M2^T) on the extended columns (direction 2 needs all
//       columns of Y), where M2 is phi_1(tau A_2);
//   S2  R = G(C2) - G(C) on the own columns;
//   P3  Y' = M1' R on the own columns, with M1' = phi_2(tau A_1), to global;
//       grid barrier B;
//   P4  C = C2 + 2 tau (Y' M2'^T) on the extended columns, with M2' = phi_2(tau A_2).
//
// The extended columns make the next step's stencil local: the halo state is
// computed by the workgroup itself (from all of Y and Y'), so no barrier is
// needed between a step's end and the next step's start.  Y and Y' use
// separate buffers, so a workgroup that runs ahead into the next step cannot
// overwrite what a slower one still reads (the barrier between them orders
// every read before the next write).
//
// The products are FP64 FMAs on the vector units: a workgroup's share is a
// 64 x 64 matrix against 4 (direction 1) or 6 (direction 2) columns, too
// narrow for 16 x 16 matrix-instruction blocks without padding, and a step's
// time goes to its barriers and exchange loads, not to these FMAs.  In each product the
// eight waves are (component c, quarter kq of the contraction index): lane i
// forms row i's partial sums over its 16 values of k for every column, the
// partial sums meet in LDS, and wave (c, q) adds the four quarters of its
// columns.  So each matrix element is read once per workgroup, and in P2/P4
// each element of Y is loaded from global memory once per workgroup, all of a
// lane's 16 loads in flight together.  The direction-1 matrices of the
// operator in use (both components, 64 KB) sit in LDS; the other operator's
// are copied in (LDS-direct loads) while a barrier and the next direction-2
// product run.  The rows of the direction-2 matrices for the extended
// columns stay in LDS for the whole launch.
//
// Exchange and barriers.  Y and Y' are written and read only with
// agent-scope atomic stores and loads, which are coherent across the chip's
// L2 caches, so no cache write-back or invalidation is needed.  A barrier
// is a counter in global memory: every wave waits for its own stores to
// complete, then after the workgroup barrier thread 0 increments the counter
// and polls it (agent-scope atomics) until it reaches the barrier's target;
// the workgroup barrier then releases the other waves, whose exchange loads
// are issued after it.  The launch is cooperative, so every workgroup is
// resident and every barrier completes; the wait is still bounded: after
// kSpinLimit polls (fewer when the host says so, for tests of this path) a
// workgroup raises the shared error flag, every
// workgroup leaves at its next barrier, and the own columns of U and V are
// filled with NaN, so an incomplete launch cannot pass for a result.
#include <cmath>
#include <cstdlib>

#include "common.h"
#include "reaction.h"

namespace adr {
namespace {

constexpr int kN1 = 64;       // rows (lanes)
constexpr int kCB = 4;        // own columns per workgroup
constexpr int kCE = kCB + 2;  // extended columns
constexpr int kMaxN2 = 64;
constexpr unsigned kSpinLimit = 1u << 20;

__global__ void k_zero_sync(unsigned* counter, int* err) {
  if (threadIdx.x == 0) {
    *counter = 0u;
    *err = 0;
  }
}

// Grid barrier: returns false when the launch is being abandoned (a barrier
// timed out in some workgroup).
__device__ __forceinline__ bool grid_sync(unsigned* counter, int* err, unsigned target,
                                          unsigned spin_limit, int* sflag) {
  __builtin_amdgcn_s_waitcnt(0);   // this wave's exchange stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int failed = 0;
    unsigned spins = 0;
    // (wrap-safe: the counter and the targets run modulo 2^32 over long launches)
    while ((int)(__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          ++spins > spin_limit) {
        failed = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (failed) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *sflag = failed;
  }
  __syncthreads();
  return *sflag == 0;
}

// LDS-direct copy of the direction-1 matrices of one operator (components 0
// and 1, 32 KB each) into dst: 64 spans of 1 KB, eight per wave; lane l of a
// span fills bytes 16 l .. 16 l + 15 of it.
__device__ __forceinline__ void dma_m1(double* dst, const double* m0, const double* m1, int wave,
                                       int lane) {
#pragma unroll
  for (int h = 0; h < 8; ++h) {
    const int span = wave * 8 + h;
    const double* src = (span < 32 ? m0 : m1) + (span % 32) * 128 + 2 * lane;
    __builtin_amdgcn_global_load_lds(src, dst + span * 128, 16, 0, 0);
  }
}

// Direction-1 product, partial sums of quarter kq: part[j] = sum over the 16
// k of the quarter of M[lane + 64 k] r[k][j], for the kCB own columns j.
__device__ __forceinline__ void dir1_partial(const double* __restrict__ M,
                                             const double (*r)[kCB], int kq, int lane,
                                             double (&part)[kCB]) {
#pragma unroll
  for (int j = 0; j < kCB; ++j) part[j] = 0.0;
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int k = 16 * kq + kk;
    const double m = M[lane + kN1 * k];
#pragma unroll
    for (int j = 0; j < kCB; ++j) part[j] = fma(m, r[k][j], part[j]);
  }
}

// Direction-2 product, quarter kq: the lane's 16 values of Y (row lane,
// columns k of the quarter; k >= n2 loads the last column again, whose
// matrix entries below are zero), then the partial sums for the kCE extended
// columns, part[je] = sum over the quarter's k of y[k] M[je][k].
__device__ __forceinline__ void dir2_load(const double* Y, int n2, int kq, int lane, double (&y)[16]) {
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int k = min(16 * kq + kk, n2 - 1);
    y[kk] = __hip_atomic_load(Y + lane + kN1 * k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}
__device__ __forceinline__ void dir2_partial(const double (&y)[16], const double (*M)[kMaxN2], int kq,
                                             double (&part)[kCE]) {
#pragma unroll
  for (int je = 0; je < kCE; ++je) {
    double sum = 0.0;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) sum = fma(y[kk], M[je][16 * kq + kk], sum);
    part[je] = sum;
  }
}

__global__ __launch_bounds__(512, 1) void k_etd_small2d(Small2dArgs a, int nsteps) {
  __shared__ __attribute__((aligned(16))) double sM1[2 * kN1 * kN1];  // [c][i + 64 k], one operator
  __shared__ double sP2[2][2][kCE][kMaxN2];  // [op][c][je]: row j0 - 1 + je of the direction-2 matrix
  __shared__ double sC[2][kCE][kN1];         // state on the extended columns
  __shared__ double sC2[2][kCE][kN1];        // C_{n2} on the extended columns
  __shared__ double sR[2][kN1][kCB];         // stage results on the own columns, [c][k][j]
  __shared__ double sPart[2][4][kCE][kN1];   // partial sums [c][kq][column][row]
  __shared__ int sflag;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n2 = a.n2;
  const int j0 = blockIdx.x * kCB;
  const unsigned G = gridDim.x;
  auto col_ok = [&](int je) { return j0 - 1 + je >= 0 && j0 - 1 + je < n2; };

  // ---- operator 0's direction-1 matrices, the direction-2 rows and the state into LDS
  dma_m1(sM1, a.P1[0][0], a.P1[0][1], wave, lane);
  for (int e = tid; e < 4 * kCE * kMaxN2; e += 512) {
    const int m = e / (kCE * kMaxN2), je = (e / kMaxN2) % kCE, k = e % kMaxN2;
    const int jg = j0 - 1 + je;
    sP2[m >> 1][m & 1][je][k] = (col_ok(je) && k < n2) ? a.P2[m >> 1][m & 1][jg + (size_t)n2 * k] : 0.0;
  }
  for (int e = tid; e < 2 * kCE * kN1; e += 512) {
    const int c = e / (kCE * kN1), je = (e / kN1) % kCE, i = e % kN1;
    const double* C = c ? a.V : a.U;
    sC[c][je][i] = col_ok(je) ? C[i + kN1 * (j0 - 1 + je)] : 0.0;
  }
  // stencil coefficients of the thread's point in S1/S2 (threads 0..255: row
  // lane, own column tid / 64)
  double b1[2][3] = {}, b2[2][3] = {};
  if (tid < kN1 * kCB) {
    const int jg = j0 + (tid >> 6);
    for (int c = 0; c < 2; ++c)
      for (int j = 0; j < 3; ++j) {
        b1[c][j] = a.band[c][0][j * kN1 + lane];
        b2[c][j] = jg < n2 ? a.band[c][1][j * n2 + jg] : 0.0;
      }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // products: component c; q is the quarter kq in the partial sums and the
  // column in the final sums (wave-uniform, so the argument pointers they
  // select are scalar loads)
  const int c = __builtin_amdgcn_readfirstlane(wave >> 2);
  const int q = __builtin_amdgcn_readfirstlane(wave & 3);
  const double tau = a.tau, tau2 = 2.0 * a.tau;
  unsigned bar = 0;
  bool ok = true;

  // the own columns' stage values (threads 0..255: point (lane, tid / 64))
  auto stage = [&](bool first) {
    if (tid >= kN1 * kCB) return;
    const int jl = tid >> 6, je = jl + 1, i = lane;
    const double u = sC[0][je][i], v = sC[1][je][i];
    double gu, gv;
    react(a.r, u, v, gu, gv);
    if (first) {
      const double um = i > 0 ? sC[0][je][i - 1] : 0.0, up = i + 1 < kN1 ? sC[0][je][i + 1] : 0.0;
      const double vm = i > 0 ? sC[1][je][i - 1] : 0.0, vp = i + 1 < kN1 ? sC[1][je][i + 1] : 0.0;
      double ku = b1[0][0] * um + b1[0][1] * u + b1[0][2] * up;
      double kv = b1[1][0] * vm + b1[1][1] * v + b1[1][2] * vp;
      ku += b2[0][0] * sC[0][je - 1][i] + b2[0][1] * u + b2[0][2] * sC[0][je + 1][i];
      kv += b2[1][0] * sC[1][je - 1][i] + b2[1][1] * v + b2[1][2] * sC[1][je + 1][i];
      sR[0][i][jl] = ku + gu;
      sR[1][i][jl] = kv + gv;
    } else {
      double gu2, gv2;
      react(a.r, sC2[0][je][i], sC2[1][je][i], gu2, gv2);
      sR[0][i][jl] = gu2 - gu;
      sR[1][i][jl] = gv2 - gv;
    }
  };
  // direction-1 product of the own columns into the exchange buffer Y[c]
  auto dir1 = [&](double* const* Y) {
    double part[kCB];
    dir1_partial(sM1 + c * kN1 * kN1, sR[c], q, lane, part);
#pragma unroll
    for (int j = 0; j < kCB; ++j) sPart[c][q][j][lane] = part[j];
    __syncthreads();
    if (j0 + q < n2) {
      const double y = (sPart[c][0][q][lane] + sPart[c][1][q][lane]) +
                       (sPart[c][2][q][lane] + sPart[c][3][q][lane]);
      __hip_atomic_store(Y[c] + lane + kN1 * (j0 + q), y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  // direction-2 product of the extended columns from the loaded y: z for the
  // columns q and q + 4
  auto dir2 = [&](const double (&y)[16], int op, double (&z)[2]) {
    double part[kCE];
    dir2_partial(y, sP2[op][c], q, part);
#pragma unroll
    for (int je = 0; je < kCE; ++je) sPart[c][q][je][lane] = part[je];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int je = q + 4 * e;
      z[e] = je < kCE ? (sPart[c][0][je][lane] + sPart[c][1][je][lane]) +
                            (sPart[c][2][je][lane] + sPart[c][3][je][lane])
                      : 0.0;
    }
  };

  for (int step = 0; step < nsteps && ok; ++step) {
    // ---- S1, P1 (operator 0's matrices are in sM1)
    stage(true);
    __syncthreads();
    dir1(a.Y[0]);
    if (!(ok = grid_sync(a.counter, a.err, G * ++bar, a.spin_limit, &sflag))) break;
    // ---- P2, with operator 1's direction-1 matrices in flight (the copy is
    // issued first: its loads hit in L2, the exchange loads do not)
    {
      double y[16], z[2];
      dma_m1(sM1, a.P1[1][0], a.P1[1][1], wave, lane);
      dir2_load(a.Y[0][c], n2, q, lane, y);
      dir2(y, 0, z);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int je = q + 4 * e;
        if (je < kCE) sC2[c][je][lane] = col_ok(je) ? sC[c][je][lane] + tau * z[e] : 0.0;
      }
    }
    __syncthreads();
    // ---- S2, P3
    stage(false);
    __builtin_amdgcn_s_waitcnt(0);   // this wave's part of the matrix copy has landed
    __syncthreads();
    dir1(a.Y[1]);
    if (!(ok = grid_sync(a.counter, a.err, G * ++bar, a.spin_limit, &sflag))) break;
    // ---- P4, with operator 0's direction-1 matrices in flight for the next step
    {
      double y[16], z[2];
      if (step + 1 < nsteps) dma_m1(sM1, a.P1[0][0], a.P1[0][1], wave, lane);
      dir2_load(a.Y[1][c], n2, q, lane, y);
      dir2(y, 1, z);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int je = q + 4 * e;
        if (je < kCE && col_ok(je)) sC[c][je][lane] = sC2[c][je][lane] + tau2 * z[e];
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  // ---- the own columns back to U, V (NaN if the launch was abandoned)
  for (int e = tid; e < 2 * kCB * kN1; e += 512) {
    const int cc = e / (kCB * kN1), jl = (e / kN1) % kCB, i = e % kN1;
    if (j0 + jl >= n2) continue;
    double* C = cc ? a.V : a.U;
    C[i + kN1 * (j0 + jl)] = ok ? sC[cc][jl + 1][i] : __builtin_nan("");
  }
}

}  // namespace

unsigned small2d_spin_limit() {
  const char* v = std::getenv("ADR_TEST_SPIN_LIMIT");
  if (!v || !*v) return kSpinLimit;
  char* end = nullptr;
  const unsigned long x = std::strtoul(v, &end, 10);
  return (end && *end == '\0' && x < kSpinLimit) ? (unsigned)x : kSpinLimit;
}

bool small2d_fits(int d, int n1, int n2) {
  return d == 2 && n1 == kN1 && n2 >= 3 && n2 <= kMaxN2;
}

hipError_t launch_etd_small2d(const Small2dArgs& a, int nsteps, hipStream_t s) {
  if (!small2d_fits(2, kN1, a.n2) || nsteps < 0 || !a.U || !a.V || !a.counter || !a.err)
    return hipErrorInvalidValue;
  for (int op = 0; op < 2; ++op)
    for (int c = 0; c < 2; ++c)
      if (!a.P1[op][c] || !a.P2[op][c] || !a.band[c][0] || !a.band[c][1] || !a.Y[op][c] ||
          reinterpret_cast<uintptr_t>(a.P1[op][c]) % 16 != 0)
        return hipErrorInvalidValue;
  if (nsteps == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_sync, dim3(1), dim3(64), 0, s, a.counter, a.err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned groups = (unsigned)((a.n2 + kCB - 1) / kCB);
  Small2dArgs args = a;
  int steps = nsteps;
  void* params[] = {&args, &steps};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_etd_small2d), dim3(groups),
                                    dim3(512), params, 0, s);
}

}  // namespace adr
