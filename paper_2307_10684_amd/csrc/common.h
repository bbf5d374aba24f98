// Internal declarations shared by the host library and the HIP kernels.
// Nothing here is part of the public ABI (include/adr.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace adr {

// Up to four tensors share one geometry in a grouped mode-product launch
// (both components of ETD2RKds; both components and both Tucker inputs of
// Lawson2b).
constexpr int kMaxGroup = 4;

enum class Elem : int { F64 = 0, F32 = 1 };

// Reaction model constants as passed to the stage kernels and
// to the FP64 mode product when it carries ETD2RKds stage 2.
struct Reaction {
  int model;
  double p[12];
};

// Geometry of one mu-mode product on an order-d tensor stored first index
// fastest: the tensor is viewed as (L, n, R) with L = prod_{nu<mu} n_nu,
// R = prod_{nu>mu} n_nu.  A fibre index x in [0, L*R) stands for (l, r) with
// x = l + L*r, and element k of fibre x sits at l + L*(k + n*r).
struct ModeArgs {
  const void* W[kMaxGroup];      // input tensors (Elem in_t)
  const void* M[kMaxGroup];      // n x n column-major matrices (FP64, or FP32 for the F32 path)
  void* out[kMaxGroup];          // output tensors (Elem out_t)
  const double* Y[kMaxGroup];    // optional FP64 addends (may alias out when out_t is F64)
  const double* Z[kMaxGroup];    // optional second FP64 addends
  double alpha, beta, gamma;     // out = alpha*(W x_mu M) + beta*Y + gamma*Z
  long long L, R, X;             // X = L*R fibres
  int n;                         // n_mu (fibre length, matrix size)
  int group;                     // number of tensors in the launch (1..kMaxGroup)
  // ETD2RKds stage 2 carried by the last product of the phi_1 Tucker operator
  // (group = 2: U then V, Y = the states C_n, out = C_{n2}):
  //   Rout[c] = G^c(out[0], out[1]) - G^c(Y[0], Y[1]); null when not fused.
  void* Rout[2];
  Reaction react;
};
// Whether launch_mode_product_f64 can carry stage 2 for this product (a.Rout
// set): an evenly tiled x-contiguous product of two tensors with addends.
bool mode_f64_stage2_fusable(const ModeArgs& a);

// One product of a grouped launch (also the per-tile view of a single product).
struct TileJob {
  const double* W;
  const double* M;
  double* out;
  const double* Y;
  const double* Z;
  double alpha, beta, gamma;
  long long L, X;
  int n;
  int n_itiles;
  long long tile_begin;   // first tile of this job in the grouped launch
};

// Tile configurations of the FP64 product (rows BI of M x fibres BX per workgroup);
// P64X64: 64x64 tiles walked by persistent workgroups (four per CU).
enum class TileCfg : int { I64X64 = 0, I64X128 = 1, I128X64 = 2, I128X128 = 3, P64X64 = 4 };
constexpr int kNumTileCfgs = 5;
void tile_cfg_dims(TileCfg c, int& BI, int& BX);
// Grouped FP64 products; `jobs` is a device array of `njobs` TileJobs whose tile
// offsets were laid out for configuration `cfg`; `ntiles` is the total.
hipError_t launch_mode_grouped_f64(TileCfg cfg, bool kfast, const TileJob* jobs, int njobs,
                                   long long ntiles, hipStream_t s);

// Launchers (return hipSuccess or the launch error).
hipError_t launch_mode_product_f64(const ModeArgs& a, hipStream_t s);

// The products along directions 1 and 2 in one pass over the (i1, i2) planes
// (FP64): out[:, :, p] = alpha * M1 W[:, :, p] M2^T (+ beta * Y[:, :, p]) for
// p < planes, every tensor n x n x planes; n = n1 = n2 must be 64 or 128
// (mode12_plane_fits) and every pointer 16-byte aligned.
bool mode12_plane_fits(int n1, int n2);
hipError_t launch_mode12_plane(int group, const double* const* W, const double* const* M1,
                               const double* const* M2, double* const* out,
                               const double* const* Y, double alpha, double beta, int n,
                               int planes, hipStream_t s);

// Reduced-precision "transposing" product (precision kLowpF32, kLowpBF16X3 or
// kLowpBF16X2, the adr_precision values):
//   out[x + X*i] = alpha * sum_k M[i,k] W[k + n*x] (+ beta * Y[x + X*i])
// W: FP32 n x X column-major; M: FP32 n x n column-major (FP32) or the split
// BF16 parts of M as transposed planes (three or two); out: FP32, or FP64 with
// the FP64 addend Y.  With the FP32 addends Z (FP64 output only):
//   out = (beta * Y + Z) + alpha * sum_k M[i,k] W[k + n*x].
constexpr int kLowpF32 = 1, kLowpBF16X3 = 2, kLowpBF16X2 = 3;
struct SplitPlanes {
  const unsigned short* p[3];   // the parts, largest first (p[2] unused with two parts)
};
hipError_t launch_tgemm_lowp(int precision, const void* const* W, const void* const* Mf32,
                             const SplitPlanes* Mp, void* const* out, const double* const* Y,
                             int group, int n, long long X, double alpha, double beta, int out_f64,
                             hipStream_t s, const float* const* Z = nullptr);
// One FP32 transposing product of a grouped launch (tiles of 128 x 128).
struct LowpJob {
  const float* W;
  const float* M;
  void* out;
  const double* Y;
  const float* Z;          // FP32 second addend (FP64 output only), or null
  double alpha, beta;
  int n;
  long long X;
  int out_f64;
  int n_itiles;
  long long tile_begin;
};
// vec: every job has n % 4 == 0 and 16-byte aligned W and M (vectorised loads)
hipError_t launch_tgemm_lowp_grouped(int precision, const LowpJob* jobs, int njobs,
                                     long long ntiles, bool vec, hipStream_t s);
// Split an FP64 n x n column-major matrix into `parts` (2 or 3) transposed bf16
// planes P[p][i*n + k]: each part is the bf16 rounding of the remainder the
// previous parts leave.
hipError_t launch_split_bf16(int n, int parts, const double* M, unsigned short* const* P,
                             hipStream_t s);

struct StageGeom {
  int d;
  int n[3];
  long long N;
  const double* band[2][3];   // tridiagonal bands (sub, diag, super) per component/direction, or null
};

// Grouped stage launches over several problems (batched and serving runs).
constexpr int kStage1Point = 0, kStage1Tile = 1;   // stage-1 kernel variants
struct StageJob {
  StageGeom g;
  Reaction r;
  int kind;                // kStage1Point or kStage1Tile (from stage1_plan)
  const double* U;
  const double* V;
  void* R[2];
  int gx, gy;              // block grid of this problem (from stage1_plan)
  long long block_begin;   // first block of this problem in the grouped launch
};
struct PointJob {
  int kind;                // 0: stage 2, 1: stage 2 from FP32 increments, 2: final C += D1 + D2
  Reaction r;
  long long N;
  const double* U;
  const double* V;
  const void* A;           // kind 0: U2 (FP64); kind 1, 2: D1u (FP32)
  const void* B;           // kind 0: V2; kind 1, 2: D1v
  const void* C2;          // kind 2: D2u (FP32)
  const void* D2;          // kind 2: D2v
  void* R[2];              // kinds 0, 1: outputs
  long long block_begin;
};
// all jobs of one launch use the variant `kind` (kStage1Point or kStage1Tile)
hipError_t launch_stage1_grouped(const StageJob* jobs, int njobs, long long nblocks, int kind,
                                 int r_f32, hipStream_t s);
hipError_t launch_pointwise_grouped(const PointJob* jobs, int njobs, long long nblocks, int r_f32,
                                    hipStream_t s);
// Stage-1 variant and block grid of one problem (gx * gy * gz blocks of 64 x 4).
int stage1_plan(const StageGeom& g, int& kind, int& gx, int& gy, int& gz);

// ETD2RKds stage 1: R^c = sum_mu C x_mu A_mu^c (stencil where a band is given,
// nothing where it is not) + G^c(U, V).  R may be FP64 or FP32.
hipError_t launch_etd_stage1(const StageGeom& g, const Reaction& r, const double* U,
                             const double* V, void* Ru, void* Rv, int r_f32, hipStream_t s);
// ETD2RKds stage 2: R^c = G^c(U2, V2) - G^c(U, V).
hipError_t launch_etd_stage2(long long N, const Reaction& r, const double* U, const double* V,
                             const double* U2, const double* V2, void* Ru, void* Rv, int r_f32,
                             hipStream_t s);
// Reduced-precision ETD2RKds with FP32 increments D1, D2 of the two Tucker operators:
// stage 2 R^c = G^c(U + D1u, V + D1v) - G^c(U, V).
hipError_t launch_etd_stage2_inc(long long N, const Reaction& r, const double* U, const double* V,
                                 const float* Du, const float* Dv, float* Ru, float* Rv,
                                 hipStream_t s);
// Whole FP64 ETD2RKds steps of a small 2D problem (n1 = 64, 3 <= n2 <= 64,
// tridiagonal operators) in one cooperative launch, the state updated in place.
// P1/P2[op][c]: the direction-1 / direction-2 matrices of component c for
// op 0 (phi_1) and op 1 (phi_2); band[c][mu] as in adr_problem; Y[op][c]:
// n1 x n2 doubles of workspace each; counter, err: a 4-byte slot each.
struct Small2dArgs {
  double* U;
  double* V;
  const double* P1[2][2];
  const double* P2[2][2];
  const double* band[2][2];
  Reaction r;
  double tau;
  int n2;
  double* Y[2][2];
  unsigned* counter;
  int* err;
  unsigned spin_limit;      // polls before a barrier wait gives up
};
bool small2d_fits(int d, int n1, int n2);
// Polls a whole-step barrier allows before the launch is abandoned: about 2^20,
// or the value of the environment variable ADR_TEST_SPIN_LIMIT when it is set
// (for tests of the abandon path).
unsigned small2d_spin_limit();
hipError_t launch_etd_small2d(const Small2dArgs& a, int nsteps, hipStream_t s);
// Lawson2b stage 1: A^c = C + tau G^c(U, V), B^c = C + tau/2 G^c(U, V).
hipError_t launch_lawson_stage1(long long N, const Reaction& r, double tau, const double* U,
                                const double* V, void* Au, void* Av, void* Bu, void* Bv, int f32,
                                hipStream_t s);
// Lawson2b stage 2: C += tau/2 G^c(U2, V2)  (C holds the second Tucker result).
hipError_t launch_lawson_stage2(long long N, const Reaction& r, double tau, double* U, double* V,
                                const double* U2, const double* V2, hipStream_t s);

// Logical tile of workgroup b in a launch of G workgroups.  Workgroups are
// dealt to the 8 XCDs round-robin and each XCD has its own L2.  Logical tiles
// are taken in chunks of C consecutive tiles, and the chunks are dealt to the
// XCDs round-robin: the tiles of a chunk (e.g. the row tiles of one fibre
// block, which read the same operand data) run on one XCD at about the same
// time and share its L2, while every XCD gets a similar mix of large and small
// jobs.  Workgroups beyond the last whole round of 8 C keep their index.
__device__ __forceinline__ long long xcd_tile(long long b, long long G, long long C = 8) {
  const long long span = 8 * C, Gs = (G / span) * span;
  if (b >= Gs) return b;
  const long long k = b % 8, j = b / 8;
  return ((j / C) * 8 + k) * C + (j % C);
}

// Dynamics indicators (trapezoidal means, increment norms, non-finite count)
// into rec[0..4]; `partial` holds 5 * indicator_blocks(N) doubles.  Up and Vp
// are both given or both null.
constexpr int kMaxIndicatorBlocks = 2048;
int indicator_blocks(long long N);
hipError_t launch_indicators(int d, const int* n, const double* U, const double* V,
                             const double* Up, const double* Vp, double* partial, double* rec,
                             hipStream_t s);

// Small dense helpers for the matrix-function precompute (n x n, column-major).
hipError_t launch_norm1(int n, const double* X, double scale, double* out, hipStream_t s);
hipError_t launch_scale_copy(long long count, const double* in, double scale, double* out,
                             hipStream_t s);
// out = sum_j c[j] * P[j] + c0 * I   (up to 8 matrices)
hipError_t launch_lincomb(int n, int count, const double* const* P, const double* c, double c0,
                          double* out, hipStream_t s);
hipError_t launch_copy_f64(const double* in, double* out, size_t count, hipStream_t s);
hipError_t launch_convert_f64_f32(const double* in, float* out, size_t count, hipStream_t s);

}  // namespace adr
