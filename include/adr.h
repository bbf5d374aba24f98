/*
 * adr.h -- C ABI of the MI355X (gfx950) ETD2RKds library, libadr.so.
 *
 * Solves two-component advection-diffusion-reaction systems on tensor-product
 * grids, in the form of Caliari & Cassini, "A second order directional split
 * exponential integrator for systems of advection-diffusion-reaction
 * equations" (arXiv 2307.10684):
 *
 *   U' = sum_mu U x_mu A_mu^u + G^u(U, V),   V' = sum_mu V x_mu A_mu^v + G^v(U, V)
 *
 * (Sec. 1 eqs. (1)-(3), Sec. 2 eq. (6)), time-stepped by ETD2RKds (Sec. 3,
 * eq. (11)) or Lawson2b (Sec. 2, eq. (7)) with a constant step tau whose small
 * matrix functions are computed once (Sec. 4, opening paragraphs).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Status: every function returns an int, ADR_OK (0) on success or a negative
 *   adr_status.  Arguments are validated before any work is enqueued; on
 *   ADR_EINVAL nothing has been written.  No C++ exception crosses the ABI.
 * - Layout: a grid tensor of order d with sizes n[0..d-1] is a dense array of
 *   N = n[0]*...*n[d-1] elements with n[0] (direction mu = 1) fastest, i.e. the
 *   vec ordering of Sec. 2.  Small n x n matrices are column-major.
 * - Memory: every pointer argument is owned by the caller.  "device" pointers
 *   are HIP device allocations on the current device; "host" pointers are
 *   ordinary CPU memory.  The library never frees caller memory.
 * - Streams: `stream` is a hipStream_t passed as void* (NULL = the legacy
 *   default stream).  Device work is enqueued asynchronously on it; unless a
 *   function says otherwise it does not synchronise.
 * - Aliasing: outputs must not alias inputs unless a function says so.
 */
#ifndef ADR_H
#define ADR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum adr_status {
  ADR_OK = 0,
  ADR_EINVAL = -1,     /* invalid argument (null pointer, size, step, enum) */
  ADR_ENOMEM = -2,     /* workspace too small or a temporary allocation failed */
  ADR_EDEVICE = -3,    /* a HIP call or kernel launch failed */
  ADR_ENOTSUP = -4,    /* valid but unsupported combination */
  ADR_ENONFINITE = -5  /* a non-finite value was found where none may be */
};

enum adr_bc { ADR_BC_NEUMANN = 0 };                 /* homogeneous Neumann, Sec. 1 */
enum adr_scheme { ADR_ETD2RKDS = 0,                 /* Sec. 3, eq. (11) */
                  ADR_LAWSON2B = 1 };               /* Sec. 2, eq. (7)  */
/* Precision of the bulk mode products (the state, the stage combinations and
 * the small matrix functions stay FP64 in every mode):
 *   ADR_BF16X3: each FP32 operand split into three bf16 parts hi + mid + lo
 *     (exact for FP32 values), six bf16 MFMA products (hi hi, hi mid, mid hi,
 *     hi lo, mid mid, lo hi) accumulated in FP32; close to FP32 accuracy.
 *   ADR_BF16X2: two parts hi + lo, three products (hi hi, hi lo, lo hi),
 *     about 2^-16 relative per product: faster, less accurate. */
enum adr_precision { ADR_F64 = 0,                   /* all arithmetic in FP64 */
                     ADR_F32 = 1,                   /* mode products in FP32 */
                     ADR_BF16X3 = 2,                /* 3-part split BF16, 6 products */
                     ADR_BF16X2 = 3 };              /* 2-part split BF16, 3 products */
/* Reaction models G^u, G^v and the order of adr_problem.params:
 *   ADR_SCHNAKENBERG (gamma, a, b):   gamma(a - u + u^2 v),  gamma(b - u^2 v)    Sec. 4.1 eq. (12)
 *   ADR_FHN          (rho, eps, a1, a0): rho(u - u^3 - v),  rho eps(u - a1 v - a0)  Secs. 4.2-4.3
 *   ADR_BRUSSELATOR  (A, B):          A - (B+1)u + u^2 v,    B u - u^2 v        Sec. 4.6 eq. (17)
 *   ADR_ZERO         ():              0, 0  (pure advection-diffusion)
 *   ADR_DIB          (rho, a1u, a2u, a3u, a4u, a1v, a2v, a3v, a4v, a5v):        Sec. 4.4 eq. (15)
 *                    rho(a1u(1-v)u - a2u u^3 - a3u(v - a4u)),
 *                    rho(a1v(1+a2v u)(1-v)(1-a3v(1-v)) - a4v v(1+a5v u)(1+a3v v)) */
enum adr_model { ADR_SCHNAKENBERG = 0, ADR_FHN = 1, ADR_BRUSSELATOR = 2, ADR_ZERO = 3,
                 ADR_DIB = 4 };
#define ADR_MAX_PARAMS 12

#define ADR_MAX_DIM 3

/* Human-readable text of a status code (static storage, never NULL). */
const char* adr_strerror(int status);

/* Library ABI version (major*10000 + minor*100 + patch). */
int adr_version(void);

/*
 * adr_build_1d_ops -- the 1D operator A = diff * d^2/dx^2 - vel * d/dx on [a, b]
 * by second-order centred finite differences with homogeneous Neumann
 * conditions embedded in the matrix (Sec. 4, opening paragraphs).  Grid nodes
 * are node-centred, x_i = a + i h, h = (b - a)/(n - 1), and the boundary rows
 * use the ghost values u_{-1} = u_1, u_n = u_{n-2}: diffusion rows
 * diff*(-2, 2)/h^2 and diff*(2, -2)/h^2, advection rows 0.
 *   n        grid points, n >= 3
 *   bc       ADR_BC_NEUMANN (the only condition the paper uses)
 *   A        host, n*n doubles, column-major; may be NULL
 *   band     host, 3*n doubles: band[i] = A[i,i-1] (band[0] = 0),
 *            band[n+i] = A[i,i], band[2n+i] = A[i,i+1] (band[3n-1] = 0); may be NULL
 * Pure host computation; errors: ADR_EINVAL (n < 3, b <= a, non-finite input,
 * unknown bc, both outputs NULL).
 */
int adr_build_1d_ops(int n, double a, double b, double diff, double vel, int bc,
                     double* A, double* band);

/*
 * adr_precompute_phi -- E = e^{tau A}, P1 = phi_1(tau A), P2 = phi_2(tau A) of
 * one n x n matrix, with phi_l(X) = int_0^1 theta^{l-1}/(l-1)! e^{(1-theta)X} dtheta
 * (Sec. 2, eq. (9)).  Computed on the device in FP64 by a degree-18 Taylor
 * polynomial of the scaled matrix tau*A/2^s followed by s steps of the
 * modified squaring of Skaflestad & Wright (cited in Sec. 4).
 *   A_dev            device, n*n doubles, column-major
 *   E_dev, P1_dev, P2_dev  device, n*n doubles each; any may be NULL (not computed)
 *   n                1 <= n <= 4096
 * Works in a per-device scratch of 14*n*n doubles that the library keeps
 * between calls (allocated, or grown, when a larger n first arrives).  Calls
 * are serialised by a lock; each synchronises `stream` twice (to read back
 * ||tau A||_1 and pick s, and before returning, so the scratch is free for
 * the next call).  Errors: ADR_EINVAL, ADR_ENOMEM, ADR_EDEVICE,
 * ADR_ENONFINITE (tau*A has a non-finite entry).
 */
int adr_precompute_phi(int n, const double* A_dev, double tau, double* E_dev,
                       double* P1_dev, double* P2_dev, void* stream);

/*
 * adr_precompute_phi_batch -- adr_precompute_phi for `count` (1..4096)
 * matrices with two synchronisations in all: the 1-norms of every tau_i A_i
 * are read back together, then each matrix's polynomial and squarings run in
 * turn on `stream` (same kernels and results as one call per matrix), and the
 * call waits for them before returning.
 *   n, tau        host arrays of `count` sizes (1..4096) and nonzero finite steps
 *   A_dev         host array of `count` device matrices (n_i x n_i, column-major)
 *   E_dev, P1_dev, P2_dev  host arrays of `count` device outputs, or NULL arrays;
 *                 an entry may be NULL (not computed), but not all three of one matrix
 * Works in the same kept per-device scratch as adr_precompute_phi, of
 * 14 n_max^2 + 1 + count doubles.  Errors as adr_precompute_phi.
 */
int adr_precompute_phi_batch(int count, const int32_t* n, const double* const* A_dev,
                             const double* tau, double* const* E_dev, double* const* P1_dev,
                             double* const* P2_dev, void* stream);

/*
 * adr_precompute_phi_noalloc -- adr_precompute_phi for callers that cannot
 * allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results, worked out in a fixed
 * array that the library keeps in each GPU's memory until the process ends
 * (14 n^2 + 1 doubles for n = ADR_PHI_NOALLOC_MAX_N: 29.4 MB per GPU).  It
 * calls no hipMalloc or hipFree.
 *   n        1 <= n <= ADR_PHI_NOALLOC_MAX_N; a larger n returns ADR_ENOMEM
 *            (the fixed array is too small) before any device work
 * Other arguments and errors as adr_precompute_phi.  All calls on a GPU share
 * its array, which keeps the last call's contents: calls are serialised by a
 * lock, and each synchronises `stream` twice (the 1-norm read-back, and before
 * returning), so no two calls use the array at once.
 */
#define ADR_PHI_NOALLOC_MAX_N 512
int adr_precompute_phi_noalloc(int n, const double* A_dev, double tau, double* E_dev,
                               double* P1_dev, double* P2_dev, void* stream);

/*
 * One problem instance: grid, model, scheme, and the device-resident small
 * matrices.  The tensors U, V are passed separately to adr_step/adr_solve.
 */
typedef struct adr_problem {
  int32_t d;                   /* space dimension, 1..3 */
  int32_t n[ADR_MAX_DIM];      /* grid sizes, n[0] fastest; entries >= d ignored; each 3..4096 */
  int32_t model;               /* enum adr_model */
  int32_t scheme;              /* enum adr_scheme */
  int32_t precision;           /* enum adr_precision */
  int32_t flags;               /* reserved, must be 0 */
  double params[ADR_MAX_PARAMS]; /* model constants, order as in enum adr_model; rest unused */
  double tau;                  /* time step, > 0 (used for the stage scalings) */
  /* phi[c][j][mu]: device n[mu] x n[mu] FP64 column-major matrices of
   * component c (0 = u, 1 = v), j = 0: e^{tau A}, 1: phi_1(tau A), 2: phi_2(tau A).
   * ETD2RKds needs j = 1, 2; Lawson2b needs j = 0. */
  const double* phi[2][3][ADR_MAX_DIM];
  /* band[c][mu]: device 3*n[mu] doubles, the tridiagonal of A_mu^c in the
   * layout of adr_build_1d_ops.  If NULL, dense[c][mu] is used instead. */
  const double* band[2][ADR_MAX_DIM];
  /* dense[c][mu]: device n[mu] x n[mu] FP64 A_mu^c (only read when band is NULL
   * and the scheme is ETD2RKds; any sparsity pattern is allowed, Sec. 1). */
  const double* dense[2][ADR_MAX_DIM];
} adr_problem;

/* Bytes of device workspace adr_step/adr_solve need for this problem (0 on invalid input). */
size_t adr_workspace_bytes(const adr_problem* p);

/*
 * adr_step -- advance (U, V) by one step of p->scheme in place.
 *   U, V   device, N doubles each (FP64 state in every precision mode)
 *   work   device, at least adr_workspace_bytes(p) bytes, 256-byte aligned
 * Enqueues 2*d mode-product launches and 2 stage launches (ETD2RKds) on
 * `stream`; no synchronisation.  FP64 ETD2RKds on 2D grids of 64 x n2
 * (3 <= n2 <= 64) with tridiagonal operators (band given) and 16-byte aligned
 * direction-1 matrices instead runs all steps of the call in one cooperative
 * launch (after a one-thread reset of its barrier counter); should that
 * launch ever abandon its steps (a grid barrier that does not complete within
 * its spin limit, about 2^20 polls; the environment variable
 * ADR_TEST_SPIN_LIMIT lowers it, for tests of this path), U and V are left NaN
 * on the abandoned columns.  Errors:
 * ADR_EINVAL, ADR_ENOMEM (work too small), ADR_ENOTSUP, ADR_EDEVICE.
 */
int adr_step(const adr_problem* p, double* U, double* V, void* work, size_t work_bytes,
             void* stream);

/* adr_solve -- nsteps >= 0 calls of adr_step with one validation (same arguments). */
int adr_solve(const adr_problem* p, double* U, double* V, int nsteps, void* work,
              size_t work_bytes, void* stream);

/*
 * adr_mode_product -- out = alpha * (W x_mu M) + beta * Y, the mu-mode product
 * of Sec. 2 ((W x_mu M)[.., i, ..] = sum_k M[i,k] W[.., k, ..]) with an
 * optional scaled addend, in FP64.
 *   d, n      tensor order (1..3) and sizes (n[0] fastest), each n >= 1
 *   mu        0-based direction (paper's mu - 1), 0 <= mu < d
 *   M         device n[mu] x n[mu] column-major
 *   W, out    device N doubles; out must not alias W
 *   Y         device N doubles or NULL (then beta is ignored); Y may alias out
 * Errors: ADR_EINVAL, ADR_EDEVICE.
 */
int adr_mode_product(int d, const int32_t* n, int mu, const double* M, const double* W,
                     double* out, double alpha, double beta, const double* Y, void* stream);

/*
 * adr_tucker -- out = alpha * (W x_1 M[0] x_2 ... x_d M[d-1]) + beta * Y, the
 * Tucker operator of Sec. 2 eq. (5), applied in the order mu = 1..d.
 *   M         array of d device matrices (n[mu] x n[mu], column-major)
 *   work      device, >= adr_tucker_workspace_bytes(d, n) bytes
 * out may not alias W; Y may alias out.  Errors as adr_mode_product, plus ADR_ENOMEM.
 */
size_t adr_tucker_workspace_bytes(int d, const int32_t* n);
int adr_tucker(int d, const int32_t* n, const double* const* M, const double* W, double* out,
               double alpha, double beta, const double* Y, void* work, size_t work_bytes,
               void* stream);

/*
 * adr_device_copy -- out[i] = in[i] for i < count (doubles), a plain streaming
 * copy used to calibrate hardware byte counters against known traffic.
 */
int adr_device_copy(const double* in, double* out, size_t count, void* stream);

/*
 * Dynamics indicators (Sec. 4, opening paragraphs): the spatial mean <C> of
 * each component, an approximation of (1/|Omega|) times the integral of the
 * field, here by the trapezoidal rule on the node-centred grid (weights 1/2 on
 * boundary nodes in each direction, normalised by prod_mu (n_mu - 1)); the
 * Frobenius norm of the time increment ||C_{n+1} - C_n||_F; and the number of
 * grid points where any input holds NaN or +-inf.  One fused, deterministic
 * reduction (no atomics).
 *
 * adr_indicators -- rec (device, 5 doubles) = { <U>, <V>, ||U - Uprev||_F,
 *   ||V - Vprev||_F, non-finite count }.  Uprev and Vprev are both device
 *   tensors or both NULL (then rec[2] = rec[3] = 0).  work: device scratch of
 *   adr_indicators_workspace_bytes(d, n) bytes.  Errors: ADR_EINVAL,
 *   ADR_ENOMEM, ADR_EDEVICE.
 */
size_t adr_indicators_workspace_bytes(int d, const int32_t* n);
int adr_indicators(int d, const int32_t* n, const double* U, const double* V,
                   const double* Uprev, const double* Vprev, double* rec, void* work,
                   size_t work_bytes, void* stream);

/*
 * adr_solve_monitored -- adr_solve, plus the indicators of every `every`-th
 * step (the increment of that step): record k = 0 .. nsteps/every - 1 at
 * rec + 5k (device), taken after step (k+1)*every.
 *   mwork   device, 256-byte aligned, adr_monitor_workspace_bytes(p) bytes
 *           (a copy of the state before each recorded step, and the
 *           reduction scratch)
 * Synchronises `stream` once at the end (only if a record was taken) and
 * returns ADR_ENONFINITE if any record counted a non-finite value (the steps
 * and records are still all done).  Other errors as adr_solve.
 */
size_t adr_monitor_workspace_bytes(const adr_problem* p);
int adr_solve_monitored(const adr_problem* p, double* U, double* V, int nsteps, int every,
                        double* rec, void* work, size_t work_bytes, void* mwork,
                        size_t mwork_bytes, void* stream);

/*
 * Grouped multi-problem ETD2RKds ("batch plans").  Sec. 3 eq. (11) is applied
 * to `count` independent problems at once; each problem keeps its own grid
 * (sizes and dimension may differ), model, constants, tau and small matrices.
 * Every phase of the step (stage 1, the d mode products of each Tucker
 * operator, stage 2, and for ADR_F32 the final update) is one launch over all
 * problems, driven by job tables the plan keeps in device memory, so one step
 * costs 2*d_max + 2 launches (+1 for ADR_F32) whatever `count` is.
 *
 * adr_batch_create -- build a plan.
 *   problems    host array of `count` (1..4096) problem descriptors; all must
 *               use ETD2RKds, the same precision (ADR_F64 or ADR_F32) and
 *               give band[c][mu] for every direction.  The structs are copied;
 *               the device buffers they point to must stay valid until
 *               adr_batch_destroy.
 *   U, V        host arrays of `count` device state pointers (N_i doubles each)
 *   work        host array of `count` device workspaces, 256-byte aligned, of
 *               at least adr_workspace_bytes(&problems[i]) bytes; they must not
 *               overlap each other or any state
 *   flags       ADR_BATCH_AUTOTUNE: time the tile shapes of every FP64 mode-
 *               product phase on the plan's own buffers and keep the fastest
 *               (cached per phase shape for the process; with the environment
 *               variable ADR_TUNE_CACHE naming a file, also across processes).
 *               The cache key is the phase's precision, direction, largest
 *               n_mu, product count and log2 of its multiply-adds.
 *               Tuning launches write only workspace, never U or V.
 *               ADR_BATCH_GRAPH: capture one step in a HIP graph that
 *               adr_batch_run replays.
 *               ADR_BATCH_PREPARED (ADR_F32): the FP32 copies of the small
 *               matrices that a plan keeps in each workspace are already there
 *               (an earlier plan over the same problem and workspace wrote
 *               them); skip rewriting them.
 *   stream      stream for the set-up work (table upload, FP32 matrix copies,
 *               tuning); synchronised before the call returns, so plans can be
 *               built on a side stream while other plans run elsewhere
 *   plan        receives the plan
 * The plan's device tables come from a pool that destroyed plans return to
 * (no device-wide synchronisation on destroy; see adr_batch_destroy).
 * Errors: ADR_EINVAL, ADR_ENOMEM (a workspace too small, or no device memory
 * for the tables), ADR_ENOTSUP (scheme, precision or a missing band),
 * ADR_EDEVICE.
 */
typedef struct adr_batch adr_batch;
enum adr_batch_flags { ADR_BATCH_AUTOTUNE = 1, ADR_BATCH_GRAPH = 2, ADR_BATCH_PREPARED = 4 };
/* ADR_BATCH_TILE(cfg): use tile configuration cfg (0..4, see adr_batch_info) for
 * every FP64 mode-product phase instead of the default or the tuner's choice. */
#define ADR_BATCH_TILE(cfg) (((cfg) + 1) << 8)
int adr_batch_create(int count, const adr_problem* problems, double* const* U,
                     double* const* V, void* const* work, const size_t* work_bytes, int flags,
                     void* stream, adr_batch** plan);
/* adr_batch_run -- enqueue nsteps >= 0 steps of every problem of the plan on `stream`. */
int adr_batch_run(adr_batch* plan, int nsteps, void* stream);
/*
 * adr_batch_info -- the tile configuration chosen for the mode products of
 * each direction mu < max_phases (0: 64x64, 1: 64x128, 2: 128x64, 3: 128x128
 * rows x fibres, one tile per workgroup; 4: 64x64 tiles walked by persistent
 * workgroups; -1 where the plan has no FP64 phase), and whether a graph was
 * captured.  Either output may be NULL when not wanted (tile_cfg only with
 * max_phases == 0).
 */
int adr_batch_info(const adr_batch* plan, int* tile_cfg, int max_phases, int* graph_captured);
/* adr_batch_destroy -- release the plan (the caller's buffers are untouched).
 * First waits, on the host, for the steps that adr_batch_run enqueued for
 * this plan on any stream (only this plan's work, no device-wide wait), so a
 * plan may be destroyed right after an asynchronous run: its job tables are
 * handed to the next plan only once no queued kernel can read them. */
int adr_batch_destroy(adr_batch* plan);

/*
 * Kernel timing.  adr_timing_enable(capacity) makes later adr_step/adr_solve/
 * adr_tucker/adr_mode_product calls record a HIP event pair around each of
 * their kernel launches, on the stream the kernel runs on, for up to
 * `capacity` launches (capacity 0 disables timing and frees the events).
 * Batch plans run without a graph are timed the same way, one record per
 * grouped launch.
 * adr_timing_read synchronises on the recorded events and returns, for the
 * kernel class `kind` (0 = mode products, 1 = stage kernels, 2 = all,
 * 3 = mode products whose epilogue also computes a stage: ETD2RKds stage 2 in
 * FP64, the new state in reduced precision, 4 = launches that run whole steps:
 * FP64 ETD2RKds on 2D grids of 64 x n2, 3 <= n2 <= 64, with tridiagonal
 * operators), the number of launches and their summed duration in milliseconds.  The record is kept until the next
 * adr_timing_enable.  Not thread-safe; intended for benchmarks.
 */
int adr_timing_enable(int capacity);
int adr_timing_read(int kind, int* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* ADR_H */
