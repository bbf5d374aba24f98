// Host-side helpers shared by the single-problem entry points (adr_api.hip)
// and the grouped multi-problem plans (batch.hip).  Internal, not ABI.
#pragma once

#include <cmath>
#include <vector>

#include "adr.h"
#include "common.h"

namespace adr {
namespace host {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ------------------------------------------------------------------ timing
struct TimingRec {
  int kind;
  int slot;
};
struct Timing {
  int capacity = 0;
  std::vector<hipEvent_t> pool;  // 2 events per slot
  std::vector<TimingRec> recs;
};
extern Timing g_timing;

template <class F>
hipError_t timed(int kind, hipStream_t s, F&& f) {
  Timing& t = g_timing;
  if (t.capacity == 0 || (int)t.recs.size() >= t.capacity) return f();
  const int slot = (int)t.recs.size();
  hipError_t e = hipEventRecord(t.pool[2 * slot], s);
  if (e != hipSuccess) return e;
  e = f();
  if (e != hipSuccess) return e;
  e = hipEventRecord(t.pool[2 * slot + 1], s);
  if (e != hipSuccess) return e;
  t.recs.push_back({kind, slot});
  return hipSuccess;
}
// timing classes: plain mode products, stage kernels, and mode products whose
// epilogue also carries a stage (ETD2RKds stage 2, or the new state)
constexpr int kKindMode = 0, kKindStage = 1, kKindModeFused = 3, kKindSteps = 4;


inline int dev_err(hipError_t e) { return e == hipSuccess ? ADR_OK : ADR_EDEVICE; }

struct Geometry {
  int d;
  int n[3];
  long long N;
};

inline bool mode_geometry(const Geometry& g, int mu, long long& L, long long& R) {
  L = 1;
  R = 1;
  for (int nu = 0; nu < mu; ++nu) L *= g.n[nu];
  for (int nu = mu + 1; nu < g.d; ++nu) R *= g.n[nu];
  return true;
}

// Workspace carve-up.  Tensors are FP64 (8 bytes) or FP32 (4 bytes) for the
// reduced-precision intermediates; reduced-precision modes also hold FP32
// copies, or the split-BF16 parts, of the small matrices.
inline int split_parts(int precision) {
  return precision == ADR_BF16X3 ? 3 : precision == ADR_BF16X2 ? 2 : 0;
}
struct Carve {
  double* U2 = nullptr;
  double* V2 = nullptr;
  float* D[2] = {};                      // reduced-precision ETD2RKds: tau * Tucker(R1; phi_1)
  void* R[4] = {};
  void* T[4] = {};
  float* phi32[2][3][3] = {};            // FP32 copies (ADR_F32)
  unsigned short* phip[2][3][3][3] = {};  // split-BF16 parts [comp][j][mu][part], transposed
  size_t bytes = 0;
};

Carve carve(const adr_problem* p, const Geometry& g, char* base);

// Matrix functions of adr_precompute_phi for one n x n matrix, worked out in
// `base` (device, phi_scratch_doubles(n) doubles, 256-byte aligned).  outs[j]
// (E, phi_1, phi_2) may be null.  Synchronises `s` twice (the 1-norm read-back
// and before returning).  Returns an adr_status.
constexpr size_t phi_scratch_doubles(int n) { return (size_t)n * n * 14 + 1; }
int precompute_phi_in(int n, const double* A_dev, double tau, double* const outs[3],
                      double* base, hipStream_t s);
// Its parts: the scaling power for ||tau A||_1, and the polynomial and squarings
// for a given power (enqueued without synchronisation).
int phi_scaling_power(double norm);
int precompute_phi_given(int n, const double* A_dev, double tau, int sq, double* const outs[3],
                         double* base, hipStream_t s);
int check_problem(const adr_problem* p, Geometry& g);
Reaction reaction_of(const adr_problem* p);
hipError_t prepare_lowp(const adr_problem* p, const Geometry& g, const Carve& c, hipStream_t s);

}  // namespace host
}  // namespace adr
