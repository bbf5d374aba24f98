// Host side of libadr.so: argument validation, workspace carving, the launch
// sequence of one ETD2RKds / Lawson2b step, the on-device matrix-function
// precompute, and kernel timing.  Implements include/adr.h.
#include "adr.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"
#include "host_common.h"

using namespace adr;
using namespace adr::host;

namespace adr {
namespace host {
Timing g_timing;
}  // namespace host
}  // namespace adr

namespace {


// ------------------------------------------------------------------ mode products
struct TuckerGroup {
  int count = 0;
  const void* in[kMaxGroup] = {};
  const double* M[kMaxGroup][3] = {};      // FP64 matrices, or FP32 copies (reduced precision)
  SplitPlanes Mp[kMaxGroup][3] = {};        // split-BF16 parts of each matrix
  void* out[kMaxGroup] = {};
  const double* Y[kMaxGroup] = {};
  const float* Z[kMaxGroup] = {};   // reduced precision: FP32 second addend of the last product
  void* t1[kMaxGroup] = {};   // ping buffer
  void* t2[kMaxGroup] = {};   // pong buffer (may be the input when it may be clobbered)
};

// out = alpha * Tucker(in; M_1..M_d) + beta * Y for every tensor of the group, applied
// mu = 1..d.  FP64 uses the general mode product on the natural layout.  The
// reduced precisions chain transposing products (each reads contiguous fibres
// and writes the next direction's fibres contiguous); their intermediates are
// FP32 and the last product writes the FP64 result in the natural layout.
// Optional ETD2RKds stage 2 carried by the last FP64 product (see ModeArgs::Rout).
struct Stage2Fuse {
  void* R[2];
  Reaction r;
};

// The FP64 mode-product arguments of direction mu of run_tucker's chain.
ModeArgs tucker_mode_args(const Geometry& g, const TuckerGroup& tg, int mu, const void* const* W,
                          void* const* out, double alpha, double beta) {
  const bool last = (mu == g.d - 1);
  ModeArgs a{};
  for (int k = 0; k < tg.count; ++k) {
    a.W[k] = W[k];
    a.out[k] = out[k];
    a.M[k] = tg.M[k][mu];
    a.Y[k] = last ? tg.Y[k] : nullptr;
    a.Z[k] = nullptr;
  }
  a.alpha = last ? alpha : 1.0;
  a.beta = last ? beta : 0.0;
  a.gamma = 0.0;
  mode_geometry(g, mu, a.L, a.R);
  a.X = a.L * a.R;
  a.n = g.n[mu];
  a.group = tg.count;
  return a;
}

// The FP64 chain takes directions 1 and 2 in one pass over the (i1, i2) planes
// where a plane fits in LDS (n1 = n2 = 64 or 128) and every tensor and matrix
// of the group is 16-byte aligned.
bool aligned16(const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }
bool tucker_plane12(const Geometry& g, const TuckerGroup& tg, int precision) {
  if (precision != ADR_F64 || g.d < 2 || !mode12_plane_fits(g.n[0], g.n[1])) return false;
  for (int k = 0; k < tg.count; ++k) {
    if (!aligned16(tg.in[k]) || !aligned16(tg.out[k]) || !aligned16(tg.M[k][0]) ||
        !aligned16(tg.M[k][1]) || (tg.Y[k] && !aligned16(tg.Y[k])))
      return false;
    if (g.d == 3 && !aligned16(tg.t1[k])) return false;
  }
  return true;
}

// The tensor that direction mu of run_tucker's chain reads (mu > 0: a ping-pong
// buffer; after the two-direction plane pass, direction 3 reads t1).
const void* tucker_input(const TuckerGroup& tg, int k, int mu, bool plane12 = false) {
  if (plane12 && mu == 2) return tg.t1[k];
  return (mu == 0) ? tg.in[k] : ((mu % 2 == 1) ? tg.t1[k] : tg.t2[k]);
}

hipError_t run_tucker(const Geometry& g, const TuckerGroup& tg, double alpha, double beta,
                      int precision, hipStream_t s, bool last_f32 = false,
                      const Stage2Fuse* fuse = nullptr) {
  const bool plane12 = tucker_plane12(g, tg, precision);
  if (plane12) {
    // directions 1 and 2 in one pass: the whole operator when d = 2, else into t1
    const double* W[kMaxGroup];
    const double* M1[kMaxGroup];
    const double* M2[kMaxGroup];
    double* out[kMaxGroup];
    const double* Y[kMaxGroup];
    const bool whole = g.d == 2;
    if (whole && fuse) return hipErrorInvalidValue;
    for (int k = 0; k < tg.count; ++k) {
      W[k] = static_cast<const double*>(tg.in[k]);
      M1[k] = tg.M[k][0];
      M2[k] = tg.M[k][1];
      out[k] = static_cast<double*>(whole ? tg.out[k] : tg.t1[k]);
      Y[k] = whole ? tg.Y[k] : nullptr;
      if (!W[k] || !out[k] || (const void*)W[k] == (const void*)out[k]) return hipErrorInvalidValue;
    }
    const int planes = g.d == 3 ? g.n[2] : 1;
    hipError_t e = timed(kKindMode, s, [&] {
      return launch_mode12_plane(tg.count, W, M1, M2, out, Y, whole ? alpha : 1.0,
                                 whole ? beta : 0.0, g.n[0], planes, s);
    });
    if (e != hipSuccess || whole) return e;
  }
  for (int mu = plane12 ? 2 : 0; mu < g.d; ++mu) {
    const bool last = (mu == g.d - 1);
    const void* W[kMaxGroup];
    void* out[kMaxGroup];
    for (int k = 0; k < tg.count; ++k) {
      W[k] = tucker_input(tg, k, mu, plane12);
      out[k] = last ? tg.out[k] : ((mu % 2 == 0) ? tg.t1[k] : tg.t2[k]);
      if (!W[k] || !out[k] || W[k] == out[k]) return hipErrorInvalidValue;
    }
    hipError_t e;
    if (precision == ADR_F64) {
      ModeArgs a = tucker_mode_args(g, tg, mu, W, out, alpha, beta);
      if (last && fuse) {
        a.Rout[0] = fuse->R[0];
        a.Rout[1] = fuse->R[1];
        a.react = fuse->r;
      }
      e = timed((last && fuse) ? kKindModeFused : kKindMode, s,
                [&] { return launch_mode_product_f64(a, s); });
    } else {
      const void* Mf[kMaxGroup];
      SplitPlanes Mp[kMaxGroup];
      const double* Y[kMaxGroup];
      const float* Z[kMaxGroup];
      bool with_z = false;
      for (int k = 0; k < tg.count; ++k) {
        Mf[k] = tg.M[k][mu];
        Mp[k] = tg.Mp[k][mu];
        Y[k] = last ? tg.Y[k] : nullptr;
        Z[k] = last ? tg.Z[k] : nullptr;
        with_z = with_z || Z[k] != nullptr;
      }
      const long long X = g.N / g.n[mu];
      e = timed(with_z ? kKindModeFused : kKindMode, s, [&] {
        return launch_tgemm_lowp(precision, W, Mf, Mp, out, Y, tg.count, g.n[mu], X,
                                 last ? alpha : 1.0, last ? beta : 0.0,
                                 (last && !last_f32) ? 1 : 0, s, with_z ? Z : nullptr);
      });
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------------ problem checks
}  // namespace

namespace adr {
namespace host {
static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_problem(const adr_problem* p, Geometry& g) {
  if (!p) return ADR_EINVAL;
  if (p->d < 1 || p->d > ADR_MAX_DIM) return ADR_EINVAL;
  if (p->model < ADR_SCHNAKENBERG || p->model > ADR_DIB) return ADR_EINVAL;
  if (p->scheme != ADR_ETD2RKDS && p->scheme != ADR_LAWSON2B) return ADR_EINVAL;
  if (p->precision < ADR_F64 || p->precision > ADR_BF16X2) return ADR_EINVAL;
  if (p->flags != 0) return ADR_EINVAL;
  if (!finite_pos(p->tau)) return ADR_EINVAL;
  for (int i = 0; i < ADR_MAX_PARAMS; ++i)
    if (!std::isfinite(p->params[i])) return ADR_EINVAL;
  g.d = p->d;
  g.N = 1;
  for (int mu = 0; mu < 3; ++mu) g.n[mu] = 1;
  for (int mu = 0; mu < p->d; ++mu) {
    if (p->n[mu] < 3 || p->n[mu] > 4096) return ADR_EINVAL;
    g.n[mu] = p->n[mu];
    g.N *= p->n[mu];
  }
  if (g.N >= (1LL << 31)) return ADR_EINVAL;
  for (int c = 0; c < 2; ++c)
    for (int mu = 0; mu < p->d; ++mu) {
      if (p->scheme == ADR_ETD2RKDS) {
        if (!p->phi[c][1][mu] || !p->phi[c][2][mu]) return ADR_EINVAL;
        if (!p->band[c][mu] && !p->dense[c][mu]) return ADR_EINVAL;
      } else {
        if (!p->phi[c][0][mu]) return ADR_EINVAL;
      }
    }
  return ADR_OK;
}

Carve carve(const adr_problem* p, const Geometry& g, char* base) {
  Carve c;
  const bool lowp = p->precision != ADR_F64;
  const size_t tb64 = align_up((size_t)g.N * sizeof(double));
  const size_t tbw = align_up((size_t)g.N * (lowp ? sizeof(float) : sizeof(double)));
  size_t off = 0;
  auto take = [&](size_t b) -> void* {
    void* ptr = base ? static_cast<void*>(base + off) : nullptr;
    off += b;
    return ptr;
  };
  if (lowp && p->scheme == ADR_ETD2RKDS) {
    // FP32 increments of the first Tucker operator replace the FP64 C_{n2}
    c.D[0] = static_cast<float*>(take(tbw));
    c.D[1] = static_cast<float*>(take(tbw));
  } else {
    c.U2 = static_cast<double*>(take(tb64));
    c.V2 = static_cast<double*>(take(tb64));
  }
  const int nin = (p->scheme == ADR_LAWSON2B) ? 4 : 2;
  for (int k = 0; k < nin; ++k) c.R[k] = take(tbw);
  // ping buffers of the Tucker chains; the reduced-precision ETD2RKds also
  // writes its second increment D2 there when d = 1 (it cannot overwrite the
  // chain's input R)
  if (g.d >= 2 || (lowp && p->scheme == ADR_ETD2RKDS))
    for (int k = 0; k < nin; ++k) c.T[k] = take(tbw);
  if (lowp) {
    for (int cc = 0; cc < 2; ++cc)
      for (int j = 0; j < 3; ++j)
        for (int mu = 0; mu < g.d; ++mu) {
          const size_t nn = (size_t)g.n[mu] * g.n[mu];
          if (p->precision == ADR_F32) {
            c.phi32[cc][j][mu] = static_cast<float*>(take(align_up(nn * sizeof(float))));
          } else {
            for (int q = 0; q < split_parts(p->precision); ++q)
              c.phip[cc][j][mu][q] = static_cast<unsigned short*>(take(align_up(nn * 2)));
          }
        }
  }
  c.bytes = off;
  return c;
}

Reaction reaction_of(const adr_problem* p) {
  Reaction r{};
  r.model = p->model;
  for (int i = 0; i < ADR_MAX_PARAMS; ++i) r.p[i] = p->params[i];
  return r;
}

// Prepare reduced-precision copies of the small matrices (once per step call).
hipError_t prepare_lowp(const adr_problem* p, const Geometry& g, const Carve& c, hipStream_t s) {
  if (p->precision == ADR_F64) return hipSuccess;
  for (int cc = 0; cc < 2; ++cc)
    for (int j = 0; j < 3; ++j)
      for (int mu = 0; mu < g.d; ++mu) {
        const double* src = p->phi[cc][j][mu];
        if (!src) continue;
        hipError_t e = (p->precision == ADR_F32)
                           ? launch_convert_f64_f32(src, c.phi32[cc][j][mu],
                                                    (size_t)g.n[mu] * g.n[mu], s)
                           : launch_split_bf16(g.n[mu], split_parts(p->precision), src,
                                               c.phip[cc][j][mu], s);
        if (e != hipSuccess) return e;
      }
  return hipSuccess;
}

}  // namespace host
}  // namespace adr

namespace {

// Small matrices of (component, function j, direction mu) in the form the
// step's precision consumes.
void set_phi(TuckerGroup& tg, int k, const adr_problem* p, const Carve& c, int comp, int j, int mu) {
  if (p->precision == ADR_F64) {
    tg.M[k][mu] = p->phi[comp][j][mu];
  } else if (p->precision == ADR_F32) {
    tg.M[k][mu] = reinterpret_cast<const double*>(c.phi32[comp][j][mu]);
  } else {
    for (int q = 0; q < 3; ++q) tg.Mp[k][mu].p[q] = c.phip[comp][j][mu][q];
  }
}

hipError_t step_etd2rkds(const adr_problem* p, const Geometry& g, const Carve& c, double* U,
                         double* V, hipStream_t s) {
  const bool lowp = p->precision != ADR_F64;
  const Reaction r = reaction_of(p);
  StageGeom sg{};
  sg.d = g.d;
  sg.N = g.N;
  for (int mu = 0; mu < 3; ++mu) sg.n[mu] = g.n[mu];
  bool dense_needed = false;
  for (int cc = 0; cc < 2; ++cc)
    for (int mu = 0; mu < g.d; ++mu) {
      sg.band[cc][mu] = p->band[cc][mu];
      if (!p->band[cc][mu]) dense_needed = true;
    }
  if (dense_needed && lowp) return hipErrorNotSupported;
  // stage 1: R^c = K^c C_n + G^c(U_n, V_n)
  hipError_t e = timed(kKindStage, s, [&] {
    return launch_etd_stage1(sg, r, U, V, c.R[0], c.R[1], lowp ? 1 : 0, s);
  });
  if (e != hipSuccess) return e;
  if (dense_needed) {
    // directions without a band: R^c += C x_mu A_mu^c with the dense matrix (FP64 only)
    for (int mu = 0; mu < g.d; ++mu) {
      ModeArgs a{};
      int k = 0;
      for (int cc = 0; cc < 2; ++cc) {
        if (p->band[cc][mu]) continue;
        a.W[k] = cc == 0 ? U : V;
        a.M[k] = p->dense[cc][mu];
        a.out[k] = c.R[cc];
        a.Y[k] = static_cast<const double*>(c.R[cc]);
        ++k;
      }
      if (k == 0) continue;
      a.group = k;
      a.alpha = 1.0;
      a.beta = 1.0;
      mode_geometry(g, mu, a.L, a.R);
      a.X = a.L * a.R;
      a.n = g.n[mu];
      e = timed(kKindMode, s, [&] { return launch_mode_product_f64(a, s); });
      if (e != hipSuccess) return e;
    }
  }
  // C_{n2} = C_n + tau * Tucker(R^c; phi_1)
  TuckerGroup tg;
  tg.count = 2;
  for (int cc = 0; cc < 2; ++cc) {
    tg.in[cc] = c.R[cc];
    tg.t1[cc] = c.T[cc];
    tg.t2[cc] = c.R[cc];
    for (int mu = 0; mu < g.d; ++mu) set_phi(tg, cc, p, c, cc, 1, mu);
  }
  if (lowp) {
    // D1 = tau * Tucker(R1; phi_1) as FP32, the states C_{n2} = C_n + D1 are
    // formed pointwise in FP64 where they are needed
    tg.out[0] = c.D[0];
    tg.out[1] = c.D[1];
    e = run_tucker(g, tg, p->tau, 0.0, p->precision, s, true);
    if (e != hipSuccess) return e;
    e = timed(kKindStage, s, [&] {
      return launch_etd_stage2_inc(g.N, r, U, V, c.D[0], c.D[1], static_cast<float*>(c.R[0]),
                                   static_cast<float*>(c.R[1]), s);
    });
    if (e != hipSuccess) return e;
    // C_{n+1} = (C_n + D1) + D2 with D2 = 2^(d-1) tau * Tucker(R2; phi_2): the last
    // product adds its result to C_n + D1 in FP64 and writes C in place
    for (int cc = 0; cc < 2; ++cc) {
      for (int mu = 0; mu < g.d; ++mu) set_phi(tg, cc, p, c, cc, 2, mu);
      tg.out[cc] = cc == 0 ? static_cast<void*>(U) : static_cast<void*>(V);
      tg.Y[cc] = cc == 0 ? U : V;
      tg.Z[cc] = static_cast<const float*>(c.D[cc]);
    }
    return run_tucker(g, tg, std::ldexp(p->tau, g.d - 1), 1.0, p->precision, s);
  }
  tg.out[0] = c.U2;
  tg.out[1] = c.V2;
  tg.Y[0] = U;
  tg.Y[1] = V;
  // stage 2: R^c = G^c(U_{n2}, V_{n2}) - G^c(U_n, V_n), in the epilogue of the
  // last product when its shape allows (the product then writes R^c into the
  // buffer it does not read: R when d = 2, T when d = 3), else as its own pass
  const int last = g.d - 1;
  Stage2Fuse fuse{};
  bool fused = false;
  const bool plane12 = tucker_plane12(g, tg, p->precision);
  if (g.d >= 2 && !(plane12 && g.d == 2)) {
    const void* W[kMaxGroup];
    void* out[kMaxGroup];
    for (int cc = 0; cc < 2; ++cc) {
      W[cc] = tucker_input(tg, cc, last, plane12);
      out[cc] = tg.out[cc];
      fuse.R[cc] = (W[cc] == c.R[cc]) ? c.T[cc] : c.R[cc];
    }
    fuse.r = r;
    fused = mode_f64_stage2_fusable(tucker_mode_args(g, tg, last, W, out, p->tau, 1.0)) &&
            fuse.R[0] != W[0] && fuse.R[1] != W[1];
  }
  e = run_tucker(g, tg, p->tau, 1.0, p->precision, s, false, fused ? &fuse : nullptr);
  if (e != hipSuccess) return e;
  if (fused) {
    // phi_2 chain from the buffer stage 2 wrote; the other one is its first ping buffer
    for (int cc = 0; cc < 2; ++cc) {
      tg.in[cc] = fuse.R[cc];
      tg.t1[cc] = (fuse.R[cc] == c.R[cc]) ? c.T[cc] : c.R[cc];
      tg.t2[cc] = fuse.R[cc];
    }
  } else {
    e = timed(kKindStage, s, [&] {
      return launch_etd_stage2(g.N, r, U, V, c.U2, c.V2, c.R[0], c.R[1], lowp ? 1 : 0, s);
    });
    if (e != hipSuccess) return e;
  }
  // C_{n+1} = C_{n2} + 2^(d-1) tau * Tucker(R^c; phi_2)
  for (int cc = 0; cc < 2; ++cc)
    for (int mu = 0; mu < g.d; ++mu) set_phi(tg, cc, p, c, cc, 2, mu);
  tg.out[0] = U;
  tg.out[1] = V;
  tg.Y[0] = c.U2;
  tg.Y[1] = c.V2;
  const double scale = std::ldexp(p->tau, g.d - 1);
  return run_tucker(g, tg, scale, 1.0, p->precision, s);
}

hipError_t step_lawson2b(const adr_problem* p, const Geometry& g, const Carve& c, double* U,
                         double* V, hipStream_t s) {
  const bool lowp = p->precision != ADR_F64;
  const Reaction r = reaction_of(p);
  // stage 1: A^c = C + tau G^c,  B^c = C + tau/2 G^c
  hipError_t e = timed(kKindStage, s, [&] {
    return launch_lawson_stage1(g.N, r, p->tau, U, V, c.R[0], c.R[1], c.R[2], c.R[3],
                                lowp ? 1 : 0, s);
  });
  if (e != hipSuccess) return e;
  // C_{n2} = Tucker(A^c; e^{tau A^c}),  C <- Tucker(B^c; e^{tau A^c}) in one grouped pass
  TuckerGroup tg;
  tg.count = 4;
  for (int k = 0; k < 4; ++k) {
    const int cc = k & 1;
    tg.in[k] = c.R[k];
    tg.t1[k] = c.T[k];
    tg.t2[k] = c.R[k];
    for (int mu = 0; mu < g.d; ++mu) set_phi(tg, k, p, c, cc, 0, mu);
  }
  tg.out[0] = c.U2;
  tg.out[1] = c.V2;
  tg.out[2] = U;
  tg.out[3] = V;
  e = run_tucker(g, tg, 1.0, 0.0, p->precision, s);
  if (e != hipSuccess) return e;
  // stage 2: C_{n+1} = Tucker(B^c; e^{tau A^c}) + tau/2 G^c(U_{n2}, V_{n2})
  return timed(kKindStage, s, [&] {
    return launch_lawson_stage2(g.N, r, p->tau, U, V, c.U2, c.V2, s);
  });
}

// Small 2D FP64 ETD2RKds problems with tridiagonal operators run whole steps
// in one cooperative launch (launch_etd_small2d).
bool small2d_step(const adr_problem* p, const Geometry& g) {
  if (p->scheme != ADR_ETD2RKDS || p->precision != ADR_F64 || !small2d_fits(g.d, g.n[0], g.n[1]))
    return false;
  for (int cc = 0; cc < 2; ++cc) {
    for (int mu = 0; mu < 2; ++mu)
      if (!p->band[cc][mu]) return false;
    // the direction-1 matrices are copied into LDS in 16-byte pieces
    for (int j = 1; j <= 2; ++j)
      if (reinterpret_cast<uintptr_t>(p->phi[cc][j][0]) % 16 != 0) return false;
  }
  return true;
}

int do_steps(const adr_problem* p, double* U, double* V, int nsteps, void* work,
             size_t work_bytes, void* stream) {
  Geometry g{};
  int st = check_problem(p, g);
  if (st != ADR_OK) return st;
  if (!U || !V || nsteps < 0) return ADR_EINVAL;
  const Carve need = carve(p, g, nullptr);
  if (!work || work_bytes < need.bytes) return ADR_ENOMEM;
  if (reinterpret_cast<uintptr_t>(work) % kAlign != 0) return ADR_EINVAL;
  if (p->scheme == ADR_ETD2RKDS && p->precision != ADR_F64)
    for (int cc = 0; cc < 2; ++cc)
      for (int mu = 0; mu < p->d; ++mu)
        if (!p->band[cc][mu]) return ADR_ENOTSUP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Carve c = carve(p, g, static_cast<char*>(work));
  if (small2d_step(p, g) && nsteps > 0) {
    // every step in one cooperative launch; the exchange buffers are the
    // stage buffers of the launch-by-launch path, its barrier counter and
    // error flag the first 8 bytes of U2
    Small2dArgs a{};
    a.U = U;
    a.V = V;
    for (int cc = 0; cc < 2; ++cc) {
      for (int op = 0; op < 2; ++op) {
        a.P1[op][cc] = p->phi[cc][1 + op][0];
        a.P2[op][cc] = p->phi[cc][1 + op][1];
      }
      a.band[cc][0] = p->band[cc][0];
      a.band[cc][1] = p->band[cc][1];
      a.Y[0][cc] = static_cast<double*>(c.R[cc]);
      a.Y[1][cc] = static_cast<double*>(c.T[cc]);
    }
    a.r = reaction_of(p);
    a.tau = p->tau;
    a.n2 = g.n[1];
    a.counter = reinterpret_cast<unsigned*>(c.U2);
    a.err = reinterpret_cast<int*>(c.U2) + 1;
    a.spin_limit = small2d_spin_limit();
    const hipError_t e = timed(kKindSteps, s, [&] { return launch_etd_small2d(a, nsteps, s); });
    return e == hipSuccess ? ADR_OK : ADR_EDEVICE;
  }
  hipError_t e = prepare_lowp(p, g, c, s);
  if (e != hipSuccess) return ADR_EDEVICE;
  for (int it = 0; it < nsteps; ++it) {
    e = (p->scheme == ADR_ETD2RKDS) ? step_etd2rkds(p, g, c, U, V, s)
                                    : step_lawson2b(p, g, c, U, V, s);
    if (e == hipErrorNotSupported) return ADR_ENOTSUP;
    if (e != hipSuccess) return ADR_EDEVICE;
  }
  return ADR_OK;
}

// ------------------------------------------------------------------ precompute helpers
hipError_t gemm(int n, const double* A, const double* B, double* C, double alpha, double beta,
                const double* Y, double gamma, const double* Z, hipStream_t s) {
  // C = alpha * A B + beta * Y + gamma * Z  as the mode-1 product of the 2-tensor B by A
  ModeArgs a{};
  a.W[0] = B;
  a.M[0] = A;
  a.out[0] = C;
  a.Y[0] = Y;
  a.Z[0] = Z;
  a.alpha = alpha;
  a.beta = beta;
  a.gamma = gamma;
  a.L = 1;
  a.R = n;
  a.X = n;
  a.n = n;
  a.group = 1;
  return launch_mode_product_f64(a, s);
}

}  // namespace

namespace adr {
namespace host {

// The scaling power of the Taylor step: the smallest s >= 0 with
// ||tau A / 2^s||_1 <= 1.
int phi_scaling_power(double norm) {
  return norm > 1.0 ? (int)std::ceil(std::log2(norm)) : 0;
}

// Degree-18 Taylor polynomials of tau A / 2^sq, then sq modified squarings, in
// `base` (phi_scratch_doubles(n) doubles), results copied to outs[j].  Enqueued
// on `s` without any synchronisation.
int precompute_phi_given(int n, const double* A_dev, double tau, int sq, double* const outs[3],
                         double* base, hipStream_t s) {
  const size_t nn = (size_t)n * n;
  double* Yp[7];
  for (int j = 1; j <= 6; ++j) Yp[j] = base + nn * (j - 1);
  double* Bb = base + nn * 6;
  double* H = base + nn * 7;
  double* cur[3] = {base + nn * 8, base + nn * 9, base + nn * 10};
  double* nxt[3] = {base + nn * 11, base + nn * 12, base + nn * 13};
  const double scale = std::ldexp(tau, -sq);
  hipError_t e = launch_scale_copy((long long)nn, A_dev, scale, Yp[1], s);
  for (int j = 2; j <= 6 && e == hipSuccess; ++j)
    e = gemm(n, Yp[j - 1], Yp[1], Yp[j], 1.0, 0.0, nullptr, 0.0, nullptr, s);
  if (e != hipSuccess) return ADR_EDEVICE;
  // Taylor polynomials of degree 18 of exp, phi_1, phi_2 (coefficients 1/(k+l)!) in
  // Paterson-Stockmeyer form: p = B0 + (B1 + (B2 + c18 Y^6) Y^6) Y^6, Bj = sum_i c_{6j+i} Y^i
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    double coef[19];
    double f = 1.0;
    for (int j = 1; j <= l; ++j) f *= j;  // l!
    for (int k = 0; k <= 18; ++k) {
      coef[k] = 1.0 / f;                  // 1/(k+l)!
      f *= (double)(k + l + 1);
    }
    auto block = [&](int j, double* out, bool add_top) {
      const double* P[8];
      double c[8];
      int cnt = 0;
      for (int i = 1; i <= 5; ++i) {
        P[cnt] = Yp[i];
        c[cnt] = coef[6 * j + i];
        ++cnt;
      }
      if (add_top) {
        P[cnt] = Yp[6];
        c[cnt] = coef[18];
        ++cnt;
      }
      return launch_lincomb(n, cnt, P, c, coef[6 * j], out, s);
    };
    e = block(2, H, true);                                                           // H = B2 + c18 Y^6
    if (e == hipSuccess) e = block(1, Bb, false);                                    // B1
    if (e == hipSuccess) e = gemm(n, H, Yp[6], nxt[l], 1.0, 1.0, Bb, 0.0, nullptr, s);  // H Y^6 + B1
    if (e == hipSuccess) e = block(0, Bb, false);                                    // B0
    if (e == hipSuccess) e = gemm(n, nxt[l], Yp[6], cur[l], 1.0, 1.0, Bb, 0.0, nullptr, s);
  }
  if (e != hipSuccess) return ADR_EDEVICE;
  // modified squaring: e^{2X} = (e^X)^2, phi_1(2X) = (e^X phi_1 + phi_1)/2,
  // phi_2(2X) = (e^X phi_2 + phi_1 + phi_2)/4
  for (int it = 0; it < sq && e == hipSuccess; ++it) {
    e = gemm(n, cur[0], cur[2], nxt[2], 0.25, 0.25, cur[1], 0.25, cur[2], s);
    if (e == hipSuccess) e = gemm(n, cur[0], cur[1], nxt[1], 0.5, 0.5, cur[1], 0.0, nullptr, s);
    if (e == hipSuccess) e = gemm(n, cur[0], cur[0], nxt[0], 1.0, 0.0, nullptr, 0.0, nullptr, s);
    for (int j = 0; j < 3; ++j) std::swap(cur[j], nxt[j]);
  }
  for (int j = 0; j < 3 && e == hipSuccess; ++j)
    if (outs[j]) e = launch_copy_f64(cur[j], outs[j], nn, s);
  if (e != hipSuccess) return ADR_EDEVICE;
  return ADR_OK;
}

// The body of adr_precompute_phi on a caller-chosen scratch: ||tau A||_1 read
// back (one synchronisation), then precompute_phi_given, then a final
// synchronisation.
int precompute_phi_in(int n, const double* A_dev, double tau, double* const outs[3],
                      double* base, hipStream_t s) {
  double* dnorm = base + (size_t)n * n * 14;
  auto fail = [&](int st) {
    (void)hipStreamSynchronize(s);
    return st;
  };
  if (launch_norm1(n, A_dev, tau, dnorm, s) != hipSuccess) return fail(ADR_EDEVICE);
  double norm = 0.0;
  if (hipMemcpyAsync(&norm, dnorm, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
    return fail(ADR_EDEVICE);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(ADR_EDEVICE);
  if (!std::isfinite(norm)) return fail(ADR_ENONFINITE);
  const int st = precompute_phi_given(n, A_dev, tau, phi_scaling_power(norm), outs, base, s);
  if (st != ADR_OK) return fail(st);
  return hipStreamSynchronize(s) == hipSuccess ? ADR_OK : ADR_EDEVICE;
}

}  // namespace host
}  // namespace adr

// ====================================================================== ABI

// scratch of adr_precompute_phi, per device
namespace {
struct PhiScratch {
  void* ptr = nullptr;
  size_t cap = 0;
};
std::mutex g_phi_mu;
std::map<int, PhiScratch> g_phi_scratch;
}  // namespace

extern "C" {

const char* adr_strerror(int status) {
  switch (status) {
    case ADR_OK: return "ok";
    case ADR_EINVAL: return "invalid argument";
    case ADR_ENOMEM: return "workspace too small or allocation failed";
    case ADR_EDEVICE: return "HIP device error";
    case ADR_ENOTSUP: return "unsupported combination";
    case ADR_ENONFINITE: return "non-finite value";
    default: return "unknown status";
  }
}

int adr_version(void) { return 10000; }

int adr_build_1d_ops(int n, double a, double b, double diff, double vel, int bc, double* A,
                     double* band) {
  if (n < 3 || !std::isfinite(a) || !std::isfinite(b) || !(b > a)) return ADR_EINVAL;
  if (!std::isfinite(diff) || !std::isfinite(vel)) return ADR_EINVAL;
  if (bc != ADR_BC_NEUMANN) return ADR_EINVAL;
  if (!A && !band) return ADR_EINVAL;
  const double h = (b - a) / (n - 1);
  const double dif = diff / (h * h);   // diffusion weight
  const double adv = vel / (2.0 * h);  // centred advection weight
  std::vector<double> lo(n, 0.0), di(n, 0.0), up(n, 0.0);
  for (int i = 1; i < n - 1; ++i) {
    lo[i] = dif + adv;   // coefficient of u_{i-1}: diff/h^2 - vel * (-1/(2h))
    di[i] = -2.0 * dif;
    up[i] = dif - adv;   // coefficient of u_{i+1}: diff/h^2 - vel * (1/(2h))
  }
  // Neumann ghost rows: u_{-1} = u_1, u_n = u_{n-2}; the centred advection cancels
  di[0] = -2.0 * dif;
  up[0] = 2.0 * dif;
  di[n - 1] = -2.0 * dif;
  lo[n - 1] = 2.0 * dif;
  if (A) {
    std::memset(A, 0, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) {
      A[i + (size_t)n * i] = di[i];
      if (i > 0) A[i + (size_t)n * (i - 1)] = lo[i];
      if (i < n - 1) A[i + (size_t)n * (i + 1)] = up[i];
    }
  }
  if (band) {
    for (int i = 0; i < n; ++i) {
      band[i] = lo[i];
      band[n + i] = di[i];
      band[2 * n + i] = up[i];
    }
  }
  return ADR_OK;
}

int adr_precompute_phi(int n, const double* A_dev, double tau, double* E_dev, double* P1_dev,
                       double* P2_dev, void* stream) {
  if (n < 1 || n > 4096 || !A_dev || !std::isfinite(tau) || tau == 0.0) return ADR_EINVAL;
  if (!E_dev && !P1_dev && !P2_dev) return ADR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // The scratch is a per-device block that grows and is kept (the call ends
  // with a synchronisation of `s`, so the next call can reuse it).  Freeing
  // it would wait for the whole device, stalling unrelated streams.
  std::lock_guard<std::mutex> lock(g_phi_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ADR_EDEVICE;
  PhiScratch& sc = g_phi_scratch[dev];
  const size_t need = sizeof(double) * phi_scratch_doubles(n);
  if (sc.cap < need) {
    if (sc.ptr) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(sc.ptr);
      sc.ptr = nullptr;
      sc.cap = 0;
    }
    if (hipMalloc(&sc.ptr, need) != hipSuccess) return ADR_ENOMEM;
    sc.cap = need;
  }
  double* outs[3] = {E_dev, P1_dev, P2_dev};
  return precompute_phi_in(n, A_dev, tau, outs, static_cast<double*>(sc.ptr), s);
}

int adr_precompute_phi_batch(int count, const int32_t* n, const double* const* A_dev,
                             const double* tau, double* const* E_dev, double* const* P1_dev,
                             double* const* P2_dev, void* stream) {
  if (count < 1 || count > 4096 || !n || !A_dev || !tau) return ADR_EINVAL;
  int nmax = 0;
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > 4096 || !A_dev[i] || !std::isfinite(tau[i]) || tau[i] == 0.0)
      return ADR_EINVAL;
    if (!(E_dev && E_dev[i]) && !(P1_dev && P1_dev[i]) && !(P2_dev && P2_dev[i])) return ADR_EINVAL;
    nmax = std::max(nmax, (int)n[i]);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_phi_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ADR_EDEVICE;
  PhiScratch& sc = g_phi_scratch[dev];
  // one work area for the matrices in turn (stream order), and the norms after it
  const size_t work = phi_scratch_doubles(nmax);
  const size_t need = sizeof(double) * (work + count);
  if (sc.cap < need) {
    if (sc.ptr) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(sc.ptr);
      sc.ptr = nullptr;
      sc.cap = 0;
    }
    if (hipMalloc(&sc.ptr, need) != hipSuccess) return ADR_ENOMEM;
    sc.cap = need;
  }
  double* base = static_cast<double*>(sc.ptr);
  double* dnorms = base + work;
  auto fail = [&](int st) {
    (void)hipStreamSynchronize(s);
    return st;
  };
  for (int i = 0; i < count; ++i)
    if (launch_norm1(n[i], A_dev[i], tau[i], dnorms + i, s) != hipSuccess) return fail(ADR_EDEVICE);
  std::vector<double> norms(count);
  if (hipMemcpyAsync(norms.data(), dnorms, sizeof(double) * count, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(ADR_EDEVICE);
  for (int i = 0; i < count; ++i)
    if (!std::isfinite(norms[i])) return fail(ADR_ENONFINITE);
  for (int i = 0; i < count; ++i) {
    double* outs[3] = {E_dev ? E_dev[i] : nullptr, P1_dev ? P1_dev[i] : nullptr,
                       P2_dev ? P2_dev[i] : nullptr};
    const int st = precompute_phi_given(n[i], A_dev[i], tau[i], phi_scaling_power(norms[i]), outs,
                                        base, s);
    if (st != ADR_OK) return fail(st);
  }
  return hipStreamSynchronize(s) == hipSuccess ? ADR_OK : ADR_EDEVICE;
}

size_t adr_workspace_bytes(const adr_problem* p) {
  Geometry g{};
  if (check_problem(p, g) != ADR_OK) return 0;
  return carve(p, g, nullptr).bytes;
}

int adr_step(const adr_problem* p, double* U, double* V, void* work, size_t work_bytes,
             void* stream) {
  return do_steps(p, U, V, 1, work, work_bytes, stream);
}

int adr_solve(const adr_problem* p, double* U, double* V, int nsteps, void* work,
              size_t work_bytes, void* stream) {
  return do_steps(p, U, V, nsteps, work, work_bytes, stream);
}

int adr_mode_product(int d, const int32_t* n, int mu, const double* M, const double* W,
                     double* out, double alpha, double beta, const double* Y, void* stream) {
  if (d < 1 || d > ADR_MAX_DIM || !n || mu < 0 || mu >= d || !M || !W || !out) return ADR_EINVAL;
  if (!std::isfinite(alpha) || (Y && !std::isfinite(beta))) return ADR_EINVAL;
  if (out == W) return ADR_EINVAL;
  Geometry g{};
  g.d = d;
  g.N = 1;
  for (int k = 0; k < 3; ++k) g.n[k] = 1;
  for (int k = 0; k < d; ++k) {
    if (n[k] < 1 || n[k] > 1 << 20) return ADR_EINVAL;
    g.n[k] = n[k];
    g.N *= n[k];
  }
  if (g.N >= (1LL << 31) || n[mu] > 4096) return ADR_EINVAL;
  ModeArgs a{};
  a.W[0] = W;
  a.M[0] = M;
  a.out[0] = out;
  a.Y[0] = Y;
  a.alpha = alpha;
  a.beta = Y ? beta : 0.0;
  mode_geometry(g, mu, a.L, a.R);
  a.X = a.L * a.R;
  a.n = n[mu];
  a.group = 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dev_err(timed(kKindMode, s, [&] { return launch_mode_product_f64(a, s); }));
}

size_t adr_tucker_workspace_bytes(int d, const int32_t* n) {
  if (d < 1 || d > ADR_MAX_DIM || !n) return 0;
  long long N = 1;
  for (int k = 0; k < d; ++k) {
    if (n[k] < 1) return 0;
    N *= n[k];
  }
  return 2 * align_up((size_t)N * sizeof(double));
}

int adr_tucker(int d, const int32_t* n, const double* const* M, const double* W, double* out,
               double alpha, double beta, const double* Y, void* work, size_t work_bytes,
               void* stream) {
  if (d < 1 || d > ADR_MAX_DIM || !n || !M || !W || !out || out == W) return ADR_EINVAL;
  if (!std::isfinite(alpha) || (Y && !std::isfinite(beta))) return ADR_EINVAL;
  Geometry g{};
  g.d = d;
  g.N = 1;
  for (int k = 0; k < 3; ++k) g.n[k] = 1;
  for (int k = 0; k < d; ++k) {
    if (n[k] < 1 || n[k] > 4096 || !M[k]) return ADR_EINVAL;
    g.n[k] = n[k];
    g.N *= n[k];
  }
  if (g.N >= (1LL << 31)) return ADR_EINVAL;
  const size_t need = adr_tucker_workspace_bytes(d, n);
  if (d > 1 && (!work || work_bytes < need)) return ADR_ENOMEM;
  TuckerGroup tg;
  tg.count = 1;
  tg.in[0] = W;
  tg.out[0] = out;
  tg.Y[0] = Y;
  if (d > 1) {
    tg.t1[0] = work;
    tg.t2[0] = static_cast<char*>(work) + need / 2;
  }
  for (int k = 0; k < d; ++k) tg.M[0][k] = M[k];
  return dev_err(run_tucker(g, tg, alpha, Y ? beta : 0.0, ADR_F64, static_cast<hipStream_t>(stream)));
}

int adr_device_copy(const double* in, double* out, size_t count, void* stream) {
  if (!in || !out) return ADR_EINVAL;
  if (count == 0) return ADR_OK;
  return dev_err(launch_copy_f64(in, out, count, static_cast<hipStream_t>(stream)));
}

size_t adr_indicators_workspace_bytes(int d, const int32_t* n) {
  if (d < 1 || d > ADR_MAX_DIM || !n) return 0;
  for (int k = 0; k < d; ++k)
    if (n[k] < 1) return 0;
  return align_up(sizeof(double) * 5 * kMaxIndicatorBlocks);
}

int adr_indicators(int d, const int32_t* n, const double* U, const double* V,
                   const double* Uprev, const double* Vprev, double* rec, void* work,
                   size_t work_bytes, void* stream) {
  if (d < 1 || d > ADR_MAX_DIM || !n || !U || !V || !rec) return ADR_EINVAL;
  if ((Uprev == nullptr) != (Vprev == nullptr)) return ADR_EINVAL;
  int nn[3] = {1, 1, 1};
  long long N = 1;
  for (int k = 0; k < d; ++k) {
    if (n[k] < 1) return ADR_EINVAL;
    nn[k] = n[k];
    N *= n[k];
  }
  if (N >= (1LL << 31)) return ADR_EINVAL;
  if (!work || work_bytes < adr_indicators_workspace_bytes(d, n)) return ADR_ENOMEM;
  return dev_err(launch_indicators(d, nn, U, V, Uprev, Vprev, static_cast<double*>(work), rec,
                                   static_cast<hipStream_t>(stream)));
}

size_t adr_monitor_workspace_bytes(const adr_problem* p) {
  Geometry g{};
  if (check_problem(p, g) != ADR_OK) return 0;
  return 2 * align_up((size_t)g.N * sizeof(double)) +
         align_up(sizeof(double) * 5 * kMaxIndicatorBlocks);
}

int adr_solve_monitored(const adr_problem* p, double* U, double* V, int nsteps, int every,
                        double* rec, void* work, size_t work_bytes, void* mwork,
                        size_t mwork_bytes, void* stream) {
  Geometry g{};
  int st = check_problem(p, g);
  if (st != ADR_OK) return st;
  if (!U || !V || !rec || nsteps < 0 || every < 1) return ADR_EINVAL;
  if (!mwork || mwork_bytes < adr_monitor_workspace_bytes(p)) return ADR_ENOMEM;
  if (reinterpret_cast<uintptr_t>(mwork) % kAlign != 0) return ADR_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(mwork);
  const size_t tb = align_up((size_t)g.N * sizeof(double));
  double* Pu = reinterpret_cast<double*>(base);
  double* Pv = reinterpret_cast<double*>(base + tb);
  double* partial = reinterpret_cast<double*>(base + 2 * tb);
  int nn[3] = {g.n[0], g.n[1], g.n[2]};
  const int records = nsteps / every;
  for (int k = 0; k < records; ++k) {
    // every-1 plain steps, then keep C_n, take the recorded step, reduce
    st = do_steps(p, U, V, every - 1, work, work_bytes, stream);
    if (st != ADR_OK) return st;
    if (launch_copy_f64(U, Pu, (size_t)g.N, s) != hipSuccess ||
        launch_copy_f64(V, Pv, (size_t)g.N, s) != hipSuccess)
      return ADR_EDEVICE;
    st = do_steps(p, U, V, 1, work, work_bytes, stream);
    if (st != ADR_OK) return st;
    if (launch_indicators(g.d, nn, U, V, Pu, Pv, partial, rec + 5 * (size_t)k, s) != hipSuccess)
      return ADR_EDEVICE;
  }
  st = do_steps(p, U, V, nsteps - records * every, work, work_bytes, stream);
  if (st != ADR_OK || records == 0) return st;
  // one synchronisation: was any recorded state non-finite?
  std::vector<double> host((size_t)records * 5);
  if (hipMemcpyAsync(host.data(), rec, host.size() * sizeof(double), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return ADR_EDEVICE;
  for (int k = 0; k < records; ++k)
    if (host[5 * (size_t)k + 4] != 0.0) return ADR_ENONFINITE;
  return ADR_OK;
}

int adr_timing_enable(int capacity) {
  if (capacity < 0) return ADR_EINVAL;
  Timing& t = g_timing;
  for (hipEvent_t ev : t.pool) (void)hipEventDestroy(ev);
  t.pool.clear();
  t.recs.clear();
  t.capacity = 0;
  if (capacity == 0) return ADR_OK;
  t.pool.resize(2 * (size_t)capacity);
  for (auto& ev : t.pool)
    if (hipEventCreate(&ev) != hipSuccess) {
      ev = nullptr;
      return ADR_EDEVICE;
    }
  t.capacity = capacity;
  return ADR_OK;
}

int adr_timing_read(int kind, int* launches, double* total_ms) {
  if (!launches || !total_ms || kind < 0 || kind > 4) return ADR_EINVAL;
  Timing& t = g_timing;
  int cnt = 0;
  double tot = 0.0;
  for (const TimingRec& r : t.recs) {
    if (kind != 2 && r.kind != kind) continue;
    hipEvent_t a = t.pool[2 * r.slot], b = t.pool[2 * r.slot + 1];
    if (hipEventSynchronize(b) != hipSuccess) return ADR_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return ADR_EDEVICE;
    ++cnt;
    tot += ms;
  }
  *launches = cnt;
  *total_ms = tot;
  return ADR_OK;
}

}  // extern "C"
