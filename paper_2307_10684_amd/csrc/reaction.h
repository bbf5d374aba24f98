// Reaction terms G^u, G^v of the models of Sec. 4 (eqs. (12)-(17)), shared by
// the stage kernels and the fused stage-2 epilogue of the FP64 mode product.
#pragma once

#include "common.h"

namespace adr {

// Reaction terms of model M (the constants' order is documented in include/adr.h);
// M = 3 is the zero reaction.  Branch-free for a fixed M, so loops over many
// points stay one basic block.
template <int M>
__device__ __forceinline__ void react_model(const Reaction& r, double u, double v, double& gu,
                                            double& gv) {
  if constexpr (M == 0) {  // Schnakenberg: gamma(a - u + u^2 v), gamma(b - u^2 v)
    const double u2v = u * u * v;
    gu = r.p[0] * (r.p[1] - u + u2v);
    gv = r.p[0] * (r.p[2] - u2v);
  } else if constexpr (M == 1) {  // FitzHugh-Nagumo: rho(u - u^3 - v), rho eps(u - a1 v - a0)
    gu = r.p[0] * (u - u * u * u - v);
    gv = r.p[0] * r.p[1] * (u - r.p[2] * v - r.p[3]);
  } else if constexpr (M == 2) {  // Brusselator: A - (B+1) u + u^2 v,  B u - u^2 v
    const double u2v = u * u * v;
    gu = r.p[0] - (r.p[1] + 1.0) * u + u2v;
    gv = r.p[1] * u - u2v;
  } else if constexpr (M == 4) {  // DIB: rho(a1u(1-v)u - a2u u^3 - a3u(v-a4u)),
                                  //      rho(a1v(1+a2v u)(1-v)(1-a3v(1-v)) - a4v v(1+a5v u)(1+a3v v))
    const double w = 1.0 - v;
    gu = r.p[0] * (r.p[1] * w * u - r.p[2] * u * u * u - r.p[3] * (v - r.p[4]));
    gv = r.p[0] * (r.p[5] * (1.0 + r.p[6] * u) * w * (1.0 - r.p[7] * w) -
                   r.p[8] * v * (1.0 + r.p[9] * u) * (1.0 + r.p[7] * v));
  } else {
    gu = 0.0;
    gv = 0.0;
  }
}

// Reaction terms of the model r.model.
__device__ __forceinline__ void react(const Reaction& r, double u, double v, double& gu,
                                      double& gv) {
  switch (r.model) {
    case 0: react_model<0>(r, u, v, gu, gv); break;
    case 1: react_model<1>(r, u, v, gu, gv); break;
    case 2: react_model<2>(r, u, v, gu, gv); break;
    case 4: react_model<4>(r, u, v, gu, gv); break;
    default: react_model<3>(r, u, v, gu, gv);
  }
}

}  // namespace adr
