"""ETD2RKds, Lawson2b and unsplit ETD2RK steps (oracle, FP64).

* ETD2RKds, Sec. 3 / eq. (11): with C in {U, V} and Phi_l^c = phi_l(tau A_mu^c),

      C_{n2}  = C_n + tau * (sum_mu C_n x_mu A_mu^c + G^c(U_n, V_n)) X_mu Phi_1^c
      C_{n+1} = C_{n2} + 2^(d-1) tau * (G^c(U_{n2}, V_{n2}) - G^c(U_n, V_n)) X_mu Phi_2^c

  where X_mu is the Tucker operator over mu = 1..d.  The factor 2^(d-1) is
  (l!)^(d-1) of the directional splitting eq. (10) for l = 2 (it is 1 for l = 1).
* Lawson2b, Sec. 2 / eq. (7): exp-Tucker operators only, no splitting error.
* ETD2RK, Sec. 2 / eq. (8): the unsplit scheme with dense phi_l(tau K); used
  only on tiny grids to measure what the splitting changes.

The small matrix functions are computed once per step size (Sec. 4, opening
paragraphs: constant tau, precompute, then step).

Parity: pinned by tests/test_oracle_integrators.py (Heun special case for
spatially constant data, single active direction equals unsplit ETD2RK,
d = 1 equals ETD2RK, closed form for g = 0, Lawson2b exact for g = 0, mean
preservation, steady states, observed order 2, axis permutation) and by the
Table 6 weak pin.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

from .matfun import phi_functions
from .models import reaction
from .operators import operator_1d, kron_sum_dense
from .tensor import tucker, kron_sum_action, vec, unvec


@dataclasses.dataclass
class Problem:
    """Semi-discrete two-component system, eq. (2)/(6): C' = K^c C + G^c(U, V)."""

    A: List[List[np.ndarray]]      # A[c][mu], c = 0 (u), 1 (v)
    model: str
    params: Sequence[float]
    tau: float

    @property
    def d(self) -> int:
        return len(self.A[0])

    @property
    def shape(self):
        return tuple(M.shape[0] for M in self.A[0])


def problem_from_workload(w) -> Problem:
    """Build the 1D operators of a ``synth.Workload`` (diffusion + advection)."""
    A = []
    for c in range(2):
        diff = w.diff[c]
        vel = w.vel_u if c == 0 else w.vel_v
        A.append([operator_1d(n, a, b, diff, vel[mu])
                  for mu, (n, (a, b)) in enumerate(zip(w.n, w.domain))])
    return Problem(A=A, model=w.model, params=tuple(w.params), tau=w.tau)


def precompute(p: Problem):
    """E, Phi_1, Phi_2 of tau*A_mu^c for every component and direction.

    Returns mats[c][j][mu] with j = 0 (exp), 1 (phi_1), 2 (phi_2).
    """
    mats = []
    for c in range(2):
        trip = [[], [], []]
        for A in p.A[c]:
            E, P1, P2 = phi_functions(p.tau * A)
            trip[0].append(E)
            trip[1].append(P1)
            trip[2].append(P2)
        mats.append(trip)
    return mats


def etd2rkds_step(U, V, p: Problem, mats, order=None):
    """One step of eq. (11).  ``order``: direction order of the Tucker operators
    (default mu = 1..d; see ``tucker``)."""
    tau, d = p.tau, p.d
    Gu, Gv = reaction(p.model, p.params, U, V)
    Ru = kron_sum_action(U, p.A[0]) + Gu
    Rv = kron_sum_action(V, p.A[1]) + Gv
    U2 = U + tau * tucker(Ru, mats[0][1], order)
    V2 = V + tau * tucker(Rv, mats[1][1], order)
    Gu2, Gv2 = reaction(p.model, p.params, U2, V2)
    c2 = 2.0 ** (d - 1)
    U1 = U2 + c2 * tau * tucker(Gu2 - Gu, mats[0][2], order)
    V1 = V2 + c2 * tau * tucker(Gv2 - Gv, mats[1][2], order)
    return np.asfortranarray(U1), np.asfortranarray(V1)


def lawson2b_step(U, V, p: Problem, mats):
    """One step of eq. (7)."""
    tau = p.tau
    Gu, Gv = reaction(p.model, p.params, U, V)
    U2 = tucker(U + tau * Gu, mats[0][0])
    V2 = tucker(V + tau * Gv, mats[1][0])
    Gu2, Gv2 = reaction(p.model, p.params, U2, V2)
    U1 = tucker(U + 0.5 * tau * Gu, mats[0][0]) + 0.5 * tau * Gu2
    V1 = tucker(V + 0.5 * tau * Gv, mats[1][0]) + 0.5 * tau * Gv2
    return np.asfortranarray(U1), np.asfortranarray(V1)


def dense_phis(p: Problem):
    """Dense K^c and phi_1(tau K^c), phi_2(tau K^c) for the unsplit scheme (tiny grids)."""
    out = []
    for c in range(2):
        K = kron_sum_dense(p.A[c])
        _, P1, P2 = phi_functions(p.tau * K)
        out.append((K, P1, P2))
    return out


def etd2rk_dense_step(U, V, p: Problem, dense):
    """One step of eq. (8) with dense matrices (no directional splitting)."""
    tau, shape = p.tau, U.shape
    u, v = vec(U), vec(V)
    (Ku, P1u, P2u), (Kv, P1v, P2v) = dense
    gu, gv = (vec(x) for x in reaction(p.model, p.params, U, V))
    u2 = u + tau * (P1u @ (Ku @ u + gu))
    v2 = v + tau * (P1v @ (Kv @ v + gv))
    gu2, gv2 = (vec(x) for x in reaction(p.model, p.params, unvec(u2, shape), unvec(v2, shape)))
    u1 = u2 + tau * (P2u @ (gu2 - gu))
    v1 = v2 + tau * (P2v @ (gv2 - gv))
    return unvec(u1, shape), unvec(v1, shape)


def split_phi_dense(As, tau: float, ell: int) -> np.ndarray:
    """(l!)^(d-1) phi_l(tau A_(x)1) ... phi_l(tau A_(x)d) as one dense matrix, eq. (10a)."""
    d = len(As)
    mats = []
    for A in As:
        E, P1, P2 = phi_functions(tau * A)
        mats.append((E, P1, P2)[ell])
    M = np.ones((1, 1))
    for mu in reversed(range(d)):
        M = np.kron(M, mats[mu])
    return (math.factorial(ell) ** (d - 1)) * M


def solve(U0, V0, p: Problem, steps: int, scheme: str = "etd2rkds", mats=None, order=None):
    """Advance (U0, V0) by ``steps`` constant steps of the chosen scheme
    (``order``: Tucker direction order of ETD2RKds, default mu = 1..d)."""
    if mats is None:
        mats = precompute(p)
    U, V = np.asfortranarray(U0, dtype=np.float64), np.asfortranarray(V0, dtype=np.float64)
    for _ in range(steps):
        if scheme == "etd2rkds":
            U, V = etd2rkds_step(U, V, p, mats, order)
        elif scheme == "lawson2b":
            U, V = lawson2b_step(U, V, p, mats)
        else:
            raise KeyError(scheme)
    return U, V
