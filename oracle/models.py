"""Pointwise reaction terms g^u(u, v), g^v(u, v) of the benchmark models (oracle).

* Schnakenberg, Sec. 4.1 / eq. (12) (also eq. (16) without advection):
  params (gamma, a, b):  g^u = gamma (a - u + u^2 v),  g^v = gamma (b - u^2 v).
* FitzHugh-Nagumo, Secs. 4.2-4.3 / eqs. (13)-(14), written as
  params (rho, eps, a1, a0):  g^u = rho (u - u^3 - v) (= rho(-u(u^2-1) - v)),
  g^v = rho eps (u - a1 v - a0).
* Advective Brusselator, Sec. 4.6 / eq. (17): params (A, B) with A = a_2^u and
  B = a_1^u:  g^u = u^2 v - (B+1) u + A,  g^v = -u^2 v + B u.
* Morpho-chemical DIB model, Sec. 4.4 / eq. (15): params
  (rho, a1u, a2u, a3u, a4u, a1v, a2v, a3v, a4v, a5v):
  g^u = rho (a1u (1 - v) u - a2u u^3 - a3u (v - a4u)),
  g^v = rho (a1v (1 + a2v u)(1 - v)(1 - a3v (1 - v)) - a4v v (1 + a5v u)(1 + a3v v)).

The reaction term holds every non-diffusive, non-advective term of the
model, the linear ones included; the matrices K^u, K^v hold only diffusion
and advection (eq. (2)).

Parity: pinned by tests/test_oracle_models.py (equilibria, hand-evaluated
values at fixed points).
"""
from __future__ import annotations

import numpy as np


def reaction(model: str, params, U: np.ndarray, V: np.ndarray):
    """Return (G^u, G^v) evaluated pointwise on the grid tensors U, V."""
    if model == "schnakenberg":
        gamma, a, b = params
        u2v = U * U * V
        return gamma * (a - U + u2v), gamma * (b - u2v)
    if model == "fhn":
        rho, eps, a1, a0 = params
        return rho * (U - U ** 3 - V), rho * eps * (U - a1 * V - a0)
    if model == "brusselator":
        A, B = params
        u2v = U * U * V
        return u2v - (B + 1.0) * U + A, -u2v + B * U
    if model == "dib":
        rho, a1u, a2u, a3u, a4u, a1v, a2v, a3v, a4v, a5v = params
        gu = rho * (a1u * (1.0 - V) * U - a2u * U ** 3 - a3u * (V - a4u))
        gv = rho * (a1v * (1.0 + a2v * U) * (1.0 - V) * (1.0 - a3v * (1.0 - V))
                    - a4v * V * (1.0 + a5v * U) * (1.0 + a3v * V))
        return gu, gv
    if model == "zero":
        return np.zeros_like(U), np.zeros_like(V)
    raise ValueError(f"unknown model {model!r}")
