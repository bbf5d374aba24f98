"""Pointwise reaction terms g^u(u, v), g^v(u, v) of the benchmark models (oracle).

* Schnakenberg, Sec. 4.1 / eq. (12) (also eq. (16) without advection):
  params (gamma, a, b):  g^u = gamma (a - u + u^2 v),  g^v = gamma (b - u^2 v).
* FitzHugh-Nagumo, Secs. 4.2-4.3 / eqs. (13)-(14), written as
  params (rho, eps, a1, a0):  g^u = rho (u - u^3 - v) (= rho(-u(u^2-1) - v)),
  g^v = rho eps (u - a1 v - a0).
* Advective Brusselator, Sec. 4.6 / eq. (17): params (A, B) with A = a_2^u and
  B = a_1^u:  g^u = u^2 v - (B+1) u + A,  g^v = -u^2 v + B u.

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
    if model == "zero":
        return np.zeros_like(U), np.zeros_like(V)
    raise ValueError(f"unknown model {model!r}")
