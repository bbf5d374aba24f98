"""Dynamics indicators of a run (oracle).

Sec. 4 (opening paragraphs) follows pattern formation through two numbers per
step: the spatial mean of u, an approximation of (1/|Omega|) * integral of
u(t_n, x) over Omega, and the Frobenius norm of the time increment
||U_{n+1} - U_n||_F.  The paper does not say which quadrature discretises the
mean.  Reading: the trapezoidal rule on the node-centred grid, i.e. weights
prod_mu w_mu(i_mu) with w = 1/2 at the two boundary nodes and 1 inside,
divided by their sum prod_mu (n_mu - 1).  (It is also the mean that pure
diffusion with the ghost-point Neumann rows preserves exactly.)

A count of non-finite grid values is kept beside them to detect blow-up.

Parity: pinned by tests/test_oracle_indicators.py (exactness of the
trapezoidal rule on multilinear data, its closed-form error on x^2, constant
increments, injected non-finite values).
"""
from __future__ import annotations

import numpy as np


def trapezoid_weights(shape) -> np.ndarray:
    """Tensor of the trapezoidal weights prod_mu w_mu(i_mu) (each n_mu >= 2)."""
    w = np.ones(tuple(shape))
    for mu, n in enumerate(shape):
        wm = np.ones(n)
        wm[0] = wm[-1] = 0.5
        sh = [1] * len(shape)
        sh[mu] = n
        w = w * wm.reshape(sh)
    return w


def spatial_mean(U: np.ndarray) -> float:
    """<U>: trapezoidal-rule mean of the grid tensor U."""
    w = trapezoid_weights(U.shape)
    return float((w * U).sum() / w.sum())


def increment_norm(U: np.ndarray, Uprev: np.ndarray) -> float:
    """||U - Uprev||_F."""
    return float(np.sqrt(((U - Uprev) ** 2).sum()))


def nonfinite_count(*tensors) -> int:
    """Number of grid points where any of the tensors holds NaN or +-inf."""
    bad = np.zeros(tensors[0].shape, dtype=bool)
    for T in tensors:
        bad |= ~np.isfinite(T)
    return int(bad.sum())


def indicators(U, V, Uprev=None, Vprev=None):
    """(<U>, <V>, ||U - Uprev||_F, ||V - Vprev||_F, non-finite count)."""
    with np.errstate(invalid="ignore", over="ignore"):
        du = increment_norm(U, Uprev) if Uprev is not None else 0.0
        dv = increment_norm(V, Vprev) if Vprev is not None else 0.0
        extra = [T for T in (Uprev, Vprev) if T is not None]
        return (spatial_mean(U), spatial_mean(V), du, dv, nonfinite_count(U, V, *extra))
