"""Error measures (oracle).

Sec. 4 (opening paragraphs): the error is the 2-norm of the relative
Frobenius errors of U and V at the final time, measured against a reference
run of the same scheme with many more steps.  Read here as
err = sqrt(e_U^2 + e_V^2) with e_C = ||C - C_ref||_F / ||C_ref||_F.  The
observed order between consecutive runs with s_{k-1} < s_k steps is
log(e_{k-1}/e_k) / log(s_k/s_{k-1}) (the "order" columns of Tables 1-6).

The GPU-vs-oracle parity measure is the relative infinity-norm error
||x - y||_inf / ||y||_inf.

Parity: pinned by tests/test_oracle_metrics.py against the orders printed in
Tables 1 and 6 computed from their printed errors.
"""
from __future__ import annotations

import math

import numpy as np


def relative_error(U, V, Uref, Vref) -> float:
    eu = np.linalg.norm(np.ravel(U - Uref)) / np.linalg.norm(np.ravel(Uref))
    ev = np.linalg.norm(np.ravel(V - Vref)) / np.linalg.norm(np.ravel(Vref))
    return float(math.hypot(eu, ev))


def observed_order(steps, errors):
    """Orders between consecutive (steps, error) pairs."""
    return [math.log(errors[k - 1] / errors[k]) / math.log(steps[k] / steps[k - 1])
            for k in range(1, len(steps))]


def rel_inf_error(x, y) -> float:
    x = np.asarray(x, dtype=np.float64).ravel()
    y = np.asarray(y, dtype=np.float64).ravel()
    den = np.abs(y).max()
    if den == 0.0:
        return float(np.abs(x - y).max())
    return float(np.abs(x - y).max() / den)
