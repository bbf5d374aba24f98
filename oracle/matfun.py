"""Small dense matrix functions e^X, phi_1(X), phi_2(X) (oracle, FP64).

Definition, eq. (9): phi_l(X) = int_0^1 theta^(l-1)/(l-1)! e^((1-theta)X) dtheta.

The paper computes these with a quadrature-based routine and a rational
matrix exponential (Sec. 4, opening paragraphs).  The oracle deliberately
uses a different, textbook route so that it shares nothing with the GPU
library: the exponential of the block upper-triangular augmented matrix

        [ X  I  0 ]            [ e^X  phi_1(X)  phi_2(X) ]
    B = [ 0  0  I ],   e^B  =  [  0      I         I     ]
        [ 0  0  0 ]            [  0      0         I     ]

(the first block row follows from integrating e^{tB} block by block and is
the identity behind eq. (9) for l = 1, 2), with e^B computed by a truncated
Taylor series after scaling B by 2^-s so that ||B/2^s||_1 <= 1/2, then s
squarings.

Parity: pinned by tests/test_oracle_matfun.py (scipy's Pade expm, the
recurrences X phi_1 = e^X - I and X phi_2 = phi_1 - I, scalar closed forms on
diagonal matrices, phi_l(0) = I/l!, eigen-decomposition of symmetric X).
"""
from __future__ import annotations

import math

import numpy as np


def expm_taylor(B: np.ndarray, theta: float = 0.5, tol: float = 1e-18,
                max_terms: int = 60) -> np.ndarray:
    """e^B by scaling (||B/2^s||_1 <= theta), Taylor series, and s squarings."""
    B = np.asarray(B, dtype=np.float64)
    norm1 = float(np.abs(B).sum(axis=0).max()) if B.size else 0.0
    s = 0
    if norm1 > theta:
        s = int(math.ceil(math.log2(norm1 / theta)))
    Y = B / (2.0 ** s)
    n = B.shape[0]
    T = np.eye(n)
    term = np.eye(n)
    for k in range(1, max_terms + 1):
        term = term @ Y / k
        T = T + term
        if np.abs(term).max() <= tol * max(np.abs(T).max(), 1e-300):
            break
    for _ in range(s):
        T = T @ T
    return T


def phi_functions(X: np.ndarray):
    """Return (e^X, phi_1(X), phi_2(X)) from the exponential of the augmented matrix."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    I = np.eye(n)
    Z = np.zeros((n, n))
    B = np.block([[X, I, Z],
                  [Z, Z, I],
                  [Z, Z, Z]])
    EB = expm_taylor(B)
    return EB[:n, :n].copy(), EB[:n, n:2 * n].copy(), EB[:n, 2 * n:].copy()


def phi_scalar(ell: int, z: float) -> float:
    """Scalar phi_l(z) = sum_k z^k / (k+l)!  (series for small |z|, closed form otherwise)."""
    if ell == 0:
        return math.exp(z)
    if abs(z) < 0.5:
        acc, term, k = 0.0, 1.0 / math.factorial(ell), 0
        while abs(term) > 1e-20:
            acc += term
            k += 1
            term = term * z / (k + ell)
        return acc
    # phi_l(z) = (phi_{l-1}(z) - 1/(l-1)!) / z
    return (phi_scalar(ell - 1, z) - 1.0 / math.factorial(ell - 1)) / z
