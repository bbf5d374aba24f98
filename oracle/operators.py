"""1D finite-difference operators and dense Kronecker sums (oracle, FP64).

Sec. 4 (opening paragraphs): every model is discretised by second-order
centred finite differences for diffusion *and* advection, with the
homogeneous Neumann conditions of eq. (1) embedded in the matrices, giving
tridiagonal n x n matrices A_mu.  The paper does not print the boundary rows;
the reading used here is the node-centred ghost-point one: nodes
x_i = a + i h with h = (b-a)/(n-1), and the ghost value u_{-1} = u_1
(resp. u_n = u_{n-2}) imposed by du/dx = 0 at the end points.  With it the
diffusion boundary rows become (-2, 2)/h^2 and (2, -2)/h^2, and the centred
advection difference vanishes on the boundary rows.

Parity: pinned by tests/test_oracle_operators.py (row sums, trapezoid
conservation, second-order consistency on cos(pi x), Kronecker structure).
"""
from __future__ import annotations

import numpy as np


def grid_nodes(n: int, a: float, b: float):
    """Node-centred grid x_i = a + i*h, h = (b-a)/(n-1)."""
    if n < 3:
        raise ValueError("need n >= 3 grid points")
    h = (b - a) / (n - 1)
    return a + h * np.arange(n, dtype=np.float64), h


def laplacian_1d(n: int, a: float, b: float) -> np.ndarray:
    """Second-order centred d^2/dx^2 with homogeneous Neumann ghost rows."""
    _, h = grid_nodes(n, a, b)
    L = np.zeros((n, n))
    for i in range(1, n - 1):
        L[i, i - 1] = 1.0
        L[i, i] = -2.0
        L[i, i + 1] = 1.0
    # ghost point u_{-1} = u_1: (u_1 - 2u_0 + u_1)/h^2
    L[0, 0] = -2.0
    L[0, 1] = 2.0
    # ghost point u_n = u_{n-2}
    L[n - 1, n - 1] = -2.0
    L[n - 1, n - 2] = 2.0
    return L / (h * h)


def advection_1d(n: int, a: float, b: float) -> np.ndarray:
    """Second-order centred d/dx; boundary rows vanish under the ghost reflection."""
    _, h = grid_nodes(n, a, b)
    C = np.zeros((n, n))
    for i in range(1, n - 1):
        C[i, i - 1] = -1.0
        C[i, i + 1] = 1.0
    return C / (2.0 * h)


def operator_1d(n: int, a: float, b: float, diff: float, vel: float) -> np.ndarray:
    """A = diff * d^2/dx^2 - vel * d/dx  (one direction of K in eq. (2))."""
    return diff * laplacian_1d(n, a, b) - vel * advection_1d(n, a, b)


def kron_sum_dense(As) -> np.ndarray:
    """K = A_d (+) ... (+) A_1 = sum_mu I_d x ... x A_mu x ... x I_1, eq. (3).

    ``As[0]`` is A_1 (the fastest index).  Only for tiny grids.
    """
    d = len(As)
    sizes = [A.shape[0] for A in As]
    N = int(np.prod(sizes))
    K = np.zeros((N, N))
    for mu in range(d):
        # Kronecker factors from the slowest direction (d) down to 1
        term = np.ones((1, 1))
        for nu in reversed(range(d)):
            term = np.kron(term, As[nu] if nu == mu else np.eye(sizes[nu]))
        K += term
    return K
