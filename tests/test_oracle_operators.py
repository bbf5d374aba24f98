"""Pins of the oracle's 1D operators and Kronecker sums against mathematics.

Sec. 4 (opening): second-order centred differences for diffusion and
advection, homogeneous Neumann conditions embedded in tridiagonal A_mu.
Eq. (3): the Kronecker sum K = A_d (+) ... (+) A_1.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("n", [3, 7, 64])
def test_rows_sum_to_zero(n):
    # constants are in the kernel of d^2/dx^2 and d/dx under Neumann conditions
    for M in (O.laplacian_1d(n, 0, 1), O.advection_1d(n, 0, 1),
              O.operator_1d(n, 0, 2, 0.3, 0.7)):
        assert np.abs(M @ np.ones(n)).max() <= 1e-12 * np.abs(M).max()


@pytest.mark.parametrize("n", [5, 33])
def test_trapezoid_weights_annihilate_laplacian(n):
    # Neumann diffusion conserves the trapezoid-rule integral: w^T L = 0
    _, h = O.grid_nodes(n, 0.0, 1.0)
    w = np.full(n, h)
    w[0] = w[-1] = h / 2
    L = O.laplacian_1d(n, 0.0, 1.0)
    assert np.abs(w @ L).max() <= 1e-12 * np.abs(L).max() * h


def test_tridiagonal():
    A = O.operator_1d(9, -1.0, 3.0, 0.2, -0.4)
    i, j = np.nonzero(A)
    assert np.all(np.abs(i - j) <= 1)


def test_second_order_consistency_on_neumann_function():
    # f = cos(pi x) on [0,1] satisfies f'(0) = f'(1) = 0; L f -> f'', C f -> f'
    errs_L, errs_C = [], []
    for n in (17, 33, 65, 129):
        x, _ = O.grid_nodes(n, 0.0, 1.0)
        f = np.cos(math.pi * x)
        errs_L.append(np.abs(O.laplacian_1d(n, 0, 1) @ f + math.pi ** 2 * f).max())
        errs_C.append(np.abs(O.advection_1d(n, 0, 1) @ f + math.pi * np.sin(math.pi * x)).max())
    for errs in (errs_L, errs_C):
        ratios = [errs[k] / errs[k + 1] for k in range(len(errs) - 1)]
        assert all(3.5 < r < 4.5 for r in ratios), ratios


def test_sign_of_advection():
    # A = diff*L - vel*C discretises diff u_xx - vel u_x  (eqs. (16)-(17))
    n = 65
    x, _ = O.grid_nodes(n, 0.0, 1.0)
    f = np.cos(math.pi * x)
    A = O.operator_1d(n, 0.0, 1.0, 0.0, 2.0)
    exact = -2.0 * (-math.pi * np.sin(math.pi * x))
    assert np.abs(A @ f - exact).max() < 1e-2


def test_kron_sum_brute_force():
    rng = np.random.default_rng(1)
    sizes = (3, 2, 4)
    As = [rng.standard_normal((n, n)) for n in sizes]
    K = O.kron_sum_dense(As)
    N = int(np.prod(sizes))
    ref = np.zeros((N, N))
    # linear index i1 + n1*(i2 + n2*i3): the first index is fastest (vec)
    for I in itertools.product(*[range(n) for n in sizes]):
        for J in itertools.product(*[range(n) for n in sizes]):
            r = I[0] + sizes[0] * (I[1] + sizes[1] * I[2])
            c = J[0] + sizes[0] * (J[1] + sizes[1] * J[2])
            val = 0.0
            for mu in range(3):
                if all(I[nu] == J[nu] for nu in range(3) if nu != mu):
                    val += As[mu][I[mu], J[mu]]
            ref[r, c] = val
    assert np.array_equal(K, ref)
