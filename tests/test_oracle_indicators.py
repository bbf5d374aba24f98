"""Pins of the dynamics indicators (Sec. 4): trapezoidal spatial mean on the
node-centred grid, Frobenius norm of the increment, non-finite count."""
import math

import numpy as np
import pytest

import oracle as O


def _nodes(n, a=0.0, b=1.0):
    return a + (b - a) * np.arange(n) / (n - 1)


@pytest.mark.parametrize("shape", [(7,), (5, 9), (4, 6, 3)])
def test_mean_is_exact_for_multilinear_data(shape):
    # the trapezoidal rule integrates functions linear in each coordinate exactly:
    # mean over [0,1]^d of prod_mu (alpha_mu x_mu + beta_mu) = prod_mu (alpha_mu/2 + beta_mu)
    rng = np.random.default_rng(len(shape))
    alpha = rng.uniform(-2, 2, len(shape))
    beta = rng.uniform(-1, 1, len(shape))
    grids = np.meshgrid(*[_nodes(n) for n in shape], indexing="ij")
    U = np.ones(shape)
    for x, a, b in zip(grids, alpha, beta):
        U = U * (a * x + b)
    want = math.prod(a / 2 + b for a, b in zip(alpha, beta))
    assert O.spatial_mean(U) == pytest.approx(want, rel=1e-14, abs=1e-15)


@pytest.mark.parametrize("n", [3, 5, 11, 64])
def test_mean_of_x_squared_has_the_trapezoid_error(n):
    # trapezoidal rule on [0,1]: T(x^2) = 1/3 + h^2/6 (error h^2/12 * (f'(1) - f'(0)));
    # a plain average of the nodes would give (2n-1)/(6(n-1)) instead
    h = 1.0 / (n - 1)
    x = _nodes(n)
    U = np.broadcast_to((x ** 2)[:, None], (n, 4)).copy()
    assert O.spatial_mean(U) == pytest.approx(1.0 / 3.0 + h * h / 6.0, rel=1e-14)
    assert abs(O.spatial_mean(U) - (2 * n - 1) / (6 * (n - 1))) > 1e-4


def test_mean_of_a_constant_and_weights_sum():
    U = np.full((6, 5, 4), 3.25)
    assert O.spatial_mean(U) == 3.25
    assert O.trapezoid_weights((6, 5, 4)).sum() == 5 * 4 * 3


def test_increment_norm_of_a_constant_shift():
    rng = np.random.default_rng(3)
    P = rng.uniform(-1, 1, (9, 8, 7))
    assert O.increment_norm(P + 0.5, P) == pytest.approx(0.5 * math.sqrt(9 * 8 * 7), rel=1e-14)
    assert O.increment_norm(P, P) == 0.0


def test_nonfinite_count():
    U = np.zeros((5, 6))
    V = np.zeros((5, 6))
    U[1, 2] = np.nan
    V[1, 2] = np.inf          # same point: counted once
    V[4, 5] = -np.inf
    P = np.zeros((5, 6))
    P[0, 0] = np.nan
    assert O.nonfinite_count(U, V) == 2
    assert O.indicators(U, V, P, None)[4] == 3
