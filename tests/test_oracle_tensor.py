"""Pins of the oracle's mu-mode product, Tucker operator and Kronecker-sum action (Sec. 2)."""
import itertools

import numpy as np
import pytest

import oracle as O


def _loops_mode_product(W, M, mu):
    out = np.zeros(W.shape)
    for idx in itertools.product(*[range(n) for n in W.shape]):
        acc = 0.0
        for k in range(W.shape[mu]):
            src = list(idx)
            src[mu] = k
            acc += M[idx[mu], k] * W[tuple(src)]
        out[idx] = acc
    return out


@pytest.mark.parametrize("shape", [(5,), (3, 4), (3, 4, 5), (2, 3, 2, 3)])
def test_mode_product_against_loops(shape):
    rng = np.random.default_rng(len(shape))
    W = rng.standard_normal(shape)
    for mu, n in enumerate(shape):
        M = rng.standard_normal((n, n))
        assert np.allclose(O.mode_product(W, M, mu), _loops_mode_product(W, M, mu),
                           rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("shape", [(4, 3), (3, 5, 4), (2, 3, 4, 2)])
def test_tucker_is_kronecker_product_on_vec(shape):
    # vec(W x_1 M_1 ... x_d M_d) = (M_d (x) ... (x) M_1) vec(W)   (eq. (5) with general M_mu)
    rng = np.random.default_rng(5)
    W = np.asfortranarray(rng.standard_normal(shape))
    Ms = [rng.standard_normal((n, n)) for n in shape]
    big = np.ones((1, 1))
    for M in reversed(Ms):
        big = np.kron(big, M)
    lhs = O.vec(O.tucker(W, Ms))
    rhs = big @ W.reshape(-1, order="F")
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


def test_two_dimensional_form():
    # 2D: e^{tau K} w = vec(e^{tau A_1} W (e^{tau A_2})^T), Sec. 2 -- here with any M_1, M_2
    rng = np.random.default_rng(9)
    W = rng.standard_normal((6, 4))
    M1, M2 = rng.standard_normal((6, 6)), rng.standard_normal((4, 4))
    assert np.allclose(O.tucker(W, [M1, M2]), M1 @ W @ M2.T, rtol=1e-14, atol=1e-14)


def test_mode_products_commute():
    rng = np.random.default_rng(2)
    W = rng.standard_normal((3, 4, 5))
    Ms = [rng.standard_normal((n, n)) for n in W.shape]
    a = O.mode_product(O.mode_product(W, Ms[0], 0), Ms[2], 2)
    b = O.mode_product(O.mode_product(W, Ms[2], 2), Ms[0], 0)
    assert np.allclose(a, b, rtol=1e-14, atol=1e-14)


def test_tucker_any_direction_order():
    # every order of the d products gives (M_d x ... x M_1) vec(W) (numpy.kron form)
    import itertools
    rng = np.random.default_rng(3)
    W = np.asfortranarray(rng.standard_normal((3, 4, 5)))
    Ms = [rng.standard_normal((n, n)) for n in W.shape]
    big = np.kron(np.kron(Ms[2], Ms[1]), Ms[0])
    rhs = big @ W.reshape(-1, order="F")
    for order in itertools.permutations(range(3)):
        lhs = O.vec(O.tucker(W, Ms, order))
        assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max(), order


def test_kron_sum_action_matches_dense():
    # K vec(W) = vec(sum_mu W x_mu A_mu), eq. (6); K from the brute-force-pinned kron_sum_dense
    rng = np.random.default_rng(4)
    shape = (4, 3, 5)
    As = [rng.standard_normal((n, n)) for n in shape]
    W = np.asfortranarray(rng.standard_normal(shape))
    K = O.kron_sum_dense(As)
    assert np.allclose(O.vec(O.kron_sum_action(W, As)), K @ O.vec(W), rtol=1e-13, atol=1e-13)


def test_vec_is_first_index_fastest():
    W = np.arange(24.0).reshape((2, 3, 4), order="F")
    assert np.array_equal(O.vec(W), np.arange(24.0))
    assert W[1, 0, 0] == 1.0 and W[0, 1, 0] == 2.0 and W[0, 0, 1] == 6.0
