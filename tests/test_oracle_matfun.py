"""Pins of the oracle's e^X, phi_1(X), phi_2(X) (eq. (9)) against independent mathematics."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O


def _phi1(z):
    return np.where(z == 0, 1.0, np.expm1(z) / np.where(z == 0, 1.0, z))


def _phi2(z):
    zz = np.where(z == 0, 1.0, z)
    return np.where(np.abs(z) < 1e-3, 0.5 + z / 6 + z * z / 24, (np.expm1(zz) - zz) / (zz * zz))


@pytest.mark.parametrize("scale", [0.1, 3.0, 40.0])
def test_expm_matches_scipy_pade(scale):
    rng = np.random.default_rng(7)
    X = rng.standard_normal((12, 12))
    X = scale * X / np.abs(X).sum(axis=0).max() - scale * np.eye(12)
    ref = sla.expm(X)
    got = O.expm_taylor(X)
    assert np.abs(got - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300) + 1e-300


@pytest.mark.parametrize("case", ["diffusion", "advection", "random"])
def test_phi_recurrences(case):
    n = 30
    if case == "diffusion":
        X = 1e-3 * O.operator_1d(n, 0, 1, 1.0, 0.0) * 0.2
    elif case == "advection":
        X = 5e-3 * O.operator_1d(n, 0, 1, 5e-3, 0.1)
    else:
        X = np.random.default_rng(3).standard_normal((n, n))
    E, P1, P2 = O.phi_functions(X)
    I = np.eye(n)
    scale = max(1.0, np.abs(X).max())
    assert np.abs(X @ P1 - (E - I)).max() <= 1e-13 * scale
    assert np.abs(X @ P2 - (P1 - I)).max() <= 1e-13 * scale


def test_phi_of_zero():
    E, P1, P2 = O.phi_functions(np.zeros((5, 5)))
    assert np.array_equal(E, np.eye(5))
    assert np.array_equal(P1, np.eye(5))
    assert np.allclose(P2, 0.5 * np.eye(5), atol=1e-17, rtol=0)


def test_diagonal_closed_forms():
    z = np.array([-1500.0, -30.0, -1.0, -1e-4, 0.0, 1e-5, 0.5, 2.0])
    E, P1, P2 = O.phi_functions(np.diag(z))
    # s squarings of the scaled Taylor value amplify its relative rounding
    # error up to 2^s times; the scaling is set by the largest |z| (+1 for
    # the identity blocks of the augmented matrix)
    s = math.ceil(math.log2((np.abs(z).max() + 1.0) / 0.5))
    tol = 2.0 ** (s + 1) * np.finfo(float).eps
    for M, ref in ((E, np.exp(z)), (P1, _phi1(z)), (P2, _phi2(z))):
        assert np.all(np.abs(np.diag(M) - ref) <= tol * np.abs(ref) + 1e-300)
        assert np.abs(M - np.diag(np.diag(M))).max() == 0.0


def test_phi_scalar_closed_forms():
    for z in (-200.0, -3.0, -0.2, 0.0, 0.3, 1.5):
        assert abs(O.phi_scalar(1, z) - float(_phi1(np.array(z)))) <= 1e-15
        assert abs(O.phi_scalar(2, z) - float(_phi2(np.array(z)))) <= 1e-15 * 0.5 + 1e-17


def test_symmetric_eigendecomposition():
    # symmetric A: phi_l(A) = Q phi_l(Lambda) Q^T
    n = 40
    L = O.laplacian_1d(n, 0, 1)
    # D^{1/2} L D^{-1/2} is symmetric for the trapezoid weights D
    w = np.ones(n); w[0] = w[-1] = 0.5
    S = np.diag(np.sqrt(w)) @ L @ np.diag(1 / np.sqrt(w))
    X = 2e-3 * (S + S.T) / 2
    lam, Q = np.linalg.eigh(X)
    E, P1, P2 = O.phi_functions(X)
    for M, f in ((E, np.exp(lam)), (P1, _phi1(lam)), (P2, _phi2(lam))):
        ref = (Q * f) @ Q.T
        assert np.abs(M - ref).max() <= 1e-13 * np.abs(ref).max()


def test_integral_definition_by_quadrature():
    # eq. (9) evaluated with 60-point Gauss-Legendre and scipy's expm at each node
    rng = np.random.default_rng(11)
    X = rng.standard_normal((8, 8)) * 0.7
    xs, ws = np.polynomial.legendre.leggauss(60)
    th, wt = 0.5 * (xs + 1), 0.5 * ws
    P1 = sum(w * sla.expm((1 - t) * X) for t, w in zip(th, wt))
    P2 = sum(w * t * sla.expm((1 - t) * X) for t, w in zip(th, wt))
    _, Q1, Q2 = O.phi_functions(X)
    assert np.abs(Q1 - P1).max() <= 1e-13 * np.abs(P1).max()
    assert np.abs(Q2 - P2).max() <= 1e-13 * np.abs(P2).max()


@pytest.mark.parametrize("n,tau,diff,vel", [(64, 1e-3, 10.0, 0.0),      # 2D Schnakenberg v
                                            (128, 1e-3, 4.0, 0.0),      # 3D FHN v
                                            (256, 5e-3, 5e-3, 0.1)])    # 3D Brusselator v
def test_benchmark_operators_against_scipy_augmented(n, tau, diff, vel):
    X = tau * O.operator_1d(n, 0, 1, diff, vel)
    I, Z = np.eye(n), np.zeros((n, n))
    B = np.block([[X, I, Z], [Z, Z, I], [Z, Z, Z]])
    ref = sla.expm(B)
    E, P1, P2 = O.phi_functions(X)
    for M, R in ((E, ref[:n, :n]), (P1, ref[:n, n:2 * n]), (P2, ref[:n, 2 * n:])):
        assert np.abs(M - R).max() <= 1e-12 * np.abs(R).max()
