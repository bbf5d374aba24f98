"""Pins of the oracle's ETD2RKds (eq. (11)) and Lawson2b (eq. (7)) steps.

None of these compares the oracle with itself: the references are scipy's
Pade exponential of the assembled N x N matrix K (a library routine the
oracle never calls), eigen-decompositions with scalar closed forms, a scalar
Heun integrator, exact conservation laws and permutation symmetry.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import synth as S


def _tiny_problem(shape, model="zero", params=(), tau=0.01, diff=(0.3, 0.7),
                  vel=(0.4, -0.2, 0.1), domain=(0.0, 1.0)):
    A = [[O.operator_1d(n, *domain, diff[c], vel[mu] * (1 + c)) for mu, n in enumerate(shape)]
         for c in range(2)]
    return O.Problem(A=A, model=model, params=params, tau=tau)


def _dense_phi(K, tau):
    """phi_0, phi_1, phi_2 of tau*K from scipy's expm of the augmented matrix."""
    N = K.shape[0]
    I, Z = np.eye(N), np.zeros((N, N))
    B = np.block([[tau * K, I, Z], [Z, Z, I], [Z, Z, Z]])
    EB = sla.expm(B)
    return EB[:N, :N], EB[:N, N:2 * N], EB[:N, 2 * N:]


def _phi1(z):
    z = np.asarray(z, dtype=complex)
    small = np.abs(z) < 1e-8
    zs = np.where(small, 1.0, z)
    return np.where(small, 1.0 + z / 2, np.expm1(zs) / zs)


# ---------------------------------------------------------------- Kronecker identity

@pytest.mark.parametrize("shape", [(4, 5), (3, 4, 5)])
def test_kronecker_sum_exponential_identity(shape):
    # e^{tau K} = e^{tau A_d} (x) ... (x) e^{tau A_1}  (eq. (5)), K assembled densely
    p = _tiny_problem(shape, tau=0.05)
    mats = O.precompute(p)
    for c in range(2):
        K = O.kron_sum_dense(p.A[c])
        ref = sla.expm(p.tau * K)
        big = np.ones((1, 1))
        for E in reversed(mats[c][0]):
            big = np.kron(big, E)
        assert np.abs(big - ref).max() <= 1e-13 * np.abs(ref).max()
        W = np.asfortranarray(np.random.default_rng(c).standard_normal(shape))
        got = O.vec(O.tucker(W, mats[c][0]))
        assert np.abs(got - ref @ O.vec(W)).max() <= 1e-13 * np.abs(ref @ O.vec(W)).max()


# ---------------------------------------------------------------- g = 0

@pytest.mark.parametrize("shape", [(5, 4), (4, 3, 5)])
def test_lawson2b_exact_for_zero_reaction(shape):
    p = _tiny_problem(shape, tau=0.03)
    mats = O.precompute(p)
    U = np.asfortranarray(np.random.default_rng(0).standard_normal(shape))
    V = np.asfortranarray(np.random.default_rng(1).standard_normal(shape))
    U1, V1 = O.lawson2b_step(U, V, p, mats)
    for C, C1, c in ((U, U1, 0), (V, V1, 1)):
        ref = sla.expm(p.tau * O.kron_sum_dense(p.A[c])) @ O.vec(C)
        assert np.abs(O.vec(C1) - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("shape", [(6, 5), (4, 5, 3)])
def test_etd2rkds_zero_reaction_closed_form(shape):
    # With g = 0, eq. (11) is C_{n+1} = C_n + tau * Tucker(K C_n; phi_1).  In the
    # eigenbasis of each A_mu this is the scalar map r = 1 + (sum z_mu) prod phi_1(z_mu).
    p = _tiny_problem(shape, tau=0.02)
    mats = O.precompute(p)
    rng = np.random.default_rng(3)
    U = np.asfortranarray(rng.standard_normal(shape))
    V = np.asfortranarray(rng.standard_normal(shape))
    U1, V1 = O.etd2rkds_step(U, V, p, mats)
    for C, C1, c in ((U, U1, 0), (V, V1, 1)):
        lams, Ss, Sis = [], [], []
        for A in p.A[c]:
            lam, Sm = np.linalg.eig(p.tau * A)
            lams.append(lam); Ss.append(Sm); Sis.append(np.linalg.inv(Sm))
        Wt = C.astype(complex)
        for mu, Si in enumerate(Sis):
            Wt = np.moveaxis(np.tensordot(Si, Wt, axes=([1], [mu])), 0, mu)
        grids = np.meshgrid(*lams, indexing="ij")
        zsum = sum(grids)
        prod = np.ones(shape, dtype=complex)
        for g in grids:
            prod = prod * _phi1(g)
        Wt = (1.0 + zsum * prod) * Wt
        for mu, Sm in enumerate(Ss):
            Wt = np.moveaxis(np.tensordot(Sm, Wt, axes=([1], [mu])), 0, mu)
        assert np.abs(Wt.imag).max() < 1e-10
        assert np.abs(C1 - Wt.real).max() <= 1e-12 * np.abs(C).max()


def test_etd2rkds_zero_reaction_local_error_is_third_order():
    # the splitting (10a) makes eq. (11) O(tau^3) locally away from e^{tau K}
    shape = (6, 5)
    rng = np.random.default_rng(8)
    U = np.asfortranarray(rng.standard_normal(shape))
    errs = []
    for tau in (0.08, 0.04, 0.02, 0.01):
        p = _tiny_problem(shape, tau=tau, diff=(0.01, 0.02), vel=(0.3, 0.2, 0.1))
        U1, _ = O.etd2rkds_step(U, U, p, O.precompute(p))
        ref = sla.expm(tau * O.kron_sum_dense(p.A[0])) @ O.vec(U)
        errs.append(np.abs(O.vec(U1) - ref).max())
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    assert all(7.0 < r < 9.0 for r in ratios), ratios


@pytest.mark.parametrize("ell", [1, 2])
def test_directional_split_factor(ell):
    # eq. (10a): phi_l(tau K) w = (l!)^(d-1) phi_l(tau A_(x)1)...phi_l(tau A_(x)d) w + O(tau^2)
    shape = (5, 4, 3)
    A = [O.operator_1d(n, 0, 1, 0.01, 0.2) for n in shape]
    K = O.kron_sum_dense(A)
    w = np.random.default_rng(1).standard_normal(K.shape[0])
    errs = []
    for tau in (0.04, 0.02, 0.01, 0.005):
        ref = _dense_phi(K, tau)[ell] @ w
        got = O.split_phi_dense(A, tau, ell) @ w
        errs.append(np.abs(got - ref).max())
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    assert all(3.5 < r < 4.5 for r in ratios), ratios


# ---------------------------------------------------------------- reductions to unsplit ETD2RK

def test_single_active_direction_equals_unsplit_etd2rk():
    # with A_mu = 0 except mu = 2, phi_l(0) = I/l! and the split is exact
    shape = (4, 5, 3)
    p = _tiny_problem(shape, model="schnakenberg", params=(200.0, 0.1, 0.9), tau=2e-3)
    for c in range(2):
        p.A[c][0] = np.zeros_like(p.A[c][0])
        p.A[c][2] = np.zeros_like(p.A[c][2])
    rng = np.random.default_rng(5)
    U = np.asfortranarray(1.0 + 0.01 * rng.standard_normal(shape))
    V = np.asfortranarray(0.9 + 0.01 * rng.standard_normal(shape))
    U1, V1 = O.etd2rkds_step(U, V, p, O.precompute(p))
    dense = []
    for c in range(2):
        K = O.kron_sum_dense(p.A[c])
        _, P1, P2 = _dense_phi(K, p.tau)
        dense.append((K, P1, P2))
    R1, R2 = O.etd2rk_dense_step(U, V, p, dense)
    assert np.abs(U1 - R1).max() <= 1e-13 and np.abs(V1 - R2).max() <= 1e-13


def test_one_dimension_equals_unsplit_etd2rk():
    p = _tiny_problem((9,), model="brusselator", params=(1.0, 3.0), tau=5e-3)
    rng = np.random.default_rng(6)
    U = np.asfortranarray(1.0 + 0.1 * rng.standard_normal(9))
    V = np.asfortranarray(3.0 + 0.1 * rng.standard_normal(9))
    U1, V1 = O.etd2rkds_step(U, V, p, O.precompute(p))
    dense = [(p.A[c][0],) + _dense_phi(p.A[c][0], p.tau)[1:] for c in range(2)]
    R1, R2 = O.etd2rk_dense_step(U, V, p, dense)
    assert np.abs(U1 - R1).max() <= 1e-14 * 4 and np.abs(V1 - R2).max() <= 1e-14 * 4


@pytest.mark.parametrize("d", [1, 2, 3])
def test_constant_data_reduces_to_heun(d):
    # A_mu 1 = 0 gives phi_l(tau A) 1 = 1/l!, so one step of eq. (11) on spatially
    # constant data is Heun's method on u' = g(u, v); this pins the 2^(d-1) factor
    shape = (5, 4, 6)[:d]
    params = (200.0, 0.1, 0.9)
    p = _tiny_problem(shape, model="schnakenberg", params=params, tau=1e-3)
    u0, v0 = 0.7, 1.3
    U = np.full(shape, u0, order="F"); V = np.full(shape, v0, order="F")
    U1, V1 = O.etd2rkds_step(U, V, p, O.precompute(p))
    g, a, b = params
    f = lambda u, v: (g * (a - u + u * u * v), g * (b - u * u * v))
    k1 = f(u0, v0)
    u2, v2 = u0 + p.tau * k1[0], v0 + p.tau * k1[1]
    k2 = f(u2, v2)
    uh, vh = u0 + p.tau / 2 * (k1[0] + k2[0]), v0 + p.tau / 2 * (k1[1] + k2[1])
    assert np.abs(U1 - uh).max() <= 1e-13 and np.abs(V1 - vh).max() <= 1e-13


# ---------------------------------------------------------------- conservation / fixed points

@pytest.mark.parametrize("scheme", ["etd2rkds", "lawson2b"])
def test_pure_diffusion_preserves_trapezoid_mean(scheme):
    # Neumann diffusion with g = 0 conserves the trapezoid-rule integral of each component
    shape = (17, 12, 9)
    p = _tiny_problem(shape, tau=1e-3, diff=(1.0, 10.0), vel=(0.0, 0.0, 0.0))
    rng = np.random.default_rng(12)
    U = np.asfortranarray(rng.uniform(0, 1, shape))
    V = np.asfortranarray(rng.uniform(0, 1, shape))
    w = np.ones(shape)
    for mu, n in enumerate(shape):
        wm = np.ones(n); wm[0] = wm[-1] = 0.5
        sh = [1] * len(shape); sh[mu] = n
        w = w * wm.reshape(sh)
    m0 = (w * U).sum() / w.sum(), (w * V).sum() / w.sum()
    U1, V1 = O.solve(U, V, p, 20, scheme)
    m1 = (w * U1).sum() / w.sum(), (w * V1).sum() / w.sum()
    assert abs(m1[0] - m0[0]) <= 1e-14 * 20 and abs(m1[1] - m0[1]) <= 1e-14 * 20
    # and the solution really changed (diffusion did act)
    assert np.abs(U1 - U).max() > 1e-3


@pytest.mark.parametrize("w", [S.with_shape(S.schnakenberg_2d(), (24, 20)),
                               S.with_shape(S.fhn_3d(), (10, 12, 8)),
                               S.with_shape(S.brusselator_3d(), (10, 8, 12))],
                         ids=lambda w: w.model)
@pytest.mark.parametrize("scheme", ["etd2rkds", "lawson2b"])
def test_homogeneous_steady_state_stays_fixed(w, scheme):
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    U = np.full(w.n, w.base[0], order="F")
    V = np.full(w.n, w.base[1], order="F")
    steps = 100
    U1, V1 = O.solve(U, V, p, steps, scheme, mats=mats)
    if scheme == "etd2rkds":
        # K 1 = 0, so only the rounding of g(u_e, v_e) = 0 moves the state
        tol = 1e-13
    else:
        # Lawson2b carries the state through e^{tau A_mu}; e^{tau A} 1 = 1 holds only
        # to the rounding of the small exponentials (pinned in the next test), and the
        # reaction couples the drift of one component into the other
        rowerr = max(sum(np.abs(E @ np.ones(E.shape[0]) - 1.0).max() for E in mats[c][0])
                     for c in range(2))
        tol = 2.0 * steps * rowerr * max(abs(w.base[0]), abs(w.base[1]), 1.0) + 1e-13
    assert np.abs(U1 - w.base[0]).max() <= tol and np.abs(V1 - w.base[1]).max() <= tol


@pytest.mark.parametrize("n,tau,diff,vel", [(24, 1e-3, 10.0, 0.0), (64, 1e-3, 10.0, 0.0),
                                            (128, 1e-3, 4.0, 0.0), (256, 5e-3, 5e-3, 0.1)])
def test_exponential_fixes_constants(n, tau, diff, vel):
    # A 1 = 0 implies e^{tau A} 1 = 1 and phi_1(tau A) 1 = 1; scaling and squaring keeps
    # this to 2^(s+1) eps where 2^s is the scaling of the augmented matrix
    A = O.operator_1d(n, 0.0, 1.0, diff, vel)
    E, P1, P2 = O.phi_functions(tau * A)
    s = math.ceil(math.log2((np.abs(tau * A).sum(axis=0).max() + 1.0) / 0.5))
    tol = 2.0 ** (s + 1) * np.finfo(float).eps
    one = np.ones(n)
    assert np.abs(E @ one - 1).max() <= tol
    assert np.abs(P1 @ one - 1).max() <= tol
    assert np.abs(P2 @ one - 0.5).max() <= tol


def test_axis_permutation_equivariance():
    w = S.with_shape(S.brusselator_3d(), (9, 9, 9)).replace(vel_u=(0.1,) * 3, vel_v=(0.1,) * 3)
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    U, V = S.initial_state(w, seed=3)
    perm = (2, 0, 1)
    U1, V1 = O.solve(U, V, p, 3, mats=mats)
    Up, Vp = O.solve(np.asfortranarray(U.transpose(perm)), np.asfortranarray(V.transpose(perm)),
                     p, 3, mats=mats)
    assert np.abs(Up - U1.transpose(perm)).max() <= 1e-14 * 10
    assert np.abs(Vp - V1.transpose(perm)).max() <= 1e-14 * 10


def test_observed_order_two():
    # 2D Schnakenberg on a 24^2 grid, T = 0.02, reference 16x finer than the finest run;
    # below 40 steps (tau*|A_v| > 10) the runs are not yet in the asymptotic regime
    w = S.with_shape(S.schnakenberg_2d(), (24, 24))
    U0, V0 = S.initial_state(w, seed=0)
    T = 0.02
    steps = [40, 80, 160]
    ref_steps = 16 * steps[-1]
    p = O.problem_from_workload(w.replace(tau=T / ref_steps))
    Ur, Vr = O.solve(U0, V0, p, ref_steps)
    errs = []
    for s in steps:
        p = O.problem_from_workload(w.replace(tau=T / s))
        U, V = O.solve(U0, V0, p, s)
        errs.append(O.relative_error(U, V, Ur, Vr))
    orders = O.observed_order(steps, errs)
    assert all(1.8 <= q <= 2.2 for q in orders), (errs, orders)
