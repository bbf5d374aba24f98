"""GPU parity of the building blocks against the oracle: the FP64 MFMA
mu-mode product and Tucker operator (Sec. 2, eq. (5)) and the on-device
matrix functions e^X, phi_1, phi_2 (eq. (9))."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O

pytestmark = pytest.mark.gpu

TOL = 1e-12  # FP64 relative infinity-norm gate


def _rand(shape, seed):
    return np.asfortranarray(np.random.default_rng(seed).standard_normal(shape))


SHAPES = [
    (7,), (64,), (300,),
    (64, 64), (33, 70), (130, 48), (256, 17), (5, 129),
    (16, 24, 40), (72, 40, 150), (64, 64, 64), (31, 17, 3), (3, 200, 9),
    # 64-row and 64x64 tiles; the largest n the boundary accepts
    (192, 128, 64), (64, 192, 48), (320, 192, 16), (4096, 24), (24, 4096),
    # few 128x128 tiles for the chip: 64x64 tiles, persistent or one per workgroup
    (384, 640), (128, 128, 128),
    # n = 320 (not a multiple of 128) with enough tiles: 64x128 persistent tiles
    (320, 192, 64),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_mode_product_every_direction(dev, shape):
    import torch
    W = _rand(shape, 1)
    Wd = dev.to_device_f64(W)
    for mu, n in enumerate(shape):
        M = _rand((n, n), 10 + mu)
        Y = _rand(shape, 20 + mu)
        out = torch.empty_like(Wd)
        dev.adr_mode_product(shape, mu, dev.to_device_f64(M), Wd, out, alpha=0.75, beta=-1.5,
                             Y=dev.to_device_f64(Y))
        torch.cuda.synchronize()
        got = dev.from_device(out, shape)
        ref = 0.75 * O.mode_product(W, M, mu) - 1.5 * Y
        assert O.rel_inf_error(got, ref) <= TOL, (shape, mu)


def test_mode_product_in_place_addend(dev):
    import torch
    shape = (40, 50, 30)
    W, Y = _rand(shape, 3), _rand(shape, 4)
    M = _rand((50, 50), 5)
    out = dev.to_device_f64(Y)
    dev.adr_mode_product(shape, 1, dev.to_device_f64(M), dev.to_device_f64(W), out, 2.0, 1.0, Y=out)
    torch.cuda.synchronize()
    ref = 2.0 * O.mode_product(W, M, 1) + Y
    assert O.rel_inf_error(dev.from_device(out, shape), ref) <= TOL


@pytest.mark.parametrize("shape", [(64, 64), (100, 37), (24, 36, 20), (130, 66, 72), (256, 256, 8),
                                   # (i1, i2) planes of 64^2 or 128^2 doubles: directions 1 and 2
                                   # in one pass over LDS-resident planes (the whole operator in 2D)
                                   (128, 128), (64, 64, 3), (128, 128, 1), (128, 128, 37), (64, 64, 200)],
                         ids=lambda s: "x".join(map(str, s)))
def test_tucker_against_oracle(dev, shape):
    import torch
    W = _rand(shape, 7)
    Ms = [_rand((n, n), 30 + k) / math.sqrt(n) for k, n in enumerate(shape)]
    Y = _rand(shape, 8)
    out = torch.empty(W.size, dtype=torch.float64, device="cuda")
    work = torch.empty(dev.adr_tucker_workspace_bytes(shape) // 8 + 1, dtype=torch.float64, device="cuda")
    dev.adr_tucker(shape, [dev.to_device_f64(M) for M in Ms], dev.to_device_f64(W), out,
                   alpha=0.5, beta=2.0, Y=dev.to_device_f64(Y), work=work)
    torch.cuda.synchronize()
    ref = 0.5 * O.tucker(W, Ms) + 2.0 * Y
    assert O.rel_inf_error(dev.from_device(out, shape), ref) <= TOL


def test_tucker_plane_pass_in_place_addend(dev):
    # the plane pass with out aliasing the addend Y (2D: the whole operator)
    import torch
    shape = (128, 128)
    W, Y = _rand(shape, 11), _rand(shape, 12)
    Ms = [_rand((128, 128), 40 + k) / math.sqrt(128) for k in range(2)]
    out = dev.to_device_f64(Y)
    work = torch.empty(dev.adr_tucker_workspace_bytes(shape) // 8 + 1, dtype=torch.float64, device="cuda")
    dev.adr_tucker(shape, [dev.to_device_f64(M) for M in Ms], dev.to_device_f64(W), out,
                   alpha=-1.25, beta=0.5, Y=out, work=work)
    torch.cuda.synchronize()
    ref = -1.25 * O.tucker(W, Ms) + 0.5 * Y
    assert O.rel_inf_error(dev.from_device(out, shape), ref) <= TOL


def test_exp_tucker_is_dense_exponential(dev):
    # eq. (5): Tucker with e^{tau A_mu} equals e^{tau K} on vec(W); K assembled densely
    import torch
    shape = (6, 5, 4)
    As = [O.operator_1d(n, 0.0, 1.0, 0.05, 0.3) for n in shape]
    tau = 0.01
    Es = [sla.expm(tau * A) for A in As]
    W = _rand(shape, 2)
    out = torch.empty(W.size, dtype=torch.float64, device="cuda")
    work = torch.empty(dev.adr_tucker_workspace_bytes(shape) // 8 + 1, dtype=torch.float64, device="cuda")
    dev.adr_tucker(shape, [dev.to_device_f64(E) for E in Es], dev.to_device_f64(W), out, work=work)
    torch.cuda.synchronize()
    ref = sla.expm(tau * O.kron_sum_dense(As)) @ O.vec(W)
    assert O.rel_inf_error(O.vec(dev.from_device(out, shape)), ref) <= 1e-12


@pytest.mark.parametrize("n,tau,diff,vel", [
    (64, 1e-3, 1.0, 0.0), (64, 1e-3, 10.0, 0.0),        # 2D Schnakenberg, u and v
    (128, 1e-3, 1.0, 0.0), (128, 1e-3, 4.0, 0.0),       # 3D FitzHugh-Nagumo
    (256, 5e-3, 1e-3, 0.1), (256, 5e-3, 5e-3, 0.025),   # 3D advective Brusselator
    (512, 1e-3, 10.0, 0.0),                             # largest batched side (tau*|A| ~ 1e4)
    (3, 0.1, 1.0, 0.0), (37, 2e-3, 0.3, 0.5), (200, 5e-3, 1.0, 0.0)])
def test_precompute_phi_against_oracle(dev, n, tau, diff, vel):
    A = O.operator_1d(n, 0.0, 1.0, diff, vel)
    E, P1, P2 = dev.adr_precompute_phi(dev.to_device_f64(A), tau)
    ref = O.phi_functions(tau * A)
    # both sides square 2^s-scaled approximations; relative rounding grows like 2^s eps
    s = max(0, math.ceil(math.log2(max(np.abs(tau * A).sum(axis=0).max(), 1.0))))
    tol = max(TOL, 8 * 2.0 ** s * np.finfo(float).eps)
    for got, want in zip((E, P1, P2), ref):
        err = O.rel_inf_error(dev.from_device(got, (n, n)), want)
        assert err <= tol, (n, err, tol)


def test_precompute_phi_invariants_on_random_matrix(dev):
    rng = np.random.default_rng(3)
    n = 50
    X = rng.standard_normal((n, n)) * 0.3
    E, P1, P2 = (dev.from_device(t, (n, n)) for t in dev.adr_precompute_phi(dev.to_device_f64(X), 1.0))
    I = np.eye(n)
    assert np.abs(X @ P1 - (E - I)).max() <= 1e-13
    assert np.abs(X @ P2 - (P1 - I)).max() <= 1e-13
    assert np.abs(E - sla.expm(X)).max() <= 1e-13 * np.abs(E).max()


def test_precompute_phi_rejects_nonfinite(dev):
    A = np.eye(8)
    A[3, 2] = np.inf
    with pytest.raises(dev.AdrError) as ei:
        dev.adr_precompute_phi(dev.to_device_f64(A), 1e-3)
    assert ei.value.status == dev.ADR_ENONFINITE


def test_device_copy(dev):
    import torch
    x = torch.randn(1000003, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    dev.adr_device_copy(x, y, x.numel())
    torch.cuda.synchronize()
    assert torch.equal(x, y)


def test_precompute_phi_batch_equals_single_calls(dev):
    # several matrices of different sizes and steps in one call (two
    # synchronisations): the same kernels as one call per matrix, so bitwise equal
    import torch
    specs = [(256, 5e-3, 1e-3, 0.1), (64, 1e-3, 10.0, 0.0), (300, 2e-3, 0.5, -0.2),
             (3, 0.1, 1.0, 0.0), (512, 1e-3, 10.0, 0.0)]
    As = [dev.to_device_f64(O.operator_1d(n, 0.0, 1.0, d, v)) for n, _, d, v in specs]
    taus = [t for _, t, _, _ in specs]
    batch = dev.adr_precompute_phi_batch(As, taus)
    torch.cuda.synchronize()
    for A, tau, got in zip(As, taus, batch):
        ref = dev.adr_precompute_phi(A, tau)
        torch.cuda.synchronize()
        for g, r in zip(got, ref):
            assert torch.equal(g, r)


def test_precompute_phi_batch_rejects_nonfinite(dev):
    good = dev.to_device_f64(np.eye(8))
    bad = np.eye(8)
    bad[1, 2] = np.nan
    with pytest.raises(dev.AdrError) as ei:
        dev.adr_precompute_phi_batch([good, dev.to_device_f64(bad)], [1e-3, 1e-3])
    assert ei.value.status == dev.ADR_ENONFINITE
