"""Reduced-precision Tucker operators (FP32 MFMA and 3-term split BF16) inside
the FP64 ETD2RKds step, checked against the FP64 oracle.

Only the bulk mu-mode products run in reduced precision; the state, the stage
combinations (C_{n2} = C_n + tau*T, C_{n+1} = C_{n2} + 2^(d-1) tau*T) and the
small matrix functions stay FP64 (Sec. 3, eq. (11)).  The products act on the
increments, so the state error stays far below the product error.

Stated tolerances (relative infinity norm per component, after the listed
steps): FP32 <= 1e-6, BF16X3 <= 1e-4.  Measured values are printed."""
import numpy as np
import pytest

import oracle as O
import synth as S

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-6, "bf16x3": 1e-4}

CASES = [
    ("bruss3d_64_100", S.brusselator_3d(64, 100), 100),
    ("bruss3d_72x40x150_10", S.with_shape(S.brusselator_3d(), (72, 40, 150)), 10),
    ("schnak2d_64_100", S.schnakenberg_2d(64, 100), 100),
    ("fhn3d_48_50", S.fhn_3d(48, 50), 50),
    ("schnak2d_130x70_20", S.with_shape(S.schnakenberg_2d(), (130, 70)), 20),
    ("bruss1d_300_50", S.with_shape(S.brusselator_3d(), (300,)), 50),
    # n = 192: 64-row tiles
    ("bruss3d_192x64x40_10", S.with_shape(S.brusselator_3d(), (192, 64, 40)), 10),
    # evenly tiled, fewer than two 128-row tiles per CU: 64-row tiles
    ("schnak2d_512x384_5", S.with_shape(S.schnakenberg_2d(), (512, 384)), 5),
]


def _run(dev, w, steps, precision, mats, scheme="etd2rkds", seed=0):
    import torch
    U0, V0 = S.initial_state(w, seed)
    s = dev.Solver(w, scheme=scheme, precision=precision, phis=mats)
    Ud, Vd = s.upload(U0, V0)
    s.solve(Ud, Vd, steps)
    torch.cuda.synchronize()
    return s.download(Ud, Vd)


@pytest.mark.parametrize("precision", ["f32", "bf16x3"])
@pytest.mark.parametrize("name,w,steps", CASES, ids=[c[0] for c in CASES])
def test_reduced_precision_step_error(dev, precision, name, w, steps):
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    U0, V0 = S.initial_state(w, 0)
    U, V = O.solve(U0, V0, p, steps, mats=mats)
    Ug, Vg = _run(dev, w, steps, precision, mats)
    eu, ev = O.rel_inf_error(Ug, U), O.rel_inf_error(Vg, V)
    print(f"{name} {precision}: rel inf err u={eu:.2e} v={ev:.2e}")
    assert eu <= TOL[precision] and ev <= TOL[precision]
    # reduced precision must not be accidentally exact (i.e. really ran)
    assert max(eu, ev) > 1e-15


@pytest.mark.parametrize("precision", ["f32", "bf16x3"])
def test_reduced_precision_full_size_256(dev, precision):
    w = S.brusselator_3d()
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    U0, V0 = S.initial_state(w, 0)
    U, V = O.solve(U0, V0, p, 1, mats=mats)
    Ug, Vg = _run(dev, w, 1, precision, mats)
    eu, ev = O.rel_inf_error(Ug, U), O.rel_inf_error(Vg, V)
    print(f"256^3 {precision} one step: u={eu:.2e} v={ev:.2e}")
    assert eu <= TOL[precision] and ev <= TOL[precision]


@pytest.mark.parametrize("precision", ["f32", "bf16x3"])
def test_reduced_precision_lawson2b(dev, precision):
    # Lawson2b carries the whole state through the products: the error is that of
    # the product precision itself (stated gates: 1e-5 FP32, 1e-3 split BF16)
    w = S.with_shape(S.brusselator_3d(), (40, 48, 56))
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    U0, V0 = S.initial_state(w, 0)
    U, V = O.solve(U0, V0, p, 10, "lawson2b", mats=mats)
    Ug, Vg = _run(dev, w, 10, precision, mats, "lawson2b")
    eu, ev = O.rel_inf_error(Ug, U), O.rel_inf_error(Vg, V)
    print(f"lawson2b {precision}: u={eu:.2e} v={ev:.2e}")
    tol = {"f32": 1e-5, "bf16x3": 1e-3}[precision]
    assert eu <= tol and ev <= tol


def test_reduced_precision_deterministic(dev):
    w = S.with_shape(S.fhn_3d(), (64, 48, 40))
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    a = _run(dev, w, 5, "bf16x3", mats)
    b = _run(dev, w, 5, "bf16x3", mats)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
