"""Reduced-precision Tucker operators (FP32 MFMA and split BF16) inside the
FP64 ETD2RKds step, checked against the FP64 oracle.

Only the bulk mu-mode products run in reduced precision; the state, the stage
combinations (C_{n2} = C_n + tau*T, C_{n+1} = C_{n2} + 2^(d-1) tau*T) and the
small matrix functions stay FP64 (Sec. 3, eq. (11)).  The products act on the
increments, so the state error stays far below the product error.

Precisions: FP32; BF16X3, each FP32 operand split exactly into three bf16
parts and multiplied by six bf16 products; BF16X2, two parts and three
products (about 2^-16 of each product).

Stated tolerances (relative infinity norm per component, after the listed
steps).  A Tucker operator is d dot products of lengths n_mu, each rounding
at a unit u relative to the increment it forms.  Where the increments are
as large as the state (FitzHugh-Nagumo, whose states lie near 0) the state
error can reach u * sum(n_mu), and the gate there is max(floor, u *
sum(n_mu)); on the other models (states near their O(1) equilibria, small
increments) it is the floor:
* FP32: u = 2^-24, floor 1e-6;
* BF16X3: u = 8 * 2^-24, floor 1e-5.  The dropped cross terms are below
  2^-22 of each product, but the bf16 matrix instruction adds each group of
  eight products after aligning them to the largest and drops the bits below
  24 (probed on gfx950), so a group can lose about seven units of 2^-24 of its
  largest product;
* BF16X2: 1e-4, except on FitzHugh-Nagumo (states within about +-0.1 of zero,
  so the relative norm magnifies the 2^-16 product error): 3e-4.
Measured values are printed."""
import numpy as np
import pytest

import oracle as O
import synth as S

pytestmark = pytest.mark.gpu

PRECISIONS = ["f32", "bf16x3", "bf16x2"]


def tolerance(precision, w):
    """The stated gate of a precision on a workload (module docstring)."""
    if precision == "bf16x2":
        return 3e-4 if w.model == "fhn" else 1e-4
    unit, floor = {"f32": (2.0 ** -24, 1e-6), "bf16x3": (8 * 2.0 ** -24, 1e-5)}[precision]
    return max(floor, unit * sum(w.n)) if w.model == "fhn" else floor

CASES = [
    ("bruss3d_64_100", S.brusselator_3d(64, 100), 100),
    ("bruss3d_72x40x150_10", S.with_shape(S.brusselator_3d(), (72, 40, 150)), 10),
    ("schnak2d_64_100", S.schnakenberg_2d(64, 100), 100),
    ("fhn3d_48_50", S.fhn_3d(48, 50), 50),
    ("schnak2d_130x70_20", S.with_shape(S.schnakenberg_2d(), (130, 70)), 20),
    ("bruss1d_300_50", S.with_shape(S.brusselator_3d(), (300,)), 50),
    # n = 192: 64-row tiles; on both models
    ("bruss3d_192x64x40_10", S.with_shape(S.brusselator_3d(), (192, 64, 40)), 10),
    ("fhn3d_192x64x40_10", S.with_shape(S.fhn_3d(), (192, 64, 40)), 10),
    # evenly tiled, fewer than two 128-row tiles per CU: 64-row tiles
    ("schnak2d_512x384_5", S.with_shape(S.schnakenberg_2d(), (512, 384)), 5),
    # n % 256 == 0 in every direction: the wide persistent split-BF16 tiles
    ("fhn3d_256x256x128_3", S.with_shape(S.fhn_3d(), (256, 256, 128)), 3),
    ("schnak2d_512x256_5", S.with_shape(S.schnakenberg_2d(), (512, 256)), 5),
]


def _run(dev, w, steps, precision, mats, scheme="etd2rkds", seed=0):
    import torch
    U0, V0 = S.initial_state(w, seed)
    s = dev.Solver(w, scheme=scheme, precision=precision, phis=mats)
    Ud, Vd = s.upload(U0, V0)
    s.solve(Ud, Vd, steps)
    torch.cuda.synchronize()
    return s.download(Ud, Vd)


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("name,w,steps", CASES, ids=[c[0] for c in CASES])
def test_reduced_precision_step_error(dev, precision, name, w, steps):
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    U0, V0 = S.initial_state(w, 0)
    U, V = O.solve(U0, V0, p, steps, mats=mats)
    Ug, Vg = _run(dev, w, steps, precision, mats)
    eu, ev = O.rel_inf_error(Ug, U), O.rel_inf_error(Vg, V)
    print(f"{name} {precision}: rel inf err u={eu:.2e} v={ev:.2e}")
    tol = tolerance(precision, w)
    assert eu <= tol and ev <= tol, (eu, ev, tol)
    # reduced precision must not be accidentally exact (i.e. really ran)
    assert max(eu, ev) > 1e-15


@pytest.mark.parametrize("precision", PRECISIONS)
def test_reduced_precision_full_size_256(dev, precision):
    w = S.brusselator_3d()
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    U0, V0 = S.initial_state(w, 0)
    U, V = O.solve(U0, V0, p, 1, mats=mats)
    Ug, Vg = _run(dev, w, 1, precision, mats)
    eu, ev = O.rel_inf_error(Ug, U), O.rel_inf_error(Vg, V)
    print(f"256^3 {precision} one step: u={eu:.2e} v={ev:.2e}")
    assert eu <= tolerance(precision, w) and ev <= tolerance(precision, w)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_reduced_precision_lawson2b(dev, precision):
    # Lawson2b carries the whole state through the products: the error is that of
    # the product precision itself (stated gates: 1e-5 FP32 and three-part split
    # BF16, 1e-3 two-part split BF16)
    w = S.with_shape(S.brusselator_3d(), (40, 48, 56))
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    U0, V0 = S.initial_state(w, 0)
    U, V = O.solve(U0, V0, p, 10, "lawson2b", mats=mats)
    Ug, Vg = _run(dev, w, 10, precision, mats, "lawson2b")
    eu, ev = O.rel_inf_error(Ug, U), O.rel_inf_error(Vg, V)
    print(f"lawson2b {precision}: u={eu:.2e} v={ev:.2e}")
    tol = {"f32": 1e-5, "bf16x3": 1e-5, "bf16x2": 1e-3}[precision]
    assert eu <= tol and ev <= tol


@pytest.mark.parametrize("w", [S.with_shape(S.fhn_3d(), (64, 48, 40)),
                               S.with_shape(S.fhn_3d(), (256, 256, 64))], ids=["generic", "wide"])
@pytest.mark.parametrize("precision", ["bf16x3", "bf16x2"])
def test_reduced_precision_deterministic(dev, w, precision):
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    a = _run(dev, w, 3, precision, mats)
    b = _run(dev, w, 3, precision, mats)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
