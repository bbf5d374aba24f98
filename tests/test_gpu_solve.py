"""GPU parity of whole ETD2RKds (Sec. 3, eq. (11)) and Lawson2b (Sec. 2,
eq. (7)) steps against the FP64 oracle, called through the C ABI.

Two kinds of runs:
* hot path: the GPU steps with the oracle's small matrices, so the comparison
  isolates the stage kernels and the mode products;
* end to end: the GPU also builds its operators (adr_build_1d_ops) and its
  matrix functions (adr_precompute_phi), as a user would.
Gate: relative infinity-norm error <= 1e-12 per component (FP64)."""
import numpy as np
import pytest

import oracle as O
import synth as S

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _oracle(w, seed, steps, scheme="etd2rkds"):
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    U0, V0 = S.initial_state(w, seed)
    U, V = O.solve(U0, V0, p, steps, scheme, mats=mats)
    return U0, V0, U, V, mats


def _gpu(dev, w, U0, V0, steps, scheme="etd2rkds", mats=None, use_band=True, chunks=None):
    import torch
    s = dev.Solver(w, scheme=scheme, phis=mats, use_band=use_band)
    Ud, Vd = s.upload(U0, V0)
    for k in (chunks or [steps]):
        s.solve(Ud, Vd, k)
    torch.cuda.synchronize()
    return s.download(Ud, Vd)


def _assert_close(got, ref, tol=TOL, joint=False):
    """Relative infinity-norm error per component.  With joint=True both
    components are measured against the larger of their two norms: used for the
    DIB model, whose u starts at the equilibrium value 0 (plus 1e-5 noise) while
    its reaction terms are O(rho a_3^u a_4^u) ~ 200, so rounding there is
    absolute and a per-component relative measure of u would be ill-conditioned."""
    if joint:
        scale = max(np.abs(ref[0]).max(), np.abs(ref[1]).max())
        eu = np.abs(got[0] - ref[0]).max() / scale
        ev = np.abs(got[1] - ref[1]).max() / scale
    else:
        eu = O.rel_inf_error(got[0], ref[0])
        ev = O.rel_inf_error(got[1], ref[1])
    assert eu <= tol and ev <= tol, (eu, ev)
    return max(eu, ev)


CASES = [
    ("schnakenberg2d_64x64_100", S.schnakenberg_2d(64, 100), 100),
    ("schnakenberg2d_130x70_30", S.with_shape(S.schnakenberg_2d(), (130, 70)), 30),
    ("fhn3d_40x36x44_20", S.with_shape(S.fhn_3d(), (40, 36, 44)), 20),
    ("bruss3d_72x40x150_10", S.with_shape(S.brusselator_3d(), (72, 40, 150)), 10),
    ("bruss1d_300_50", S.with_shape(S.brusselator_3d(), (300,)), 50),
    ("fhn3d_3x3x3_5", S.with_shape(S.fhn_3d(), (3, 3, 3)), 5),
    # Sec. 4.4 DIB model (eq. (15)) on [0,20]^2, and the advective Schnakenberg
    # experiment of Sec. 4.5 (eq. (16), Gaussian-bump data) at its own 80^3 grid
    ("dib2d_96x80_40", S.with_shape(S.dib_2d(200, 1250), (96, 80)), 40),
    ("paper_schnak3d_80_10", S.paper_schnakenberg_3d(80, 50), 10),
    # evenly tiled grids: the last product of the phi_1 operator also computes
    # stage 2 (64x64 persistent tiles at these sizes, 128x128 at 256^3)
    ("schnakenberg2d_256x128_20", S.with_shape(S.schnakenberg_2d(), (256, 128)), 20),
    ("bruss3d_64x128x64_10", S.with_shape(S.brusselator_3d(), (64, 128, 64)), 10),
    ("dib2d_128x256_10", S.with_shape(S.dib_2d(200, 1250), (128, 256)), 10),
    # n % 64 == 0 but not % 128: 64-row tiles for the products and stage 2
    ("schnakenberg2d_128x192_20", S.with_shape(S.schnakenberg_2d(), (128, 192)), 20),
    # stage 2 carried by persistent 64x64 tiles (few tiles for the chip)
    ("schnakenberg2d_384x384_3", S.with_shape(S.schnakenberg_2d(), (384, 384)), 3),
    # stage 2 on 64x128 tiles (256 pairs of 128x128 tiles would leave half the
    # persistent workgroups idle)
    ("bruss3d_128x128x256_1", S.with_shape(S.brusselator_3d(), (128, 128, 256)), 1),
    ("fhn3d_192x128x64_5", S.with_shape(S.fhn_3d(), (192, 128, 64)), 5),
    # strided direction with L % 128 != 0, L % 64 == 0: 64x64 tiles
    ("bruss3d_64x192x48_5", S.with_shape(S.brusselator_3d(), (64, 192, 48)), 5),
    # 128^2 and 64^2 (i1, i2) planes: directions 1 and 2 in one pass over LDS
    ("fhn3d_128x128x40_10", S.with_shape(S.fhn_3d(), (128, 128, 40)), 10),
    ("bruss3d_64x64x96_10", S.with_shape(S.brusselator_3d(), (64, 64, 96)), 10),
    ("schnakenberg2d_128x128_20", S.with_shape(S.schnakenberg_2d(), (128, 128)), 20),
    # 3D grids of 2^20 points or more: stage 1 on LDS tiles, the planes split
    # over as many blocks per tile column as the chip holds at once (1-2 planes
    # each here, uneven); the last case has partial tiles in i1 and i2 as well
    ("fhn3d_64x128x128_5", S.with_shape(S.fhn_3d(), (64, 128, 128)), 5),
    ("bruss3d_256x64x72_3", S.with_shape(S.brusselator_3d(), (256, 64, 72)), 3),
    ("bruss3d_100x90x120_3", S.with_shape(S.brusselator_3d(), (100, 90, 120)), 3),
    # thin 3D grid: 256 tiles per plane, so 4 planes over 3 blocks per tile column
    ("fhn3d_512x512x4_2", S.with_shape(S.fhn_3d(), (512, 512, 4)), 2),
    # 2D grids of 64 x n2 (n2 <= 64): every step in one cooperative launch, four
    # columns per workgroup; a last workgroup with fewer columns (30, 3), the
    # advective Brusselator (non-symmetric bands) and the DIB model
    ("schnakenberg2d_64x30_40", S.with_shape(S.schnakenberg_2d(), (64, 30)), 40),
    ("fhn2d_64x3_20", S.with_shape(S.fhn_3d(), (64, 3)), 20),
    ("bruss2d_64x64_30", S.with_shape(S.brusselator_3d(), (64, 64)), 30),
    ("dib2d_64x48_20", S.with_shape(S.dib_2d(200, 1250), (64, 48)), 20),
]


@pytest.mark.parametrize("name,w,steps", CASES, ids=[c[0] for c in CASES])
def test_etd2rkds_hot_path(dev, name, w, steps):
    U0, V0, U, V, mats = _oracle(w, 0, steps)
    got = _gpu(dev, w, U0, V0, steps, mats=mats)
    _assert_close(got, (U, V), joint=(w.model == "dib"))


E2E = CASES[:4] + [CASES[6], CASES[8]]


@pytest.mark.parametrize("name,w,steps", E2E, ids=[c[0] for c in E2E])
def test_etd2rkds_end_to_end(dev, name, w, steps):
    U0, V0, U, V, _ = _oracle(w, 1, steps)
    got = _gpu(dev, w, U0, V0, steps)
    _assert_close(got, (U, V), joint=(w.model == "dib"))


@pytest.mark.parametrize("name,w,steps", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_lawson2b(dev, name, w, steps):
    U0, V0, U, V, mats = _oracle(w, 2, steps, "lawson2b")
    got = _gpu(dev, w, U0, V0, steps, "lawson2b", mats=mats)
    _assert_close(got, (U, V))


@pytest.mark.parametrize("name,w,steps", [CASES[1], CASES[3]], ids=[CASES[1][0], CASES[3][0]])
def test_dense_kronecker_action_path(dev, name, w, steps):
    # without the tridiagonal bands the library applies K C with dense mode products
    U0, V0, U, V, mats = _oracle(w, 3, steps)
    got = _gpu(dev, w, U0, V0, steps, mats=mats, use_band=False)
    _assert_close(got, (U, V))


def test_full_size_fhn_128(dev):
    w = S.fhn_3d()                           # 128^3, tau = 1e-3
    U0, V0, U, V, mats = _oracle(w, 0, 2)
    _assert_close(_gpu(dev, w, U0, V0, 2, mats=mats), (U, V))


def test_full_size_brusselator_256(dev):
    w = S.brusselator_3d()                   # 256^3, tau = 5e-3: the benchmark workload
    U0, V0, U, V, mats = _oracle(w, 0, 1)
    _assert_close(_gpu(dev, w, U0, V0, 1, mats=mats), (U, V))


def test_full_size_brusselator_256_end_to_end(dev):
    w = S.brusselator_3d()
    U0, V0, U, V, _ = _oracle(w, 5, 1)
    _assert_close(_gpu(dev, w, U0, V0, 1), (U, V))


def test_largest_2d_grid(dev):
    w = S.with_shape(S.schnakenberg_2d(), (1024, 1024))
    U0, V0, U, V, mats = _oracle(w, 0, 1)
    _assert_close(_gpu(dev, w, U0, V0, 1, mats=mats), (U, V))


def test_bitwise_determinism_and_resume(dev):
    w = S.with_shape(S.brusselator_3d(), (64, 48, 80))
    U0, V0 = S.initial_state(w, 4)
    a = _gpu(dev, w, U0, V0, 20)
    b = _gpu(dev, w, U0, V0, 20)
    c = _gpu(dev, w, U0, V0, 20, chunks=[7, 13])
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y) and np.array_equal(x, z)


def test_whole_step_launch_abandons_to_nan(dev, monkeypatch):
    # a grid barrier that gives up (forced here by a spin limit of 0 polls, set
    # from the host) ends the launch with NaN in U and V instead of a result,
    # and the next call with the normal limit steps correctly again
    w = S.with_shape(S.schnakenberg_2d(), (64, 64))
    U0, V0, U, V, mats = _oracle(w, 7, 10)
    monkeypatch.setenv("ADR_TEST_SPIN_LIMIT", "0")
    bad = _gpu(dev, w, U0, V0, 10, mats=mats)
    assert np.isnan(bad[0]).all() and np.isnan(bad[1]).all()
    monkeypatch.delenv("ADR_TEST_SPIN_LIMIT")
    _assert_close(_gpu(dev, w, U0, V0, 10, mats=mats), (U, V))


def test_whole_step_launch_resumes_bitwise(dev):
    # the 64 x n2 path runs a solve call's steps in one launch; splitting the
    # steps over several calls gives the same bits
    w = S.with_shape(S.brusselator_3d(), (64, 40))
    U0, V0 = S.initial_state(w, 6)
    a = _gpu(dev, w, U0, V0, 30)
    b = _gpu(dev, w, U0, V0, 30, chunks=[1, 7, 22])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("w", [S.schnakenberg_2d(64, 1), S.fhn_3d(48, 1), S.brusselator_3d(40, 1)],
                         ids=lambda w: w.model)
@pytest.mark.parametrize("scheme", ["etd2rkds", "lawson2b"])
def test_homogeneous_steady_state_fixed(dev, w, scheme):
    U0 = np.full(w.n, w.base[0], order="F")
    V0 = np.full(w.n, w.base[1], order="F")
    U, V = _gpu(dev, w, U0, V0, 100, scheme)
    assert np.abs(U - w.base[0]).max() <= 1e-11 and np.abs(V - w.base[1]).max() <= 1e-11


def test_zero_steps_leaves_state(dev):
    w = S.with_shape(S.fhn_3d(), (20, 21, 22))
    U0, V0 = S.initial_state(w, 0)
    U, V = _gpu(dev, w, U0, V0, 0)
    assert np.array_equal(U, U0) and np.array_equal(V, V0)


@pytest.mark.parametrize("shape", [(4096,), (4096, 24), (24, 4096)], ids=["1d", "2d_long_x1", "2d_long_x2"])
def test_largest_direction_steady_state(dev, shape):
    # n_mu = 4096, the largest size the boundary accepts: operators and matrix
    # functions built on the device, 10 steps from the homogeneous equilibrium
    # (1, 3) of the Brusselator stay there to rounding
    w = S.with_shape(S.brusselator_3d(), shape)
    U0 = np.full(w.n, w.base[0], order="F")
    V0 = np.full(w.n, w.base[1], order="F")
    U, V = _gpu(dev, w, U0, V0, 10)
    assert np.abs(U - w.base[0]).max() <= 1e-11 and np.abs(V - w.base[1]).max() <= 1e-11
