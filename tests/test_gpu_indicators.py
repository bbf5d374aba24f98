"""The fused indicator reduction (adr_indicators) and the monitored solve
(adr_solve_monitored) against the oracle's indicators (Sec. 4): trapezoidal
spatial means, Frobenius norms of the increment, non-finite counts.

Means and norms are sums in another order than the oracle's: relative
tolerance 1e-13 (N up to 2^24 terms of like sign in FP64 with pairwise-style
block sums); counts must be exact."""
import numpy as np
import pytest

import oracle as O
import synth as S

pytestmark = pytest.mark.gpu


def _check(rec, ref):
    for k in range(4):
        assert rec[k] == pytest.approx(ref[k], rel=1e-13, abs=1e-300), (k, rec[k], ref[k])
    assert rec[4] == ref[4]


@pytest.mark.parametrize("shape", [(300,), (130, 70), (37, 29, 11), (3, 3, 3), (256, 256, 256)],
                         ids=lambda s: "x".join(map(str, s)))
def test_indicators_match_oracle(dev, shape):
    import torch
    rng = np.random.default_rng(len(shape) * 7 + shape[0])
    U, V, P, Q = (np.asfortranarray(rng.uniform(-1, 2, shape)) for _ in range(4))
    d = [dev.to_device_f64(x) for x in (U, V, P, Q)]
    rec = dev.adr_indicators(shape, d[0], d[1], d[2], d[3])
    torch.cuda.synchronize()
    _check(rec.cpu().numpy(), O.indicators(U, V, P, Q))
    rec = dev.adr_indicators(shape, d[0], d[1])
    torch.cuda.synchronize()
    _check(rec.cpu().numpy(), O.indicators(U, V))


def test_indicators_count_nonfinite(dev):
    import torch
    shape = (40, 33, 9)
    rng = np.random.default_rng(5)
    U, V, P, Q = (np.asfortranarray(rng.uniform(0, 1, shape)) for _ in range(4))
    U[3, 4, 5] = np.nan
    V[3, 4, 5] = np.inf
    V[39, 32, 8] = -np.inf
    P[0, 0, 0] = np.nan
    d = [dev.to_device_f64(x) for x in (U, V, P, Q)]
    rec = dev.adr_indicators(shape, *d).cpu().numpy()
    torch.cuda.synchronize()
    assert rec[4] == O.indicators(U, V, P, Q)[4] == 3


@pytest.mark.parametrize("w,steps,every", [
    (S.with_shape(S.schnakenberg_2d(), (96, 80)), 12, 3),
    (S.with_shape(S.fhn_3d(), (24, 20, 28)), 10, 4),
    (S.with_shape(S.dib_2d(), (64, 64)), 6, 1),
    # evenly tiled: stage 2 runs in the epilogue of the last phi_1 product
    (S.with_shape(S.schnakenberg_2d(), (128, 256)), 8, 2),
    (S.with_shape(S.brusselator_3d(), (64, 32, 128)), 4, 2),
], ids=["schnak2d", "fhn3d", "dib2d", "schnak2d_fused", "bruss3d_fused"])
def test_solve_monitored_matches_oracle(dev, w, steps, every):
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    U0, V0 = S.initial_state(w, 4)
    U, V = U0, V0
    ref = []
    for n in range(1, steps + 1):
        Up, Vp = U, V
        U, V = O.etd2rkds_step(U, V, p, mats)
        if n % every == 0:
            ref.append(O.indicators(U, V, Up, Vp))
    s = dev.Solver(w, phis=mats)
    Ud, Vd = s.upload(U0, V0)
    recs, st = s.solve_monitored(Ud, Vd, steps, every)
    assert st == dev.ADR_OK
    assert recs.shape == (steps // every, 5)
    for got, want in zip(recs, ref):
        for k in range(4):
            assert got[k] == pytest.approx(want[k], rel=1e-11), (k, got[k], want[k])
        assert got[4] == 0
    Ug, Vg = s.download(Ud, Vd)
    # DIB: u sits at its equilibrium 0; measure both fields against the larger
    # norm (rounding in its O(200) reaction terms is absolute)
    scale = max(np.abs(U).max(), np.abs(V).max()) if w.model == "dib" else None
    for g, r in ((Ug, U), (Vg, V)):
        den = scale if scale is not None else np.abs(r).max()
        assert np.abs(g - r).max() / den <= 1e-12


def test_solve_monitored_pure_diffusion_keeps_the_mean(dev):
    # g = 0 with Neumann rows: the trapezoidal mean is invariant (any grid size)
    w = S.with_shape(S.brusselator_3d(), (64, 48, 40)).replace(
        model="zero", params=(), vel_u=(0.0,) * 3, vel_v=(0.0,) * 3)
    s = dev.Solver(w)
    U0, V0 = S.initial_state(w, 1)
    Ud, Vd = s.upload(U0, V0)
    recs, st = s.solve_monitored(Ud, Vd, 20, 5)
    m0 = O.spatial_mean(U0), O.spatial_mean(V0)
    assert st == dev.ADR_OK
    for r in recs:
        assert abs(r[0] - m0[0]) <= 1e-13 * abs(m0[0]) * 20
        assert abs(r[1] - m0[1]) <= 1e-13 * abs(m0[1]) * 20
        assert r[2] > 0 and r[3] > 0


def test_solve_monitored_reports_nonfinite_state(dev):
    w = S.with_shape(S.schnakenberg_2d(), (64, 64))
    s = dev.Solver(w)
    U0, V0 = S.initial_state(w, 2)
    U0[10, 20] = np.nan
    Ud, Vd = s.upload(U0, V0)
    recs, st = s.solve_monitored(Ud, Vd, 4, 2)
    assert st == dev.ADR_ENONFINITE
    assert all(r[4] >= 1 for r in recs)
