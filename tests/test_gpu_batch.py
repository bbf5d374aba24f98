"""Grouped multi-problem ETD2RKds plans (adr_batch_*), called through the C ABI.

Many independent problems of different dimension, grid size, model and step
size advance together, one grouped launch per phase of Sec. 3 eq. (11).
Checks:
* every instance of a mixed plan matches the FP64 oracle (<= 1e-12 relative
  infinity norm per component; FP32 products <= 1e-6);
* each instance alone (a plan of one) gives bitwise the result it gives in the
  mix: the grouped kernels sum every output in the same order whatever the
  neighbours and tile shape;
* a captured graph replayed several times, with eager work in between, equals
  eager grouped launches bitwise;
* autotuning picks a valid tile shape per direction, leaves U and V untouched
  and does not change the results;
* the 64-instance batched Schnakenberg workload (sides 64..512) matches the
  single-problem path and, on sampled instances, the oracle."""
import numpy as np
import pytest

import oracle as O
import synth as S

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6}

MIX = [
    S.schnakenberg_2d(64, 10),
    S.with_shape(S.schnakenberg_2d(), (130, 70)),
    S.with_shape(S.fhn_3d(), (40, 36, 44)),
    S.with_shape(S.brusselator_3d(), (300,)),
    S.with_shape(S.fhn_3d(), (3, 3, 3)),
    S.with_shape(S.brusselator_3d(), (72, 40, 150)),
    # over 2^20 points: its stage 1 takes the LDS-tiled kernel inside the grouped launch
    S.with_shape(S.schnakenberg_2d(), (1100, 960)),
]
STEPS = 6


def _oracle(w, seed, steps):
    p = O.problem_from_workload(w)
    mats = O.precompute(p)
    U0, V0 = S.initial_state(w, seed)
    U, V = O.solve(U0, V0, p, steps, "etd2rkds", mats=mats)
    return U0, V0, U, V, mats


@pytest.fixture(scope="module")
def mix_ref():
    return [_oracle(w, 10 + k, STEPS) for k, w in enumerate(MIX)]


def _setup(dev, works, refs, precision="f64"):
    solvers, states = [], []
    for w, (U0, V0, _, _, mats) in zip(works, refs):
        s = dev.Solver(w, precision=precision, phis=mats)
        solvers.append(s)
        states.append(s.upload(U0, V0))
    return solvers, states


def _run_batch(dev, works, refs, steps, precision="f64", flags=0, chunks=None, between=None):
    import torch
    solvers, states = _setup(dev, works, refs, precision)
    b = dev.Batch(solvers, states, flags)
    for k in (chunks or [steps]):
        b.run(k)
        if between is not None:
            between()
    torch.cuda.synchronize()
    info = b.info()
    b.close()
    return [s.download(*st) for s, st in zip(solvers, states)], info


def _err(got, ref):
    return max(O.rel_inf_error(got[0], ref[0]), O.rel_inf_error(got[1], ref[1]))


@pytest.mark.parametrize("precision,flags", [("f64", 0), ("f64", 2), ("f64", 3), ("f32", 0), ("f32", 2)],
                         ids=["f64", "f64_graph", "f64_tuned_graph", "f32", "f32_graph"])
def test_batch_matches_oracle(dev, mix_ref, precision, flags):
    got, info = _run_batch(dev, MIX, mix_ref, STEPS, precision, flags)
    for w, g, r in zip(MIX, got, mix_ref):
        e = _err(g, (r[2], r[3]))
        print(f"{w.name} {w.n} {precision} flags={flags}: rel inf err {e:.2e}")
        assert e <= TOL[precision], (w.name, e)
        if precision == "f32":
            assert e > 1e-15
    assert info[1] == bool(flags & dev.ADR_BATCH_GRAPH)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_alone_equals_in_mix(dev, mix_ref, precision):
    mixed, _ = _run_batch(dev, MIX, mix_ref, STEPS, precision)
    for k, w in enumerate(MIX):
        alone, _ = _run_batch(dev, [w], [mix_ref[k]], STEPS, precision)
        assert np.array_equal(alone[0][0], mixed[k][0]) and np.array_equal(alone[0][1], mixed[k][1]), w.name


def test_batch_graph_replays_equal_eager(dev, mix_ref):
    import torch

    def eager_work():
        x = torch.arange(1 << 20, device="cuda", dtype=torch.float64)
        torch.cuda.synchronize()
        assert float(x.sum()) == float((1 << 20) * ((1 << 20) - 1) // 2)

    eager, _ = _run_batch(dev, MIX, mix_ref, STEPS, "f64", 0)
    graph, info = _run_batch(dev, MIX, mix_ref, STEPS, "f64", dev.ADR_BATCH_GRAPH,
                             chunks=[1, 2, 1, 2], between=eager_work)
    assert info[1]
    for e, g in zip(eager, graph):
        assert np.array_equal(e[0], g[0]) and np.array_equal(e[1], g[1])


def test_batch_autotune(dev, mix_ref):
    import torch
    solvers, states = _setup(dev, MIX, mix_ref)
    b = dev.Batch(solvers, states, dev.ADR_BATCH_AUTOTUNE)
    torch.cuda.synchronize()
    cfgs, graph = b.info()
    assert not graph
    assert all(c in (0, 1, 2, 3, 4) for c in cfgs), cfgs
    # tuning writes workspace only
    for s, st, r in zip(solvers, states, mix_ref):
        U, V = s.download(*st)
        assert np.array_equal(U, r[0]) and np.array_equal(V, r[1])
    b.run(STEPS)
    torch.cuda.synchronize()
    tuned = [s.download(*st) for s, st in zip(solvers, states)]
    b.close()
    plain, _ = _run_batch(dev, MIX, mix_ref, STEPS, "f64", 0)
    for t, p in zip(tuned, plain):
        assert np.array_equal(t[0], p[0]) and np.array_equal(t[1], p[1])


@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4], ids=["64x64", "64x128", "128x64", "128x128", "64x64_persistent"])
def test_batch_every_tile_configuration(dev, mix_ref, cfg):
    # each configuration of the grouped FP64 product gives the plan's default
    # result bitwise (same summation order) and the oracle's within 1e-12
    plain, _ = _run_batch(dev, MIX, mix_ref, STEPS, "f64", 0)
    forced, info = _run_batch(dev, MIX, mix_ref, STEPS, "f64", dev.ADR_BATCH_TILE(cfg))
    assert all(c == cfg for c in info[0][:3]), info
    for w, f, p, r in zip(MIX, forced, plain, mix_ref):
        assert np.array_equal(f[0], p[0]) and np.array_equal(f[1], p[1]), w.name
        assert _err(f, (r[2], r[3])) <= TOL["f64"]


def test_batch_rejects_unsupported(dev, mix_ref):
    w = MIX[0]
    U0, V0, _, _, mats = mix_ref[0]
    s = dev.Solver(w, scheme="lawson2b", phis=mats)
    st = s.upload(U0, V0)
    with pytest.raises(dev.AdrError) as ei:
        dev.Batch([s], [st])
    assert ei.value.status == dev.ADR_ENOTSUP


@pytest.mark.parametrize("precision,steps", [("f64", 3), ("f32", 3)])
def test_batched_schnakenberg_64(dev, precision, steps):
    """The 64-instance workload (sides drawn from 64..512): every instance
    against the single-problem path, sampled instances against the oracle."""
    import torch
    works = S.batched_schnakenberg_2d(64, steps)
    refs = []
    for k, w in enumerate(works):
        U0, V0 = S.initial_state(w, 100 + k)
        refs.append((U0, V0, None, None, None))
    # matrix functions from the device (as a user would), shared by both paths
    solvers, states = [], []
    for w, r in zip(works, refs):
        s = dev.Solver(w, precision=precision)
        solvers.append(s)
        states.append(s.upload(r[0], r[1]))
    b = dev.Batch(solvers, states, dev.ADR_BATCH_GRAPH | (dev.ADR_BATCH_AUTOTUNE if precision == "f64" else 0))
    b.run(steps)
    torch.cuda.synchronize()
    b.close()
    got = [s.download(*st) for s, st in zip(solvers, states)]
    worst = 0.0
    for s, r, g in zip(solvers, refs, got):
        Ud, Vd = s.upload(r[0], r[1])
        s.solve(Ud, Vd, steps)
        torch.cuda.synchronize()
        single = s.download(Ud, Vd)
        worst = max(worst, _err(g, single))
    print(f"batch vs single-problem path ({precision}): max rel inf err {worst:.2e}")
    assert worst <= (1e-13 if precision == "f64" else 1e-6)
    sides = [w.n[0] for w in works]
    sample = sorted({int(np.argmax(sides)), int(np.argmin(sides)), 7})
    for k in sample:
        w = works[k]
        p = O.problem_from_workload(w)
        U, V = O.solve(refs[k][0], refs[k][1], p, steps, "etd2rkds", mats=O.precompute(p))
        e = _err(got[k], (U, V))
        print(f"instance {k} side {w.n[0]} ({precision}): rel inf err vs oracle {e:.2e}")
        assert e <= TOL[precision]


def test_destroy_right_after_async_run(dev, mix_ref):
    # plan A runs on a side stream and is destroyed at once, without a
    # synchronisation; plan B, built right after, may take A's pooled job-table
    # block.  destroy waits for A's queued steps first, so both stay exact.
    import torch
    side = torch.cuda.Stream()
    sa, sta = _setup(dev, MIX[:3] + MIX[6:], mix_ref[:3] + mix_ref[6:])
    torch.cuda.synchronize()
    a = dev.Batch(sa, sta, dev.ADR_BATCH_GRAPH, stream=side)
    a.run(STEPS)
    a.close()
    sb, stb = _setup(dev, MIX[3:6], mix_ref[3:6])
    b = dev.Batch(sb, stb)
    b.run(STEPS)
    torch.cuda.synchronize()
    b.close()
    for s, st, r in zip(sa + sb, sta + stb, mix_ref[:3] + mix_ref[6:] + mix_ref[3:6]):
        e = _err(s.download(*st), (r[2], r[3]))
        assert e <= TOL["f64"], (s.workload.name, e)
