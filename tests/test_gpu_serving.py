"""The continuous-batching serving loop on the GPU (GpuBackend + Engine).

A stream of mixed 1D/2D/3D requests with different models, step sizes and
step counts arrives while others run; each result must equal the result of
the same request served alone, and match the FP64 oracle, within the stated
tolerance: <= 1e-12 relative infinity norm per component for FP64; for FP32
products the rounding bound of the d length-n_mu dot products,
sum_mu n_mu * 2^-24 (at least 1e-6), since the requests here draw tau up to
5e-3 and the increments are then a large part of the state.  (Rounds of a
lane with several requests run the grouped kernels; a lane with one request
runs the single-problem kernels, which round the addends in another order,
so results agree to rounding, not bitwise.)  A tight HBM budget makes
requests queue without changing any result beyond that tolerance."""
import numpy as np
import pytest

import oracle as O
import synth as S

pytestmark = pytest.mark.gpu


def _stream(serving, count=8, seed=0):
    rng = np.random.default_rng(seed)
    shapes = [(64, 64), (96, 80), (24, 24, 24), (32, 28, 20), (200,), (48, 48)]
    makers = [S.schnakenberg_2d, S.fhn_3d, S.brusselator_3d]
    jobs = []
    t = 0.0
    for k in range(count):
        t += float(rng.exponential(0.004))
        w = S.with_shape(makers[k % 3](), shapes[k % len(shapes)])
        w = w.replace(tau=float(np.exp(rng.uniform(np.log(1e-4), np.log(5e-3)))))
        steps = int(rng.integers(5, 26))
        sd = int(rng.integers(1 << 20))
        jobs.append(serving.Job(k, t, w, steps, lambda w=w, s=sd: S.initial_state(w, s)))
    return jobs


def _oracle(job):
    p = O.problem_from_workload(job.workload)
    U, V = job.initial()
    return O.solve(U, V, p, job.steps, "etd2rkds", mats=O.precompute(p))


def _err(a, b):
    return max(O.rel_inf_error(a[0], b[0]), O.rel_inf_error(a[1], b[1]))


@pytest.fixture(scope="module")
def serving(dev):
    from paper_2307_10684_amd import serving as sv
    return sv


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_serving_mix_equals_alone_and_oracle(serving, precision):
    jobs = _stream(serving)
    be = serving.GpuBackend(precision)
    eng = serving.Engine(be, budget_bytes=8 << 30, max_chunk=4)
    mix = eng.run(jobs)
    st = eng.stats
    print(f"{precision}: {st}")
    assert st["peak_active"] >= 3, "requests did not overlap"
    assert all(c.status == "ok" for c in mix)
    for c, j in zip(mix, jobs):
        tol = 1e-12 if precision == "f64" else max(1e-6, sum(j.workload.n) * 2.0 ** -24)
        alone = serving.Engine(be, budget_bytes=8 << 30, max_chunk=7).run([j])[0]
        assert _err(alone.result, c.result) <= tol, j.workload.name
        e = _err(c.result, _oracle(j))
        print(f"request {j.rid} {j.workload.n} {j.steps} steps: rel inf err {e:.2e}")
        assert e <= tol


def test_serving_tight_budget_queues_without_changing_results(serving):
    jobs = _stream(serving, seed=1)
    be = serving.GpuBackend("f64")
    free = serving.Engine(be, budget_bytes=8 << 30, max_chunk=5).run(jobs)
    # room for two requests beside the memory the backend holds for good (its
    # work areas, grown to the largest side by the first run)
    assert all(be.held_extra(j) == 0 for j in jobs)
    budget = be.held() + 2 * max(be.footprint(j) for j in jobs)
    eng = serving.Engine(be, budget_bytes=budget, max_chunk=5)
    tight = eng.run(jobs)
    assert all(c.status == "ok" for c in tight)
    assert eng.stats["peak_bytes"] <= budget
    assert max(c.wait for c in tight) > 0.0
    for a, b in zip(free, tight):
        assert _err(a.result, b.result) <= 1e-12


def test_sequential_plain_path_agrees(serving):
    jobs = _stream(serving, count=5, seed=2)
    be = serving.GpuBackend("f64")
    seq, stats = serving.run_sequential(be, jobs)
    mix = serving.Engine(be, budget_bytes=8 << 30).run(jobs)
    for a, b in zip(seq, mix):
        assert _err(a.result, b.result) <= 1e-13
    assert stats["grid_point_steps"] == sum(j.steps * j.N for j in jobs)
