"""Scheduling logic of the continuous-batching serving loop, on the CPU.

The engine (paper_2307_10684_amd.serving.Engine) is driven by a stand-in
backend that executes the steps with the FP64 oracle and models device time on
a virtual clock, so admission, HBM-budget accounting, slot limits, round
pipelining and result delivery are checked without a GPU.  The GPU backend is
exercised by tests/test_gpu_serving.py."""
import importlib.util
import os
import sys

import numpy as np
import pytest

import oracle as O
import synth as S

_spec = importlib.util.spec_from_file_location(
    "adr_serving", os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                "paper_2307_10684_amd", "serving.py"))
serving = importlib.util.module_from_spec(_spec)
sys.modules["adr_serving"] = serving
_spec.loader.exec_module(serving)   # pure Python: no library or GPU needed


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class FakeBackend:
    """Executes rounds with the oracle; one serial device whose time per round is
    cost * (grid points * steps) of the members."""

    def __init__(self, clock, cost=1e-6, setup=1e-4):
        self.clock, self.cost, self.setup = clock, cost, setup
        self.device_free = {}      # lane -> time its stream is free
        self.mem = 0
        self.peak_mem = 0
        self.live = 0
        self.peak_live = 0
        self.outstanding = set()
        self.peak_outstanding = 0
        self.rounds = []
        self.plans_alive = 0
        self._tok = 0

    def footprint(self, job):
        n = job.workload.n
        return 16 * job.N * 8 + 2 * sum(4 * k * k for k in n) * 8

    def admit(self, job):
        p = O.problem_from_workload(job.workload)
        U, V = job.initial()
        self.clock.t += self.setup
        self.mem += self.footprint(job)
        self.peak_mem = max(self.peak_mem, self.mem)
        self.live += 1
        self.peak_live = max(self.peak_live, self.live)
        return {"job": job, "p": p, "mats": O.precompute(p), "U": U.copy(), "V": V.copy(),
                "steps": 0, "out": None, "released": False}

    def plan(self, handles):
        self.plans_alive += 1
        return list(handles)

    def _round(self, plan, steps, lane=0):
        for h in plan:
            assert not h["released"], "a released request was launched"
            for _ in range(steps):
                h["U"], h["V"] = O.etd2rkds_step(h["U"], h["V"], h["p"], h["mats"])
            h["steps"] += steps
        start = max(self.device_free.get(lane, 0.0), self.clock.t)
        self.device_free[lane] = start + self.cost * steps * sum(h["job"].N for h in plan)
        self._tok += 1
        tok = ("round", self._tok, self.device_free[lane])
        self.outstanding.add(tok[1])
        self.peak_outstanding = max(self.peak_outstanding, len(self.outstanding))
        self.rounds.append(([h["job"].rid for h in plan], steps, lane))
        return tok

    def launch(self, plan, steps, lane=0):
        return self._round(plan, steps, lane)

    def solve_alone(self, h, steps):
        return self._round([h], steps)

    def fetch(self, h, after):
        h["out"] = (h["U"].copy(), h["V"].copy())
        return ("fetch", None, after[2] if after else self.clock.t)

    def ready(self, token):
        done = self.clock.t >= token[2]
        if done and token[0] == "round":
            self.outstanding.discard(token[1])
        return done

    def wait(self, token):
        if token[0] == "round":
            self.outstanding.discard(token[1])
        self.clock.t = max(self.clock.t, token[2])

    def result(self, h):
        return h["out"]

    def release(self, h):
        assert not h["released"]
        h["released"] = True
        self.mem -= self.footprint(h["job"])
        self.live -= 1

    def release_plan(self, plan):
        self.plans_alive -= 1


def _jobs(count=8, seed=0, spacing=0.002, steps=(3, 13)):
    rng = np.random.default_rng(seed)
    shapes = [(8, 8), (10, 7), (6, 6, 6), (5, 7, 6), (12,)]
    makers = [S.schnakenberg_2d, S.fhn_3d, S.brusselator_3d]
    jobs = []
    t = 0.0
    for k in range(count):
        t += float(rng.exponential(spacing))
        shape = shapes[int(rng.integers(len(shapes)))]
        w = S.with_shape(makers[int(rng.integers(3))](), shape)
        w = w.replace(tau=float(rng.uniform(1e-4, 5e-3)))
        nsteps = int(rng.integers(steps[0], steps[1]))
        seed_k = int(rng.integers(1 << 20))
        jobs.append(serving.Job(k, t, w, nsteps, lambda w=w, s=seed_k: S.initial_state(w, s)))
    return jobs


def _alone(job):
    p = O.problem_from_workload(job.workload)
    mats = O.precompute(p)
    U, V = job.initial()
    for _ in range(job.steps):
        U, V = O.etd2rkds_step(U, V, p, mats)
    return U, V


def _engine(clock, be, **kw):
    kw.setdefault("budget_bytes", 1 << 30)
    return serving.Engine(be, clock=clock, sleep=clock.sleep, **kw)


def test_every_result_equals_the_request_solved_alone():
    clock = Clock()
    be = FakeBackend(clock)
    jobs = _jobs(10)
    eng = _engine(clock, be, max_chunk=4)
    done = eng.run(jobs)
    assert [c.rid for c in done] == list(range(10))
    for c, j in zip(done, jobs):
        assert c.status == "ok"
        U, V = _alone(j)
        assert np.array_equal(c.result[0], U) and np.array_equal(c.result[1], V)
        assert j.arrival <= c.admitted <= c.finished
    assert be.live == 0 and be.mem == 0 and be.plans_alive == 0
    assert eng.stats["grid_point_steps"] == sum(j.steps * j.N for j in jobs)


def test_requests_join_while_others_run():
    clock = Clock()
    be = FakeBackend(clock, cost=2e-6)
    jobs = _jobs(8, seed=1, spacing=0.001)
    done = _engine(clock, be, max_chunk=2).run(jobs)
    # some round holds several requests, and some request joined a running mix
    assert max(len(r[0]) for r in be.rounds) >= 3
    joined = any(a.admitted > b.admitted and a.admitted < b.finished
                 for a in done for b in done if a.rid != b.rid)
    assert joined
    # no round takes a request past its step count (results equal alone)
    for c, j in zip(done, jobs):
        U, _ = _alone(j)
        assert np.array_equal(c.result[0], U)


def test_budget_is_never_exceeded_and_excess_requests_wait():
    clock = Clock()
    be = FakeBackend(clock)
    jobs = _jobs(10, seed=2, spacing=1e-4)
    budget = 2 * max(be.footprint(j) for j in jobs)
    eng = _engine(clock, be, budget_bytes=budget, max_chunk=3)
    done = eng.run(jobs)
    assert all(c.status == "ok" for c in done)
    assert be.peak_mem <= budget and eng.stats["peak_bytes"] <= budget
    assert max(c.wait for c in done) > 0.0       # some request was queued, none failed
    # first come, first served
    order = [c.rid for c in sorted(done, key=lambda c: (c.admitted, c.rid))]
    assert order == sorted(order)


def test_slot_limit_and_pipeline_depth():
    clock = Clock()
    be = FakeBackend(clock)
    eng = _engine(clock, be, max_active=3, depth=2, max_chunk=2)
    eng.run(_jobs(9, seed=3, spacing=1e-5))
    assert be.peak_live <= 3 and eng.stats["peak_active"] <= 3
    assert be.peak_outstanding <= 2


def test_lanes_separate_small_and_large_requests():
    clock = Clock()
    be = FakeBackend(clock)
    jobs = _jobs(10, seed=7, spacing=1e-4)
    flops = sorted(serving.step_flops(j.workload) for j in jobs)
    bound = flops[len(flops) // 2]
    eng = _engine(clock, be, lane_bounds=[bound], max_chunk=3)
    done = eng.run(jobs)
    lane = {j.rid: int(serving.step_flops(j.workload) >= bound) for j in jobs}
    for members, _, ln in be.rounds:
        assert all(lane[r] == ln for r in members)
    assert {ln for _, _, ln in be.rounds} == {0, 1}
    for c, j in zip(done, jobs):
        U, V = _alone(j)
        assert np.array_equal(c.result[0], U) and np.array_equal(c.result[1], V)
    assert be.plans_alive == 0 and be.live == 0
    with pytest.raises(ValueError):
        _engine(clock, be, lane_bounds=[2.0, 1.0])


def test_request_larger_than_the_budget_is_rejected_not_stalled():
    clock = Clock()
    be = FakeBackend(clock)
    jobs = _jobs(4, seed=4)
    big = S.with_shape(S.fhn_3d(), (40, 40, 40))
    jobs.append(serving.Job(99, 0.0005, big, 5, lambda: S.initial_state(big, 0)))
    budget = max(be.footprint(j) for j in jobs[:4]) * 2
    done = _engine(clock, be, budget_bytes=budget).run(jobs)
    st = {c.rid: c.status for c in done}
    assert st[99] == "rejected"
    assert all(st[k] == "ok" for k in range(4))


def test_zero_steps_returns_the_initial_state():
    clock = Clock()
    be = FakeBackend(clock)
    jobs = _jobs(3, seed=5)
    w = S.with_shape(S.schnakenberg_2d(), (9, 9))
    jobs.append(serving.Job(7, 0.0, w, 0, lambda: S.initial_state(w, 3)))
    done = {c.rid: c for c in _engine(clock, be).run(jobs)}
    U0, V0 = S.initial_state(w, 3)
    assert np.array_equal(done[7].result[0], U0) and np.array_equal(done[7].result[1], V0)


def test_negative_steps_and_bad_settings_raise():
    clock = Clock()
    be = FakeBackend(clock)
    w = S.with_shape(S.schnakenberg_2d(), (9, 9))
    with pytest.raises(ValueError):
        _engine(clock, be).run([serving.Job(0, 0.0, w, -1, lambda: S.initial_state(w, 0))])
    with pytest.raises(ValueError):
        _engine(clock, be, max_chunk=0)


def test_sequential_path_matches_and_batching_lowers_latency():
    jobs = _jobs(8, seed=6, spacing=1e-4, steps=(4, 9))
    c1 = Clock()
    be1 = FakeBackend(c1, cost=1e-5, setup=0.0)
    seq, seq_stats = serving.run_sequential(be1, jobs, clock=c1, sleep=c1.sleep)
    c2 = Clock()
    be2 = FakeBackend(c2, cost=1e-5, setup=0.0)
    eng = _engine(c2, be2, max_chunk=4)
    mix = eng.run(jobs)
    for a, b in zip(seq, mix):
        assert np.array_equal(a.result[0], b.result[0]) and np.array_equal(a.result[1], b.result[1])
    assert seq_stats["grid_point_steps"] == eng.stats["grid_point_steps"]
    # the model device is serial, so batching cannot be faster in total, but the
    # short requests no longer wait behind long ones
    assert eng.stats["p50_latency_s"] <= seq_stats["p50_latency_s"] * 1.5


class FailingBackend(FakeBackend):
    """Set-up of the listed requests raises (as a device allocation might)."""

    def __init__(self, clock, fail_rids, **kw):
        super().__init__(clock, **kw)
        self.fail_rids = set(fail_rids)

    def admit(self, job):
        if job.rid in self.fail_rids:
            raise MemoryError(f"no device memory for request {job.rid}")
        return super().admit(job)


def test_a_failed_setup_fails_alone():
    clock = Clock()
    be = FailingBackend(clock, fail_rids={2, 5})
    jobs = _jobs(8, seed=8)
    done = {c.rid: c for c in _engine(clock, be, max_chunk=3).run(jobs)}
    assert done[2].status == "failed" and "MemoryError" in done[2].error
    assert done[5].status == "failed"
    for j in jobs:
        if j.rid in (2, 5):
            continue
        U, V = _alone(j)
        assert done[j.rid].status == "ok"
        assert np.array_equal(done[j.rid].result[0], U) and np.array_equal(done[j.rid].result[1], V)
    assert be.live == 0 and be.mem == 0 and be.plans_alive == 0


def test_cancellation_of_running_and_queued_requests():
    clock = Clock()
    be = FakeBackend(clock, cost=1e-5)
    jobs = _jobs(6, seed=9, spacing=1e-4, steps=(20, 30))
    t_cut = 0.004
    # a running request cancelled mid-run, and one cancelled while still queued
    jobs[1].cancelled = lambda: clock.t > t_cut
    late = S.with_shape(S.schnakenberg_2d(), (9, 9))
    jobs.append(serving.Job(50, 0.01, late, 5, lambda: S.initial_state(late, 1),
                            cancelled=lambda: True))
    eng = _engine(clock, be, max_chunk=2)
    done = {c.rid: c for c in eng.run(jobs)}
    assert done[1].status == "cancelled" and done[1].result is None
    assert done[50].status == "cancelled"
    assert eng.stats["cancelled"] == 2
    steps_run = {}
    for members, steps, _ in be.rounds:
        for r in members:
            steps_run[r] = steps_run.get(r, 0) + steps
    assert 0 < steps_run.get(1, 0) < jobs[1].steps      # it ran, then stopped
    assert 50 not in steps_run                          # never admitted to a round
    for j in jobs:
        if j.rid in (1, 50):
            continue
        U, V = _alone(j)
        assert done[j.rid].status == "ok"
        assert np.array_equal(done[j.rid].result[0], U) and np.array_equal(done[j.rid].result[1], V)
    assert be.live == 0 and be.mem == 0 and be.plans_alive == 0


class HeldBackend(FakeBackend):
    """A backend that keeps a work area growing with the largest grid side it
    has set up (like the library's matrix-function scratch) and a fixed one."""

    def __init__(self, clock, base=10_000, per_side2=100, **kw):
        super().__init__(clock, **kw)
        self.base, self.per_side2, self.side = base, per_side2, 0

    def _area(self, side):
        return self.per_side2 * side * side

    def held(self):
        return self.base + self._area(self.side)

    def held_extra(self, job):
        side = max(job.workload.n)
        return max(0, self._area(side) - self._area(self.side))

    def admit(self, job):
        h = super().admit(job)
        self.side = max(self.side, max(job.workload.n))
        return h


def test_held_memory_counts_against_the_budget():
    # the kept work area is part of every admission check: with it the device
    # never goes over the budget, and a request whose growth of the area cannot
    # fit even on an empty device is rejected
    clock = Clock()
    be = HeldBackend(clock, cost=1e-7)
    small_w = S.with_shape(S.schnakenberg_2d(), (16, 16))
    small = [serving.Job(k, 0.0, small_w, 3, lambda: S.initial_state(small_w, 0))
             for k in range(4)]
    big_w = S.with_shape(S.schnakenberg_2d(), (40, 40))
    big = serving.Job(9, 0.0, big_w, 2, lambda: S.initial_state(big_w, 0))
    fp_small = be.footprint(small[0])
    # three small requests fit the budget, but not beside the held memory
    budget = be.base + be._area(16) + 3 * fp_small - 1
    assert 3 * fp_small <= budget
    eng = serving.Engine(be, budget_bytes=budget, max_active=8, max_chunk=2,
                         clock=clock, sleep=clock.sleep)
    done = eng.run(small + [big])
    status = {c.rid: c.status for c in done}
    assert status[9] == "rejected"                      # 100 * 40^2 alone exceeds the budget
    assert all(status[k] == "ok" for k in range(4))
    assert be.peak_mem + be.held() <= budget
    assert eng.stats["peak_bytes"] <= budget and eng.stats["held_bytes"] == be.held()
    # counting the held memory, two small requests run at once, not three
    assert eng.stats["peak_active"] == 2
