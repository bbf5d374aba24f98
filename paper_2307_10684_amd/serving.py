"""Continuous-batching serving loop for ETD2RKds solves on one GPU.

Requests (a grid, a reaction model, a step size, a step count and initial
data) arrive over time.  The engine admits them by an HBM budget and a slot
limit, keeps each admitted solve's state tensors, operators and matrix
functions resident on the device, and advances every admitted solve together:
one grouped plan (``adr_batch_*``) steps all of them in ``2*d_max + 2``
launches per step, so the work of different requests overlaps inside the same
kernels.  The loop runs in rounds of at most ``max_chunk`` steps; a round
never takes a request past its step count, and a finished request's state is
copied back while the next round already runs.  Rounds are pipelined
``depth`` deep: while the device works on round k, the host admits new
arrivals (building their operators and matrix functions on a side stream) and
queues round k+1 with a plan that includes them.  Requests of very different
size run in separate lanes (plans on separate streams) so that a small
request is not held to the step rate of a large one.

The engine is pure scheduling logic.  The device work goes through a backend
object; ``GpuBackend`` below drives the HIP library, and the tests drive the
same engine with a CPU stand-in.

Backend protocol::

    footprint(job) -> int          device bytes the request holds while admitted
    admit(job) -> handle           allocate, build operators, matrix functions, upload state
    plan(handles) -> plan          grouped plan over the handles (in this order)
    launch(plan, steps, lane) -> token   enqueue `steps` steps of every member on the
                                   lane's stream
    fetch(handle, after) -> token  enqueue the download of a state after round `after`
    ready(token) -> bool           whether the token's work is done (no blocking)
    wait(token)                    block until the token's work is done
    result(handle) -> (U, V)       host arrays (after the fetch token completed)
    release(handle)                free the request's device memory
    release_plan(plan)             free a plan (no run of it is pending)
    solve_alone(handle, steps) -> token   (sequential reference path)

Optional: ``held() -> int`` device bytes the backend holds outside any request
(work areas kept until the process ends), and ``held_extra(job) -> int`` the
bytes admitting ``job`` would add to that for good (a kept work area that has
to grow).  The engine counts both against the budget.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Job:
    """One request.  ``workload`` carries the problem description (grid ``n``,
    ``domain``, ``diff``, ``vel_u``, ``vel_v``, ``model``, ``params``, ``tau``);
    ``initial`` returns the host initial state (U0, V0), first index fastest."""
    rid: int
    arrival: float                  # seconds after the stream starts
    workload: Any
    steps: int
    initial: Callable[[], tuple]
    # polled between rounds: once it returns True the request is dropped
    # (queued or running) and completes with status "cancelled"
    cancelled: Optional[Callable[[], bool]] = None

    @property
    def N(self) -> int:
        return int(np.prod(self.workload.n))


@dataclasses.dataclass
class Completion:
    rid: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    grid_points: int
    status: str = "ok"              # "ok", "rejected" (larger than the whole budget),
                                    # "failed" (set-up raised), "cancelled"
    result: Optional[tuple] = None
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def wait(self) -> float:
        return self.admitted - self.arrival


@dataclasses.dataclass
class _Slot:
    serial: int                     # admission order (identifies the slot in plans)
    job: Job
    handle: Any
    bytes: int
    admitted: float
    left: int                       # steps not yet enqueued


@dataclasses.dataclass
class _Round:
    token: Any
    plan: int                       # serial of the plan
    members: List[_Slot]
    steps: int
    finishing: List[_Slot]
    fetches: List[Any]


class _Lane:
    """Requests of one size class: their own plan, rounds and stream."""

    def __init__(self, index: int):
        self.index = index
        self.inflight: collections.deque = collections.deque()
        self.plan_id = None
        self.members = ()


def step_flops(workload) -> float:
    """Multiply-adds x 2 of one ETD2RKds step's four Tucker operators on the
    grid: 8 * N * sum(n_mu) (Sec. 3, eq. (11); Sec. 2 for the mode products)."""
    n = [int(x) for x in workload.n]
    return 8.0 * float(np.prod(n)) * float(sum(n))


class Engine:
    """Continuous batching over a backend (see the module docstring).

    Admitted requests are split into lanes by the work of one step
    (``lane_bounds``, ascending thresholds in flops; the default puts steps of
    4 GFLOP and more, about what fills the device for one step, in their own
    lane): each lane has its own
    plan, its own rounds and its own device stream, so small requests keep
    their own step rate beside large ones and their kernels fill the compute
    units that the large ones leave idle.  The loop polls the rounds in flight
    (``backend.ready``), so arrivals are admitted as soon as they come.
    """

    def __init__(self, backend, budget_bytes: int, max_active: int = 64, max_chunk: int = 32,
                 depth: int = 2, keep_results: bool = True,
                 lane_bounds: Sequence[float] = (4e9,),
                 poll_s: float = 2e-4,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        if budget_bytes <= 0 or max_active < 1 or max_chunk < 1 or depth < 1 or poll_s <= 0:
            raise ValueError("budget_bytes, max_active, max_chunk, depth and poll_s must be positive")
        if list(lane_bounds) != sorted(lane_bounds):
            raise ValueError("lane_bounds must be ascending")
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.max_chunk = int(max_chunk)
        self.depth = int(depth)
        self.keep_results = keep_results
        self.lane_bounds = [float(b) for b in lane_bounds]
        self.poll_s = float(poll_s)
        self.clock = clock
        self.sleep = sleep
        self.stats = {}

    def lane_of(self, job: Job) -> int:
        f = step_flops(job.workload)
        return sum(1 for b in self.lane_bounds if f >= b)

    def run(self, jobs: Sequence[Job]) -> List[Completion]:
        be = self.backend
        for j in jobs:
            if j.steps < 0:
                raise ValueError(f"request {j.rid}: negative step count")
        pending = collections.deque(sorted(jobs, key=lambda j: (j.arrival, j.rid)))
        queue: collections.deque = collections.deque()
        slots: List[_Slot] = []
        lanes = [_Lane(k) for k in range(len(self.lane_bounds) + 1)]
        lane_of_slot = {}
        done: List[Completion] = []
        used = 0
        peak_used = peak_active = rounds = nplans = 0
        serial = 0
        plans = {}                  # plan serial -> [backend plan, references]
        t0 = self.clock()

        def now():
            return self.clock() - t0

        def drop_plan(pid):
            plans[pid][1] -= 1
            if plans[pid][1] == 0:
                be.release_plan(plans.pop(pid)[0])

        def finish(s: _Slot, t: float, result=None, status="ok"):
            nonlocal used
            done.append(Completion(s.job.rid, s.job.arrival, s.admitted, t, s.job.steps,
                                   s.job.N, status, result))
            used -= s.bytes
            slots.remove(s)
            lane_of_slot.pop(s.serial, None)
            be.release(s.handle)

        def is_cancelled(job: Job) -> bool:
            return job.cancelled is not None and bool(job.cancelled())

        def in_flight(s: _Slot) -> bool:
            return any(s in r.members for ln in lanes for r in ln.inflight)

        while True:
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            # cancellations: queued requests leave at once; admitted ones once no
            # round that includes them is in flight
            for job in [j for j in queue if is_cancelled(j)]:
                queue.remove(job)
                done.append(Completion(job.rid, job.arrival, now(), now(), job.steps, job.N,
                                       "cancelled"))
            for sl in [x for x in slots if is_cancelled(x.job) and not in_flight(x)]:
                finish(sl, now(), None, "cancelled")
            # admission: first come, first served, while slots and budget allow; memory
            # the backend keeps for good (and its growth for this request) counts too
            while queue and len(slots) < self.max_active:
                job = queue[0]
                need = int(be.footprint(job))
                held = int(be.held()) if hasattr(be, "held") else 0
                extra = int(be.held_extra(job)) if hasattr(be, "held_extra") else 0
                if held + extra + need > self.budget:
                    queue.popleft()
                    done.append(Completion(job.rid, job.arrival, now(), now(), job.steps, job.N,
                                           "rejected"))
                    continue
                if held + extra + used + need > self.budget:
                    break
                queue.popleft()
                try:
                    handle = be.admit(job)
                except Exception as exc:   # a request that cannot be set up fails alone
                    done.append(Completion(job.rid, job.arrival, now(), now(), job.steps, job.N,
                                           "failed", error=f"{type(exc).__name__}: {exc}"))
                    continue
                used += need
                serial += 1
                s = _Slot(serial, job, handle, need, now(), job.steps)
                slots.append(s)
                lane_of_slot[s.serial] = self.lane_of(job)
                held_now = int(be.held()) if hasattr(be, "held") else 0
                peak_used = max(peak_used, used + held_now)
                peak_active = max(peak_active, len(slots))
                if job.steps == 0:
                    res = None
                    if self.keep_results:
                        tok = be.fetch(handle, None)
                        be.wait(tok)
                        res = be.result(handle)
                    finish(s, now(), res)

            progressed = False
            # completed rounds (oldest first in each lane)
            for ln in lanes:
                while ln.inflight:
                    r = ln.inflight[0]
                    if not (be.ready(r.token) and all(be.ready(f) for f in r.fetches)):
                        break
                    ln.inflight.popleft()
                    for s in r.finishing:
                        finish(s, now(), be.result(s.handle) if self.keep_results else None)
                    drop_plan(r.plan)
                    progressed = True
            # new rounds
            for ln in lanes:
                runnable = [s for s in slots if s.left > 0 and lane_of_slot[s.serial] == ln.index
                            and not is_cancelled(s.job)]
                if not runnable:
                    if ln.plan_id is not None:
                        drop_plan(ln.plan_id)
                        ln.plan_id, ln.members = None, ()
                    continue
                if len(ln.inflight) >= self.depth:
                    continue
                members = tuple(s.serial for s in runnable)
                if ln.plan_id is None or members != ln.members:
                    if ln.plan_id is not None:
                        drop_plan(ln.plan_id)
                    serial += 1
                    nplans += 1
                    ln.plan_id, ln.members = serial, members
                    plans[ln.plan_id] = [be.plan([s.handle for s in runnable]), 1]
                steps = min(self.max_chunk, min(s.left for s in runnable))
                token = be.launch(plans[ln.plan_id][0], steps, ln.index)
                plans[ln.plan_id][1] += 1
                rounds += 1
                for s in runnable:
                    s.left -= steps
                finishing = [s for s in runnable if s.left == 0]
                fetches = [be.fetch(s.handle, token) if self.keep_results else token
                           for s in finishing]
                ln.inflight.append(_Round(token, ln.plan_id, runnable, steps, finishing, fetches))
                progressed = True
            if progressed:
                continue
            if any(ln.inflight for ln in lanes):
                self.sleep(self.poll_s)
                continue
            if pending:
                self.sleep(max(0.0, pending[0].arrival - now()))
                continue
            if queue:   # nothing active, yet the head does not fit: cannot happen
                raise RuntimeError("admission stalled with an idle device")
            break
        assert not plans, "plans left behind"
        end = now()
        ok = [c for c in done if c.status == "ok"]
        lat = np.array([c.latency for c in ok]) if ok else np.zeros(1)
        gps = sum(c.steps * c.grid_points for c in ok)
        self.stats = {
            "requests": len(done),
            "rejected": sum(1 for c in done if c.status == "rejected"),
            "failed": sum(1 for c in done if c.status == "failed"),
            "cancelled": sum(1 for c in done if c.status == "cancelled"),
            "makespan_s": end, "grid_point_steps": gps,
            "throughput": gps / end if end > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_wait_s": float(np.mean([c.wait for c in ok])) if ok else 0.0,
            "peak_bytes": peak_used, "peak_active": peak_active,
            "held_bytes": int(be.held()) if hasattr(be, "held") else 0,
            "rounds": rounds, "plans_built": nplans, "lanes": len(lanes),
        }
        return sorted(done, key=lambda c: c.rid)


def run_sequential(backend, jobs: Sequence[Job], keep_results: bool = True,
                   clock: Callable[[], float] = time.perf_counter,
                   sleep: Callable[[float], None] = time.sleep):
    """The plain path for comparison: requests in arrival order, one at a time,
    each set up and solved alone (adr_solve), no batching or overlap."""
    t0 = clock()
    done = []
    for job in sorted(jobs, key=lambda j: (j.arrival, j.rid)):
        t = clock() - t0
        if job.arrival > t:
            sleep(job.arrival - t)
        admitted = clock() - t0
        h = backend.admit(job)
        tok = backend.solve_alone(h, job.steps)
        backend.wait(tok)
        res = None
        if keep_results:
            f = backend.fetch(h, tok)
            backend.wait(f)
            res = backend.result(h)
        done.append(Completion(job.rid, job.arrival, admitted, clock() - t0, job.steps, job.N,
                               "ok", res))
        backend.release(h)
    end = clock() - t0
    lat = np.array([c.latency for c in done]) if done else np.zeros(1)
    gps = sum(c.steps * c.grid_points for c in done)
    stats = {"requests": len(done), "makespan_s": end, "grid_point_steps": gps,
             "throughput": gps / end if end > 0 else 0.0,
             "p50_latency_s": float(np.percentile(lat, 50)),
             "p99_latency_s": float(np.percentile(lat, 99))}
    return done, stats


# ----------------------------------------------------------------------------- GPU backend

class _Handle:
    __slots__ = ("solver", "U", "V", "hostU", "hostV", "shape")


class GpuBackend:
    """Backend on the HIP library: per-request operators and matrix functions
    built on a set-up stream (adr_build_1d_ops; adr_precompute_phi_batch for
    the request's distinct matrices, two synchronisations), grouped
    plans (adr_batch_*) run on one compute stream per lane, results copied back
    on a copy stream into pinned host memory.  All streams have the default
    priority."""

    def __init__(self, precision: str = "f64", device: str = "cuda", graph: bool = False):
        import torch
        if precision not in ("f64", "f32"):
            raise ValueError("serving runs FP64 or FP32 products")
        self.torch = torch
        self.precision = precision
        self.device = device
        self.graph = graph          # capture each plan's step in a HIP graph
        self.lanes = {}             # lane -> compute stream (created on first use)
        self.setup = torch.cuda.Stream(device)
        self.copy = torch.cuda.Stream(device)
        # the matrix functions are computed in a work area the library keeps per
        # device and grows to the largest side it has seen (14 n^2 + 1 + count
        # doubles; see adr_precompute_phi_batch)
        self._phi_side = 0

    # the library's fixed work area of adr_precompute_phi_noalloc (held once the
    # library is loaded) plus the kept work area of the matrix-function precompute
    _NOALLOC_BYTES = 8 * (14 * 512 * 512 + 1)

    @staticmethod
    def _phi_area(side: int) -> int:
        return 8 * (14 * side * side + 1 + 6) if side > 0 else 0

    def held(self) -> int:
        return self._NOALLOC_BYTES + self._phi_area(self._phi_side)

    def held_extra(self, job: Job) -> int:
        side = max(int(x) for x in job.workload.n)
        return max(0, self._phi_area(side) - self._phi_area(self._phi_side))

    def _lane(self, lane: int):
        if lane not in self.lanes:
            self.lanes[lane] = self.torch.cuda.Stream(self.device)
        return self.lanes[lane]

    def footprint(self, job: Job) -> int:
        from . import workspace_bytes_for
        w = job.workload
        n = [int(x) for x in w.n]
        N = int(np.prod(n))
        ops = sum(2 * (4 * k * k + 3 * k) * 8 for k in n)   # per component: E, phi1, phi2, A, band
        return 2 * N * 8 + workspace_bytes_for(n, self.precision) + ops

    def admit(self, job: Job):
        from . import Solver, adr_batch_create, adr_batch_destroy
        torch = self.torch
        h = _Handle()
        with torch.cuda.stream(self.setup):
            s = Solver(job.workload, precision=self.precision, device=self.device,
                       stream=self.setup)
            U0, V0 = job.initial()
            h.U, h.V = s.upload(U0, V0)
        if self.precision == "f32":
            # a plan of one writes the FP32 matrix copies into the workspace once;
            # the serving plans then skip that (ADR_BATCH_PREPARED)
            p = adr_batch_create([s.problem], [h.U], [h.V], [s.work], 0, self.setup)
            adr_batch_destroy(p)
        self.setup.synchronize()
        self._phi_side = max(self._phi_side, max(int(x) for x in job.workload.n))
        h.solver = s
        h.shape = s.shape
        h.hostU = h.hostV = None
        return h

    def plan(self, handles):
        from . import ADR_BATCH_GRAPH, ADR_BATCH_PREPARED, adr_batch_create
        if len(handles) == 1:
            # a lane with one request steps it with the single-problem path, whose
            # tile shapes are chosen for that problem alone
            return ("single", handles[0])
        flags = ADR_BATCH_PREPARED if self.precision == "f32" else 0
        if self.graph:
            flags |= ADR_BATCH_GRAPH
        return adr_batch_create([h.solver.problem for h in handles], [h.U for h in handles],
                                [h.V for h in handles], [h.solver.work for h in handles], flags,
                                self.setup)

    def launch(self, plan, steps: int, lane: int = 0):
        from . import adr_batch_run, adr_solve
        st = self._lane(lane)
        if isinstance(plan, tuple):
            h = plan[1]
            adr_solve(h.solver.problem, h.U, h.V, steps, h.solver.work, st)
        else:
            adr_batch_run(plan, steps, st)
        ev = self.torch.cuda.Event()
        ev.record(st)
        return ev

    def solve_alone(self, h, steps: int):
        from . import adr_solve
        st = self._lane(0)
        adr_solve(h.solver.problem, h.U, h.V, steps, h.solver.work, st)
        ev = self.torch.cuda.Event()
        ev.record(st)
        return ev

    def fetch(self, h, after):
        torch = self.torch
        if after is not None:
            self.copy.wait_event(after)
        else:
            self.copy.wait_stream(self.setup)
        with torch.cuda.stream(self.copy):
            h.hostU = torch.empty(h.U.numel(), dtype=torch.float64, pin_memory=True)
            h.hostV = torch.empty(h.V.numel(), dtype=torch.float64, pin_memory=True)
            h.hostU.copy_(h.U, non_blocking=True)
            h.hostV.copy_(h.V, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(self.copy)
        return ev

    def ready(self, token) -> bool:
        return token.query()

    def wait(self, token):
        token.synchronize()

    def result(self, h):
        shape = tuple(h.shape)
        U = np.asfortranarray(h.hostU.numpy().reshape(shape, order="F").copy())
        V = np.asfortranarray(h.hostV.numpy().reshape(shape, order="F").copy())
        return U, V

    def release(self, h):
        h.solver = h.U = h.V = h.hostU = h.hostV = None

    def release_plan(self, plan):
        from . import adr_batch_destroy
        if not isinstance(plan, tuple):
            adr_batch_destroy(plan)
