"""Full-length GPU parity of the configured runs against the FP64 oracle.

* 3D FitzHugh-Nagumo 128^3, tau = 1e-3, 200 ETD2RKds steps (FP64), compared
  every 50 steps;
* 3D advective Brusselator 256^3, tau = 5e-3, 100 ETD2RKds steps, compared
  every 20 steps, in FP64 and with the Tucker products in FP32, in three-part
  split BF16 and in two-part split BF16, all against the same FP64 oracle
  trajectory.

The GPU runs are end to end, in the configuration the benchmark times: the
library builds the operators (adr_build_1d_ops) and their matrix functions
(adr_precompute_phi) itself.  Each checkpoint is a test of its own; the runs
advance lazily, so a checkpoint selected alone still starts from step 0.

Gates (relative infinity norm per component): FP64 1e-12; the reduced
precisions take the gates of tests/test_gpu_lowp.py (for this Brusselator:
FP32 1e-6, three-part split BF16 1e-5, two-part split BF16 1e-4).  The oracle
run with the Tucker directions reversed (tests/mode_order_drift.py) measures
how far rounding alone moves these trajectories; the FP64 gate lies above it.
"""
import numpy as np
import pytest

import oracle as O
import synth as S

pytestmark = pytest.mark.gpu

def _tol(prec, w):
    if prec == "f64":
        return 1e-12
    from test_gpu_lowp import tolerance
    return tolerance(prec, w)


class _Run:
    """One oracle trajectory and the GPU trajectories of several precisions
    from the same seeded initial state, advanced together to checkpoints."""

    def __init__(self, dev, w, precisions, seed=0):
        self.dev, self.w = dev, w
        self.p = O.problem_from_workload(w)
        self.mats = O.precompute(self.p)
        U0, V0 = S.initial_state(w, seed)
        self.ref, self.ref_step = (U0, V0), 0
        self.gpu = {}
        for prec in precisions:
            s = dev.Solver(w, precision=prec)
            self.gpu[prec] = [s, s.upload(U0, V0), 0]

    def oracle_at(self, step):
        assert step >= self.ref_step
        self.ref = O.solve(*self.ref, self.p, step - self.ref_step, mats=self.mats)
        self.ref_step = step
        return self.ref

    def gpu_at(self, prec, step):
        import torch
        entry = self.gpu[prec]
        s, (Ud, Vd), done = entry
        assert step >= done
        s.solve(Ud, Vd, step - done)
        torch.cuda.synchronize()
        entry[2] = step
        return s.download(Ud, Vd)


@pytest.fixture(scope="module")
def runs(dev):
    cache = {}
    yield cache
    cache.clear()
    import torch
    torch.cuda.empty_cache()


def _check(runs, dev, key, w, precisions, prec, step):
    if key not in runs:
        import torch
        runs.clear()                 # one configured run on the device at a time
        torch.cuda.empty_cache()
        runs[key] = _Run(dev, w, precisions)
    r = runs[key]
    U, V = r.oracle_at(step)
    Ug, Vg = r.gpu_at(prec, step)
    eu, ev = O.rel_inf_error(Ug, U), O.rel_inf_error(Vg, V)
    print(f"{key} {prec} step {step}: rel inf err u={eu:.3e} v={ev:.3e}")
    assert np.isfinite(Ug).all() and np.isfinite(Vg).all()
    assert eu <= _tol(prec, w) and ev <= _tol(prec, w), (eu, ev)
    if prec != "f64":
        assert max(eu, ev) > 1e-15   # the reduced precision really ran


FHN_STEPS = [50, 100, 150, 200]


@pytest.mark.parametrize("step", FHN_STEPS, ids=[f"step{k}" for k in FHN_STEPS])
def test_fhn_128_200_steps(dev, runs, step):
    w = S.fhn_3d()                                  # 128^3, tau = 1e-3, 200 steps
    assert w.n == (128, 128, 128) and w.steps == 200
    _check(runs, dev, "fhn3d_128", w, ("f64",), "f64", step)


BRUSS_PRECISIONS = ("f64", "f32", "bf16x3", "bf16x2")
BRUSS_CASES = [(k, prec) for k in (20, 40, 60, 80, 100) for prec in BRUSS_PRECISIONS]


@pytest.mark.parametrize("step,prec", BRUSS_CASES, ids=[f"{p}-step{k}" for k, p in BRUSS_CASES])
def test_brusselator_256_100_steps(dev, runs, step, prec):
    w = S.brusselator_3d()                          # 256^3, tau = 5e-3, 100 steps
    assert w.n == (256, 256, 256) and w.steps == 100
    _check(runs, dev, "brusselator3d_256", w, BRUSS_PRECISIONS, prec, step)
