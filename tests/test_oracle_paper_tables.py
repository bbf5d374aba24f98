"""Weak pins of the whole oracle against the errors printed in Tables 4 and 6.

The advective Brusselator experiment has deterministic initial data, so the
oracle can rerun it: 64^3 grid, T = 1, errors of ETD2RKds and Lawson2b against
a reference run with many more steps.  Matching the printed errors pins the
grid convention, the boundary rows, the matrix functions, the reaction terms
and the structure of both schemes at once.  The paper does not state the
reference step count; here the reference is a Richardson extrapolation of
two fine runs, so that its own error is third order.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import synth as S

TAB = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def _run(steps, scheme="etd2rkds"):
    w = S.paper_brusselator_3d(64, steps=steps)
    p = O.problem_from_workload(w)
    U0, V0 = S.initial_state(w)
    return O.solve(U0, V0, p, steps, scheme)


def _reference(s1, s2):
    U1, V1 = _run(s1)
    U2, V2 = _run(s2)
    return (4 * U2 - U1) / 3, (4 * V2 - V1) / 3


def test_table6_etd2rkds_first_row():
    row = TAB["table6_brusselator3d"]["etd2rkds"]
    Ur, Vr = _reference(200, 400)
    err = O.relative_error(*_run(50), Ur, Vr)
    assert err == pytest.approx(row["error"][0], rel=0.01)


@pytest.mark.slow
@pytest.mark.parametrize("scheme", ["etd2rkds", "lawson2b"])
def test_table6_all_rows(scheme):
    row = TAB["table6_brusselator3d"][scheme]
    Ur, Vr = _reference(800, 1600)
    errs = [O.relative_error(*_run(s, scheme), Ur, Vr) for s in row["steps"]]
    for got, want in zip(errs, row["error"]):
        assert got == pytest.approx(want, rel=0.01)
    assert np.allclose(np.round(O.observed_order(row["steps"], errs), 2), row["order"], atol=0.02)


@pytest.mark.slow
def test_table4_dib_etd2rkds():
    """Sec. 4.4 / Table 4: DIB model on 200^2, T = 2.5.  The paper's noise comes
    from MATLAB's generator (seed 123), which is not reproduced; with seeded
    noise of the same law the errors agree to within 10% and the orders to
    0.05 (measured: 1.18e-2, 8.12e-3, 5.94e-3, 4.53e-3; orders 2.03)."""
    row = TAB["table4_dib2d"]["etd2rkds"]

    def run(steps):
        w = S.dib_2d(200, steps)
        p = O.problem_from_workload(w)
        U0, V0 = S.initial_state(w, 123)
        return O.solve(U0, V0, p, steps)

    U1, V1 = run(4000)
    U2, V2 = run(8000)
    Ur, Vr = (4 * U2 - U1) / 3, (4 * V2 - V1) / 3
    errs = [O.relative_error(*run(s), Ur, Vr) for s in row["steps"]]
    for got, want in zip(errs, row["error"]):
        assert got == pytest.approx(want, rel=0.10)
    assert np.allclose(O.observed_order(row["steps"], errs), row["order"], atol=0.05)
