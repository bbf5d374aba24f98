"""Pins of the reaction terms: equilibria stated in the paper and hand-evaluated points."""
import json
import os

import numpy as np
import pytest

import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "reaction_points.json")))


@pytest.mark.parametrize("model,params,ue,ve", [
    # Sec. 4.1: (a + b, b/(a+b)^2)
    ("schnakenberg", (200.0, 0.1, 0.9), 1.0, 0.9),
    ("schnakenberg", (1000.0, 0.1305, 0.7695), 0.9, 0.7695 / 0.81),
    # Sec. 4.3: (0, 0)
    ("fhn", (24.649, 11.0, 0.1, 0.0), 0.0, 0.0),
    ("fhn", (1.0, 0.1, 2.0, 0.0), 0.0, 0.0),
    # Sec. 4.6: (a_2, a_1/a_2) = (A, B/A)
    ("brusselator", (2.0, 1.0), 2.0, 0.5),
    ("brusselator", (1.0, 3.0), 1.0, 3.0),
    # Sec. 4.4: (0, a_4^u), with a_4^v chosen by the formula printed there
    ("dib", (6.25, 10.0, 1.0, 66.0, 0.5, 3.0, 2.5, 0.2,
             3.0 * 0.5 * (1 - 0.2 + 0.2 * 0.5) / (0.5 * (1 + 0.2 * 0.5)), 1.5), 0.0, 0.5),
])
def test_equilibria(model, params, ue, ve):
    gu, gv = O.reaction(model, params, np.array([ue]), np.array([ve]))
    scale = max(abs(p) for p in params)
    assert abs(gu[0]) <= 1e-14 * scale and abs(gv[0]) <= 1e-14 * scale


@pytest.mark.parametrize("case", GOLD["points"], ids=lambda c: c["model"])
def test_hand_evaluated_points(case):
    # values worked out by hand from the model equations (arithmetic in the fixture)
    gu, gv = O.reaction(case["model"], case["params"], np.array([case["u"]]), np.array([case["v"]]))
    assert gu[0] == pytest.approx(case["gu"], rel=1e-15, abs=1e-15)
    assert gv[0] == pytest.approx(case["gv"], rel=1e-15, abs=1e-15)


def test_dib_a4v_of_the_workload_makes_the_equilibrium():
    import synth as S
    w = S.dib_2d(16)
    gu, gv = O.reaction("dib", w.params, np.array([w.base[0]]), np.array([w.base[1]]))
    assert abs(gu[0]) <= 1e-13 and abs(gv[0]) <= 1e-13
    # and it is not an equilibrium for a perturbed a_4^v
    p = list(w.params)
    p[8] *= 1.01
    _, gv2 = O.reaction("dib", p, np.array([0.0]), np.array([0.5]))
    assert abs(gv2[0]) > 1e-3
