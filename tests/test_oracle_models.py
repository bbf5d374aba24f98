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
])
def test_equilibria(model, params, ue, ve):
    gu, gv = O.reaction(model, params, np.array([ue]), np.array([ve]))
    scale = max(abs(p) for p in params)
    assert abs(gu[0]) <= 1e-14 * scale and abs(gv[0]) <= 1e-14 * scale


@pytest.mark.parametrize("case", GOLD["points"], ids=lambda c: c["model"])
def test_hand_evaluated_points(case):
    gu, gv = O.reaction(case["model"], case["params"], np.array([case["u"]]), np.array([case["v"]]))
    assert gu[0] == pytest.approx(case["gu"], rel=1e-15, abs=1e-15)
    assert gv[0] == pytest.approx(case["gv"], rel=1e-15, abs=1e-15)
