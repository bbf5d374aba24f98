"""Pins of the error/order formulas against the orders printed in the paper's tables."""
import json
import os

import numpy as np
import pytest

import oracle as O

TAB = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


@pytest.mark.parametrize("key,scheme", [("table1_schnakenberg2d", "etd2rkds"),
                                        ("table5_schnakenberg3d", "etd2rkds"),
                                        ("table6_brusselator3d", "etd2rkds"),
                                        ("table6_brusselator3d", "lawson2b")])
def test_observed_order_reproduces_printed_orders(key, scheme):
    row = TAB[key][scheme]
    orders = O.observed_order(row["steps"], row["error"])
    assert np.allclose(np.round(orders, 2), row["order"], atol=0.011)


def test_relative_error_combines_components_in_two_norm():
    U = np.ones((3, 3)); V = 2 * np.ones((3, 3))
    # e_U = 0.1, e_V = 0.05*... chosen so the combined value is sqrt(0.1^2 + 0.2^2)
    err = O.relative_error(1.1 * U, 1.2 * V, U, V)
    assert err == pytest.approx(np.hypot(0.1, 0.2), rel=1e-14)


def test_rel_inf_error():
    assert O.rel_inf_error([1.0, 2.0], [1.0, 4.0]) == 0.5
    assert O.rel_inf_error([0.0], [0.0]) == 0.0
