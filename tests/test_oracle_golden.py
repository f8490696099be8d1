"""The oracle reproduces its frozen outputs (tests/golden/oracle_regression.json,
written by tests/golden/make_golden.py from the oracle alone)."""
import json
import os

import pytest

from tests.golden.make_golden import run_case

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name", ["c1_2000", "c2_300", "c1_single_order_seed5"])
def test_oracle_matches_golden(oracle, name):
    with open(os.path.join(HERE, "oracle_regression.json")) as f:
        gold = json.load(f)["cases"][name]
    got = run_case(gold["input"])
    exp = gold["output"]
    assert got["stats"] == exp["stats"]
    assert got["image_sum"] == pytest.approx(exp["image_sum"], rel=1e-12)
    assert got["grad_dot_beta"] == pytest.approx(exp["grad_dot_beta"], rel=1e-10, abs=1e-300)
    for (i, v), (j, w) in zip(got["image_top"], exp["image_top"]):
        assert i == j and v == pytest.approx(w, rel=1e-12)
    for (i, v), (j, w) in zip(got["grad_top"], exp["grad_top"]):
        assert i == j and v == pytest.approx(w, rel=1e-10)
