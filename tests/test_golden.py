"""The oracle against its committed regression fixtures (tests/golden/,
written by tests/golden/make_golden.py from the oracle alone; the paper
prints no worked example to store instead)."""
import json
import os

import numpy as np
import pytest

from tests.golden import make_golden as mg

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def stored():
    with open(os.path.join(HERE, "oracle_regression.json")) as f:
        return json.load(f)


def test_c1_jk_unchanged(stored):
    now, ref = mg.c1_fixture(), stored["c1"]
    assert now["tr_PJ"] == pytest.approx(ref["tr_PJ"], rel=1e-13)
    assert now["tr_PK"] == pytest.approx(ref["tr_PK"], rel=1e-13)
    assert np.allclose(now["J_row0"], ref["J_row0"], rtol=0, atol=1e-13)
    assert np.allclose(now["K_row0"], ref["K_row0"], rtol=0, atol=1e-13)


def test_twocomp_energy_unchanged(stored):
    assert mg.twocomp_fixture()["E2_2c"] == pytest.approx(stored["twocomp"]["E2_2c"], rel=1e-12)


def test_boys_unchanged(stored):
    now = mg.boys_fixture()
    assert np.allclose(now["F"], stored["boys"]["F"], rtol=1e-15, atol=0)
