"""Pins of the oracle's residence-time and solvation-number sampler (Sec. 5,
Eqs. 7-8): straight-line motion whose shell occupancy is known by hand, with
and without the excursion tolerance, and a static FCC lattice."""
import numpy as np
import pytest

import oracle
from residence_cases import BALLISTIC_EXPECTED, BALLISTIC_SOLVATION, ballistic_system, fcc_system


@pytest.mark.parametrize("tol", [3, 2])
def test_ballistic_occupancy_windows(tol):
    o = oracle.md(ballistic_system(tol))
    np.testing.assert_allclose(o["res_acf"], BALLISTIC_EXPECTED[tol]["res_acf"], rtol=1e-15, atol=0)
    np.testing.assert_array_equal(o["res_cnt"], BALLISTIC_EXPECTED[tol]["res_cnt"])
    assert (o["solvation_sum"], o["solvation_cnt"]) == BALLISTIC_SOLVATION


def test_static_fcc_first_shell():
    o = oracle.md(fcc_system())
    # samples at steps 0, 2, 4, 6; one solute with 12 first-shell neighbours
    assert o["solvation_cnt"] == 4 and o["solvation_sum"] == 48
    # origins at 0, 2, 4, 6; lags 0..2; nobody moves, so every fraction is 1
    np.testing.assert_array_equal(o["res_cnt"], [4, 3, 2])
    np.testing.assert_array_equal(o["res_acf"], [4, 3, 2])
