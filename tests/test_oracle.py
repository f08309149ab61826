"""The CPU oracle against its pins (hand-worked values, closed forms, brute
force, library routines, invariants).  CPU only."""
import numpy as np
import pytest

import oracle
import oracle_pins as pins


@pytest.fixture(scope="module")
def orc():
    oracle.build(force=False)
    return oracle.default()


def test_golden(orc):
    pins.check_golden(orc)


def test_closed_forms(orc):
    pins.check_closed_forms(orc)


def test_brute_force(orc):
    pins.check_brute_force(orc)


def test_invariants(orc):
    pins.check_invariants(orc)


def test_cancellation(orc):
    pins.check_cancellation(orc)


def test_segmented(orc):
    pins.check_segmented(orc)


def test_bad_arguments(orc):
    with pytest.raises(ValueError):
        orc.scan(np.zeros(4, np.int32), "int32", 7)
    with pytest.raises(ValueError):
        orc.segscan(np.zeros(4, np.int32), np.array([1, 4]), "int32", "add")
    with pytest.raises(ValueError):
        orc.segscan(np.zeros(4, np.int32), np.array([0, 3, 2, 4]), "int32", "add")
    with pytest.raises(TypeError):
        orc.scan(np.zeros(4, np.float64), "float32", "add")


def test_error_ratio():
    y64 = np.array([0.0, 1.0, 3.0])
    a = np.array([0.0, 1.0, 3.0])
    assert oracle.float_error_ratio(np.array([0.0, 1.0, 3.0], np.float32), y64, a) == (0.0, 0)
    r, j = oracle.float_error_ratio(np.array([0.0, 1.5, 3.0], np.float32), y64, a)
    assert j == 1 and r == 0.5
    r, j = oracle.float_error_ratio(np.array([1e-30, 1.0, 3.0], np.float32), y64, a)
    assert r == float("inf") and j == 0
