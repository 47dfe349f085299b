"""Pins of the relative error of Sec. 4 (the measure every parity gate uses).

Each expected value is worked out by hand from the definition
sqrt(sum |u_a - u_d|^2 / sum |u_d|^2): a dropped square root, a denominator
taken from u_a instead of u_d, or a missing modulus changes every one of them.
"""
import numpy as np
import pytest

from oracle import rel_err


@pytest.mark.parametrize("eps", [1e-3, 0.5, -0.25, 2.0])
def test_scaled_copy_gives_the_scale(eps):
    # u_a = (1 + eps) u_d  ->  |eps| |u_d| / |u_d| = |eps|, for any u_d
    rng = np.random.default_rng(0)
    u_d = rng.standard_normal((7, 3)) + 1j * rng.standard_normal((7, 3))
    assert rel_err((1 + eps) * u_d, u_d) == pytest.approx(abs(eps), rel=1e-12)


def test_one_differing_entry():
    # u_d = (1, 1, 1, 1), u_a differs by 3 in one entry: sqrt(9 / 4) = 1.5
    # (no square root: 2.25; denominator from u_a: 3 / sqrt(19) = 0.688)
    u_d = np.ones(4, dtype=np.complex128)
    u_a = u_d.copy()
    u_a[2] += 3.0
    assert rel_err(u_a, u_d) == pytest.approx(1.5, rel=1e-15)


def test_complex_entries_use_the_modulus():
    # u_d = (1 + i, 2): sum |u_d|^2 = 2 + 4 = 6; the difference (0, i) has |.|^2 = 1
    u_d = np.array([1 + 1j, 2.0])
    u_a = np.array([1 + 1j, 2.0 + 1j])
    assert rel_err(u_a, u_d) == pytest.approx(np.sqrt(1.0 / 6.0), rel=1e-15)
    # a purely imaginary error of the same size as a real one counts the same
    assert rel_err(np.array([1 + 1j, 3.0]), u_d) == pytest.approx(np.sqrt(1.0 / 6.0), rel=1e-15)


def test_sums_run_over_all_columns():
    # two columns, errors 1 and 2 on norms^2 4 and 16: sqrt((1 + 4) / 20) = 0.5
    u_d = np.array([[2.0, 4.0]])
    u_a = np.array([[3.0, 6.0]])
    assert rel_err(u_a, u_d) == pytest.approx(0.5, rel=1e-15)


def test_identical_is_zero_and_is_symmetric_only_when_it_should_be():
    u = np.array([1.0, -2.0, 0.5j])
    assert rel_err(u, u) == 0.0
    # not symmetric: the reference norm is the denominator
    a, d = np.array([2.0]), np.array([1.0])
    assert rel_err(a, d) == pytest.approx(1.0)
    assert rel_err(d, a) == pytest.approx(0.5)
