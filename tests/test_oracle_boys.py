"""Pins of the oracle's Boys function F_m(T) = int_0^1 t^(2m) exp(-T t^2) dt
(the moment function behind the Rys weights of Section 2, eq. rys1) against
values fixed by mathematics, not by the oracle's own formula."""
import math

import mpmath
import numpy as np
import pytest

from oracle import oracle as o


def boys_mp(m, T):
    """Independent definition: F_m(T) = 1F1(m+1/2; m+3/2; -T) / (2m+1)."""
    with mpmath.workdps(40):
        return float(mpmath.hyp1f1(m + 0.5, m + 1.5, -mpmath.mpf(T)) / (2 * m + 1))


def test_boys_at_zero():
    F = o.boys(16, 0.0)
    for m in range(17):
        assert F[m] == pytest.approx(1.0 / (2 * m + 1), rel=1e-15)


@pytest.mark.parametrize("T", [1e-12, 1e-6, 0.01, 0.3, 1.0, 2.5, 7.0, 12.0, 19.9, 29.99, 30.0, 30.01, 45.0, 80.0, 300.0])
def test_boys_vs_mpmath(T):
    F = o.boys(16, T)
    for m in range(17):
        ref = boys_mp(m, T)
        assert abs(F[m] - ref) <= 2e-14 * ref, (m, T, F[m], ref)


def test_boys_large_T_closed_form():
    # F_m(T) -> (2m-1)!! / 2^(m+1) * sqrt(pi / T^(2m+1)) up to exp(-T) terms
    T = 200.0
    F = o.boys(12, T)
    for m in range(13):
        dfm = 1.0
        for k in range(2 * m - 1, 0, -2):
            dfm *= k
        ref = dfm / 2 ** (m + 1) * math.sqrt(math.pi / T ** (2 * m + 1))
        assert F[m] == pytest.approx(ref, rel=1e-14)


def test_boys_f0_is_erf():
    for T in (0.05, 0.7, 3.0, 11.0, 25.0, 40.0):
        ref = 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
        assert o.boys(0, T)[0] == pytest.approx(ref, rel=1e-14)


def test_boys_recursion_identity():
    # (2m+1) F_m(T) = 2T F_(m+1)(T) + exp(-T), checked between grid points
    for T in np.linspace(0.013, 60.0, 97):
        F = o.boys(14, T)
        for m in range(14):
            lhs = (2 * m + 1) * F[m]
            rhs = 2 * T * F[m + 1] + math.exp(-T)
            assert lhs == pytest.approx(rhs, rel=1e-13)
