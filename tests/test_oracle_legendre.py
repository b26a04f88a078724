"""Pins of the oracle's Legendre functions against things other than itself.

Each test fixes a part of Sec. 2.1 / Algorithm 2 that a plausible mistake
would break: the recurrence sign of Eq. (assLegRec), the seed exponent of
Eq. (pmm), the coefficient of Eq. (pm1m), the normalisation, the phase
convention and the rescaling of Sec. 2.2.2.
"""
import math
from fractions import Fraction
from math import factorial

import mpmath
import numpy as np
import pytest
import scipy.special as sps

from oracle import ref

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _xs(theta):
    return math.cos(theta), math.sin(theta)


def _xs_consistent(theta):
    # x as a double, s = sqrt(1 - x^2) correctly rounded from that x, so that
    # the pair is consistent to half an ulp of s (near the poles the ulp of x
    # alone moves P_l0 by l(l+1)/2 ulp)
    x = math.cos(theta)
    mpmath.mp.dps = 40
    return x, float(mpmath.sqrt(1 - mpmath.mpf(x) ** 2))


def test_mu_matches_printed_factorial_formula():
    # Eq. (pmm): mu_m = sqrt((2m+1)!/(4 pi)) / (2^m m!), exact big-integer form
    mu = ref.mu(300)
    mpmath.mp.dps = 50
    for m in [0, 1, 2, 3, 10, 57, 100, 299, 300]:
        exact = mpmath.sqrt(mpmath.mpf(factorial(2 * m + 1)) / (4 * mpmath.pi)) / (
            mpmath.mpf(2) ** m * factorial(m))
        assert abs(mu[m] / float(exact) - 1) < 1e-14 * (1 + m / 10)


@pytest.mark.parametrize("theta", [0.0, 1e-3, 0.4, 1.1, math.pi / 2, 2.5, math.pi - 1e-2])
def test_closed_forms_low_degree(theta):
    # Y_00, Y_10 ~ cos, Y_11 ~ sin and the l = 2 row, no Condon-Shortley phase
    x, s = _xs(theta)
    pi = math.pi
    exp = {
        (0, 0): 1 / math.sqrt(4 * pi),
        (1, 0): math.sqrt(3 / (4 * pi)) * x,
        (1, 1): math.sqrt(3 / (8 * pi)) * s,
        (2, 0): math.sqrt(5 / (4 * pi)) * (3 * x * x - 1) / 2,
        (2, 1): math.sqrt(15 / (8 * pi)) * x * s,
        (2, 2): math.sqrt(15 / (32 * pi)) * s * s,
        (3, 3): math.sqrt(35 / (64 * pi)) * s ** 3,
        (3, 2): math.sqrt(105 / (32 * pi)) * x * s * s,
    }
    for (l, m), v in exp.items():
        got = ref.legendre(3, m, x, s)[l]
        assert abs(got - v) <= 1.5e-15 * max(1.0, abs(v)), (l, m, got, v)


def _equator_value(l, m):
    # P_lm(0) of the orthonormal functions, exact rational inside the sqrt
    if (l + m) % 2:
        return 0.0
    num = Fraction(factorial(l - m) * factorial(l + m))
    den = Fraction((2 ** l * factorial((l - m) // 2) * factorial((l + m) // 2)) ** 2)
    sign = -1 if ((l - m) // 2) % 2 else 1
    return sign * math.sqrt((2 * l + 1) / (4 * math.pi)) * math.sqrt(num / den)


def test_equator_closed_form():
    for m in [0, 1, 2, 5, 12, 31]:
        lam = ref.legendre(60, m, 0.0, 1.0)
        for l in range(m, 61):
            v = _equator_value(l, m)
            assert abs(lam[l] - v) <= 2e-15 * max(1.0, abs(v)) + 1e-300, (l, m)


@pytest.mark.parametrize("theta", [3e-4, 1e-3, 0.05, 0.3, 1.2, math.pi / 2, 2.0, 3.0])
def test_addition_theorem(theta):
    # sum_m |Y_lm|^2 = (2l+1)/(4 pi): P_l0^2 + 2 sum_{m>=1} P_lm^2
    L = 1024
    x, s = _xs_consistent(theta)
    tot = np.zeros(L + 1)
    for m in range(L + 1):
        lam = ref.legendre(L, m, x, s)
        tot += (1.0 if m == 0 else 2.0) * lam * lam
    ell = np.arange(L + 1)
    err = np.max(np.abs(tot / ((2 * ell + 1) / (4 * np.pi)) - 1))
    assert err < 2e-11, err


@pytest.mark.slow
def test_addition_theorem_l4096():
    L = 4096
    for theta in [4e-4, 0.7]:
        x, s = _xs_consistent(theta)
        tot = np.zeros(L + 1)
        for m in range(L + 1):
            lam = ref.legendre(L, m, x, s)
            tot += (1.0 if m == 0 else 2.0) * lam * lam
        ell = np.arange(L + 1)
        err = np.max(np.abs(tot / ((2 * ell + 1) / (4 * np.pi)) - 1))
        assert err < 1e-10, (theta, err)


def test_parity():
    # P_lm(-x) = (-1)^(l+m) P_lm(x): north/south symmetry of Sec. 2.2.1
    for theta in [0.2, 0.9, 1.4]:
        x, s = _xs(theta)
        for m in [0, 1, 7, 40]:
            a = ref.legendre(200, m, x, s)
            b = ref.legendre(200, m, -x, s)
            sign = np.array([(-1) ** (l + m) for l in range(201)])
            assert np.array_equal(b, sign * a)


def test_scipy_spherical_harmonics():
    # scipy's Y_l^m carries the Condon-Shortley phase (-1)^m
    L = 120
    for theta in [0.05, 0.7, 1.9, 3.1]:
        x, s = _xs(theta)
        for m in [0, 1, 2, 9, 33, 80, 120]:
            lam = ref.legendre(L, m, x, s)
            ell = np.arange(m, L + 1)
            y = sps.sph_harm_y(ell, m, theta, 0.0).real * (-1) ** m
            sc = np.sqrt((2 * ell + 1) / (4 * np.pi))
            assert np.max(np.abs(lam[m:] - y) / sc) < 1e-12, (theta, m)


@pytest.mark.parametrize("l,m,theta", [
    (4096, 60, "pole"),         # seed sin^60 ~ 1e-205: scaled exponent needed
    (4096, 1500, math.pi / 6),  # seed 2^-1500 underflows, value O(1)
    (4096, 2000, 0.6),
])
def test_mpmath_large_degree(l, m, theta):
    # Independent special-function evaluation (hypergeometric) at l = 4096.
    # The oracle takes x and s separately; its result scales as
    # (s / sqrt(1-x^2))^m in s, so the mpmath value at x is rescaled to the s
    # actually passed.
    if theta == "pole":
        N = 2048
        omz = 1.0 / (3.0 * N * N)
        x = 1.0 - omz
        s = math.sqrt(omz * (1.0 + x))
    else:
        x, s = _xs(theta)
    mpmath.mp.dps = 40
    X = mpmath.mpf(x)
    v = (-1) ** m * mpmath.sqrt((2 * l + 1) / (4 * mpmath.pi) * mpmath.factorial(l - m)
                                / mpmath.factorial(l + m)) * mpmath.legenp(l, m, X, maxprec=20000)
    v *= (mpmath.mpf(s) / mpmath.sqrt(1 - X * X)) ** m
    got = ref.legendre(l, m, x, s)[l]
    assert abs(got / float(v) - 1) < 2e-12, (got, float(v))


def test_mu_seed_underflow_is_zero_not_nan():
    lam = ref.legendre(300, 300, 1.0, 0.0)
    assert lam[300] == 0.0 and np.all(np.isfinite(lam))
    lam = ref.legendre(300, 0, 1.0, 0.0)
    ell = np.arange(301)
    # P_l0(1) = sqrt((2l+1)/(4 pi)) (P_l(1) = 1)
    # the recurrence at x = 1 drifts by about l ulp
    assert np.max(np.abs(lam / np.sqrt((2 * ell + 1) / (4 * np.pi)) - 1)) < 4e-13
