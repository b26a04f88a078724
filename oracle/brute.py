"""Brute-force spherical harmonic synthesis for small l_max (test infrastructure).

Independent of the recurrence: the associated Legendre functions come from
Rodrigues' formula with exact rational polynomial coefficients,

    P_l(x)    = 1 / (2^l l!) d^l/dx^l (x^2 - 1)^l,
    P_lm(x)   = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) (1-x^2)^{m/2} d^m/dx^m P_l(x),

(the orthonormal functions of Sec. 2.1 without a Condon-Shortley phase,
which is what Eq. (pmm) with mu_m > 0 gives), evaluated in 40-digit mpmath
arithmetic.  The map is then the literal double sum of Eq. (alm2mapDef),

    s(theta, phi) = sum_{l <= lmax} sum_{m=-l}^{l} a_lm Y_lm(theta, phi),

over every pixel, with a_{l,-m} = (-1)^m conj(a_lm) and
Y_{l,-m} = (-1)^m P_lm e^{-i m phi} (Sec. 2.1).  The analysis is the literal
weighted sum of Eq. (map2almDef) with the conjugate harmonic,

    a_lm = sum_pixels w_p s_p conj(Y_lm(theta_p, phi_p)),  m >= 0.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import comb, factorial

import mpmath
import numpy as np

mpmath.mp.dps = 40


@lru_cache(maxsize=None)
def _dm_legendre_poly(l: int, m: int) -> tuple:
    """Coefficients c_k (ascending powers) of d^m/dx^m P_l(x), exact."""
    # (x^2 - 1)^l = sum_k C(l,k) (-1)^(l-k) x^(2k)
    coef = {}
    for k in range(l + 1):
        coef[2 * k] = Fraction(comb(l, k) * (-1) ** (l - k))
    # l + m derivatives, then divide by 2^l l!
    for _ in range(l + m):
        coef = {p - 1: c * p for p, c in coef.items() if p > 0}
    den = Fraction(2 ** l * factorial(l))
    deg = max(coef) if coef else 0
    return tuple(coef.get(p, Fraction(0)) / den for p in range(deg + 1))


def plm(l: int, m: int, x, s) -> mpmath.mpf:
    """Orthonormal P_lm at x = cos theta, s = sin theta (mpmath value)."""
    x = mpmath.mpf(float(x))
    s = mpmath.mpf(float(s))
    c = _dm_legendre_poly(l, m)
    poly = mpmath.mpf(0)
    for ck in reversed(c):
        poly = poly * x + mpmath.mpf(ck.numerator) / ck.denominator
    norm = mpmath.sqrt(mpmath.mpf(2 * l + 1) / (4 * mpmath.pi)
                       * mpmath.mpf(factorial(l - m)) / factorial(l + m))
    return norm * s ** m * poly


def plm_table(lmax: int, x, s) -> np.ndarray:
    """[lmax+1, lmax+1] float64 table T[l, m] = P_lm(x) (0 for m > l)."""
    t = np.zeros((lmax + 1, lmax + 1))
    for l in range(lmax + 1):
        for m in range(l + 1):
            t[l, m] = float(plm(l, m, x, s))
    return t


def alm2map_brute(lmax: int, geom, alm) -> np.ndarray:
    """Literal sum over l and m = -l..l at every pixel (full m set)."""
    out = np.zeros(int(geom.npix))
    idx = {}
    off = 0
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            idx[(l, m)] = off + (l - m)
        off += lmax - m + 1
    a = np.asarray(alm, dtype=np.complex128)
    for r in range(geom.nrings):
        T = plm_table(lmax, geom.cth[r], geom.sth[r])
        n = int(geom.nphi[r])
        phi = float(geom.phi0[r]) + 2.0 * np.pi * np.arange(n) / n
        acc = np.zeros(n, dtype=np.complex128)
        for l in range(lmax + 1):
            for m in range(-l, l + 1):
                am = abs(m)
                if m >= 0:
                    alm_v = a[idx[(l, m)]] if m > 0 else a[idx[(l, 0)]].real
                    y = T[l, am] * np.exp(1j * m * phi)
                else:
                    alm_v = (-1) ** am * np.conj(a[idx[(l, am)]])
                    y = (-1) ** am * T[l, am] * np.exp(1j * m * phi)
                acc += alm_v * y
        s0 = int(geom.ringstart[r])
        out[s0:s0 + n] = acc.real
        assert np.max(np.abs(acc.imag)) <= 1e-12 * max(1.0, np.max(np.abs(acc.real)))
    return out


def map2alm_brute(lmax: int, geom, m_in, ring_weight) -> np.ndarray:
    """Literal weighted sum over every pixel (full m set), complex128 [nalm]."""
    m_in = np.asarray(m_in, dtype=np.float64)
    out = np.zeros((lmax + 1) * (lmax + 2) // 2, dtype=np.complex128)
    for r in range(geom.nrings):
        T = plm_table(lmax, geom.cth[r], geom.sth[r])
        n = int(geom.nphi[r])
        s0 = int(geom.ringstart[r])
        phi = float(geom.phi0[r]) + 2.0 * np.pi * np.arange(n) / n
        sw = float(ring_weight[r]) * m_in[s0:s0 + n]
        off = 0
        for m in range(lmax + 1):
            e = np.sum(sw * np.exp(-1j * m * phi))
            for l in range(m, lmax + 1):
                out[off + (l - m)] += T[l, m] * e
            off += lmax - m + 1
    return out
