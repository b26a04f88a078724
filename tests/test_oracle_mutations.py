"""The pins catch plausible mistakes: each planted mistake in a copy of the C
oracle (built into a temporary directory on the CPU) must fail at least one
independent check (brute-force sum, addition theorem, mpmath value)."""
import ctypes
import math
import os
import shutil
import subprocess

import mpmath
import numpy as np
import pytest

import workloads as W
from oracle import brute

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "sht_oracle.c")

MUTATIONS = {
    # recurrence sign as printed in Eq. (assLegRec)
    "recurrence_plus": [("(x * v1 - v0 / b[j - 1])", "(x * v1 + v0 / b[j - 1])")],
    # seed exponent m instead of m/2 (Eq. pmm as printed): s^(2m)
    "seed_exponent_m": [("int p = m;", "int p = 2 * m;")],
    # second seed with the wrong beta index (Eq. pm1m)
    "pm1m_index": [("v1 = b[1] * x * v0;", "v1 = b[2] * x * v0;")],
    # mu_m running product off by one
    "mu_ratio": [("sqrt((2.0 * m + 1.0) / (2.0 * m))", "sqrt((2.0 * m + 2.0) / (2.0 * m))")],
    # rescale bookkeeping: exponent not advanced (value scaled back wrongly)
    "rescale_exponent": [("            k += 1;\n            scale", "            k += 0;\n            scale")],
    # dropped conjugate-symmetric half: imaginary part of a_lm ignored
    "drop_imag": [("if (m > 0) dim += a[2 * j + 1] * P[j];", "if (m > 0) dim += 0.0 * P[j];")],
}


def _build(tmp, name, subs):
    src = open(SRC).read()
    hit = 0
    for a, b in subs:
        if a in src:
            src = src.replace(a, b)
            hit += 1
    assert hit, f"mutation {name} did not apply"
    c = os.path.join(tmp, f"{name}.c")
    so = os.path.join(tmp, f"{name}.so")
    open(c, "w").write(src)
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           c, "-o", so, "-lm"])
    L = ctypes.CDLL(so)
    d = ctypes.POINTER(ctypes.c_double)
    L.oracle_lambda.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, d]
    L.oracle_delta.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                               ctypes.c_int, d, d, d, d, ctypes.c_int]
    return L


def _lam(L, lmax, m, x, s):
    out = np.empty(lmax + 1)
    L.oracle_lambda(lmax, m, x, s, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def _pins_fail(L):
    dp = ctypes.POINTER(ctypes.c_double)
    # 1. brute force at lmax = 12 on HEALPix nside 4 (Delta only: compare maps)
    lmax = 12
    g = W.healpix_geometry(4)
    a = W.random_alm(lmax, [3])
    mv = np.arange(lmax + 1, dtype=np.int32)
    dl = np.empty((g.nrings, lmax + 1), complex)
    L.oracle_delta(lmax, lmax + 1, mv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), g.nrings,
                   g.cth.ctypes.data_as(dp), g.sth.ctypes.data_as(dp),
                   a.view(np.float64).ctypes.data_as(dp), dl.view(np.float64).ctypes.data_as(dp), 1)
    from oracle import ref
    m1 = ref.map_from_delta(mv, g, dl)
    m2 = brute.alm2map_brute(lmax, g, a)
    if np.linalg.norm(m1 - m2) > 1e-12 * np.linalg.norm(m2):
        return "brute"
    # 2. addition theorem at l <= 1024 near a pole and at mid latitude
    for th in [0.02, 0.7]:
        x = math.cos(th)
        s = math.sqrt((1 - x) * (1 + x))
        tot = np.zeros(1025)
        for m in range(1025):
            tot += (1.0 if m == 0 else 2.0) * _lam(L, 1024, m, x, s) ** 2
        ell = np.arange(1025)
        if np.max(np.abs(tot / ((2 * ell + 1) / (4 * np.pi)) - 1)) > 1e-9:
            return "addition"
    # 3. mpmath at l = 4096, m = 1500 (rescaling needed)
    x, s = math.cos(math.pi / 6), math.sin(math.pi / 6)
    mpmath.mp.dps = 30
    X = mpmath.mpf(x)
    v = (-1) ** 1500 * mpmath.sqrt(8193 / (4 * mpmath.pi) * mpmath.factorial(2596)
                                   / mpmath.factorial(5596)) * mpmath.legenp(4096, 1500, X)
    v *= (mpmath.mpf(s) / mpmath.sqrt(1 - X * X)) ** 1500
    if abs(_lam(L, 4096, 1500, x, s)[4096] / float(v) - 1) > 1e-10:
        return "mpmath"
    return None


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    L = _build(str(tmp_path), name, MUTATIONS[name])
    assert _pins_fail(L) is not None, f"mutation {name} passed every pin"


def test_unmutated_oracle_passes_same_pins(tmp_path):
    L = _build(str(tmp_path), "none", [("#define ORACLE_S 256", "#define ORACLE_S 256")])
    assert _pins_fail(L) is None
