"""FP64 CPU oracle: Python side (test infrastructure only).

The Legendre stage runs in the plain C file ``sht_oracle.c`` (loaded with
ctypes); the per-ring Fourier step is written here with numpy.

Per-ring synthesis (Eq. Delta2map, Sec. 2.1):
    s(theta_r, phi_j) = sum_{m=-mmax}^{mmax} Delta_m(theta_r) e^{i m phi_j},
    phi_j = phi0_r + 2 pi j / nphi_r,  Delta_{-m} = conj(Delta_m)  (Eq. DeltaDef).
Writing e^{i m phi_j} = e^{i m phi0} e^{2 pi i m j / n}, the sum becomes an
inverse DFT of length n once every mode m is moved to bin m mod n: modes
beyond the ring's bandwidth are wrapped and co-added, missing modes are zero
(the rule stated at the end of Sec. 2.2.2).

Adjoint (transpose with respect to the real inner product of the stored
coefficients, m >= 0): per ring G_k = sum_j g_j e^{-2 pi i j k / n} (forward
DFT), Dt_m = c_m e^{-i m phi0} G_{m mod n} with c_0 = 1, c_m = 2 for m > 0,
then out_lm = sum_r P_lm(cos theta_r) Dt_m(r).  The factor c_m and the
conjugate phase follow from differentiating s = sum_l Re(a_l0) P_l0 +
2 Re sum_{m>0} e^{i m phi} sum_l a_lm P_lm with respect to Re and Im of a_lm.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sht_oracle.c")
_SO = os.path.join(_HERE, "_build", "libsht_oracle.so")
_lock = threading.Lock()
_lib = None


COMPILE_FLAGS = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                 "-fno-fast-math", "-std=c11", "-D_GNU_SOURCE"]


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, no contraction, OpenMP)."""
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call([*COMPILE_FLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_SO):
                build(force=True)
            L = ctypes.CDLL(_SO)
            d = ctypes.POINTER(ctypes.c_double)
            i32 = ctypes.POINTER(ctypes.c_int32)
            L.oracle_mu.argtypes = [ctypes.c_int, d]
            L.oracle_mu.restype = None
            L.oracle_lambda.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_double, d]
            L.oracle_lambda.restype = ctypes.c_int
            L.oracle_delta.argtypes = [ctypes.c_int, ctypes.c_int, i32, ctypes.c_int,
                                       d, d, d, d, ctypes.c_int]
            L.oracle_delta.restype = ctypes.c_int
            L.oracle_delta_adjoint.argtypes = L.oracle_delta.argtypes
            L.oracle_delta_adjoint.restype = ctypes.c_int
            L.oracle_max_threads.argtypes = []
            L.oracle_max_threads.restype = ctypes.c_int
            _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def mu(mmax: int) -> np.ndarray:
    """mu_m of Eq. (pmm) for m = 0..mmax."""
    out = np.empty(mmax + 1)
    lib().oracle_mu(int(mmax), _dp(out))
    return out


def legendre(lmax: int, m: int, x: float, s: float) -> np.ndarray:
    """P_lm(x) for l = 0..lmax (zero for l < m) at x = cos theta, s = sin theta."""
    out = np.empty(lmax + 1)
    rc = lib().oracle_lambda(int(lmax), int(m), float(x), float(s), _dp(out))
    if rc:
        raise ValueError(f"oracle_lambda failed ({rc})")
    return out


def _mset(lmax, mval):
    if mval is None:
        return np.arange(lmax + 1, dtype=np.int32)
    return np.ascontiguousarray(mval, dtype=np.int32)


def delta(lmax: int, mval, cth, sth, alm, nthreads: int = 0) -> np.ndarray:
    """Delta_m(theta_r) (Eq. DeltaDef) for all rings and m: complex [nrings, nm]."""
    mval = _mset(lmax, mval)
    cth = np.ascontiguousarray(cth, dtype=np.float64)
    sth = np.ascontiguousarray(sth, dtype=np.float64)
    a = np.ascontiguousarray(alm, dtype=np.complex128).view(np.float64)
    out = np.empty((len(cth), len(mval)), dtype=np.complex128)
    rc = lib().oracle_delta(int(lmax), len(mval), _ip(mval), len(cth), _dp(cth), _dp(sth),
                            _dp(a), _dp(out.view(np.float64)), int(nthreads))
    if rc:
        raise ValueError(f"oracle_delta failed ({rc})")
    return out


def delta_adjoint(lmax: int, mval, cth, sth, dt, nthreads: int = 0) -> np.ndarray:
    """out_lm = sum_r P_lm(cos theta_r) dt_m(r): complex [nalm] (m-major)."""
    mval = _mset(lmax, mval)
    cth = np.ascontiguousarray(cth, dtype=np.float64)
    sth = np.ascontiguousarray(sth, dtype=np.float64)
    d = np.ascontiguousarray(dt, dtype=np.complex128)
    assert d.shape == (len(cth), len(mval))
    n = int(np.sum(lmax - mval.astype(np.int64) + 1))
    out = np.empty(n, dtype=np.complex128)
    rc = lib().oracle_delta_adjoint(int(lmax), len(mval), _ip(mval), len(cth), _dp(cth),
                                    _dp(sth), _dp(d.view(np.float64)),
                                    _dp(out.view(np.float64)), int(nthreads))
    if rc:
        raise ValueError(f"oracle_delta_adjoint failed ({rc})")
    return out


# ----------------------------------------------------------------- Fourier step

def ring_synthesis(delta_row, mval, phi0: float, nphi: int) -> np.ndarray:
    """Pixels of one ring from its Delta_m, m in mval (wrap rule + inverse DFT)."""
    n = int(nphi)
    mval = np.asarray(mval, dtype=np.int64)
    d = np.asarray(delta_row, dtype=np.complex128)
    ph = np.exp(1j * (mval.astype(np.float64) * phi0))
    D = d * ph
    D = np.where(mval == 0, D.real + 0j, D)
    F = np.zeros(n, dtype=np.complex128)
    np.add.at(F, mval % n, D)
    pos = mval > 0
    np.add.at(F, (-mval[pos]) % n, np.conj(D[pos]))
    z = np.fft.ifft(F) * n          # sum_k F_k e^{+2 pi i j k / n}
    return z.real.copy()


def ring_synthesis_direct(delta_row, mval, phi0: float, nphi: int) -> np.ndarray:
    """Literal Eq. (Delta2map) at every pixel: sum over m = -mmax..mmax."""
    n = int(nphi)
    mval = np.asarray(mval, dtype=np.int64)
    d = np.asarray(delta_row, dtype=np.complex128)
    phi = phi0 + 2.0 * np.pi * np.arange(n) / n
    out = np.zeros(n, dtype=np.complex128)
    for m, dm in zip(mval, d):
        if m == 0:
            out += dm.real
        else:
            out += dm * np.exp(1j * m * phi) + np.conj(dm) * np.exp(-1j * m * phi)
    return out.real.copy()


def ring_analysis(g, mval, phi0: float) -> np.ndarray:
    """Adjoint of ring_synthesis: Dt_m = c_m e^{-i m phi0} G_{m mod n}."""
    g = np.asarray(g, dtype=np.float64)
    n = g.shape[0]
    mval = np.asarray(mval, dtype=np.int64)
    G = np.fft.fft(g)               # sum_j g_j e^{-2 pi i j k / n}
    ph = np.exp(-1j * (mval.astype(np.float64) * phi0))
    c = np.where(mval == 0, 1.0, 2.0)
    out = c * ph * G[mval % n]
    out = np.where(mval == 0, out.real + 0j, out)
    return out


# ------------------------------------------------------------ whole transform

def alm2map_delta(lmax, mval, geom, alm, nthreads=0):
    return delta(lmax, mval, geom.cth, geom.sth, alm, nthreads)


def map_from_delta(mval, geom, dl, rings=None) -> np.ndarray:
    mval = np.asarray(mval)
    out = np.zeros(int(geom.npix))
    rr = range(geom.nrings) if rings is None else rings
    for k, r in enumerate(rr):
        row = dl[r] if rings is None else dl[k]
        s0, n = int(geom.ringstart[r]), int(geom.nphi[r])
        out[s0:s0 + n] = ring_synthesis(row, mval, float(geom.phi0[r]), n)
    return out


def alm2map(lmax: int, geom, alm, mval=None, nthreads: int = 0) -> np.ndarray:
    """Full FP64 alm2map of one map: real float64 [npix], RING order."""
    mval = _mset(lmax, mval)
    dl = delta(lmax, mval, geom.cth, geom.sth, alm, nthreads)
    return map_from_delta(mval, geom, dl)


def alm2map_rings(lmax: int, geom, alm, rings, mval=None, nthreads: int = 0):
    """Pixels of a subset of rings only: list of float64 arrays (one per ring)."""
    mval = _mset(lmax, mval)
    rings = np.asarray(rings, dtype=np.int64)
    dl = delta(lmax, mval, geom.cth[rings], geom.sth[rings], alm, nthreads)
    return [ring_synthesis(dl[k], mval, float(geom.phi0[r]), int(geom.nphi[r]))
            for k, r in enumerate(rings)]


def alm2map_adjoint(lmax: int, geom, m_in, mval=None, nthreads: int = 0) -> np.ndarray:
    """Adjoint of alm2map: complex128 [nalm] (m-major), Im of m = 0 entries is 0."""
    mval = _mset(lmax, mval)
    m_in = np.asarray(m_in, dtype=np.float64)
    dt = np.empty((geom.nrings, len(mval)), dtype=np.complex128)
    for r in range(geom.nrings):
        s0, n = int(geom.ringstart[r]), int(geom.nphi[r])
        dt[r] = ring_analysis(m_in[s0:s0 + n], mval, float(geom.phi0[r]))
    return delta_adjoint(lmax, mval, geom.cth, geom.sth, dt, nthreads)


def map2alm(lmax: int, geom, m_in, ring_weight, niter: int = 0, mval=None,
            nthreads: int = 0) -> np.ndarray:
    """Quadrature-weighted analysis (Eq. map2almDef read with conj(Y_lm) and a
    weight w_r per pixel of ring r): a = D adjoint(w s), D = 1 for m = 0 and
    1/2 for m > 0 (the adjoint counts m and -m together), then `niter` Jacobi
    steps a <- a + D adjoint(w (s - alm2map(a)))."""
    mval = _mset(lmax, mval)
    m_in = np.asarray(m_in, dtype=np.float64)
    w = np.asarray(ring_weight, dtype=np.float64)
    wpix = np.zeros(int(geom.npix))
    for r in range(geom.nrings):
        s0, n = int(geom.ringstart[r]), int(geom.nphi[r])
        wpix[s0:s0 + n] = w[r]
    dfac = np.concatenate([np.full(lmax - int(m) + 1, 1.0 if m == 0 else 0.5) for m in mval])
    a = dfac * alm2map_adjoint(lmax, geom, wpix * m_in, mval, nthreads)
    for _ in range(niter):
        res = m_in - alm2map(lmax, geom, a, mval, nthreads)
        a = a + dfac * alm2map_adjoint(lmax, geom, wpix * res, mval, nthreads)
    return a
