"""Seeded synthetic inputs: ring geometries and harmonic coefficients.

This module holds no arithmetic of the transform itself.  It only builds the
inputs that both the HIP path and the CPU oracle consume:

* iso-latitude ring geometries (HEALPix-style, Gauss-Legendre), given as
  per-ring cos(theta), sin(theta), phi_0, pixel count and pixel offset;
* Gaussian random a_lm with a prescribed power spectrum C_l, drawn from
  counter-free seeded PCG64 streams (``numpy.random.default_rng([cfg, i])``)
  in m-major order (for each m: l = m..lmax, real part then imaginary part);
* seeded N(0, 1) pixel data for the loss of the differentiation workload.

The paper (Sec. 2.2.1) assumes iso-latitude rings placed symmetrically about
the equator; it does not fix the pixelization used in its experiments
(Sec. 6).  The HEALPix rings follow Gorski et al. (2005), which the paper
cites for the serial transform.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Geometry", "healpix_geometry", "gl_geometry", "ecp_geometry",
    "nalm", "mvals", "alm_offsets", "random_alm", "random_map", "CONFIGS",
    "config_alm", "config_geometry",
]


@dataclass
class Geometry:
    """Ring geometry of a pixelized sphere (RING order).

    cth, sth : cos/sin of the ring colatitude (float64 [nrings])
    phi0     : azimuth of the ring's first pixel (float64 [nrings])
    nphi     : pixels in the ring (int64 [nrings])
    ringstart: offset of the ring's first pixel in the map (int64 [nrings])
    npix     : total pixels (max of ringstart + nphi)
    weight   : optional quadrature weight per ring (float64 [nrings])
    """
    cth: np.ndarray
    sth: np.ndarray
    phi0: np.ndarray
    nphi: np.ndarray
    ringstart: np.ndarray
    npix: int
    name: str = ""
    weight: np.ndarray | None = None

    @property
    def nrings(self) -> int:
        return int(self.cth.shape[0])

    @property
    def theta(self) -> np.ndarray:
        return np.arctan2(self.sth, self.cth)

    def subset(self, rings) -> "Geometry":
        """Geometry of a subset of rings, each keeping its pixel offset."""
        rings = np.asarray(rings, dtype=np.int64)
        return Geometry(self.cth[rings].copy(), self.sth[rings].copy(),
                        self.phi0[rings].copy(), self.nphi[rings].copy(),
                        self.ringstart[rings].copy(), self.npix,
                        self.name + "[subset]",
                        None if self.weight is None else self.weight[rings].copy())


def healpix_geometry(nside: int) -> Geometry:
    """HEALPix ring geometry (Gorski et al. 2005), 4*nside-1 rings north to south.

    North cap i < N: 1 - z = i^2 / (3 N^2), nphi = 4 i, phi0 = pi / (4 i).
    Belt N <= i <= 3N: z = 2 (2N - i) / (3N), nphi = 4N,
      phi0 = pi / (4N) if (i - N) is even else 0.
    South cap: mirror of ring 4N - i with z negated, so every north/south pair
    has bitwise opposite cos(theta) and bitwise equal sin(theta).
    """
    N = int(nside)
    if N < 1:
        raise ValueError("nside must be >= 1")
    R = 4 * N - 1
    cth = np.empty(R)
    sth = np.empty(R)
    phi0 = np.empty(R)
    nphi = np.empty(R, dtype=np.int64)
    start = np.empty(R, dtype=np.int64)
    for i in range(1, 2 * N + 1):           # north cap and northern belt incl. equator
        if i < N:
            omz = (i * i) / (3.0 * N * N)   # 1 - z, one rounding
            z = 1.0 - omz
            s = math.sqrt(omz * (1.0 + z))
            n = 4 * i
            p0 = math.pi / (4.0 * i)
            st = 2 * i * (i - 1)
        else:
            z = 2.0 * (2 * N - i) / (3.0 * N)
            s = math.sqrt((1.0 - z) * (1.0 + z))
            n = 4 * N
            p0 = math.pi / (4.0 * N) if (i - N) % 2 == 0 else 0.0
            st = 2 * N * (N - 1) + 4 * N * (i - N)
        r = i - 1
        cth[r], sth[r], phi0[r], nphi[r], start[r] = z, s, p0, n, st
        if i < 2 * N:                        # mirror ring 4N - i
            j = 4 * N - i
            rs = j - 1
            cth[rs] = -z
            sth[rs] = s
            phi0[rs] = p0
            nphi[rs] = n
            if i < N:
                start[rs] = 12 * N * N - 2 * i * (i + 1)
            else:
                start[rs] = 2 * N * (N - 1) + 4 * N * (j - N)
    cth[2 * N - 1] = 0.0
    sth[2 * N - 1] = 1.0
    return Geometry(cth, sth, phi0, nphi, start, 12 * N * N, f"healpix{N}")


def gl_geometry(nrings: int, nphi: int, phi0: float = 0.0) -> Geometry:
    """Gauss-Legendre rings: nodes of numpy's leggauss, north to south.

    The nodes returned by numpy are symmetric by construction, so pairs have
    bitwise opposite cos(theta).  weight holds w_i * 2 pi / nphi, the weight
    of one pixel of ring i.
    """
    x, w = np.polynomial.legendre.leggauss(int(nrings))
    order = np.argsort(-x, kind="stable")
    x = x[order].copy()
    w = w[order].copy()
    # exact antisymmetry of the nodes (numpy already symmetrizes them)
    n = len(x)
    for i in range(n // 2):
        x[n - 1 - i] = -x[i]
        w[n - 1 - i] = w[i]
    if n % 2:
        x[n // 2] = 0.0
    s = np.sqrt((1.0 - x) * (1.0 + x))
    nphi_a = np.full(n, int(nphi), dtype=np.int64)
    start = np.arange(n, dtype=np.int64) * int(nphi)
    return Geometry(x, s, np.full(n, float(phi0)), nphi_a, start, n * int(nphi),
                    f"gl{nrings}x{nphi}", weight=w * (2.0 * np.pi / nphi))


def ecp_geometry(nrings: int, nphi: int) -> Geometry:
    """Equidistant-cylindrical rings at theta_i = pi (i + 1/2) / nrings."""
    th = np.pi * (np.arange(nrings) + 0.5) / nrings
    x = np.cos(th)
    s = np.sin(th)
    n = len(x)
    for i in range(n // 2):
        x[n - 1 - i] = -x[i]
        s[n - 1 - i] = s[i]
    if n % 2:
        x[n // 2] = 0.0
        s[n // 2] = 1.0
    return Geometry(x, s, np.zeros(n), np.full(n, int(nphi), dtype=np.int64),
                    np.arange(n, dtype=np.int64) * int(nphi), n * int(nphi),
                    f"ecp{nrings}x{nphi}")


def mvals(lmax: int, mmax: int | None = None) -> np.ndarray:
    mmax = lmax if mmax is None else mmax
    return np.arange(mmax + 1, dtype=np.int32)


def alm_offsets(lmax: int, mval) -> np.ndarray:
    """Start of each m's l = m..lmax run in the m-major packed array."""
    mval = np.asarray(mval, dtype=np.int64)
    lens = lmax - mval + 1
    return np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)


def nalm(lmax: int, mval=None) -> int:
    if mval is None:
        return (lmax + 1) * (lmax + 2) // 2
    return int(alm_offsets(lmax, mval)[-1])


def _cl(lmax: int, spectrum: str) -> np.ndarray:
    ell = np.arange(lmax + 1, dtype=np.float64)
    cl = np.zeros(lmax + 1)
    if spectrum == "inv_l_lp1":          # C_l = 1 / (l (l + 1)), l >= 2
        cl[2:] = 1.0 / (ell[2:] * (ell[2:] + 1.0))
    elif spectrum == "inv_l2":           # C_l = l^-2, l >= 2
        cl[2:] = 1.0 / (ell[2:] ** 2)
    elif spectrum == "flat":
        cl[:] = 1.0
    else:
        raise ValueError(spectrum)
    return cl


def random_alm(lmax: int, seed, mval=None, spectrum: str = "inv_l_lp1") -> np.ndarray:
    """One map's Gaussian a_lm (complex128 [nalm], m-major packed).

    E|a_lm|^2 = C_l; a_l0 is real with variance C_l, Re/Im of m > 0 have
    variance C_l / 2.  Draw order: for each m, l = m..lmax, (re, im).
    """
    mval = mvals(lmax) if mval is None else np.asarray(mval, dtype=np.int32)
    rng = np.random.default_rng(seed)
    off = alm_offsets(lmax, mval)
    z = rng.standard_normal((int(off[-1]), 2))
    cl = _cl(lmax, spectrum)
    out = np.empty(int(off[-1]), dtype=np.complex128)
    for i, m in enumerate(mval):
        ell = np.arange(m, lmax + 1)
        seg = slice(off[i], off[i + 1])
        if m == 0:
            out[seg] = z[seg, 0] * np.sqrt(cl[ell])
        else:
            sd = np.sqrt(cl[ell] / 2.0)
            out[seg] = z[seg, 0] * sd + 1j * (z[seg, 1] * sd)
    return out


def random_map(npix: int, seed) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(int(npix))


# Workloads: the small FP64 case, the full-size FP64 case, the batched mixed
# precision case, the batched uneven case and the differentiation case.
CONFIGS = {
    1: dict(name="fp64_l64_n32", lmax=64, nside=32, nmaps=1, spectrum="inv_l_lp1",
            precision="fp64"),
    2: dict(name="fp64_l4096_n2048", lmax=4096, nside=2048, nmaps=1, spectrum="inv_l_lp1",
            precision="fp64"),
    3: dict(name="mixed_l4096_n2048_x16", lmax=4096, nside=2048, nmaps=16,
            spectrum="inv_l_lp1", precision="mixed"),
    4: dict(name="uneven_x64", lmax_choices=(256, 512, 1024, 2048), nmaps=64,
            spectrum="inv_l2", precision="fp64"),
    5: dict(name="grad_l1024_n512_x8", lmax=1024, nside=512, nmaps=8, spectrum="inv_l_lp1",
            precision="fp64"),
}


def config_geometry(cfg_id: int) -> Geometry:
    return healpix_geometry(CONFIGS[cfg_id]["nside"])


def config_alm(cfg_id: int, map_idx: int = 0, lmax: int | None = None) -> np.ndarray:
    c = CONFIGS[cfg_id]
    L = c["lmax"] if lmax is None else lmax
    return random_alm(L, [cfg_id, map_idx], spectrum=c["spectrum"])


def uneven_lmax(n: int = 64, seed=(4, 1000)) -> list[int]:
    """The l_max of each map of the batched uneven workload (uniform draw)."""
    rng = np.random.default_rng(list(seed))
    ch = CONFIGS[4]["lmax_choices"]
    return [int(ch[i]) for i in rng.integers(0, len(ch), size=n)]
