"""Pins of the oracle's whole transform and of its Fourier step.

* brute force: the literal double sum of Eq. (alm2mapDef) at every pixel with
  exact-rational Legendre functions (l_max <= 16), and at sampled pixels of
  the l_max = 64, nside = 32 workload with scipy's spherical harmonics;
* the per-ring Fourier step against the literal sum of Eq. (Delta2map) for
  rings with fewer, equal and more pixels than modes (the wrap rule of
  Sec. 2.2.2);
* Gauss-Legendre quadrature round trip (orthonormality of Sec. 2.1);
* adjoint dot-product identity;
* invariants: linearity, rotation about the axis, m = 0 rings, the pole.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import brute, ref


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_l64_nside32_against_scipy_literal_sum():
    """The l_max = 64, nside = 32 workload at every 16th pixel against the
    literal sum over l and m = -l..l of Eq. (alm2mapDef), with
    a_{l,-m} = (-1)^m conj(a_lm) (Sec. 2.1) and scipy's Y_lm, which carries
    the Condon-Shortley phase the paper's mu_m (Eq. pmm) does not:
    Y_lm(paper) = (-1)^m Y_lm(scipy) for every m of either sign."""
    sps = pytest.importorskip("scipy.special")
    lmax, nside = 64, 32
    g = W.healpix_geometry(nside)
    a = W.config_alm(1)
    off = W.alm_offsets(lmax, W.mvals(lmax))
    th = np.repeat(g.theta, g.nphi)
    ph = np.concatenate([g.phi0[r] + 2 * np.pi * np.arange(g.nphi[r]) / g.nphi[r]
                         for r in range(g.nrings)])
    pix = np.arange(0, g.npix, 16)
    th, ph = th[pix], ph[pix]
    s = np.zeros(len(pix), dtype=np.complex128)
    for ell in range(lmax + 1):
        for mu in range(-ell, ell + 1):
            m = abs(mu)
            alm = a[off[m] + ell - m]
            if m == 0:
                alm = complex(alm.real, 0.0)
            amu = alm if mu >= 0 else (-1) ** m * np.conj(alm)
            s += amu * (-1) ** mu * sps.sph_harm_y(ell, mu, th, ph)
    assert np.max(np.abs(s.imag)) < 1e-13 * np.max(np.abs(s.real))
    e = ref.alm2map(lmax, g, a)[pix]
    assert _rel(s.real, e) < 1e-13
    assert np.max(np.abs(s.real - e)) < 1e-13 * np.max(np.abs(e))


@pytest.mark.parametrize("lmax,nside", [(8, 4), (16, 8), (16, 2)])
def test_brute_force_healpix(lmax, nside):
    g = W.healpix_geometry(nside)
    a = W.random_alm(lmax, [77, lmax, nside])
    m1 = ref.alm2map(lmax, g, a)
    m2 = brute.alm2map_brute(lmax, g, a)
    assert _rel(m1, m2) < 1e-14


def test_brute_force_odd_rings_and_im_a_l0_ignored():
    g = W.ecp_geometry(9, 7)            # odd ring count and odd nphi < 2 lmax + 1
    lmax = 12
    a = W.random_alm(lmax, [78], spectrum="flat")
    a2 = a.copy()
    off = W.alm_offsets(lmax, W.mvals(lmax))
    a2[off[0]:off[1]] += 1j * 3.0       # imaginary part of a_l0 must not matter
    m1 = ref.alm2map(lmax, g, a2)
    m2 = brute.alm2map_brute(lmax, g, a)
    assert _rel(m1, m2) < 1e-14


def test_partial_m_set_sums_to_full():
    lmax = 24
    g = W.healpix_geometry(8)
    a = W.random_alm(lmax, [5])
    full = ref.alm2map(lmax, g, a)
    off = W.alm_offsets(lmax, W.mvals(lmax))
    parts = [np.array([0, 3, 5, 24], np.int32), np.array([1, 2, 4], np.int32),
             np.arange(6, 24, dtype=np.int32)]
    tot = np.zeros_like(full)
    for ms in parts:
        sub = np.concatenate([a[off[m]:off[m + 1]] for m in ms])
        tot += ref.alm2map(lmax, g, sub, mval=ms)
    assert _rel(tot, full) < 1e-14


@pytest.mark.parametrize("nphi", [1, 2, 3, 4, 7, 8, 16, 20, 21, 40, 41, 64, 100])
def test_ring_fourier_step_vs_literal_sum(nphi):
    rng = np.random.default_rng(nphi)
    mmax = 20
    mval = np.arange(mmax + 1)
    d = rng.standard_normal(mmax + 1) + 1j * rng.standard_normal(mmax + 1)
    d[0] = d[0].real
    for phi0 in [0.0, 0.3, math.pi / nphi]:
        a = ref.ring_synthesis(d, mval, phi0, nphi)
        b = ref.ring_synthesis_direct(d, mval, phi0, nphi)
        assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b)) + 1e-13


def test_ring_analysis_is_adjoint_of_synthesis():
    rng = np.random.default_rng(3)
    mval = np.array([0, 1, 2, 5, 9, 13, 30])
    for n in [5, 8, 12, 31, 64]:
        d = rng.standard_normal(len(mval)) + 1j * rng.standard_normal(len(mval))
        d[0] = d[0].real
        g = rng.standard_normal(n)
        lhs = np.dot(ref.ring_synthesis(d, mval, 0.37, n), g)
        dt = ref.ring_analysis(g, mval, 0.37)
        rhs = np.sum(d.real * dt.real + d.imag * dt.imag)
        # the m = 0 stored coefficient is real: only its real part pairs
        assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


@pytest.mark.parametrize("lmax", [8, 32, 64])
def test_gauss_legendre_round_trip(lmax):
    # nrings = lmax + 1 GL rings, nphi >= 2 lmax + 1: quadrature is exact for
    # the product of two band-limited functions, so D * adjoint(w s) = a with
    # D = 1 for m = 0 and 1/2 for m > 0.
    g = W.gl_geometry(lmax + 1, 2 * lmax + 2)
    a = W.random_alm(lmax, [11, lmax])
    s = ref.alm2map(lmax, g, a)
    w = np.repeat(g.weight, g.nphi)
    back = ref.alm2map_adjoint(lmax, g, w * s)
    off = W.alm_offsets(lmax, W.mvals(lmax))
    back[off[1]:] *= 0.5
    assert np.max(np.abs(back - a)) < 1e-13 * np.max(np.abs(a)) * lmax


@pytest.mark.parametrize("nside,lmax", [(4, 10), (16, 40)])
def test_adjoint_dot_product(nside, lmax):
    g = W.healpix_geometry(nside)
    a = W.random_alm(lmax, [21])
    d = W.random_map(g.npix, [22])
    lhs = np.dot(ref.alm2map(lmax, g, a), d)
    at = ref.alm2map_adjoint(lmax, g, d)
    rhs = np.sum(a.real * at.real + a.imag * at.imag)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    off = W.alm_offsets(lmax, W.mvals(lmax))
    assert np.all(at[off[0]:off[1]].imag == 0)


def test_linearity_and_rotation():
    lmax, nside = 24, 8
    g = W.healpix_geometry(nside)
    a = W.random_alm(lmax, [31])
    b = W.random_alm(lmax, [32])
    ma, mb = ref.alm2map(lmax, g, a), ref.alm2map(lmax, g, b)
    assert _rel(ref.alm2map(lmax, g, 2.0 * a - 3.0 * b), 2 * ma - 3 * mb) < 1e-14
    # rotation by alpha about the axis: a_lm e^{-i m alpha} gives the map at phi - alpha
    alpha = 0.123
    mv = np.concatenate([np.full(lmax - m + 1, m) for m in range(lmax + 1)])
    ar = a * np.exp(-1j * mv * alpha)
    g2 = W.Geometry(g.cth, g.sth, g.phi0 + alpha, g.nphi, g.ringstart, g.npix)
    assert _rel(ref.alm2map(lmax, g2, ar), ma) < 1e-13


def test_m0_only_constant_rings_and_pole():
    lmax = 30
    off = W.alm_offsets(lmax, W.mvals(lmax))
    a = np.zeros(off[-1], complex)
    a[:off[1]] = np.random.default_rng(4).standard_normal(lmax + 1)
    g = W.healpix_geometry(8)
    m = ref.alm2map(lmax, g, a)
    for r in range(g.nrings):
        ring = m[g.ringstart[r]:g.ringstart[r] + g.nphi[r]]
        assert np.ptp(ring) < 1e-14 * max(1, np.max(np.abs(ring)))
    # a ring at the north pole (x = 1, s = 0): s = sum_l a_l0 sqrt((2l+1)/(4 pi))
    pole = W.Geometry(np.array([1.0]), np.array([0.0]), np.array([0.0]),
                      np.array([3], np.int64), np.array([0], np.int64), 3)
    b = W.random_alm(lmax, [6])
    v = ref.alm2map(lmax, pole, b)
    ell = np.arange(lmax + 1)
    exp = np.sum(b[:lmax + 1].real * np.sqrt((2 * ell + 1) / (4 * np.pi)))
    assert np.max(np.abs(v - exp)) < 1e-14 * abs(exp) * 10


def test_even_parity_alm_gives_symmetric_map():
    lmax = 20
    a = W.random_alm(lmax, [8])
    for m in range(lmax + 1):
        off = W.alm_offsets(lmax, W.mvals(lmax))
        for l in range(m, lmax + 1):
            if (l + m) % 2:
                a[off[m] + l - m] = 0
    g = W.healpix_geometry(8)
    s = ref.alm2map(lmax, g, a)
    R = g.nrings
    for r in range(R // 2):
        rs = R - 1 - r
        n = g.ringstart
        assert np.allclose(s[n[r]:n[r] + g.nphi[r]], s[n[rs]:n[rs] + g.nphi[rs]],
                           rtol=0, atol=1e-14)


# ---- quadrature-weighted analysis (map2alm)

def test_map2alm_matches_literal_sum():
    # D adjoint(w s) against the literal sum of Eq. (map2almDef) with the
    # conjugate harmonic and a weight per ring (Rodrigues P_lm, mpmath).
    nside, lmax = 2, 5
    g = W.healpix_geometry(nside)
    rng = np.random.default_rng(41)
    s = rng.standard_normal(g.npix)
    w = 0.5 + rng.random(g.nrings)
    got = ref.map2alm(lmax, g, s, w)
    want = brute.map2alm_brute(lmax, g, s, w)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("lmax", [8, 24])
def test_map2alm_gauss_legendre_exact(lmax):
    # exact quadrature: map2alm inverts alm2map on lmax + 1 GL rings
    g = W.gl_geometry(lmax + 1, 2 * lmax + 2)
    a = W.random_alm(lmax, [42, lmax])
    back = ref.map2alm(lmax, g, ref.alm2map(lmax, g, a), g.weight)
    assert np.max(np.abs(back - a)) < 1e-13 * np.max(np.abs(a)) * lmax


def test_map2alm_jacobi_refinement_converges():
    # HEALPix with the uniform weight 4 pi / npix is not exact; the Jacobi
    # steps shrink the error of a band-limited map geometrically
    nside, lmax = 8, 12
    g = W.healpix_geometry(nside)
    a = W.random_alm(lmax, [43])
    s = ref.alm2map(lmax, g, a)
    w = np.full(g.nrings, 4.0 * np.pi / g.npix)
    errs = [np.max(np.abs(ref.map2alm(lmax, g, s, w, niter=k) - a)) for k in (0, 1, 3)]
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1]
    assert errs[2] < 1e-3 * np.max(np.abs(a))
