"""GPU parity at the library's advertised limits.

* ring lengths up to SHT_MAX_NPHI = 16384 in the synthesis and its adjoint
  (the 8192-point FFT class, odd 7-smooth lengths above 4096, the split
  Bluestein step at 16380), and the lengths the header documents as
  unsupported (a half length above 4096 that is odd and not 7-smooth, or an
  odd length above 4096 that is not 7-smooth) refused at plan time;
* l_max 8192 on a band of HEALPix nside-4096 rings from the pole ring to the
  equator, in every precision (rings of 16384 pixels, seeds that underflow to
  2^-40000 near the pole);
* the adjoint and map2alm at l_max 4096 on 256 rings of the nside-2048 grid.

Bounds: FP64 relative L2 <= 1e-12 per map (element-wise for the ring
Fourier steps, scaled by log2 n as in the other ring tests); mixed forms
<= 1e-6 per map.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import ref

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {"fp64": 1e-12, "fp32_mfma": 1e-6, "bf16x3_mfma": 1e-6, "f16x2_mfma": 1e-6}


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1010_1260_amd as P
    return P


def _dev():
    return torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _compact(g, rings):
    """The given rings of g as a geometry of their own, pixels packed."""
    rings = np.asarray(rings, dtype=np.int64)
    nphi = g.nphi[rings].copy()
    start = np.concatenate([[0], np.cumsum(nphi)[:-1]]).astype(np.int64)
    return W.Geometry(g.cth[rings].copy(), g.sth[rings].copy(), g.phi0[rings].copy(), nphi,
                      start, int(nphi.sum()))


SUPPORTED = [4375, 6561, 8190, 12000, 16380, 16384]
UNSUPPORTED = [4097, 8191, 9998, 16382]


@pytest.mark.parametrize("nphi", SUPPORTED)
def test_long_ring_synthesis_and_analysis(P, nphi):
    _say("long ring", nphi)
    rng = np.random.default_rng(7000 + nphi)
    mmax = 300
    mval = np.arange(mmax + 1, dtype=np.int32)
    nr = 2
    phi0 = np.array([np.pi / nphi, 0.37])
    geo = W.Geometry(np.array([0.6, -0.6]), np.array([0.8, 0.8]), phi0,
                     np.full(nr, nphi, np.int64), np.arange(nr) * nphi, nr * nphi)
    plan = P.Plan(mmax, geo, mval=mval)
    dl = rng.standard_normal((nr, mmax + 1)) + 1j * rng.standard_normal((nr, mmax + 1))
    dl[:, 0] = dl[:, 0].real
    d_dev = torch.from_numpy(np.ascontiguousarray(dl.T)).to(_dev()).reshape(1, mmax + 1, nr)
    got = plan.delta2map(d_dev).cpu().numpy()[0]
    exp = ref.map_from_delta(mval, geo, dl)
    scale = max(1, np.log2(nphi + 1))
    assert np.max(np.abs(got - exp)) < 1e-13 * np.max(np.abs(exp)) * scale
    g = rng.standard_normal(nr * nphi)
    gota = plan.map2delta_adjoint(torch.from_numpy(g).to(_dev()).reshape(1, -1)).cpu().numpy()[0].T
    for r in range(nr):
        expa = ref.ring_analysis(g[r * nphi:(r + 1) * nphi], mval, phi0[r])
        assert np.max(np.abs(gota[r] - expa)) < 1e-13 * np.max(np.abs(expa)) * scale


@pytest.mark.parametrize("nphi", UNSUPPORTED)
def test_unsupported_ring_lengths_refused(P, nphi):
    from paper_1010_1260_amd import _lib as L
    _say("unsupported ring", nphi)
    geo = W.Geometry(np.array([0.6]), np.array([0.8]), np.zeros(1), np.array([nphi], np.int64),
                     np.zeros(1, np.int64), nphi)
    with pytest.raises(L.ShtError) as e:
        P.Plan(64, geo)
    assert e.value.code == L.SHT_ERR_UNSUPPORTED


@pytest.fixture(scope="module")
def band8192():
    """Rings of HEALPix nside 4096: the first four (sin theta down to
    2e-4), two more in the cap, the last cap ring, two belt rings and the
    equator, with the mirrors of the first, a cap and a belt ring."""
    g = W.healpix_geometry(4096)
    R = g.nrings
    rings = [0, 1, 2, 3, 200, 2000, 4094, 6000, 7000, 8191, R - 1, R - 1 - 2000, R - 1 - 6000]
    return _compact(g, rings)


@pytest.mark.parametrize("prec", list(TOL))
def test_lmax8192_band(P, band8192, prec):
    lmax = 8192
    nmaps = 1 if prec == "fp64" else 2
    _say("lmax 8192 band", prec, nmaps)
    g = band8192
    alms = [W.random_alm(lmax, [8192, i]) for i in range(nmaps)]
    plan = P.Plan(lmax, g, nmaps=nmaps, precision=prec)
    got = plan.alm2map(torch.from_numpy(np.stack(alms)).to(_dev())).cpu().numpy()
    for i in range(nmaps):
        exp = ref.alm2map(lmax, g, alms[i])
        assert _rel(got[i], exp) < TOL[prec], i


@pytest.fixture(scope="module")
def band4096():
    """256 rings of HEALPix nside 2048, all paired: the 64 rings nearest the
    north pole, 64 belt rings, and their mirrors."""
    g = W.healpix_geometry(2048)
    R = g.nrings
    north = list(range(64)) + list(range(3000, 3064))
    return _compact(g, north + [R - 1 - r for r in north])


def test_adjoint_and_map2alm_lmax4096_band(P, band4096):
    lmax = 4096
    _say("adjoint + map2alm lmax 4096 band")
    g = band4096
    plan = P.Plan(lmax, g)
    s = W.random_map(g.npix, [4096, 1])
    s_dev = torch.from_numpy(s).to(_dev()).reshape(1, -1)
    got = plan.alm2map_adjoint(s_dev).cpu().numpy()[0]
    exp = ref.alm2map_adjoint(lmax, g, s)
    assert _rel(got, exp) < 1e-12
    # dot-product identity <alm2map(a), s> = <a, adjoint(s)>
    a = W.random_alm(lmax, [4096, 2])
    fwd = plan.alm2map(torch.from_numpy(a).to(_dev()).reshape(1, -1)).cpu().numpy()[0]
    lhs = float(np.dot(fwd, s))
    rhs = float(np.sum(a.real * got.real + a.imag * got.imag))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    w = np.full(g.nrings, 4.0 * np.pi / 50331648)
    for niter in (0, 1):
        got2 = plan.map2alm(s_dev, w, niter=niter).cpu().numpy()[0]
        exp2 = ref.map2alm(lmax, g, s, w, niter=niter)
        assert _rel(got2, exp2) < 1e-12, niter
