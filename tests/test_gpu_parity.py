"""GPU parity: the HIP path through the C ABI against the CPU oracle.

FP64 bound (element-wise, relative to the data's scale): the two sides run
the same recurrence with different rounding (normalised vs plain form, FMA
contraction, summation order), so they agree to a few hundred ulp of the
largest values; relative L2 <= 1e-12 per map is the contract.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def _to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(_dev())


# ---------------------------------------------------------------- Legendre

@pytest.mark.parametrize("lmax,nside", [(64, 32), (200, 64), (513, 100)])
def test_delta_parity_healpix(P, lmax, nside):
    _say("delta healpix", lmax, nside)
    g = W.healpix_geometry(nside)
    a = W.random_alm(lmax, [101, lmax])
    plan = P.Plan(lmax, g)
    d = plan.alm2delta(_to_dev(a).reshape(1, -1)).cpu().numpy()[0].T   # -> [ring][m]
    e = ref.delta(lmax, None, g.cth, g.sth, a)
    assert _rel(d, e) < 1e-12
    assert np.max(np.abs(d - e)) < 1e-12 * np.max(np.abs(e))


def test_delta_pairing_matches_unpaired(P):
    _say("delta pairing vs unpaired")
    lmax, nside = 150, 40
    g = W.healpix_geometry(nside)
    a = W.random_alm(lmax, [102])
    d1 = P.Plan(lmax, g).alm2delta(_to_dev(a).reshape(1, -1)).cpu().numpy()
    p2 = P.Plan(lmax, g, pairing=False)
    assert p2.npairs == g.nrings
    d2 = p2.alm2delta(_to_dev(a).reshape(1, -1)).cpu().numpy()
    assert _rel(d1, d2) < 1e-13


def test_delta_partial_mset_ragged_and_batch(P):
    _say("delta partial m-set, ragged rings, 3 maps")
    lmax = 97
    mval = np.array([0, 1, 5, 6, 7, 40, 41, 90, 97], np.int32)
    g = W.ecp_geometry(37, 21)          # odd ring count, rings not multiple of 64
    alms = [W.random_alm(lmax, [103, i], mval=mval) for i in range(3)]
    plan = P.Plan(lmax, g, mval=mval, nmaps=3)
    d = np.swapaxes(plan.alm2delta(_to_dev(np.stack(alms))).cpu().numpy(), 1, 2)
    for i in range(3):
        e = ref.delta(lmax, mval, g.cth, g.sth, alms[i])
        assert _rel(d[i], e) < 1e-12


def test_delta_edge_cases(P):
    _say("delta edge cases")
    # lmax = 0
    g = W.healpix_geometry(2)
    a = np.array([0.7 + 0.3j])
    d = P.Plan(0, g).alm2delta(_to_dev(a).reshape(1, -1)).cpu().numpy()[0].T
    assert np.allclose(d[:, 0], 0.7 / np.sqrt(4 * np.pi), rtol=1e-15, atol=0)
    # single m = lmax, and rings at the poles (s = 0) and equator
    geo = W.Geometry(np.array([1.0, 0.6, 0.0, -0.6, -1.0]), np.array([0.0, 0.8, 1.0, 0.8, 0.0]),
                     np.zeros(5), np.array([1, 3, 5, 3, 1], np.int64),
                     np.array([0, 1, 4, 9, 12], np.int64), 13)
    for lmax, mval in [(40, np.array([40], np.int32)), (40, np.array([0, 1, 2], np.int32)),
                       (1, None)]:
        al = W.random_alm(lmax, [104, lmax], mval=mval, spectrum="flat")
        plan = P.Plan(lmax, geo, mval=mval)
        d = plan.alm2delta(_to_dev(al).reshape(1, -1)).cpu().numpy()[0].T
        e = ref.delta(lmax, mval, geo.cth, geo.sth, al)
        assert np.max(np.abs(d - e)) <= 1e-13 * max(1.0, np.max(np.abs(e)))


def test_delta_deep_rescaling(P):
    _say("delta deep rescaling near the pole, lmax 2048")
    lmax = 2048
    th = np.array([1e-4, 3e-3, 0.05, 0.6])
    x, s = np.cos(th), np.sin(th)
    geo = W.Geometry(x, s, np.zeros(4), np.full(4, 8, np.int64), np.arange(4) * 8, 32)
    a = W.random_alm(lmax, [105], spectrum="flat")
    d = P.Plan(lmax, geo).alm2delta(_to_dev(a).reshape(1, -1)).cpu().numpy()[0].T
    e = ref.delta(lmax, None, x, s, a)
    for r in range(4):
        assert _rel(d[r], e[r]) < 1e-11, r


# ------------------------------------------------------------------ Fourier

# 44, 52, 356, 8156: HEALPix polar-cap lengths 4 p with p prime (half-split
# Bluestein)
@pytest.mark.parametrize("nphi", [1, 2, 3, 4, 5, 6, 7, 8, 11, 12, 13, 16, 30, 31, 44, 52, 64, 97,
                                  100, 128, 210, 254, 255, 256, 356, 1000, 1024, 2046, 4094,
                                  4096, 8156, 8190, 8192])
def test_ring_synthesis_parity(P, nphi):
    _say("ring synthesis nphi", nphi)
    rng = np.random.default_rng(nphi)
    mmax = 300
    mval = np.arange(mmax + 1, dtype=np.int32)
    nr = 3
    phi0 = np.array([0.0, np.pi / nphi, 0.37])
    geo = W.Geometry(np.array([0.6, 0.0, -0.6]), np.array([0.8, 1.0, 0.8]), phi0,
                     np.full(nr, nphi, np.int64), np.arange(nr) * nphi, nr * nphi)
    dl = rng.standard_normal((nr, mmax + 1)) + 1j * rng.standard_normal((nr, mmax + 1))
    dl[:, 0] = dl[:, 0].real
    plan = P.Plan(mmax, geo, mval=mval)
    got = plan.delta2map(_to_dev(np.ascontiguousarray(dl.T)).reshape(1, mmax + 1, nr)).cpu().numpy()[0]
    exp = ref.map_from_delta(mval, geo, dl)
    assert np.max(np.abs(got - exp)) < 1e-13 * np.max(np.abs(exp)) * max(1, np.log2(nphi + 1))


@pytest.mark.parametrize("nphi", [1, 2, 3, 6, 7, 12, 31, 44, 52, 100, 254, 356, 1000, 4094,
                                  4096, 8156])
def test_ring_analysis_parity(P, nphi):
    _say("ring analysis nphi", nphi)
    rng = np.random.default_rng(1000 + nphi)
    mmax = 260
    mval = np.arange(mmax + 1, dtype=np.int32)
    nr = 2
    phi0 = np.array([0.1, 0.0])
    geo = W.Geometry(np.array([0.6, -0.6]), np.array([0.8, 0.8]), phi0,
                     np.full(nr, nphi, np.int64), np.arange(nr) * nphi, nr * nphi)
    g = rng.standard_normal(nr * nphi)
    plan = P.Plan(mmax, geo, mval=mval)
    got = plan.map2delta_adjoint(_to_dev(g).reshape(1, -1)).cpu().numpy()[0].T   # -> [ring][m]
    for r in range(nr):
        exp = ref.ring_analysis(g[r * nphi:(r + 1) * nphi], mval, phi0[r])
        assert np.max(np.abs(got[r] - exp)) < 1e-13 * np.max(np.abs(exp)) * max(1, np.log2(nphi + 1))


# ------------------------------------------------------------ whole transform

@pytest.mark.parametrize("lmax,nside", [(64, 32), (128, 64), (300, 128)])
def test_alm2map_parity_healpix(P, lmax, nside):
    _say("alm2map healpix", lmax, nside)
    g = W.healpix_geometry(nside)
    a = W.random_alm(lmax, [106, lmax])
    got = P.Plan(lmax, g).alm2map(_to_dev(a).reshape(1, -1)).cpu().numpy()[0]
    exp = ref.alm2map(lmax, g, a)
    assert _rel(got, exp) < 1e-12


def test_alm2map_gl_and_odd_rings(P):
    _say("alm2map GL and ECP odd")
    for lmax, g in [(40, W.gl_geometry(41, 81)), (33, W.ecp_geometry(35, 67))]:
        a = W.random_alm(lmax, [107, lmax])
        got = P.Plan(lmax, g).alm2map(_to_dev(a).reshape(1, -1)).cpu().numpy()[0]
        exp = ref.alm2map(lmax, g, a)
        assert _rel(got, exp) < 1e-12


def test_adjoint_parity_and_dot_product(P):
    _say("adjoint parity + dot test")
    lmax, nside, nmaps = 96, 48, 2
    g = W.healpix_geometry(nside)
    plan = P.Plan(lmax, g, nmaps=nmaps)
    maps = np.stack([W.random_map(g.npix, [108, i]) for i in range(nmaps)])
    got = plan.alm2map_adjoint(_to_dev(maps)).cpu().numpy()
    alms = np.stack([W.random_alm(lmax, [109, i]) for i in range(nmaps)])
    fwd = plan.alm2map(_to_dev(alms)).cpu().numpy()
    for i in range(nmaps):
        exp = ref.alm2map_adjoint(lmax, g, maps[i])
        assert _rel(got[i], exp) < 1e-12
        lhs = float(np.dot(fwd[i], maps[i]))
        rhs = float(np.sum(alms[i].real * got[i].real + alms[i].imag * got[i].imag))
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_determinism(P):
    _say("determinism")
    lmax, nside = 128, 64
    g = W.healpix_geometry(nside)
    a = _to_dev(W.random_alm(lmax, [110])).reshape(1, -1)
    plan = P.Plan(lmax, g)
    m1 = plan.alm2map(a).cpu().numpy()
    m2 = plan.alm2map(a).cpu().numpy()
    assert np.array_equal(m1, m2)
    mp = _to_dev(W.random_map(g.npix, [111])).reshape(1, -1)
    b1 = plan.alm2map_adjoint(mp).cpu().numpy()
    b2 = plan.alm2map_adjoint(mp).cpu().numpy()
    assert np.array_equal(b1, b2)


def test_error_paths(P):
    _say("error paths")
    import ctypes
    from paper_1010_1260_amd import _lib as L
    g = W.healpix_geometry(4)
    plan = P.Plan(8, g)
    lib = L.load()
    a = torch.zeros((1, plan.nalm), dtype=torch.complex128, device=_dev())
    m = torch.zeros((1, plan.npix), dtype=torch.float64, device=_dev())
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=_dev())
    v = ctypes.c_void_p
    assert lib.sht_alm2map(plan.handle, v(a.data_ptr()), v(m.data_ptr()), v(ws.data_ptr()),
                           16, None) == L.SHT_ERR_WORKSPACE
    assert lib.sht_alm2map(plan.handle, None, v(m.data_ptr()), v(ws.data_ptr()),
                           ws.numel(), None) == L.SHT_ERR_INVALID_ARG
    assert lib.sht_alm2map(None, v(a.data_ptr()), v(m.data_ptr()), v(ws.data_ptr()),
                           ws.numel(), None) == L.SHT_ERR_BAD_HANDLE
    assert lib.sht_alm2map(plan.handle, v(a.data_ptr()), v(m.data_ptr()), v(ws.data_ptr()),
                           ws.numel(), None) == L.SHT_OK
    torch.cuda.synchronize()


# --------------------------------------------------------- full-size sample

@pytest.mark.slow
def test_alm2map_l4096_nside2048_sampled_rings(P):
    """Full-size FP64 workload in the benchmark's launch configuration; the
    oracle recomputes a sample of rings (poles, caps, belt, equator)."""
    _say("alm2map l4096 nside2048 sampled")
    cfg = W.CONFIGS[2]
    L, N = cfg["lmax"], cfg["nside"]
    g = W.healpix_geometry(N)
    a = W.config_alm(2)
    plan = P.Plan(L, g)
    got = plan.alm2map(_to_dev(a).reshape(1, -1))
    torch.cuda.synchronize()
    got = got.cpu().numpy()[0]
    rings = [0, 1, 7, 100, N - 2, N - 1, N, 2 * N - 1, 3 * N, 4 * N - 3, 4 * N - 2]
    exp = ref.alm2map_rings(L, g, a, rings)
    num = den = 0.0
    for r, e in zip(rings, exp):
        s0, n = int(g.ringstart[r]), int(g.nphi[r])
        gg = got[s0:s0 + n]
        num += float(np.sum((gg - e) ** 2))
        den += float(np.sum(e ** 2))
        assert np.max(np.abs(gg - e)) < 1e-11 * max(np.max(np.abs(e)), 1e-300), r
    assert np.sqrt(num / den) < 1e-12
