"""GPU map2alm (quadrature-weighted analysis, Eq. map2almDef) through the C ABI
against the CPU oracle, plus its exactness on Gauss-Legendre rings and the
convergence of the Jacobi refinement at the differentiation workload's size.
FP64 bound as for the other transforms (relative L2 <= 1e-12 per map);
refinement through a mixed-precision alm2map: <= 1e-6."""
import ctypes
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


def _to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(_dev())


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("niter", [0, 2])
def test_map2alm_parity_healpix(P, niter):
    nside, lmax = 16, 30
    _say("map2alm healpix", nside, lmax, "niter", niter)
    g = W.healpix_geometry(nside)
    rng = np.random.default_rng(51)
    maps = np.stack([W.random_map(g.npix, [52, b]) for b in range(2)])
    w = 0.5 + rng.random(g.nrings)
    plan = P.Plan(lmax, g, nmaps=2)
    got = plan.map2alm(_to_dev(maps), w, niter=niter).cpu().numpy()
    for b in range(2):
        want = ref.map2alm(lmax, g, maps[b], w, niter=niter)
        assert _rel(got[b], want) < 1e-12
        assert np.max(np.abs(got[b] - want)) < 1e-12 * np.max(np.abs(want))


def test_map2alm_partial_m_set(P):
    nside, lmax = 8, 20
    _say("map2alm partial m-set", nside, lmax)
    g = W.healpix_geometry(nside)
    mval = np.array([0, 3, 4, 11, 20], dtype=np.int32)
    s = W.random_map(g.npix, [53])
    w = np.full(g.nrings, 4.0 * np.pi / g.npix)
    plan = P.Plan(lmax, g, mval=mval)
    got = plan.map2alm(_to_dev(s).reshape(1, -1), w, niter=1).cpu().numpy()[0]
    want = ref.map2alm(lmax, g, s, w, niter=1, mval=mval)
    assert _rel(got, want) < 1e-12


def test_map2alm_gauss_legendre_inverts_alm2map(P):
    lmax = 96
    _say("map2alm GL round trip", lmax)
    g = W.gl_geometry(lmax + 1, 2 * lmax + 2)
    a = W.random_alm(lmax, [54])
    plan = P.Plan(lmax, g)
    s = plan.alm2map(_to_dev(a).reshape(1, -1))
    back = plan.map2alm(s, g.weight).cpu().numpy()[0]
    assert np.max(np.abs(back - a)) < 1e-12 * np.max(np.abs(a))


def test_map2alm_refinement_differentiation_size(P):
    # the differentiation workload's geometry (l_max 1024, nside 512): for a
    # band-limited map the refinement error falls with every step
    lmax, nside = 1024, 512
    _say("map2alm refinement", lmax, nside)
    g = W.healpix_geometry(nside)
    a = W.random_alm(lmax, [5, 0])
    plan = P.Plan(lmax, g)
    s = plan.alm2map(_to_dev(a).reshape(1, -1))
    w = np.full(g.nrings, 4.0 * np.pi / g.npix)
    at = _to_dev(a).reshape(1, -1)
    errs = [float(torch.linalg.norm(plan.map2alm(s, w, niter=k) - at) / torch.linalg.norm(at))
            for k in (0, 1, 3)]
    _say("errors", errs)
    assert errs[1] < errs[0] and errs[2] < errs[1]


def test_map2alm_mixed_plan_refinement(P):
    nside, lmax = 16, 24
    _say("map2alm mixed refinement", nside, lmax)
    g = W.healpix_geometry(nside)
    maps = np.stack([W.random_map(g.npix, [55, b]) for b in range(3)])
    w = np.full(g.nrings, 4.0 * np.pi / g.npix)
    for prec in ("fp32_mfma", "bf16x3_mfma", "f16x2_mfma"):
        plan = P.Plan(lmax, g, nmaps=3, precision=prec)
        got = plan.map2alm(_to_dev(maps), w, niter=2).cpu().numpy()
        for b in range(3):
            want = ref.map2alm(lmax, g, maps[b], w, niter=2)
            assert _rel(got[b], want) < 1e-6, prec


def test_map2alm_error_paths(P):
    from paper_1010_1260_amd import _lib as L
    _say("map2alm error paths")
    g = W.healpix_geometry(4)
    plan = P.Plan(8, g)
    lib = L.load()
    s = torch.zeros(1, g.npix, dtype=torch.float64, device=_dev())
    w = torch.ones(g.nrings, dtype=torch.float64, device=_dev())
    a = torch.empty(1, plan.nalm, dtype=torch.complex128, device=_dev())
    ws = plan.workspace()
    vp = ctypes.c_void_p
    args = lambda niter, tmp, wsb: (plan.handle, vp(s.data_ptr()), vp(w.data_ptr()),
                                    vp(a.data_ptr()), niter, tmp, vp(ws.data_ptr()), wsb, None)
    assert lib.sht_map2alm(*args(1, None, ws.numel())) == L.SHT_ERR_INVALID_ARG
    assert lib.sht_map2alm(*args(-1, None, ws.numel())) == L.SHT_ERR_INVALID_ARG
    assert lib.sht_map2alm(*args(101, vp(s.data_ptr()), ws.numel())) == L.SHT_ERR_INVALID_ARG
    assert lib.sht_map2alm(*args(0, None, 16)) == L.SHT_ERR_WORKSPACE
    assert lib.sht_map2alm(plan.handle, vp(s.data_ptr()), None, vp(a.data_ptr()), 0, None,
                           vp(ws.data_ptr()), ws.numel(), None) == L.SHT_ERR_INVALID_ARG
    assert lib.sht_map2alm(*args(0, None, ws.numel())) == L.SHT_OK
    torch.cuda.synchronize()
