"""GPU parity of the mixed-precision batched Legendre stage (FP64 recurrence,
FP32, 3-way split BF16 or 2-way split FP16 matrix-core contraction) against
the FP64 oracle.  Bound: relative L2
error <= 1e-6 per map (the target for the mixed forms); the emulated error of
the two-level FP32 accumulation is about 1e-7."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import ref

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-6


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


PRECS = ["fp32_mfma", "bf16x3_mfma", "f16x2_mfma"]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("lmax,nside,nmaps", [(64, 32, 1), (200, 64, 3), (255, 100, 16),
                                              (130, 40, 17), (31, 16, 2), (0, 2, 1), (1, 2, 2)])
def test_mixed_delta_and_map_parity(P, lmax, nside, nmaps, prec):
    _say("mixed delta/map", prec, lmax, nside, nmaps)
    g = W.healpix_geometry(nside)
    alms = np.stack([W.random_alm(lmax, [301, lmax, i], spectrum="flat" if lmax < 2 else "inv_l_lp1")
                     for i in range(nmaps)])
    plan = P.Plan(lmax, g, nmaps=nmaps, precision=prec)
    a = torch.from_numpy(alms).to(_dev())
    d = np.swapaxes(plan.alm2delta(a).cpu().numpy(), 1, 2)   # -> [map][ring][m]
    mp = plan.alm2map(a).cpu().numpy()
    for i in range(nmaps):
        e = ref.delta(lmax, None, g.cth, g.sth, alms[i])
        assert _rel(d[i], e) < TOL, i
        em = ref.map_from_delta(np.arange(lmax + 1), g, e)
        assert _rel(mp[i], em) < TOL, i


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_partial_mset_ragged(P, prec):
    _say("mixed partial m-set, ragged", prec)
    lmax = 97
    mval = np.array([0, 1, 5, 6, 7, 40, 41, 90, 97], np.int32)
    g = W.ecp_geometry(37, 21)
    alms = np.stack([W.random_alm(lmax, [302, i], mval=mval) for i in range(5)])
    plan = P.Plan(lmax, g, mval=mval, nmaps=5, precision=prec)
    d = np.swapaxes(plan.alm2delta(torch.from_numpy(alms).to(_dev())).cpu().numpy(), 1, 2)
    for i in range(5):
        e = ref.delta(lmax, mval, g.cth, g.sth, alms[i])
        assert _rel(d[i], e) < TOL


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_matches_fp64_path(P, prec):
    _say("mixed vs fp64 kernel", prec)
    lmax, nside, nmaps = 300, 128, 4
    g = W.healpix_geometry(nside)
    alms = np.stack([W.random_alm(lmax, [303, i]) for i in range(nmaps)])
    a = torch.from_numpy(alms).to(_dev())
    m64 = P.Plan(lmax, g, nmaps=nmaps).alm2map(a).cpu().numpy()
    m32 = P.Plan(lmax, g, nmaps=nmaps, precision=prec).alm2map(a).cpu().numpy()
    for i in range(nmaps):
        assert _rel(m32[i], m64[i]) < TOL


@pytest.mark.slow
@pytest.mark.parametrize("prec", PRECS)
def test_mixed_l4096_nside2048_x16_sampled(P, prec):
    _say("mixed l4096 nside2048 x16 sampled rings", prec)
    L, N, nmaps = 4096, 2048, 16
    g = W.healpix_geometry(N)
    alms = [W.random_alm(L, [3, i]) for i in range(nmaps)]
    plan = P.Plan(L, g, nmaps=nmaps, precision=prec)
    out = plan.alm2map(torch.from_numpy(np.stack(alms)).to(_dev()))
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    rings = [0, 3, 300, N - 1, 2 * N - 1, 3 * N + 5, 4 * N - 2]
    for i in [0, 7, 15]:
        exp = ref.alm2map_rings(L, g, alms[i], rings)
        num = den = 0.0
        for r, e in zip(rings, exp):
            s0, n = int(g.ringstart[r]), int(g.nphi[r])
            num += float(np.sum((out[i, s0:s0 + n] - e) ** 2))
            den += float(np.sum(e ** 2))
        assert np.sqrt(num / den) < TOL, i


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_coefficient_range(P, prec):
    """Coefficients spread over many binades: whole maps scaled by 1e-25 and
    1e25 (inside the FP32 range the mixed forms accumulate in), and one map
    whose m-blocks differ by up to 1e30.  The split-FP16 form rescales per
    map and 128-row block of l, so its error stays that of the FP32 form."""
    _say("mixed coefficient range", prec)
    lmax, nside = 300, 96
    g = W.healpix_geometry(nside)
    mv = np.arange(lmax + 1)
    off = W.alm_offsets(lmax, mv)
    base = [W.random_alm(lmax, [305, i]) for i in range(4)]
    wild = base[3].copy()
    for m in range(lmax + 1):
        wild[off[m]:off[m] + lmax - m + 1] *= 10.0 ** (30 * ((m % 7) / 6.0) - 15)
    # l-dependent spread inside an m as well: 128-row blocks of very different size
    ll = np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])
    wild *= 10.0 ** (((ll // 64) % 3) * 6.0 - 6.0)
    alms = np.stack([base[0] * 1e-25, base[1] * 1e25, base[2], wild])
    plan = P.Plan(lmax, g, nmaps=4, precision=prec)
    mp = plan.alm2map(torch.from_numpy(alms).to(_dev())).cpu().numpy()
    for i in range(4):
        em = ref.alm2map(lmax, g, alms[i])
        assert np.all(np.isfinite(mp[i])), i
        assert _rel(mp[i], em) < TOL, i


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_bluestein_fast_rings(P, prec):
    """Rings of 4 i pixels with i not 7-smooth take the mixed forms' complex64
    Bluestein path (even- and odd-indexed convolutions side by side, lengths
    21 to 4096): from heavy aliasing (44 pixels at m_max 4096) to rings longer
    than m_max, beside 7-smooth and odd rings, at odd pixel offsets (unaligned
    stores), ring by ring against the oracle."""
    _say("mixed Bluestein fast-path rings", prec)
    L, N = 4096, 2048
    g0 = W.healpix_geometry(N)
    # north-cap ring i - 1 has 4 i pixels; 2048 and 1536 are 7-smooth, the
    # equator ring 2 N - 1 has 4 N
    ivals = [11, 13, 22, 97, 509, 1021, 1023, 1031, 2039, 2047, 2048, 1536]
    rings = [i - 1 for i in ivals] + [2 * N - 1]
    # plus an odd ring, and 7560 pixels: half length 3780 = 4 x 7 x 5 x 27 is
    # 7-smooth, but its radix-7 pass would need three butterflies per thread
    # on the fast path, so the mixed forms take it through Bluestein
    nphi = np.array([int(g0.nphi[r]) for r in rings] + [4093, 7560], np.int64)
    cth = np.append(g0.cth[rings], [0.3, -0.55])
    sth = np.sqrt(1.0 - cth * cth)
    phi0 = np.append(g0.phi0[rings], [0.1, 0.0])
    start = np.concatenate([[1], 1 + np.cumsum(nphi[:-1] + 1)]).astype(np.int64)
    g = W.Geometry(cth, sth, phi0, nphi, start, int(start[-1] + nphi[-1]), "bluestein rings")
    nmaps = 2
    alms = np.stack([W.random_alm(L, [306, i]) for i in range(nmaps)])
    plan = P.Plan(L, g, nmaps=nmaps, precision=prec)
    out = plan.alm2map(torch.from_numpy(alms).to(_dev())).cpu().numpy()
    for i in range(nmaps):
        exp = ref.alm2map_rings(L, g, alms[i], list(range(len(nphi))))
        num = den = 0.0
        for r, e in enumerate(exp):
            got = out[i, start[r]:start[r] + nphi[r]]
            assert _rel(got, e) < 4 * TOL, (i, r, int(nphi[r]))
            num += float(np.sum((got - e) ** 2))
            den += float(np.sum(e ** 2))
        assert np.sqrt(num / den) < TOL, i
        # the gaps between the rings stay untouched
        gaps = np.ones(out.shape[1], bool)
        for r in range(len(nphi)):
            gaps[start[r]:start[r] + nphi[r]] = False
        assert np.all(out[i, gaps] == 0.0), i
    # the same plan's Fourier stage from a caller's complex128 Delta (the FP64
    # size-class kernels take these rings then)
    dls = [ref.delta(L, None, g.cth, g.sth, alms[i]) for i in range(nmaps)]
    d_dev = torch.from_numpy(np.stack([np.ascontiguousarray(d.T) for d in dls])).to(_dev())
    got = plan.delta2map(d_dev).cpu().numpy()
    for i in range(nmaps):
        em = ref.map_from_delta(np.arange(L + 1), g, dls[i])
        assert _rel(got[i], em) < 1e-12, i


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_gappy_mset_fast_paths(P, prec):
    """A gappy m-set (the fold looks each mode's position up) on HEALPix
    rings, so that both ring fast paths (smooth belt and caps, and the
    Bluestein caps of 4 i pixels with i not 7-smooth) take it, against the
    oracle."""
    _say("mixed gappy m-set on the ring fast paths", prec)
    lmax, nside, nmaps = 300, 64, 3
    mval = np.array([0, 1, 2, 5, 17, 40, 41, 100, 150, 199, 200, 263, 299, 300], np.int32)
    g = W.healpix_geometry(nside)
    alms = np.stack([W.random_alm(lmax, [307, i], mval=mval) for i in range(nmaps)])
    plan = P.Plan(lmax, g, mval=mval, nmaps=nmaps, precision=prec)
    got = plan.alm2map(torch.from_numpy(alms).to(_dev())).cpu().numpy()
    for i in range(nmaps):
        assert _rel(got[i], ref.alm2map(lmax, g, alms[i], mval=mval)) < TOL, i
