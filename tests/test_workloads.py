"""Input generators: HEALPix ring invariants and seeded coefficient draws."""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("N", [1, 2, 4, 32, 512, 2048])
def test_healpix_invariants(N):
    g = W.healpix_geometry(N)
    assert g.nrings == 4 * N - 1
    assert int(np.sum(g.nphi)) == 12 * N * N == g.npix
    # contiguous, increasing ring starts
    assert g.ringstart[0] == 0
    assert np.all(g.ringstart[1:] == g.ringstart[:-1] + g.nphi[:-1])
    # bitwise north/south symmetry and the equator
    R = g.nrings
    assert np.array_equal(g.cth, -g.cth[::-1])
    assert np.array_equal(g.sth, g.sth[::-1])
    assert g.cth[2 * N - 1] == 0.0 and g.sth[2 * N - 1] == 1.0
    assert np.allclose(g.cth ** 2 + g.sth ** 2, 1.0, rtol=0, atol=4e-16)
    assert np.all(np.diff(g.cth) < 0)
    if N > 1:
        assert g.cth[0] == 1.0 - 1.0 / (3.0 * N * N)
        assert g.nphi[0] == 4 and g.nphi[N - 1] == 4 * N
    assert R == len(g.phi0)


def test_config_sizes():
    g = W.healpix_geometry(2048)
    assert g.npix == 50_331_648 and g.nrings == 8191
    assert W.nalm(4096) == 8_394_753
    g = W.healpix_geometry(32)
    assert g.npix == 12_288 and g.nrings == 127
    assert W.nalm(64) == 2145


def test_random_alm_statistics_and_seeding():
    L = 512
    a = W.random_alm(L, [1, 0])
    b = W.random_alm(L, [1, 0])
    c = W.random_alm(L, [1, 1])
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    off = W.alm_offsets(L, W.mvals(L))
    assert np.all(a[off[0]:off[1]].imag == 0)
    ell = np.concatenate([np.arange(m, L + 1) for m in range(L + 1)])
    assert np.all(a[ell < 2] == 0)
    # E|a_lm|^2 = C_l = 1/(l(l+1)): pooled estimate over many (l, m)
    sel = ell >= 2
    ratio = np.abs(a[sel]) ** 2 * ell[sel] * (ell[sel] + 1.0)
    assert abs(np.mean(ratio) - 1) < 0.02


def test_uneven_lmax_draw():
    ls = W.uneven_lmax()
    assert len(ls) == 64 and set(ls) <= {256, 512, 1024, 2048}
    assert ls == W.uneven_lmax()
