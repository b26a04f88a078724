"""Batched uneven transforms: one persistent Legendre launch for maps of
different l_max / nside, autotuned launch shape, HIP graph replay.

The persistent kernel's atomic counter only hands out tiles, and every
tile's arithmetic is that of the single-plan kernel, so the batch must equal
the single-plan transforms bitwise, for every launch shape; the single-plan
path is itself checked against the oracle.
"""
import os
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


def _setup(P, lmaxes, seed0):
    plans, alms, singles = [], [], []
    for i, L in enumerate(lmaxes):
        g = W.healpix_geometry(max(1, L // 2))
        p = P.Plan(L, g)
        a = torch.from_numpy(W.random_alm(L, [seed0, i], spectrum="inv_l2")).to(_dev())
        plans.append(p)
        alms.append(a)
        singles.append(p.alm2map(a.reshape(1, -1)).reshape(-1))
    return plans, alms, singles


def test_batch_equals_single_plans_every_config(P):
    _say("batch vs single plans, all launch shapes")
    lmaxes = [16, 64, 32, 128, 16, 96, 64, 2, 0, 128, 50, 33]
    plans, alms, singles = _setup(P, lmaxes, 601)
    b = P.Batch(plans)
    for ch in (1, 2, 4):
        for w in (1, 4, 8, 16, 32):   # every entry of the default table among them
            b.set_config(ch, w)
            outs = b.alm2map(alms)
            torch.cuda.synchronize()
            for i in range(len(plans)):
                assert torch.equal(outs[i], singles[i]), (ch, w, i)
    # the single-plan path against the oracle for two of the maps
    for i in (3, 10):
        L = lmaxes[i]
        g = W.healpix_geometry(max(1, L // 2))
        exp = ref.alm2map(L, g, alms[i].cpu().numpy())
        got = singles[i].cpu().numpy()
        assert np.linalg.norm(got - exp) <= 1e-12 * np.linalg.norm(exp)


def test_batch_default_shape_follows_size(P):
    """The default launch shape comes from the size table: (2 chains, 4 waves
    per CU) up to 4 tiles of 128 ring pairs per CU, (4, 8) up to 16, (4, 16)
    above."""
    _say("batch default shape by size")
    ncu = torch.cuda.get_device_properties(_dev()).multi_processor_count

    def tiles_per_cu(plans):
        return sum(((p.npairs + 127) // 128) * ((p.nm + 1) // 2) for p in plans) / ncu

    for lmax, nmaps in [(16, 1), (256, 8), (512, 32)]:
        plans = [P.Plan(lmax, W.healpix_geometry(lmax // 2)) for _ in range(nmaps)]
        t = tiles_per_cu(plans)
        exp = (2, 4) if t <= 4 else ((4, 8) if t <= 16 else (4, 16))
        assert P.Batch(plans).config == exp, (lmax, nmaps, t)


def test_batch_autotune_and_cache(P, tmp_path):
    _say("batch autotune + cache")
    plans, alms, singles = _setup(P, [64, 128, 32, 128, 96], 602)
    b = P.Batch(plans)
    outs = b.new_maps()
    cache = str(tmp_path / "tune.txt")
    cfg = b.autotune(alms, outs, cache)
    assert cfg[0] in (1, 2, 4) and cfg[1] in (4, 8, 16)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:3] == [str(cfg[0]), str(cfg[1])]
    b2 = P.Batch(plans)
    b2.set_config(1, 1)
    assert b2.autotune(alms, b2.new_maps(), cache) == cfg     # read from the cache
    assert len(open(cache).read().strip().splitlines()) == 1
    outs = b2.alm2map(alms)
    torch.cuda.synchronize()
    for i in range(len(plans)):
        assert torch.equal(outs[i], singles[i])


def test_batch_graph_replay(P):
    _say("batch graph capture and replay")
    plans, alms, singles = _setup(P, [128, 64, 96, 32], 603)
    b = P.Batch(plans)
    outs = b.new_maps()
    s = torch.cuda.Stream(device=_dev())
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        b.capture(alms, outs, s)
    s.synchronize()
    other = P.Plan(64, W.healpix_geometry(32))
    oa = torch.from_numpy(W.random_alm(64, [604])).to(_dev()).reshape(1, -1)
    for rep in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        b.replay(s)
        s.synchronize()
        for i in range(len(plans)):
            assert torch.equal(outs[i], singles[i]), (rep, i)
        # eager work between replays
        other.alm2map(oa)
        torch.cuda.synchronize()


@pytest.mark.slow
def test_batch_uneven_64_maps(P):
    """The batched uneven workload: 64 maps, l_max uniform over {256, 512,
    1024, 2048}, nside = l_max / 2, C_l = l^-2, autotuned, graph replayed."""
    _say("batch uneven 64 maps")
    lmaxes = W.uneven_lmax()
    plans, alms, singles = _setup(P, lmaxes, 4)
    b = P.Batch(plans)
    outs = b.new_maps()
    b.autotune(alms, outs)
    s = torch.cuda.Stream(device=_dev())
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        b.capture(alms, outs, s)
    for o in outs:
        o.zero_()
    torch.cuda.synchronize()
    b.replay(s)
    s.synchronize()
    for i in range(len(plans)):
        assert torch.equal(outs[i], singles[i]), i
    # oracle on sampled rings of the largest map
    i = int(np.argmax(lmaxes))
    L = lmaxes[i]
    g = W.healpix_geometry(L // 2)
    rings = [0, 5, L // 2, L - 1, 3 * (L // 2), 4 * (L // 2) - 2]
    exp = ref.alm2map_rings(L, g, alms[i].cpu().numpy(), rings)
    got = outs[i].cpu().numpy()
    num = den = 0.0
    for r, e in zip(rings, exp):
        s0, n = int(g.ringstart[r]), int(g.nphi[r])
        num += float(np.sum((got[s0:s0 + n] - e) ** 2))
        den += float(np.sum(e ** 2))
    assert np.sqrt(num / den) < 1e-12


def test_batch_two_streams_distinct_workspaces(P):
    """Transforms of one batch enqueued on two streams at once, each with the
    workspace the binding keeps for its stream: the persistent kernel's work
    counter lives in the workspace, so the launches hand out their own tiles
    and both equal the single-plan maps bitwise."""
    _say("one batch on two streams with distinct workspaces")
    lmaxes = [256, 128, 512, 64, 256, 96, 384, 128]
    plans, alms, singles = _setup(P, lmaxes, 604)
    b = P.Batch(plans)
    b.set_config(1, 2)   # few persistent waves: each launch runs long enough to overlap
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        ws1 = b.workspace()
    with torch.cuda.stream(s2):
        ws2 = b.workspace()
    assert ws1.data_ptr() != ws2.data_ptr()
    res = []
    for rep in range(3):
        with torch.cuda.stream(s1):
            o1 = b.alm2map(alms)
        with torch.cuda.stream(s2):
            o2 = b.alm2map(alms)
        res.append((o1, o2))
    torch.cuda.synchronize()
    for rep, (o1, o2) in enumerate(res):
        for i in range(len(plans)):
            assert torch.equal(o1[i], singles[i]), (rep, 1, i)
            assert torch.equal(o2[i], singles[i]), (rep, 2, i)
