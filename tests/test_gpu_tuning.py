"""Launch shape of the FP64 forward Legendre kernel (ring pairs per lane) and
its autotuner: every shape gives bitwise the same result, the autotuner keeps
a valid shape and honours its cache, and the mixed plans reject the setting.
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


@pytest.mark.parametrize("lmax,nside,nmaps", [(200, 64, 2), (97, 50, 3), (300, 150, 1)])
def test_every_shape_bitwise_equal(P, lmax, nside, nmaps):
    """Ring-pair counts 128, 100 and 300: full, partial and ragged last
    blocks at 64, 128 and 256 pairs per wave."""
    _say("fwd chains bitwise", lmax, nside, nmaps)
    g = W.healpix_geometry(nside)
    alms = np.stack([W.random_alm(lmax, [601, i]) for i in range(nmaps)])
    a = torch.from_numpy(alms).to(_dev())
    plan = P.Plan(lmax, g, nmaps=nmaps)
    assert plan.config in (1, 2, 4)
    outs = {}
    for ch in (1, 2, 4):
        plan.set_config(ch)
        assert plan.config == ch
        outs[ch] = (plan.alm2delta(a).cpu(), plan.alm2map(a).cpu())
    for ch in (2, 4):
        assert torch.equal(outs[ch][0], outs[1][0]), ch
        assert torch.equal(outs[ch][1], outs[1][1]), ch
    for i in range(nmaps):
        assert _rel(outs[1][1][i].numpy(), ref.alm2map(lmax, g, alms[i])) < 1e-12


def test_autotune_and_cache(P, tmp_path):
    _say("plan autotune + cache")
    lmax, nside = 256, 128
    g = W.healpix_geometry(nside)
    a = torch.from_numpy(W.random_alm(lmax, [602])).to(_dev())
    cache = str(tmp_path / "tune.txt")
    p1 = P.Plan(lmax, g)
    best = p1.autotune(a, cache_path=cache)
    assert best in (1, 2, 4)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].split()[1] == str(best)
    p2 = P.Plan(lmax, g)
    p2.set_config(4 if best != 4 else 1)
    assert p2.autotune(a, cache_path=cache) == best           # from the cache, no new line
    assert len(open(cache).read().splitlines()) == 1
    m1 = p1.alm2map(a).cpu()
    p1.set_config(1)
    assert torch.equal(m1, p1.alm2map(a).cpu())


def test_config_errors(P):
    _say("plan config errors")
    g = W.healpix_geometry(16)
    p = P.Plan(32, g)
    for bad in (0, 3, 8, -1):
        with pytest.raises(P.ShtError):
            p.set_config(bad)
    pm = P.Plan(32, g, nmaps=2, precision="fp32_mfma")
    with pytest.raises(P.ShtError):
        pm.set_config(1)
    a = torch.zeros((2, pm.nalm), dtype=torch.complex128, device=_dev())
    before = pm.config
    assert pm.autotune(a) == before                           # nothing to tune
    with pytest.raises(ValueError):
        p.alm2map(torch.zeros(p.nalm, dtype=torch.complex128, device=_dev()),
                  out=torch.empty(p.npix - 1, dtype=torch.float64, device=_dev()))


def test_default_shape_follows_size(P):
    """The size table picks one pair per lane for launches too small to fill
    the chip and two for large ones."""
    _say("default shape by size")
    small = P.Plan(64, W.healpix_geometry(32))
    large = P.Plan(2048, W.healpix_geometry(1024))
    assert small.config == 1
    assert large.config == 2


def test_stale_error_of_the_caller_is_not_reported(P):
    """A failed HIP call of the caller (here an invalid device index, which
    changes nothing) must not surface as an error of the next library call
    that launches kernels (plan creation launches the Bluestein table
    kernel for rings of 44 pixels and others at nside 32)."""
    import ctypes
    _say("stale caller error")
    hip = ctypes.CDLL("libamdhip64.so")
    assert hip.hipSetDevice(ctypes.c_int(9999)) != 0
    plan = P.Plan(64, W.healpix_geometry(32))
    a = torch.from_numpy(W.random_alm(64, [603])).to(_dev())
    assert hip.hipSetDevice(ctypes.c_int(9999)) != 0
    plan.alm2map(a)
    torch.cuda.synchronize()


def test_forward_workspace_suffices_for_synthesis(P):
    """Synthesis runs in forward_workspace_bytes and refuses one byte less;
    workspace_bytes covers every call (the adjoint also keeps partial sums
    per block of 256 ring pairs) and the adjoint refuses one byte less."""
    import ctypes
    from paper_1010_1260_amd import _lib as L
    _say("forward-only workspace")
    lmax, nside, nmaps = 128, 160, 3
    g = W.healpix_geometry(nside)
    plan = P.Plan(lmax, g, nmaps=nmaps)
    fwd = int(plan.info.forward_workspace_bytes)
    full = int(plan.workspace_bytes)
    assert 0 < fwd <= full
    alms = np.stack([W.random_alm(lmax, [604, i]) for i in range(nmaps)])
    a = torch.from_numpy(alms).to(_dev())
    ws = torch.empty(fwd, dtype=torch.uint8, device=_dev())
    out = torch.empty((nmaps, plan.npix), dtype=torch.float64, device=_dev())
    lib = L.load()
    st = ctypes.c_void_p(torch.cuda.current_stream(_dev()).cuda_stream)
    vp = ctypes.c_void_p
    assert lib.sht_alm2map(plan.handle, vp(a.data_ptr()), vp(out.data_ptr()), vp(ws.data_ptr()),
                           fwd, st) == L.SHT_OK
    assert lib.sht_alm2map(plan.handle, vp(a.data_ptr()), vp(out.data_ptr()), vp(ws.data_ptr()),
                           fwd - 1, st) == L.SHT_ERR_WORKSPACE
    adj = torch.empty((nmaps, plan.nalm), dtype=torch.complex128, device=_dev())
    wsf = torch.empty(full, dtype=torch.uint8, device=_dev())
    assert lib.sht_alm2map_adjoint(plan.handle, vp(out.data_ptr()), vp(adj.data_ptr()),
                                   vp(wsf.data_ptr()), full - 1, st) == L.SHT_ERR_WORKSPACE
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for i in range(nmaps):
        assert _rel(got[i], ref.alm2map(lmax, g, alms[i])) < 1e-12


def test_decision_log(P, tmp_path):
    """SHT_LOG=1 makes plan and batch creation and the autotuner report their
    decisions on stderr; without it the library prints nothing."""
    import subprocess
    import sys as _sys
    _say("decision log")
    root = __import__("os").path.dirname(__import__("os").path.dirname(__import__("os").path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import torch, workloads as W\n"
        "from paper_1010_1260_amd import Plan, Batch\n"
        "p = Plan(128, W.healpix_geometry(64))\n"
        "a = torch.from_numpy(W.random_alm(128, [7])).to('cuda:0').reshape(1, -1)\n"
        "p.autotune(a)\n"
        "b = Batch([p, Plan(64, W.healpix_geometry(32))])\n"
        "torch.cuda.synchronize()\n" % root)
    env = dict(__import__("os").environ, SHT_LOG="1")
    r = subprocess.run([_sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    for key in ("sht: plan l_max=128", "sht: plan synthesis rings: fast path",
                "sht: plan fast ring nphi=256: half length 128 = 16x8",
                "sht: autotune plan:", "sht: batch maps=2"):
        assert key in r.stderr, (key, r.stderr)
    env["SHT_LOG"] = "0"
    r = subprocess.run([_sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=120)
    assert r.returncode == 0 and "sht:" not in r.stderr
