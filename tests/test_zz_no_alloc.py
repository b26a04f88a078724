"""sht_alm2map_noalloc (workspace in the library's fixed device array) gives
bitwise the results of sht_alm2map with a caller workspace, through the C
ABI, on two calls in a row with the second input smaller than the first, in
FP64 and in a mixed form; plans whose workspace exceeds the array are refused.
"""
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


def _both(P, lmax, nside, nmaps, precision, seed):
    from paper_1010_1260_amd import _lib as L
    lib = L.load()
    vp = ctypes.c_void_p
    g = W.healpix_geometry(nside)
    plan = P.Plan(lmax, g, nmaps=nmaps, precision=precision)
    assert int(plan.info.forward_workspace_bytes) <= L.SHT_NOALLOC_SCRATCH_BYTES
    alms = np.stack([W.random_alm(lmax, [seed, i]) for i in range(nmaps)])
    a = torch.from_numpy(alms).to(_dev())
    ws = torch.empty(int(plan.info.forward_workspace_bytes), dtype=torch.uint8, device=_dev())
    ref_out = torch.empty((nmaps, plan.npix), dtype=torch.float64, device=_dev())
    out = torch.full((nmaps, plan.npix), float("nan"), dtype=torch.float64, device=_dev())
    st = vp(torch.cuda.current_stream(_dev()).cuda_stream)
    assert lib.sht_alm2map(plan.handle, vp(a.data_ptr()), vp(ref_out.data_ptr()),
                           vp(ws.data_ptr()), ws.numel(), st) == L.SHT_OK
    assert lib.sht_alm2map_noalloc(plan.handle, vp(a.data_ptr()), vp(out.data_ptr()),
                                   st) == L.SHT_OK
    torch.cuda.synchronize()
    return g, alms, out.cpu().numpy(), ref_out.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "f16x2_mfma"])
def test_noalloc_matches_alm2map_twice(P, precision):
    """First call l_max 256 / nside 128 / 2 maps, then l_max 48 / nside 24 /
    1 map on the same device array: both equal sht_alm2map bitwise and the
    oracle to the form's bound."""
    tol = 1e-12 if precision == "fp64" else 1e-6
    for (lmax, nside, nmaps, seed) in [(256, 128, 2, 901), (48, 24, 1, 902)]:
        _say("noalloc", precision, lmax, nside, nmaps)
        g, alms, got, exp = _both(P, lmax, nside, nmaps, precision, seed)
        assert np.array_equal(got, exp)
        for i in range(nmaps):
            o = ref.alm2map(lmax, g, alms[i])
            assert np.linalg.norm(got[i] - o) / np.linalg.norm(o) < tol


def test_noalloc_refuses_large_plans_and_bad_args(P):
    from paper_1010_1260_amd import _lib as L
    lib = L.load()
    vp = ctypes.c_void_p
    _say("noalloc limits")
    plan = P.Plan(2048, W.healpix_geometry(1024))
    assert int(plan.info.forward_workspace_bytes) > L.SHT_NOALLOC_SCRATCH_BYTES
    a = torch.zeros((1, plan.nalm), dtype=torch.complex128, device=_dev())
    out = torch.empty((1, plan.npix), dtype=torch.float64, device=_dev())
    st = vp(torch.cuda.current_stream(_dev()).cuda_stream)
    assert lib.sht_alm2map_noalloc(plan.handle, vp(a.data_ptr()), vp(out.data_ptr()),
                                   st) == L.SHT_ERR_WORKSPACE
    assert lib.sht_alm2map_noalloc(plan.handle, None, vp(out.data_ptr()),
                                   st) == L.SHT_ERR_INVALID_ARG
    assert lib.sht_alm2map_noalloc(None, vp(a.data_ptr()), vp(out.data_ptr()),
                                   st) == L.SHT_ERR_BAD_HANDLE
