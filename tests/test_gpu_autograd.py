"""Differentiation through the hand-written adjoint (torch.autograd.Function).

Workload: 8 maps, l_max = 1024, HEALPix nside = 512; loss
0.5 ||alm2map(a) - d||^2 with d ~ N(0, 1) per pixel (seeded).  The gradient
from backward (the adjoint applied to alm2map(a) - d) is checked against
central finite differences (h = 1e-6, FP64) on more than 64 coordinates --
real and imaginary parts, m = 0, m = l, l = l_max -- and along random
directions, and against the CPU oracle's adjoint.
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


def test_gradcheck_tiny(P):
    _say("gradcheck tiny")
    lmax = 6
    g = W.healpix_geometry(2)
    plan = P.Plan(lmax, g, nmaps=2)
    a = torch.from_numpy(np.stack([W.random_alm(lmax, [501, i], spectrum="flat")
                                   for i in range(2)])).to(_dev()).requires_grad_(True)
    f = lambda x: P.alm2map(x, plan)  # noqa: E731
    assert torch.autograd.gradcheck(f, (a,), eps=1e-6, atol=1e-9, rtol=1e-7)


@pytest.fixture(scope="module")
def c5(P):
    cfg = W.CONFIGS[5]
    L, N, B = cfg["lmax"], cfg["nside"], cfg["nmaps"]
    g = W.healpix_geometry(N)
    alms = np.stack([W.config_alm(5, i) for i in range(B)])
    data = np.stack([W.random_map(g.npix, [5, 100 + i]) for i in range(B)])
    plan = P.Plan(L, g, nmaps=B)
    return dict(L=L, N=N, B=B, g=g, alms=alms, data=data, plan=plan)


def _grad(P, c):
    a = torch.from_numpy(c["alms"]).to(_dev()).requires_grad_(True)
    d = torch.from_numpy(c["data"]).to(_dev())
    s = P.alm2map(a, c["plan"])
    loss = 0.5 * torch.sum((s - d) ** 2)
    loss.backward()
    return a.grad.detach().cpu().numpy(), s.detach()


def _fd_coords(L, off):
    # (m, l, part) triples: m = 0 (real only), m = l, l = lmax, interior, both parts
    coords = []
    for m, l in [(0, 2), (0, 17), (0, L), (1, 1), (1, 5), (2, 2), (7, 300), (64, 64), (100, 1000),
                 (511, 512), (700, 1024), (1023, 1023), (1024, 1024), (3, L), (512, L), (9, 9)]:
        for part in (0, 1):
            if m == 0 and part == 1:
                continue
            coords.append((int(off[m] + (l - m)), part))
    rng = np.random.default_rng(77)
    while len(coords) < 72:
        m = int(rng.integers(0, L + 1))
        l = int(rng.integers(m, L + 1))
        part = int(rng.integers(0, 2)) if m > 0 else 0
        coords.append((int(off[m] + (l - m)), part))
    return coords


def test_c5_gradient_vs_central_differences(P, c5):
    _say("c5 gradient vs central differences")
    c = c5
    L, B = c["L"], c["B"]
    grad, _ = _grad(P, c)
    off = W.alm_offsets(L, W.mvals(L))
    coords = _fd_coords(L, off)
    h = 1e-6
    d = torch.from_numpy(c["data"]).to(_dev())
    base = torch.from_numpy(c["alms"]).to(_dev())
    plan = c["plan"]
    # perturb one coordinate per map per transform pair (the loss is a sum over maps)
    for start in range(0, len(coords), B):
        chunk = coords[start:start + B]
        ap = base.clone()
        am = base.clone()
        for b, (idx, part) in enumerate(chunk):
            delta = h if part == 0 else 1j * h
            ap[b, idx] += delta
            am[b, idx] -= delta
        sp = plan.alm2map(ap)
        sm = plan.alm2map(am)
        # L+ - L- = 0.5 sum (s+ - s-)(s+ + s- - 2 d), evaluated without cancellation
        dl = 0.5 * torch.sum((sp - sm) * (sp + sm - 2 * d), dim=1).cpu().numpy()
        for b, (idx, part) in enumerate(chunk):
            fd = dl[b] / (2 * h)
            gv = grad[b, idx].real if part == 0 else grad[b, idx].imag
            assert abs(fd - gv) <= 1e-5 * abs(gv) + 1e-7, (b, idx, part, fd, gv)
    # random directions
    rng = np.random.default_rng(78)
    for _ in range(4):
        v = np.stack([W.random_alm(L, [rng.integers(1 << 30)], spectrum="flat") for _ in range(B)])
        vt = torch.from_numpy(v).to(_dev())
        sp = plan.alm2map(base + h * vt)
        sm = plan.alm2map(base - h * vt)
        dl = float(0.5 * torch.sum((sp - sm) * (sp + sm - 2 * d)).cpu()) / (2 * h)
        gd = float(np.sum(grad.real * v.real + grad.imag * v.imag))
        assert abs(dl - gd) <= 1e-5 * abs(gd), (dl, gd)
    # Im a_l0 does not enter the map: its gradient is exactly zero
    assert np.all(grad[:, off[0]:off[1]].imag == 0)


def test_c5_adjoint_vs_cpu_adjoint_and_dot(P, c5):
    _say("c5 adjoint vs cpu adjoint")
    c = c5
    L, B, g = c["L"], c["B"], c["g"]
    plan = c["plan"]
    res = torch.from_numpy(c["data"]).to(_dev())
    gpu = plan.alm2map_adjoint(res).cpu().numpy()
    for b in (0, B - 1):
        exp = ref.alm2map_adjoint(L, g, c["data"][b])
        err = np.linalg.norm(gpu[b] - exp) / np.linalg.norm(exp)
        assert err < 1e-12, (b, err)
    fwd = plan.alm2map(torch.from_numpy(c["alms"]).to(_dev())).cpu().numpy()
    for b in range(B):
        lhs = float(np.dot(fwd[b], c["data"][b]))
        rhs = float(np.sum(c["alms"][b].real * gpu[b].real + c["alms"][b].imag * gpu[b].imag))
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0), b
