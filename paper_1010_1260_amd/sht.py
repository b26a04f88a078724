"""PyTorch-facing wrapper of the C ABI: plans, device buffers, streams, autograd.

PyTorch provides device memory and the current HIP stream; every step of the
transform runs in the library's kernels (see include/sht.h).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


def _cur_stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream_workspace(cache: dict, dev: torch.device, nbytes: int) -> torch.Tensor:
    """The workspace of at least `nbytes` kept in `cache` for the current
    stream of `dev`, allocated on that stream (torch's caching allocator
    then only hands its memory out again in that stream's order)."""
    need = max(1, int(nbytes))
    key = _cur_stream(dev)
    ws = cache.get(key)
    if ws is None or ws.numel() < need:
        cache.pop(key, None)
        with torch.cuda.device(dev):
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
        cache[key] = ws
    return ws


class Plan:
    """A transform plan for one ring geometry, band limit and m-set.

    geom: any object with numpy arrays cth, sth, phi0, nphi, ringstart
    (e.g. ``workloads.healpix_geometry``).  The plan's tables live on
    ``device`` (default: the current CUDA/HIP device).
    """

    PRECISIONS = {"fp64": 0, "fp32_mfma": 1, "bf16x3_mfma": 2, "f16x2_mfma": 3}

    def __init__(self, lmax: int, geom, mval=None, nmaps: int = 1, pairing: bool = True,
                 device=None, precision: str = "fp64"):
        lib = L.load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.lmax = int(lmax)
        self.mval = (np.arange(self.lmax + 1, dtype=np.int32) if mval is None
                     else np.ascontiguousarray(mval, dtype=np.int32))
        self.nmaps = int(nmaps)
        self._cth = np.ascontiguousarray(geom.cth, dtype=np.float64)
        self._sth = np.ascontiguousarray(geom.sth, dtype=np.float64)
        self._phi0 = np.ascontiguousarray(geom.phi0, dtype=np.float64)
        self._nphi = np.ascontiguousarray(geom.nphi, dtype=np.int64)
        rs = getattr(geom, "ringstart", None)
        self._start = None if rs is None else np.ascontiguousarray(rs, dtype=np.int64)
        d = L.GeometryDesc()
        d.lmax = self.lmax
        d.nm = len(self.mval)
        d.mval = self.mval.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.nrings = len(self._cth)
        d.cth = self._cth.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.sth = self._sth.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.phi0 = self._phi0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.nphi = self._nphi.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        d.ringstart = (None if self._start is None
                       else self._start.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        d.nmaps = self.nmaps
        if precision not in self.PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(self.PRECISIONS)}")
        self.precision = precision
        d.precision = self.PRECISIONS[precision]
        d.flags = 0 if pairing else L.SHT_FLAG_NO_PAIRING
        d.npix = int(getattr(geom, "npix", 0) or 0)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(lib.sht_plan(ctypes.byref(h), ctypes.byref(d)), "sht_plan")
        self._h = h
        info = L.PlanInfo()
        L.check(lib.sht_plan_get_info(h, ctypes.byref(info)), "sht_plan_get_info")
        self.info = info
        self.nalm = int(info.nalm)
        self.npix = int(info.npix)
        self.nrings = int(info.nrings)
        self.nm = int(info.nm)
        self.npairs = int(info.npairs)
        covered = int(np.sum(self._nphi))
        self._full_cover = covered == self.npix
        self._ws = {}

    # ----------------------------------------------------------------- misc
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.load().sht_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    @property
    def workspace_bytes(self) -> int:
        return int(self.info.workspace_bytes)

    def workspace(self, full: bool = True) -> torch.Tensor:
        """Device scratch for the plan's calls on the current stream:
        synthesis needs only the forward part (full=False); the adjoint and
        map2alm need all of it.  The plan keeps one workspace per stream,
        allocated on that stream and grown on the first call that needs more,
        so calls on different streams never share one (the library's rule for
        concurrent calls), and memory dropped when a workspace grows is only
        reused by work ordered after the calls that used it."""
        return _stream_workspace(self._ws, self.device,
                                 self.workspace_bytes if full
                                 else int(self.info.forward_workspace_bytes))

    @property
    def config(self) -> int:
        """Ring pairs per lane of the FP64 forward Legendre kernel."""
        c = ctypes.c_int32()
        L.check(L.load().sht_plan_get_config(self._h, ctypes.byref(c)), "sht_plan_get_config")
        return int(c.value)

    def set_config(self, chains: int):
        L.check(L.load().sht_plan_set_config(self._h, chains), "sht_plan_set_config")

    def autotune(self, alm: torch.Tensor, out: torch.Tensor | None = None,
                 cache_path: str | None = None) -> int:
        """Time every launch shape on these buffers and keep the fastest."""
        a = self._alm_in(alm)
        out = self._new_map() if out is None else \
            self._check_out(out, torch.float64, self.nmaps * self.npix, "out")
        ws = self.workspace(full=False)
        cp = cache_path.encode() if cache_path else None
        L.check(L.load().sht_plan_autotune(self._h, _ptr(a), _ptr(out), _ptr(ws), ws.numel(),
                                           cp, ctypes.c_void_p(_cur_stream(self.device))),
                "sht_plan_autotune")
        return self.config

    def _alm_in(self, alm: torch.Tensor) -> torch.Tensor:
        if alm.dtype != torch.complex128:
            raise TypeError("alm must be complex128")
        if alm.device != self.device:
            raise ValueError("alm must be on the plan's device")
        a = alm.reshape(self.nmaps, self.nalm) if alm.dim() == 1 and self.nmaps == 1 else alm
        if tuple(a.shape) != (self.nmaps, self.nalm):
            raise ValueError(f"alm must have shape ({self.nmaps}, {self.nalm})")
        return a.contiguous()

    def _map_in(self, m: torch.Tensor) -> torch.Tensor:
        if m.dtype != torch.float64:
            raise TypeError("map must be float64")
        if m.device != self.device:
            raise ValueError("map must be on the plan's device")
        mm = m.reshape(self.nmaps, self.npix) if m.dim() == 1 and self.nmaps == 1 else m
        if tuple(mm.shape) != (self.nmaps, self.npix):
            raise ValueError(f"map must have shape ({self.nmaps}, {self.npix})")
        return mm.contiguous()

    def _check_out(self, out: torch.Tensor, dtype, numel: int, what: str) -> torch.Tensor:
        """A caller-supplied output must match exactly: the kernels write
        through its raw pointer."""
        if out.dtype != dtype or out.device != self.device or not out.is_contiguous() \
                or out.numel() != numel:
            raise ValueError(f"{what} must be a contiguous {dtype} tensor of {numel} elements "
                             f"on {self.device}")
        return out

    def _new_map(self) -> torch.Tensor:
        f = torch.empty if self._full_cover else torch.zeros
        return f((self.nmaps, self.npix), dtype=torch.float64, device=self.device)

    # ---------------------------------------------------------- transforms
    def alm2map(self, alm: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        a = self._alm_in(alm)
        out = self._new_map() if out is None else \
            self._check_out(out, torch.float64, self.nmaps * self.npix, "out")
        ws = self.workspace(full=False)
        L.check(L.load().sht_alm2map(self._h, _ptr(a), _ptr(out), _ptr(ws), ws.numel(),
                                     ctypes.c_void_p(_cur_stream(self.device))), "sht_alm2map")
        return out

    def alm2map_adjoint(self, m: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        mm = self._map_in(m)
        out = torch.empty((self.nmaps, self.nalm), dtype=torch.complex128,
                          device=self.device) if out is None else \
            self._check_out(out, torch.complex128, self.nmaps * self.nalm, "out")
        ws = self.workspace()
        L.check(L.load().sht_alm2map_adjoint(self._h, _ptr(mm), _ptr(out), _ptr(ws), ws.numel(),
                                             ctypes.c_void_p(_cur_stream(self.device))),
                "sht_alm2map_adjoint")
        return out

    def map2alm(self, m: torch.Tensor, ring_weight, niter: int = 0,
                out: torch.Tensor | None = None) -> torch.Tensor:
        """Quadrature-weighted analysis (sht_map2alm): D adjoint(w s), refined
        by `niter` steps a <- a + map2alm(s - alm2map(a)).  ring_weight: the
        weight of one pixel of each ring (float64 [nrings])."""
        mm = self._map_in(m)
        w = torch.as_tensor(ring_weight, dtype=torch.float64).to(self.device).contiguous()
        if tuple(w.shape) != (self.nrings,):
            raise ValueError("ring_weight must have one entry per ring")
        out = torch.empty((self.nmaps, self.nalm), dtype=torch.complex128,
                          device=self.device) if out is None else \
            self._check_out(out, torch.complex128, self.nmaps * self.nalm, "out")
        tmp = torch.empty((self.nmaps, self.npix), dtype=torch.float64,
                          device=self.device) if niter > 0 else None
        ws = self.workspace()
        L.check(L.load().sht_map2alm(self._h, _ptr(mm), _ptr(w), _ptr(out), int(niter),
                                     None if tmp is None else _ptr(tmp), _ptr(ws), ws.numel(),
                                     ctypes.c_void_p(_cur_stream(self.device))),
                "sht_map2alm")
        return out

    def alm2delta(self, alm: torch.Tensor) -> torch.Tensor:
        a = self._alm_in(alm)
        out = torch.empty((self.nmaps, self.nm, self.nrings), dtype=torch.complex128,
                          device=self.device)
        ws = self.workspace(full=False)
        L.check(L.load().sht_alm2delta(self._h, _ptr(a), _ptr(out), _ptr(ws), ws.numel(),
                                       ctypes.c_void_p(_cur_stream(self.device))),
                "sht_alm2delta")
        return out

    def delta2map(self, delta: torch.Tensor) -> torch.Tensor:
        if delta.dtype != torch.complex128 or tuple(delta.shape) != (self.nmaps, self.nm,
                                                                     self.nrings):
            raise ValueError("delta must be complex128 (nmaps, nm, nrings)")
        dl = delta.contiguous()
        out = self._new_map()
        L.check(L.load().sht_delta2map(self._h, _ptr(dl), _ptr(out),
                                       ctypes.c_void_p(_cur_stream(self.device))),
                "sht_delta2map")
        return out

    def map2delta_adjoint(self, m: torch.Tensor) -> torch.Tensor:
        mm = self._map_in(m)
        out = torch.empty((self.nmaps, self.nm, self.nrings), dtype=torch.complex128,
                          device=self.device)
        L.check(L.load().sht_map2delta_adjoint(self._h, _ptr(mm), _ptr(out),
                                               ctypes.c_void_p(_cur_stream(self.device))),
                "sht_map2delta_adjoint")
        return out

    def delta2alm_adjoint(self, delta: torch.Tensor) -> torch.Tensor:
        if delta.dtype != torch.complex128 or tuple(delta.shape) != (self.nmaps, self.nm,
                                                                     self.nrings):
            raise ValueError("delta must be complex128 (nmaps, nm, nrings)")
        dl = delta.contiguous()
        out = torch.empty((self.nmaps, self.nalm), dtype=torch.complex128, device=self.device)
        ws = self.workspace()
        L.check(L.load().sht_delta2alm_adjoint(self._h, _ptr(dl), _ptr(out), _ptr(ws),
                                               ws.numel(),
                                               ctypes.c_void_p(_cur_stream(self.device))),
                "sht_delta2alm_adjoint")
        return out


class AlmToMap(torch.autograd.Function):
    """map = alm2map(alm); backward applies the hand-written adjoint.

    The gradient with respect to a complex coefficient is
    dL/dRe(a) + i dL/dIm(a) (PyTorch's convention for real losses); the
    imaginary part of a_l0 does not enter the map, so its gradient is 0.
    """

    @staticmethod
    def forward(ctx, alm, plan):
        ctx.plan = plan
        return plan.alm2map(alm)

    @staticmethod
    def backward(ctx, grad_map):
        return ctx.plan.alm2map_adjoint(grad_map.contiguous()).reshape(
            ctx.plan.nmaps, ctx.plan.nalm), None


def alm2map(alm: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable alm2map (autograd through AlmToMap)."""
    return AlmToMap.apply(alm, plan)


class Batch:
    """Maps of different l_max / geometry transformed together.

    One persistent Legendre launch for all maps (work tiles sorted longest
    first), one Fourier launch per ring size class; optional autotuning of the
    launch shape and HIP graph capture.  The single-map FP64 plans must stay
    alive as long as the batch (the batch keeps references to them).
    """

    def __init__(self, plans):
        lib = L.load()
        self.plans = list(plans)
        self.device = self.plans[0].device
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(lib.sht_plan_batch(ctypes.byref(h), arr, len(self.plans)), "sht_plan_batch")
        self._h = h
        n = ctypes.c_size_t()
        L.check(lib.sht_batch_workspace_size(h, ctypes.byref(n)), "sht_batch_workspace_size")
        self.workspace_bytes = int(n.value)
        self._ws = {}
        self._keep = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.load().sht_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self) -> torch.Tensor:
        """The batch workspace for the current stream (one per stream, so
        that batched transforms on different streams never share one)."""
        return _stream_workspace(self._ws, self.device, self.workspace_bytes)

    def new_maps(self):
        return [p._new_map().reshape(-1) for p in self.plans]

    def _ptrs(self, alms, outs):
        if len(alms) != len(self.plans) or len(outs) != len(self.plans):
            raise ValueError("one coefficient array and one map per plan")
        for p, a, o in zip(self.plans, alms, outs):
            if a.dtype != torch.complex128 or a.numel() != p.nalm or not a.is_contiguous():
                raise ValueError("alm arrays must be contiguous complex128 of each plan's nalm")
            if o.dtype != torch.float64 or o.numel() != p.npix or not o.is_contiguous():
                raise ValueError("maps must be contiguous float64 of each plan's npix")
        pa = torch.tensor([a.data_ptr() for a in alms], dtype=torch.int64, device=self.device)
        po = torch.tensor([o.data_ptr() for o in outs], dtype=torch.int64, device=self.device)
        return pa, po

    def alm2map(self, alms, outs=None):
        outs = self.new_maps() if outs is None else outs
        pa, po = self._ptrs(alms, outs)
        ws = self.workspace()
        L.check(L.load().sht_alm2map_batch(self._h, _ptr(pa), _ptr(po), _ptr(ws), ws.numel(),
                                           ctypes.c_void_p(_cur_stream(self.device))),
                "sht_alm2map_batch")
        return outs

    @property
    def config(self):
        c = ctypes.c_int32()
        w = ctypes.c_int32()
        L.check(L.load().sht_batch_get_config(self._h, ctypes.byref(c), ctypes.byref(w)),
                "sht_batch_get_config")
        return int(c.value), int(w.value)

    def set_config(self, chains: int, waves_per_cu: int):
        L.check(L.load().sht_batch_set_config(self._h, chains, waves_per_cu),
                "sht_batch_set_config")

    def autotune(self, alms, outs, cache_path: str | None = None):
        pa, po = self._ptrs(alms, outs)
        ws = self.workspace()
        cp = cache_path.encode() if cache_path else None
        L.check(L.load().sht_batch_autotune(self._h, _ptr(pa), _ptr(po), _ptr(ws), ws.numel(),
                                            cp, ctypes.c_void_p(_cur_stream(self.device))),
                "sht_batch_autotune")
        return self.config

    def capture(self, alms, outs, stream: torch.cuda.Stream):
        """Capture one batched transform into a HIP graph on `stream`."""
        with torch.cuda.stream(stream):
            pa, po = self._ptrs(alms, outs)
            ws = self.workspace()
        # the graph replays with these buffers: keep them alive with it
        self._keep = (pa, po, ws, list(alms), list(outs))
        L.check(L.load().sht_batch_graph_capture(self._h, _ptr(pa), _ptr(po), _ptr(ws),
                                                 ws.numel(), ctypes.c_void_p(stream.cuda_stream)),
                "sht_batch_graph_capture")

    def replay(self, stream: torch.cuda.Stream | None = None):
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        L.check(L.load().sht_batch_graph_launch(self._h, ctypes.c_void_p(s.cuda_stream)),
                "sht_batch_graph_launch")
