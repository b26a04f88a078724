#!/usr/bin/env python3
"""Benchmark: alm2map maps/s at l_max = 4096, HEALPix nside = 2048 on one MI355X,
mixed precision against FP64.

Workloads (seeded Gaussian a_lm, C_l = 1/(l(l+1)), HEALPix rings,
50,331,648 pixels, 8191 rings; inputs resident in HBM before timing):
  * mixed: a batch of 16 maps; FP64 recurrence, matrix-core contraction in
    each mixed form (FP32, 3-way split BF16, 2-way split FP16), FP64 ring
    Fourier synthesis -- the headline value is the fastest form;
  * fp64:  one map at a time, everything FP64 -- the comparison.
One step is the whole transform of one batch through the C ABI (coefficient
prescale, Legendre stage, per-ring Fourier synthesis).  Stage durations come
from HIP events the library records on the launch stream around each kernel.
Beside the headline: the l_max 64 / nside 32 single map (launch-latency
bound), the 64-map uneven batch (one persistent launch replayed from a HIP
graph), map2alm, the differentiation workload, each mixed map's error
against the CPU oracle on sampled rings, and the oracle's own rate on the
host (all threads and one thread).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "maps/s at ℓmax=4096,nside=2048: mixed-precision vs FP64, rel err≤1e-6"
PEAK_FP64 = 78.6e12    # MI355X FP64 vector FLOP/s
PEAK_FP32_MFMA = 157.3e12
PEAK_BF16_MFMA = 2.5e15   # dense
PEAK_F16_MFMA = 2.5e15    # dense
# mixed forms: matrix-core peak of the operand type, kernel, matrix-core
# products per useful product, dtype label
FORMS = {
    "fp32_mfma": (PEAK_FP32_MFMA, "k_legendre_mfma_f32", 1, "f32"),
    "bf16x3_mfma": (PEAK_BF16_MFMA, "k_legendre_mfma_bf16x3", 6, "bf16x3"),
    "f16x2_mfma": (PEAK_F16_MFMA, "k_legendre_mfma_f16x2", 3, "f16x2"),
}
PEAK_HBM = 8.0e12      # bytes/s


def _hip():
    lib = ctypes.CDLL("libamdhip64.so")
    lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
    lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                        ctypes.c_void_p]
    return lib


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def recorded_traffic(key):
    """HBM bytes per launch recorded from rocprofv3 counters (profiles/traffic.json),
    or None when absent or when the kernel's sources (its file and the headers
    it includes, hashed together) changed since."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[key]
        h = hashlib.sha256()
        for s in rec["sources"]:
            h.update(open(os.path.join(ROOT, s), "rb").read())
        if h.hexdigest()[:16] != rec["sources_sha256_16"]:
            return None
        return float(rec["bytes_per_launch"])
    except (OSError, KeyError, ValueError, TypeError):
        return None


def run_plan(plan, alm, steps, warmup, lib, hip, torch, np):
    """Time `steps` transforms after `warmup`; returns wall seconds, stage ms, output."""
    dev = plan.device
    out = torch.empty((plan.nmaps, plan.npix), dtype=torch.float64, device=dev)
    ws = plan.workspace(full=False)
    sh = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    nev = 4
    evs = []
    for _ in range(steps * nev):
        e = ctypes.c_void_p()
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
        evs.append(e)
    EvArr = ctypes.c_void_p * nev
    args = (plan.handle, ctypes.c_void_p(alm.data_ptr()), ctypes.c_void_p(out.data_ptr()),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), sh)
    for _ in range(warmup):
        assert lib.sht_alm2map(*args) == 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        arr = EvArr(*[evs[i * nev + k].value for k in range(nev)])
        assert lib.sht_alm2map_events(*args, arr) == 0
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = np.zeros((steps, nev - 1))
    f = ctypes.c_float()
    for i in range(steps):
        for k in range(nev - 1):
            assert hip.hipEventElapsedTime(ctypes.byref(f), evs[i * nev + k],
                                           evs[i * nev + k + 1]) == 0
            st[i, k] = f.value
    for e in evs:
        hip.hipEventDestroy(e)
    return wall, st.mean(axis=0), out


def run_uneven(args, torch, np, W, dev):
    """64 maps, l_max uniform over {256, 512, 1024, 2048}, nside = l_max / 2,
    C_l = l^-2: one batch (persistent Legendre launch, autotuned, replayed
    from a HIP graph) against the same maps one plan at a time."""
    from paper_1010_1260_amd import Batch, Plan
    lmaxes = W.uneven_lmax()
    plans, alms = [], []
    for i, L in enumerate(lmaxes):
        plans.append(Plan(L, W.healpix_geometry(L // 2), device=dev))
        alms.append(torch.from_numpy(W.random_alm(L, [4, i], spectrum="inv_l2")).to(dev))
    b = Batch(plans)
    outs = b.new_maps()
    t0 = time.perf_counter()
    cfg = b.autotune(alms, outs)
    tune_s = time.perf_counter() - t0
    s = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        b.capture(alms, outs, s)
    for _ in range(args.warmup):
        b.replay(s)
    s.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(args.steps):
        b.replay(s)
    e1.record(s)
    s.synchronize()
    t_batch = e0.elapsed_time(e1) / args.steps
    # same maps, one single-map transform after another
    singles = [(p, a.reshape(1, -1)) for p, a in zip(plans, alms)]
    for p, a in singles:
        p.alm2map(a)
    torch.cuda.synchronize()
    e0.record()
    for p, a in singles:
        p.alm2map(a)
    e1.record()
    torch.cuda.synchronize()
    t_seq = e0.elapsed_time(e1)
    # algorithmic Legendre flops of the batch: 8 per (ring pair, l, m)
    flops = float(sum(p.npairs * p.nalm * 8 for p in plans))
    return {"maps": len(plans), "lmax_counts": {str(L): lmaxes.count(L) for L in sorted(set(lmaxes))},
            "ms_per_batch_graph": t_batch, "maps_per_s": len(plans) / (t_batch * 1e-3),
            "ms_one_plan_at_a_time": t_seq, "speedup_vs_one_at_a_time": t_seq / t_batch,
            "legendre_flops": flops, "overall_TFLOPs_legendre_work": flops / (t_batch * 1e-3) / 1e12,
            "tuned_chains_waves_per_cu": list(cfg), "autotune_s": tune_s}


def run_transfer(plan, alms_np, torch, np, reps=3):
    """Transfer-inclusive rate of one batch: a_lm from pinned host memory to
    the device, the transform, the maps back to pinned host memory (the
    paper's GPU timing spans kernel launch to result retrieval, Sec. 6).
    Reported beside the headline, never as it."""
    dev = plan.device
    h_alm = torch.empty((plan.nmaps, plan.nalm), dtype=torch.complex128, pin_memory=True)
    h_alm.copy_(torch.from_numpy(np.stack(alms_np)))
    h_map = torch.empty((plan.nmaps, plan.npix), dtype=torch.float64, pin_memory=True)
    d_alm = torch.empty((plan.nmaps, plan.nalm), dtype=torch.complex128, device=dev)
    d_map = torch.empty((plan.nmaps, plan.npix), dtype=torch.float64, device=dev)

    def once():
        d_alm.copy_(h_alm, non_blocking=True)
        plan.alm2map(d_alm, out=d_map)
        h_map.copy_(d_map, non_blocking=True)

    once()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        once()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    h2d = float(h_alm.numel() * 16)
    d2h = float(h_map.numel() * 8)
    return {"ms_per_batch": ms, "maps_per_s": plan.nmaps / (ms * 1e-3),
            "h2d_bytes": h2d, "d2h_bytes": d2h,
            "host_link_GBps_if_serial": (h2d + d2h) / (ms * 1e-3) / 1e9,
            "buffers": "pinned host (hipHostMalloc through torch), one stream, no overlap"}


def run_small(torch, np, W, dev, reps=200):
    """l_max 64, HEALPix nside 32, one FP64 map: launch-latency bound, timed
    over `reps` back-to-back transforms; checked against the oracle."""
    from oracle import ref
    from paper_1010_1260_amd import Plan
    c = W.CONFIGS[1]
    L, N = c["lmax"], c["nside"]
    geom = W.healpix_geometry(N)
    plan = Plan(L, geom, device=dev)
    a_np = W.config_alm(1)
    a = torch.from_numpy(a_np).to(dev).reshape(1, -1)
    out = torch.empty((1, plan.npix), dtype=torch.float64, device=dev)
    for _ in range(10):
        plan.alm2map(a, out=out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.alm2map(a, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    exp = ref.alm2map(L, geom, a_np)
    got = out[0].cpu().numpy()
    return {"lmax": L, "nside": N, "maps": 1, "precision": "fp64", "reps": reps,
            "ms_per_map": ms, "maps_per_s": 1e3 / ms,
            "rel_err_vs_oracle": float(np.linalg.norm(got - exp) / np.linalg.norm(exp))}


def _time_calls(fn, torch, reps=5, warm=2):
    """Median of `reps` timed calls of fn (HIP events on the current stream)."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def shape_sweep(torch, np, W, dev):
    """Launch shapes over sizes (the source of the libraries' default tables):
    the FP64 forward Legendre kernel's ring pairs per lane {1, 2, 4} on HEALPix
    grids (nside = l_max / 2, Legendre stage only), and the batch's (chains per
    lane, persistent waves per CU) on batches of uniform and uneven l_max.
    Prints one JSON line."""
    from paper_1010_1260_amd import Batch, Plan
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    fwd = []
    for L, nm in [(64, 1), (64, 16), (128, 1), (128, 16), (256, 1), (256, 4), (256, 16),
                  (512, 1), (512, 4), (512, 16), (1024, 1), (1024, 4), (1024, 16),
                  (2048, 1), (2048, 4), (4096, 1)]:
        g = W.healpix_geometry(L // 2)
        plan = Plan(L, g, nmaps=nm, device=dev)
        a = torch.from_numpy(np.stack([W.random_alm(L, [9, i]) for i in range(nm)])).to(dev)
        waves1 = ((plan.npairs + 63) // 64) * ((plan.nm + 1) // 2) * nm / ncu
        default = plan.config
        ms = {}
        for ch in (1, 2, 4):
            plan.set_config(ch)
            ms[ch] = _time_calls(lambda: plan.alm2delta(a), torch)
        fwd.append({"lmax": L, "nside": L // 2, "maps": nm, "waves_per_cu_at_1": waves1,
                    "ms": ms, "fastest": min(ms, key=ms.get), "default": default})
        del plan, a
    batches = {"uniform 128 x4": [128] * 4, "uniform 256 x4": [256] * 4,
               "uniform 512 x4": [512] * 4, "uniform 256 x16": [256] * 16,
               "uniform 256 x64": [256] * 64, "uniform 512 x32": [512] * 32,
               "uniform 1024 x16": [1024] * 16, "uniform 2048 x8": [2048] * 8,
               "uniform 2048 x32": [2048] * 32, "uneven x64": W.uneven_lmax(),
               "uneven x16": W.uneven_lmax()[:16]}
    bat = []
    for name, lm in batches.items():
        plans = [Plan(L, W.healpix_geometry(L // 2), device=dev) for L in lm]
        alms = [torch.from_numpy(W.random_alm(L, [10, i])).to(dev) for i, L in enumerate(lm)]
        b = Batch(plans)
        outs = b.new_maps()
        default = b.config
        ms = {}
        for ch in (1, 2, 4):
            for wv in (4, 8, 16, 32):
                b.set_config(ch, wv)
                ms[f"{ch},{wv}"] = _time_calls(lambda: b.alm2map(alms, outs), torch)
        tiles = sum(((p.npairs + 127) // 128) * ((p.nm + 1) // 2) for p in plans)
        bat.append({"batch": name, "maps": len(lm), "tiles_per_cu_at_128_pairs": tiles / ncu,
                    "ms": ms, "fastest": min(ms, key=ms.get), "default": list(default)})
        del b, plans, alms, outs
        torch.cuda.empty_cache()
    print(json.dumps({"shape_sweep": {"device_cus": ncu, "fp64_forward": fwd, "batch": bat}}),
          flush=True)


def run_grad(args, torch, np, W, dev):
    """The differentiation workload: 8 maps, l_max 1024, nside 512, loss
    0.5 ||alm2map(a) - d||^2 with d ~ N(0, 1) per pixel; one step = forward
    transform, loss, backward through the hand-written adjoint."""
    from paper_1010_1260_amd import Plan, alm2map
    c = W.CONFIGS[5]
    L, N, B = c["lmax"], c["nside"], c["nmaps"]
    geom = W.healpix_geometry(N)
    plan = Plan(L, geom, nmaps=B, device=dev)
    a0 = torch.from_numpy(np.stack([W.config_alm(5, i) for i in range(B)])).to(dev)
    d = torch.from_numpy(np.stack([W.random_map(geom.npix, [5, 100 + i])
                                   for i in range(B)])).to(dev)

    def step():
        a = a0.clone().requires_grad_(True)
        loss = 0.5 * ((alm2map(a, plan) - d) ** 2).sum()
        loss.backward()
        return a.grad

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    n = 5
    for _ in range(n):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / n
    return {"maps": B, "lmax": L, "nside": N, "ms_forward_backward": ms,
            "maps_per_s": B / (ms * 1e-3)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--lmax", type=int, default=4096)
    ap.add_argument("--nside", type=int, default=2048)
    ap.add_argument("--nmaps", type=int, default=16, help="batch of the mixed-precision run")
    ap.add_argument("--only", choices=["all", "fp64", *FORMS], default="all")
    ap.add_argument("--no-transfer", action="store_true",
                    help="skip the transfer-inclusive (pinned host buffers) timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the batched uneven workload (64 maps, l_max in "
                         "{256..2048}, one persistent launch, autotuned, graph replay)")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the l_max 64 / nside 32 single-map timing")
    ap.add_argument("--shape-sweep", action="store_true",
                    help="only time the launch shapes of the FP64 forward kernel and of the "
                         "batch over sizes (the source of the default tables) and exit")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before timing, copy this many MiB device to device (a copy of known "
                         "size for scaling hardware byte counters)")
    ap.add_argument("--cpu-ring-stride", type=int, default=8,
                    help="oracle timed on every k-th ring (bounded CPU sample)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the transform runs on one GPU (--gpus {args.gpus} requested); "
              "sharding over maps or ring pairs across GPUs is not implemented", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import workloads as W
    from paper_1010_1260_amd import Plan
    from paper_1010_1260_amd import _lib as L

    lib = L.load()
    hip = _hip()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.shape_sweep:
        shape_sweep(torch, np, W, dev)
        return 0
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    Lmax, N, B = args.lmax, args.nside, args.nmaps
    geom = W.healpix_geometry(N)
    alms_np = [W.random_alm(Lmax, [3, i]) for i in range(B)]
    res = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "data": "synthetic (seeded Gaussian a_lm, C_l = 1/(l(l+1)), HEALPix rings)"}

    mixed_runs = {}
    fp64 = None
    for prec in FORMS:
        if args.only in ("all", prec):
            plan = Plan(Lmax, geom, nmaps=B, precision=prec, device=dev)
            alm = torch.from_numpy(np.stack(alms_np)).to(dev)
            wall, st, out = run_plan(plan, alm, args.steps, args.warmup, lib, hip, torch, np)
            mixed_runs[prec] = dict(plan=plan, wall=wall, st=st, out=out)
            del alm
            if args.only == "all":
                # keep only the output of the run that may become the headline
                pass
    if args.only in ("all", "fp64"):
        plan64 = Plan(Lmax, geom, nmaps=1, device=dev)
        alm0 = torch.from_numpy(alms_np[0]).to(dev).reshape(1, -1)
        wall, st, out = run_plan(plan64, alm0, args.steps, args.warmup, lib, hip, torch, np)
        fp64 = dict(plan=plan64, wall=wall, st=st, out=out)
        # map2alm (quadrature-weighted analysis) of that map on the same plan:
        # uniform pixel weight 4 pi / npix, no refinement and 3 refinement steps
        w = torch.full((geom.nrings,), 4.0 * np.pi / geom.npix, dtype=torch.float64, device=dev)
        a2m = {}
        for niter in (0, 3):
            plan64.map2alm(out, w, niter=niter)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(2):
                back = plan64.map2alm(out, w, niter=niter)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 2
            err = float(torch.linalg.norm(back - alm0) / torch.linalg.norm(alm0))
            a2m[f"niter{niter}"] = {"ms": ms, "maps_per_s": 1e3 / ms, "rel_err_vs_alm": err}
            del back
        fp64["map2alm"] = a2m
    mixed = None
    if mixed_runs:
        best = max(mixed_runs, key=lambda k: 1.0 / mixed_runs[k]["wall"])
        mixed = mixed_runs[best]
        mixed["prec"] = best

    npairs = (mixed or fp64)["plan"].npairs
    nalm = (mixed or fp64)["plan"].nalm
    # Fourier stage, algorithmic bytes per map: Delta read once (complex128 in
    # FP64, complex64 in the mixed forms) and the map written once
    fft_bytes_fp64 = 16.0 * geom.nrings * (Lmax + 1) + 8.0 * geom.npix
    fft_bytes_mixed = 8.0 * geom.nrings * (Lmax + 1) + 8.0 * geom.npix
    if fp64 is not None:
        t = fp64["wall"] / args.steps
        leg = float(fp64["st"][1])
        flops = float(npairs) * float(nalm) * 8.0
        fp64_info = {
            "maps_per_s": 1.0 / t, "ms_per_step": t * 1e3,
            "stages_ms": {"prescale": float(fp64["st"][0]), "legendre": leg,
                          "ring_synthesis": float(fp64["st"][2])},
            "legendre_roofline": {"bound": "alu", "achieved": flops / (leg * 1e-3) / 1e12,
                                  "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                                  "frac": flops / (leg * 1e-3) / PEAK_FP64,
                                  "kernel": f"k_legendre_fwd<{fp64['plan'].config}>",
                                  "flops_per_launch": flops},
            "fourier_GBps": fft_bytes_fp64 / (float(fp64["st"][2]) * 1e-3) / 1e9,
            "fourier_frac_hbm": fft_bytes_fp64 / (float(fp64["st"][2]) * 1e-3) / PEAK_HBM,
            "map2alm": fp64["map2alm"],
        }
        res["fp64"] = fp64_info
    if mixed is not None:
        forms = {}
        for prec, run in mixed_runs.items():
            t = run["wall"] / args.steps
            leg = float(run["st"][1])
            # algorithmic contraction flops: 4 per (ring pair, l, m, map) (complex
            # accumulate of a real P_lm); the FP64 recurrence (4 per (pair, l, m))
            # runs on the vector units beside it
            flops = float(npairs) * float(nalm) * 4.0 * B
            peak, kern, nprod, _ = FORMS[prec]
            executed = flops * nprod
            traffic = recorded_traffic(f"{kern}|lmax={Lmax}|nside={N}|nmaps={B}")
            forms[prec] = {
                "maps_per_s": B / t, "ms_per_step": t * 1e3,
                "stages_ms": {"prescale": float(run["st"][0]), "legendre": leg,
                              "ring_synthesis": float(run["st"][2])},
                "roofline": {"bound": "mfma", "achieved": flops / (leg * 1e-3) / 1e12,
                             "peak": peak / 1e12, "unit": "TFLOP/s",
                             "frac": flops / (leg * 1e-3) / peak, "traffic": traffic,
                             "kernel": kern, "flops_per_launch": flops,
                             "executed_mfma_flops_per_launch": executed,
                             "executed_frac": executed / (leg * 1e-3) / peak},
            }
        best = mixed["prec"]
        t = mixed["wall"] / args.steps
        fb = forms[best]
        res.update({
            "value": B / t, "unit": "maps/s", "ms_per_step": t * 1e3,
            "dtype": FORMS[best][3] + " matrix-core contraction + f64 recurrence and alias "
                     "fold + f32 ring FFT",
            "config": {"workload": f"alm2map mixed precision, batch of {B} maps, lmax={Lmax}, "
                                   f"HEALPix nside={N}", "lmax": Lmax, "nside": N,
                       "nmaps": B, "precision": best, "npix": geom.npix,
                       "nrings": geom.nrings},
            "stages_ms": fb["stages_ms"],
            "roofline": fb["roofline"],
            "mixed_forms": forms,
            "fourier_stage": {"bytes_per_launch": fft_bytes_mixed * B,
                              "bytes_note": "complex64 Delta read once + float64 map written "
                                            "once",
                              "achieved_GBps": fft_bytes_mixed * B /
                              (fb["stages_ms"]["ring_synthesis"] * 1e-3) / 1e9,
                              "frac_hbm": fft_bytes_mixed * B /
                              (fb["stages_ms"]["ring_synthesis"] * 1e-3) / PEAK_HBM},
        })
        if fp64 is not None:
            res["speedup_mixed_vs_fp64"] = res["value"] / res["fp64"]["maps_per_s"]
            p64 = fp64["plan"]
            refs = []
            for i in range(B):
                a = torch.from_numpy(alms_np[i]).to(dev).reshape(1, -1)
                refs.append(p64.alm2map(a)[0].clone())
            for prec, run in mixed_runs.items():
                errs = [float(torch.linalg.norm(run["out"][i] - refs[i]) / torch.linalg.norm(refs[i]))
                        for i in range(B)]
                forms[prec]["rel_err_vs_fp64_gpu"] = {"max": max(errs), "mean": float(np.mean(errs)),
                                                      "maps": B}
            res["rel_err_mixed_vs_fp64_gpu"] = forms[best]["rel_err_vs_fp64_gpu"]
            del refs
        if not args.no_transfer:
            res["transfer_inclusive"] = run_transfer(mixed["plan"], alms_np, torch, np)
    else:
        t = fp64["wall"] / args.steps
        res.update({"value": 1.0 / t, "unit": "maps/s", "ms_per_step": t * 1e3, "dtype": "f64",
                    "config": {"workload": f"alm2map FP64, 1 map, lmax={Lmax}, HEALPix nside={N}",
                               "lmax": Lmax, "nside": N, "nmaps": 1, "precision": "fp64"},
                    "roofline": dict(res["fp64"]["legendre_roofline"], traffic=None)})

    if not args.no_uneven:
        res["uneven_batch"] = run_uneven(args, torch, np, W, dev)
    if not args.no_small:
        res["small_lmax64_nside32"] = run_small(torch, np, W, dev)
    if args.only in ("all", "fp64"):
        res["differentiation"] = run_grad(args, torch, np, W, dev)

    if not args.no_cpu_baseline:
        from oracle import ref
        rings = np.arange(0, geom.nrings, args.cpu_ring_stride)
        th = ref.max_threads()
        tc0 = time.perf_counter()
        exp = ref.alm2map_rings(Lmax, geom, alms_np[0], rings, nthreads=th)
        tc = time.perf_counter() - tc0
        # every ring costs the same Legendre work: scale the sample to a map
        cpu_maps_per_s = (len(rings) / geom.nrings) / tc
        # one thread on a smaller sample (every 128th ring)
        rings1 = np.arange(0, geom.nrings, 128)
        t10 = time.perf_counter()
        ref.alm2map_rings(Lmax, geom, alms_np[0], rings1, nthreads=1)
        t1 = time.perf_counter() - t10
        try:
            aff = len(os.sched_getaffinity(0))
        except (AttributeError, OSError):
            aff = None
        res["cpu_baseline"] = {"value": cpu_maps_per_s, "unit": "maps/s", "cores": th,
                               "kind": "oracle",
                               "sample": f"map 0, {len(rings)} of {geom.nrings} rings (every "
                                         f"{args.cpu_ring_stride}th), {tc:.1f} s wall, scaled "
                                         f"by ring count; CPU: {_cpu_model()}",
                               "threads_used": th, "os_cpu_count": os.cpu_count(),
                               "affinity_cpus": aff,
                               "value_1thread": (len(rings1) / geom.nrings) / t1,
                               "sample_1thread": f"map 0, {len(rings1)} rings (every 128th), "
                                                 f"{t1:.1f} s wall",
                               "compiler": " ".join(ref.COMPILE_FLAGS)}
        errs = {}
        for name, runinfo in list(mixed_runs.items()) + [("fp64", fp64)]:
            if runinfo is None:
                continue
            got = runinfo["out"][0].cpu().numpy()
            num = den = 0.0
            for r, e in zip(rings, exp):
                s0, n = int(geom.ringstart[r]), int(geom.nphi[r])
                num += float(np.sum((got[s0:s0 + n] - e) ** 2))
                den += float(np.sum(e ** 2))
            errs[name] = float(np.sqrt(num / den))
        res["rel_err_vs_oracle_sampled_rings_map0"] = errs
        # every map of the mixed batch against the oracle on every 64th ring
        if mixed_runs:
            rings64 = np.arange(0, geom.nrings, 64)
            exps = [ref.alm2map_rings(Lmax, geom, alms_np[i], rings64, nthreads=th)
                    for i in range(B)]
            per = {}
            for name, runinfo in mixed_runs.items():
                outc = runinfo["out"].cpu().numpy()
                e_i = []
                for i in range(B):
                    num = den = 0.0
                    for r, e in zip(rings64, exps[i]):
                        s0, n = int(geom.ringstart[r]), int(geom.nphi[r])
                        num += float(np.sum((outc[i, s0:s0 + n] - e) ** 2))
                        den += float(np.sum(e ** 2))
                    e_i.append(float(np.sqrt(num / den)))
                per[name] = {"max": max(e_i), "mean": float(np.mean(e_i)), "per_map": e_i}
            res["rel_err_vs_oracle_per_map"] = {
                "rings": f"{len(rings64)} of {geom.nrings} (every 64th), all {B} maps",
                "forms": per}
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
