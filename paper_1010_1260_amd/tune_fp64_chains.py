"""Measure the FP64 forward Legendre kernel's launch shape (ring pairs per
lane: 1, 2 or 4) over problem sizes and print the table the library's
default rule is read from (Sec. 5: the best launch parameters depend on the
input size).

Run on the GPU from the repository root:

    python3 -m paper_1010_1260_amd.tune_fp64_chains

Each row times the Legendre stage (sht_alm2delta) of a HEALPix plan with
nside = l_max / 2 on seeded coefficients: two warm-up calls, then the median
of five timed calls per shape, with HIP events on the launch stream.
"""
from __future__ import annotations

import statistics
import sys

import numpy as np
import torch

from . import Plan

SIZES = [(64, 32, (1, 16)), (128, 64, (1, 16)), (256, 128, (1, 4, 16)),
         (512, 256, (1, 4, 16)), (1024, 512, (1, 4, 16)), (2048, 1024, (1, 4)),
         (4096, 2048, (1,))]
CHAINS = (1, 2, 4)


def _geometry(nside: int):
    import workloads as W
    return W.healpix_geometry(nside)


def _alms(lmax: int, nmaps: int, dev) -> torch.Tensor:
    rng = np.random.default_rng([lmax, nmaps])
    n = (lmax + 1) * (lmax + 2) // 2
    a = rng.standard_normal((nmaps, n)) + 1j * rng.standard_normal((nmaps, n))
    return torch.from_numpy(a).to(dev)


def time_stage(plan: Plan, alm: torch.Tensor, reps: int = 5) -> float:
    for _ in range(2):
        plan.alm2delta(alm)
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.alm2delta(alm)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return statistics.median(ts)


def main() -> int:
    if not torch.cuda.is_available():
        print("needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda", 0)
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    print(f"device: {torch.cuda.get_device_name(dev)}, {ncu} compute units")
    print("| l_max | nside | maps | waves/CU at 1 pair/lane | 1 (ms) | 2 (ms) | 4 (ms) "
          "| fastest | default |")
    print("|---|---|---|---|---|---|---|---|---|")
    for lmax, nside, nmaps_list in SIZES:
        g = _geometry(nside)
        for nmaps in nmaps_list:
            plan = Plan(lmax, g, nmaps=nmaps)
            default = plan.config
            alm = _alms(lmax, nmaps, dev)
            waves = -(-plan.npairs // 64) * ((plan.nm + 1) // 2) * nmaps / ncu
            t = {}
            for ch in CHAINS:
                plan.set_config(ch)
                t[ch] = time_stage(plan, alm)
            best = min(t, key=t.get)
            print(f"| {lmax} | {nside} | {nmaps} | {waves:.1f} | {t[1]:.3f} | {t[2]:.3f} "
                  f"| {t[4]:.3f} | {best} | {default} |", flush=True)
            plan.close()
            del alm
            torch.cuda.empty_cache()
    return 0


if __name__ == "__main__":
    sys.exit(main())
