#!/usr/bin/env python
"""Throughput of the IFGF-accelerated matvec on one MI355X.

Workload (default): a dielectric sphere of radius 5 (10 vacuum wavelengths
across, eps_r = 2.25 inside, vacuum outside: k_int = 3 pi, k_ext = 2 pi),
cube-sphere map with 6 x 16 x 16 patches of 10 x 10 Chebyshev nodes
(153,600 points), one right-hand side of i.i.d. complex normal densities.

A step is one forward evaluation of the hot path on that input, with every
input resident in HBM before the timed region starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IFGF N-Müller matvecs/s + GMRES time-to-1e-4 residual, mixed/learned vs FP64"

# algorithmic flops per work unit of each kernel (FMA = 2, transcendental = 1)
def flops_per_unit(name, npts):
    if name == "near":          # (target, source) pair, both wavenumbers
        return 280.0
    if name == "leaf":          # (interpolation point, source) pair
        return 160.0
    if name == "targets":       # (target, cousin box): value 16 + derivative 12 complex columns
        return 4.0 * npts * 16 + 4.0 * npts * 12 + 10.0 * npts + 300.0
    if name == "propagate":     # (parent interpolation point, child box)
        return 4.0 * npts * 16 + 2.0 * npts + 150.0
    return 0.0


PEAK = {"f64": 78.6e12, "f32_valu": 78.6e12, "f32_mfma": 157.3e12, "hbm": 8.0e12}


def cpu_baseline(surface, ks, w, sample_rows, seed=2):
    """Time the oracle's O(N^2) direct sum on a sample of rows."""
    import numpy as np
    from threadpoolctl import threadpool_info
    import synth
    from oracle import direct
    phi = synth.complex_normal((8, surface.n), seed)
    rows = np.arange(sample_rows)
    t0 = time.perf_counter()
    direct.regular_sums(surface.x, surface.normal, w, phi, ks, targets=rows, block=64)
    dt = time.perf_counter() - t0
    per_matvec = dt * surface.n / sample_rows
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": 1.0 / per_matvec, "unit": "matvecs/s", "cores": threads, "kind": "oracle",
            "sample": f"O1 direct regular sums (8 densities x 2 wavenumbers, S and n.grad S) for "
                      f"{sample_rows} of {surface.n} target rows, {dt:.1f} s, extrapolated x{surface.n // sample_rows}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--Ps", type=int, default=3)
    ap.add_argument("--Pa", type=int, default=5)
    ap.add_argument("--cpu-rows", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2408_02274_amd import IFGFPlan

    surf = synth.cube_sphere(16, 10, 5.0)
    ks = (3.0 * math.pi, 2.0 * math.pi)          # (k_int, k_ext)
    w = np.full(surf.n, 4.0 * math.pi * 25.0 / surf.n)
    prec = 0 if args.precision == "fp64" else 1
    t0 = time.perf_counter()
    plan = IFGFPlan(surf.x, surf.normal, w, ks[0], ks[1], 1e-3, Ps=args.Ps, Pa=args.Pa,
                    precision=prec)
    plan_s = time.perf_counter() - t0
    print(f"[bench] plan built in {plan_s:.1f} s", file=sys.stderr, flush=True)
    dens = torch.from_numpy(synth.complex_normal((1, 8, surf.n), 2)).to("cuda")
    out = torch.empty((1, 2, 14, surf.n), dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        plan.apply(dens, out)
    torch.cuda.synchronize()
    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.apply(dens, out, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = plan.stats()
    plan.set_timing(False)
    ms_per_step = elapsed / args.steps * 1e3
    value = args.steps / elapsed

    npts = st["Ps"] * st["Pa"] * st["Pa"]
    timing = st.get("timing", {})
    kern = {}
    for name, t in timing.items():
        fl = flops_per_unit(name, npts) * t["units"]
        kern[name] = {"launches": t["launches"], "ms": t["ms"], "flop": fl}
    dom = max(kern, key=lambda k: kern[k]["ms"])
    d = kern[dom]
    achieved = d["flop"] / (d["ms"] * 1e-3)
    peak = PEAK["f64"] if args.precision == "fp64" else PEAK["f32_valu"]
    roof = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
            "avg_launch_ms": d["ms"] / d["launches"]}
    res = {
        "metric": METRIC, "value": value, "unit": "matvecs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "IFGF raw sums (8 densities x 2 wavenumbers, S and n.grad S) on a "
                               "sphere of radius 5, 6x16x16 patches x 10x10 nodes (153,600 points), "
                               "k_int = 3 pi, k_ext = 2 pi, 1 RHS",
                   "Ps": st["Ps"], "Pa": st["Pa"], "D": st["D"], "plan_seconds": plan_s},
        "roofline": roof,
        "kernels_ms_per_step": {k: v["ms"] / args.steps for k, v in kern.items()},
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(surf, ks, w, args.cpu_rows)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
