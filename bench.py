#!/usr/bin/env python
"""Throughput of the IFGF-accelerated N-Mueller forward map on one MI355X,
and GMRES time to a 1e-4 true residual.

Workload (default): a dielectric sphere of radius 5 (10 vacuum wavelengths
across; eps_r = 2.25 inside, vacuum outside: k_int = 3 pi, k_ext = 2 pi),
equiangular cube-sphere map with 6 x 16 x 16 patches of 10 x 10 Chebyshev
nodes (153,600 points, 614,400 unknowns), IFGF tolerance 1e-4.

A step is one N-Mueller matrix-vector product A y (densities, IFGF sums of
S and n.grad S for 8 densities x 2 wavenumbers, near-field corrections,
operator assembly) on i.i.d. complex normal unknowns, everything resident
in HBM before the timed region.  The headline form is the mixed one: IFGF
cone grids and interpolation in FP32, corrections, assembly and GMRES in
FP64.  The plain FP64 form of the same operator is timed beside it.

After the timed steps, GMRES solves of a plane-wave right-hand side (+z,
polarised x) to a 1e-4 true FP64 residual: mixed, FP64, and flexible GMRES
with the identity-part scaling D^-1.  The learned preconditioner (trained
parameters from paper_2408_02274_amd/weights) is timed on a held-out body of
the ellipsoid family it was trained on, against plain GMRES there.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IFGF N-Müller matvecs/s + GMRES time-to-1e-4 residual, mixed/learned vs FP64"
WEIGHTS = os.path.join(ROOT, "paper_2408_02274_amd", "weights", "precond_nc10.npz")
TRAFFIC = os.path.join(ROOT, "profiles", "propagate_fp32_sphere153k_hbm_traffic.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2408_02274_amd", "csrc", "ifgf_mfma.hip")


def flops_per_unit(name, npts):
    """Algorithmic flops per work unit (FMA = 2 flops, transcendental = 1,
    real x complex multiply-add = 4)."""
    return {
        "near": 280.0,                                   # (target, source) pair, 2 wavenumbers
        "leaf": 160.0,                                   # (interpolation point, source) pair
        "targets": 4.0 * npts * 16 + 4.0 * npts * 12 + 10.0 * npts + 300.0,   # (target, cousin box)
        "propagate": 4.0 * npts * 16 + 2.0 * npts + 150.0,                    # (parent point, child box)
        "nm_correct": 224.0,                             # (target, singular-patch node) pair
    }.get(name, 0.0)


def bytes_per_unit(name):
    return {"nm_correct": 68.0}.get(name, 0.0)


PEAK = {"fp64": 78.6e12, "fp32_valu_nopk": 78.6e12, "fp32_mfma": 157.3e12, "hbm": 8.0e12}


def kernel_sha(path=KERNEL_SRC):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_per_launch(kernel, precision, points, Ps, Pa):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when there is none for this kernel, precision and
    workload (points, orders) or the kernel source changed since the counters
    were taken."""
    if not os.path.exists(TRAFFIC):
        return None
    vals = {}
    for line in open(TRAFFIC):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel") != kernel or vals.get("precision") != precision:
        return None
    if vals.get("points") != str(points) or vals.get("orders") != f"{Ps},{Pa}":
        return None
    if vals.get("kernel_source_sha256") != kernel_sha():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_sample(args, npatch, log, mie_solution=None):
    """O1 (direct sums, singular corrections, assembly) on the nodes of
    `npatch` patches drawn from seed 2, run by the oracle's own program over a
    process pool of the host cores (one BLAS thread per worker); optionally the
    Mie error of a solution.  Returns the oracle's arrays and timings."""
    import tempfile
    import subprocess
    import numpy as np
    nproc = min(16, os.cpu_count() or 1)
    out = os.path.join(tempfile.mkdtemp(), "o1.npz")
    cmd = [sys.executable, "-m", "oracle.sample", "--npf", str(args.npf), "--nc", str(args.nc),
           "--radius", str(args.radius), "--npatch", str(npatch), "--nproc", str(nproc), "--out", out]
    if mie_solution is not None:
        cmd += ["--mie-solution", mie_solution]
    t0 = time.perf_counter()
    subprocess.run(cmd, cwd=ROOT, check=True, timeout=1200)
    log(f"oracle sample ({npatch} patches, {nproc} processes) in {time.perf_counter() - t0:.1f} s")
    return dict(np.load(out))


def o2_config1_seconds(Ps, Pa):
    """Wall time of one reference-IFGF evaluation (O2, single process) on the
    1,536-point unit sphere (24 patches x 8 x 8 nodes, k_int = 3 pi, k_ext = 2 pi)
    at the given orders: context for the CPU cost of the method itself."""
    import synth
    from oracle import ifgf_ref
    s = synth.cube_sphere(2, 8, 1.0)
    import numpy as np
    w = np.full(s.n, 4 * math.pi / s.n)
    phi = synth.complex_normal((8, s.n), 1)
    t0 = time.perf_counter()
    ifgf_ref.ReferenceIFGF(s.x, s.normal, w, (3 * math.pi, 2 * math.pi), ifgf_ref.Params(Ps=Ps, Pa=Pa)).apply(phi)
    return time.perf_counter() - t0


def batching(log, reps=5):
    """64 random right-hand sides on the unit sphere (24 patches x 8 x 8
    nodes, k_ext = 2 pi, eps_r 2.25): one-at-a-time applies, one batched
    apply (column batch chosen by the autotuner), one graph launch of the
    batched apply, and GMRES for 64 plane waves in lock-step vs one at a
    time."""
    import torch
    import synth
    from paper_2408_02274_amd import NMullerGraph, NMullerOperator
    from paper_2408_02274_amd import binding as B
    s = synth.cube_sphere(2, 8, 1.0)
    op = NMullerOperator(s, 1.0, 2.25, tol=1e-4, precision=B.IFGF_FP32, max_nrhs=64, batch_columns=4)
    cols = B.ifgf_autotune(op.ifgf_handle())
    y = torch.from_numpy(synth.complex_normal((64, 4, s.n), 3)).to("cuda")
    out = torch.empty_like(y)

    def clock(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_loop = clock(lambda: [op.apply(y[r:r + 1], out[r:r + 1]) for r in range(64)])
    t_batch = clock(lambda: op.apply(y, out))
    g = NMullerGraph([op], [y], [out])
    t_graph = clock(g.launch)
    res = {"workload": "config-1 sphere (1,536 points), 64 RHS, mixed form",
           "rhs_matvecs_per_s_looped": 64 / t_loop, "rhs_matvecs_per_s_batched": 64 / t_batch,
           "rhs_matvecs_per_s_graph": 64 / t_graph, "graph_nodes": g.nodes, "autotuned_columns": cols,
           "ms_looped": t_loop * 1e3, "ms_batched": t_batch * 1e3, "ms_graph": t_graph * 1e3}
    g.close()
    # GMRES for 64 plane waves (directions uniform on the sphere, polarisations
    # uniform in the tangent plane): lock-step batch vs one solve at a time
    import numpy as np
    d, pol = synth.plane_wave_batch(64, 3)
    ke = 2 * math.pi
    ph = np.exp(1j * ke * (s.x @ d.T)).T                   # [64][n]
    E = pol[:, None, :] * ph[:, :, None]
    H = np.cross(d, pol)[:, None, :] * ph[:, :, None]
    b = op.rhs(torch.from_numpy(E).to("cuda"), torch.from_numpy(H).to("cuda"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = op.solve(b, rtol=1e-4, maxit=300)
    torch.cuda.synchronize()
    t_lock = time.perf_counter() - t0
    t0 = time.perf_counter()
    lone = [op.solve(b[r:r + 1].contiguous(), rtol=1e-4, maxit=300)[1][0] for r in range(64)]
    torch.cuda.synchronize()
    t_lone = time.perf_counter() - t0
    res["gmres_64_plane_waves"] = {
        "rtol": 1e-4, "lockstep_seconds": t_lock, "one_at_a_time_seconds": t_lone,
        "iterations_total": sum(i["iters"] for i in info), "iterations_max": max(i["iters"] for i in info),
        "all_converged": all(i["converged"] for i in info) and all(i["converged"] for i in lone),
        "lockstep_speedup": t_lone / t_lock}
    op.close()
    log(f"batching: {res}")
    return res


def bodies32(log, reps=5):
    """32 uneven ellipsoids (a, b, c ~ U[0.5, 3], eps_r ~ U[1.5, 4], seeds
    1000 + i; patches per face ceil(sqrt(A / 1.5)) for surface area A, so a
    patch is about (0.5 wavelengths)^2; 10 x 10 nodes), mixed form: 32 looped
    applies vs one graph launch of all 32.  The host plans take minutes."""
    import torch
    import synth
    from paper_2408_02274_amd import NMullerGraph, NMullerOperator
    from paper_2408_02274_amd import binding as B

    def area(a, b, c, p=1.6075):   # Knud Thomsen's approximation
        return 4 * math.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3) ** (1 / p)

    ops, ys, outs, npts = [], [], [], []
    t0 = time.perf_counter()
    for i, (a, b, c, eps) in enumerate(synth.ellipsoid_batch(32, 1000)):
        npf = max(1, math.ceil(math.sqrt(area(a, b, c) / 1.5)))
        s = synth.ellipsoid(a, b, c, npf, 10)
        ops.append(NMullerOperator(s, 1.0, eps, tol=1e-4, precision=B.IFGF_FP32))
        ys.append(torch.from_numpy(synth.complex_normal((1, 4, s.n), 100 + i)).to("cuda"))
        outs.append(torch.empty_like(ys[-1]))
        npts.append(s.n)
        log(f"body {i}: n = {s.n}, plans {time.perf_counter() - t0:.0f} s")
    plan_s = time.perf_counter() - t0

    def clock(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    t_loop = clock(lambda: [op.apply(y, o) for op, y, o in zip(ops, ys, outs)])
    g = NMullerGraph(ops, ys, outs)
    t_graph = clock(g.launch)
    res = {"workload": "32 ellipsoids, seeds 1000..1031, mixed form", "points_total": int(sum(npts)),
           "points_min": int(min(npts)), "points_max": int(max(npts)), "plan_seconds": plan_s,
           "ms_looped": t_loop * 1e3, "ms_graph": t_graph * 1e3, "batch_matvecs_per_s_graph": 1 / t_graph,
           "body_matvecs_per_s_graph": 32 / t_graph, "graph_nodes": g.nodes}
    g.close()
    for op in ops:
        op.close()
    log(f"bodies32: {res}")
    return res


def learned_preconditioner(log, seed=5003):
    """The learned FGMRES preconditioner on a held-out body of the family it
    was trained on (ellipsoid semi-axes U[0.5, 2], eps_r U[2, 12], 6 x 6 x 6
    patches of 10 x 10 nodes, plane wave from the seed): plain GMRES, FGMRES
    with M = D^-1 alone, and FGMRES with the trained network, each to a 1e-4
    true FP64 residual on the mixed operator."""
    import numpy as np
    from paper_2408_02274_amd import precond
    z = np.load(WEIGHTS)
    params, dims = z["params"], [int(v) for v in z["dims"]]
    surf, eps, axes = precond.body(seed)
    t0 = time.perf_counter()
    op = precond.make_operator(surf, eps)
    b = precond.plane_wave_rhs(op, surf, seed)
    log(f"learned-preconditioner body {seed}: n = {surf.n}, eps_r {eps:.2f}, plan {time.perf_counter() - t0:.1f} s")
    r = precond.evaluate(op, b, params, dims, rtol=1e-4, maxit=800)
    op.close()
    out = {"workload": f"held-out ellipsoid seed {seed}: semi-axes {np.round(axes, 3).tolist()}, eps_r "
                       f"{eps:.3f}, {surf.n} points, plane wave from the seed",
           "weights": "paper_2408_02274_amd/weights/precond_nc10.npz"}
    for k in ("plain", "scaling_only", "learned"):
        out[k] = {"iters": r[k]["iters"], "seconds": r[k]["wall"], "true_relres": r[k]["true_relres"],
                  "converged": r[k]["converged"], "fallbacks": r[k]["fallbacks"]}
    out["learned_vs_plain_seconds"] = r["learned"]["wall"] / r["plain"]["wall"]
    out["learned_vs_scaling_only_seconds"] = r["learned"]["wall"] / r["scaling_only"]["wall"]
    out["note"] = ("the network is judged against M = D^-1 alone, its fixed part: a ratio above 1 means the "
                   "learned correction costs time")
    log(f"learned preconditioner: {out}")
    return out


def waveguide(args, log):
    """The large workload shaped like the paper's waveguide example (Sec. IV):
    rounded rectangular box 40 x 1 x 0.5 wavelengths with edge radius 0.1,
    patches of about 0.087 wavelengths with 10 x 10 nodes (16,704 patches,
    1,670,400 points), eps 12.1 inside and 2.1 outside (k_int = 21.86, k_ext =
    9.105).  Timed: one evaluation of the IFGF sums (16 S + 12 n.grad S at both
    wavenumbers, the T_IFGF part of the paper's forward map) in FP32 with
    FP32-sized workspaces, tol 1e-4; the error against the oracle's direct sums
    on 4,096 random nodes; device memory of the plan.  The N-Mueller corrections
    of this surface (about 1.6e9 (target, node) pairs at 64 bytes in FP64) do
    not fit one GPU beside the cone buffers and are not built here."""
    import numpy as np
    import torch
    import synth
    from paper_2408_02274_amd import IFGFPlan
    from paper_2408_02274_amd import binding as B
    surf = synth.rounded_box((20.0, 0.5, 0.25), 0.1, 0.087, 10)
    ks = (2 * math.pi * math.sqrt(12.1), 2 * math.pi * math.sqrt(2.1))
    area = 8 * (20 * 0.5 + 20 * 0.25 + 0.5 * 0.25)            # outer box; the rounding removes < 1%
    wconst = area / surf.n
    free0 = torch.cuda.mem_get_info()[0]
    t0 = time.perf_counter()
    plan = IFGFPlan(surf.x, surf.normal, np.full(surf.n, wconst), ks[0], ks[1], 1e-4,
                    precision=B.IFGF_FP32, fp32_workspaces=1, verbose=1)
    plan_s = time.perf_counter() - t0
    free1 = torch.cuda.mem_get_info()[0]
    log(f"waveguide plan: n = {surf.n}, {plan_s:.1f} s, {(free0 - free1) / 2**30:.1f} GiB on the device")
    phi = torch.from_numpy(synth.complex_normal((1, 8, surf.n), 3)).to("cuda")
    out = torch.empty((1, 2, 14, surf.n), dtype=torch.complex128, device="cuda")
    for _ in range(args.warmup):
        plan.apply(phi, out)
    torch.cuda.synchronize()
    plan.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.apply(phi, out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = plan.stats()
    plan.set_timing(False)
    g = out.cpu().numpy()[0]
    npts = st["Ps"] * st["Pa"] * st["Pa"]
    kern = kernel_table(st, args.steps, npts)
    dom = max(kern, key=lambda k: kern[k]["ms"])
    d = kern[dom]
    achieved = d["flop"] / (d["ms"] * 1e-3)
    roof = {"bound": "mfma", "kernel": dom, "achieved": achieved / 1e12, "peak": PEAK["fp32_mfma"] / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK["fp32_mfma"], "traffic": None,
            "avg_launch_ms": d["ms"] / d["launches"], "flop_per_launch": d["flop"] / d["launches"]}
    res = {"metric": "IFGF sums evaluations/s (T_IFGF part of the N-Mueller forward map)",
           "value": args.steps / el, "unit": "evaluations/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"rounded box 40 x 1 x 0.5 wavelengths, edge radius 0.1, {surf.P} patches x "
                                  f"10 x 10 nodes ({surf.n} points), k_int = {ks[0]:.3f}, k_ext = {ks[1]:.3f}, "
                                  f"IFGF tol 1e-4, FP32 cone grids and FP32-sized workspaces",
                      "Ps": st["Ps"], "Pa": st["Pa"], "D": st["D"], "plan_seconds": round(plan_s, 1),
                      "device_GiB": round((free0 - free1) / 2**30, 2), "plan_device_bytes": st["device_bytes"]},
           "roofline": roof,
           "kernels_ms_per_step": {k: round(v["ms"] / args.steps, 3) for k, v in kern.items()},
           "paper_context": "Table I row 5 (1,572,864 points): T_IFGF 50.14 s on 128 EPYC 7763 cores"}
    plan.close()
    if not args.no_cpu:
        import tempfile
        import subprocess
        nproc = min(16, os.cpu_count() or 1)
        o = os.path.join(tempfile.mkdtemp(), "o1.npz")
        cmd = [sys.executable, "-m", "oracle.sample", "--geometry", "rounded_box", "--nc", "10",
               "--direct-rows", "4096", "--k-int", repr(ks[0]), "--k-ext", repr(ks[1]),
               "--weight", repr(wconst), "--nproc", str(nproc), "--out", o]
        subprocess.run(cmd, cwd=ROOT, check=True, timeout=1200)
        o1 = dict(np.load(o))
        rows = o1["rows"]
        gs = g[:, :, rows]

        def rel(a, b):
            return float(np.linalg.norm(a - b) / np.linalg.norm(b))

        res["err_vs_o1"] = {"S": max(rel(gs[q, :8], o1["SD"][q, :8]) for q in range(2)),
                            "D": max(rel(gs[q, 8:], o1["SD"][q, 8:]) for q in range(2)),
                            "rows": "4096 random nodes (seed 2), densities from seed 3"}
        t = float(o1["seconds_direct"])
        res["cpu_baseline"] = {
            "value": rows.size / (t * surf.n), "unit": "evaluations/s", "cores": nproc, "kind": "oracle",
            "sample": f"oracle O1 direct sums (S and n.grad S, 8 densities x 2 wavenumbers) on {rows.size} of "
                      f"{surf.n} nodes took {t:.1f} s over {nproc} worker processes; extrapolated "
                      f"x{surf.n / rows.size:.0f} to one evaluation", "cpu_model": cpu_model()}
        log(f"waveguide errors vs O1: {res['err_vs_o1']}")
    return res


def kernel_table(st, steps, npts):
    kern = {}
    for name, t in st.get("timing", {}).items():
        kern[name] = {"launches": t["launches"], "ms": t["ms"],
                      "flop": flops_per_unit(name, npts) * t["units"],
                      "bytes": bytes_per_unit(name) * t["units"]}
    return kern


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--nrhs", type=int, default=1,
                    help="right-hand sides per step (stacked into the cone-data columns)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32"],
                    help="IFGF form of the timed steps: fp32 = mixed (default), fp64 = plain")
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--npf", type=int, default=16, help="patches per cube face edge")
    ap.add_argument("--nc", type=int, default=10, help="Chebyshev nodes per patch direction")
    ap.add_argument("--radius", type=float, default=5.0)
    ap.add_argument("--oracle-patches", type=int, default=41,
                    help="patches whose nodes the oracle evaluates (41 x 100 points at the default size)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-gmres", action="store_true")
    ap.add_argument("--no-fp64-gmres", action="store_true", help="skip the FP64-form GMRES solve")
    ap.add_argument("--maxit", type=int, default=400)
    ap.add_argument("--no-fp64-form", action="store_true", help="skip timing the FP64 form beside the mixed one")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-RHS batching measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner solves")
    ap.add_argument("--ifgf-only", action="store_true",
                    help="time the raw IFGF sums only (no N-Mueller plan: seconds to set up)")
    ap.add_argument("--waveguide", action="store_true",
                    help="the 1.67M-point rounded-box waveguide workload instead (IFGF sums; ~6 minutes)")
    ap.add_argument("--bodies32", action="store_true",
                    help="also time the 32-ellipsoid batch (host plans take ~5 minutes)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="also run one device copy of MIB MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); sharding across GPUs "
              "is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2408_02274_amd import NMullerOperator
    from paper_2408_02274_amd import binding as B

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.waveguide:
        print(json.dumps(waveguide(args, log)), flush=True)
        return

    if args.copy_calib > 0:
        nb = args.copy_calib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nb} bytes read, {nb} bytes written")
        del src, dst

    surf = synth.cube_sphere(args.npf, args.nc, args.radius)
    eps_e, eps_i = 1.0, 2.25
    fp32 = args.precision == "fp32"
    prec = B.IFGF_FP32 if fp32 else B.IFGF_FP64
    t0 = time.perf_counter()
    if args.ifgf_only:
        from paper_2408_02274_amd import IFGFPlan
        ks = (2 * math.pi * math.sqrt(eps_i), 2 * math.pi * math.sqrt(eps_e))
        w = np.full(surf.n, 4.0 * math.pi * args.radius ** 2 / surf.n)
        op = IFGFPlan(surf.x, surf.normal, w, ks[0], ks[1], args.tol, precision=prec, max_nrhs=args.nrhs)
        ih = op.handle
        y = torch.from_numpy(synth.complex_normal((args.nrhs, 8, surf.n), 2)).to("cuda")
        out = torch.empty((args.nrhs, 2, 14, surf.n), dtype=torch.complex128, device="cuda")
        args.no_gmres = True
    else:
        op = NMullerOperator(surf, eps_e, eps_i, tol=args.tol, precision=prec, max_nrhs=args.nrhs)
        ih = op.ifgf_handle()
        y = torch.from_numpy(synth.complex_normal((args.nrhs, 4, surf.n), 2)).to("cuda")
        out = torch.empty_like(y)
    plan_s = time.perf_counter() - t0
    log(f"plan built in {plan_s:.1f} s (n = {surf.n})")
    stream = torch.cuda.current_stream()

    def timed_steps(steps, warmup):
        for _ in range(warmup):
            op.apply(y, out, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        B.ifgf_set_timing(ih, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            op.apply(y, out, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = B.ifgf_stats(ih)
        B.ifgf_set_timing(ih, False)
        return el, st

    elapsed, st = timed_steps(args.steps, args.warmup)
    log(f"{args.steps} matvecs ({args.precision}) in {elapsed:.3f} s")
    ms_per_step = elapsed / args.steps * 1e3
    value = args.steps * args.nrhs / elapsed
    npts = st["Ps"] * st["Pa"] * st["Pa"]
    kern = kernel_table(st, args.steps, npts)
    out_main = out.clone()

    # IFGF sums of seeded densities (phi seed 3) in the working form: compared
    # with the oracle's direct sums on sampled rows at the end
    def ifgf_sums():
        phi = torch.from_numpy(synth.complex_normal((1, 8, surf.n), 3)).to("cuda")
        sd = torch.empty((1, 2, 14, surf.n), dtype=torch.complex128, device="cuda")
        B.ifgf_apply(ih, phi, 1, sd)
        torch.cuda.synchronize()
        return sd.cpu().numpy()[0]

    gpu_forms = {}
    if not args.ifgf_only and args.nrhs == 1:
        gpu_forms[args.precision] = {"SD": ifgf_sums(), "Ay": out_main.cpu().numpy()[0]}

    # the plain FP64 form of the same operator, and the mixed form's deviation from it
    fp64_form = None
    if fp32 and not args.no_fp64_form:
        B.ifgf_set_precision(ih, B.IFGF_FP64)
        el64, st64 = timed_steps(max(1, min(args.steps, 3)), 1)
        n64 = max(1, min(args.steps, 3))
        dev = float(torch.linalg.norm(out_main - out) / torch.linalg.norm(out))
        if "fp32" in gpu_forms:
            gpu_forms["fp64"] = {"SD": ifgf_sums(), "Ay": out.cpu().numpy()[0]}
        B.ifgf_set_precision(ih, B.IFGF_FP32)
        k64 = kernel_table(st64, n64, npts)
        fp64_form = {"matvecs_per_s": n64 * args.nrhs / el64, "ms_per_step": el64 / n64 * 1e3,
                     "speedup_mixed_over_fp64": value / (n64 * args.nrhs / el64),
                     "mixed_vs_fp64_rel_l2": dev,
                     "kernels_ms_per_step": {k: round(v["ms"] / n64, 4) for k, v in k64.items()}}
        log(f"FP64 form: {fp64_form['ms_per_step']:.1f} ms/step; mixed deviates by {dev:.2e}")

    dom = max(kern, key=lambda k: kern[k]["ms"])
    d = kern[dom]
    avg_launch_s = d["ms"] * 1e-3 / d["launches"]
    if d["flop"] > 0:
        achieved = d["flop"] / (d["ms"] * 1e-3)
        mfma = dom in ("propagate",)          # contraction on the matrix cores
        if mfma:
            peak = PEAK["fp32_mfma"] if fp32 else PEAK["fp64"]
        else:
            peak = PEAK["fp32_valu_nopk"] if fp32 else PEAK["fp64"]
        roof = {"bound": "mfma" if mfma else "alu", "kernel": dom, "achieved": achieved / 1e12,
                "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak}
    else:
        achieved = d["bytes"] / (d["ms"] * 1e-3)
        roof = {"bound": "hbm", "kernel": dom, "achieved": achieved / 1e9, "peak": 8000.0,
                "unit": "GB/s", "frac": achieved / PEAK["hbm"]}
    tr = traffic_per_launch(dom, args.precision, surf.n, st["Ps"], st["Pa"]) if args.nrhs == 1 else None
    roof["traffic"] = tr
    if tr is not None:
        roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        roof["traffic_GBps"] = tr / avg_launch_s / 1e9
    roof["avg_launch_ms"] = avg_launch_s * 1e3
    roof["flop_per_launch"] = d["flop"] / d["launches"]

    gm = None
    if not args.no_gmres:
        ke = 2 * math.pi * math.sqrt(eps_e)
        ph = np.exp(1j * ke * surf.x[:, 2])
        E = np.zeros((1, surf.n, 3), complex)
        H = np.zeros_like(E)
        E[0, :, 0] = ph
        H[0, :, 1] = (ke / (2 * math.pi)) * ph
        b = op.rhs(torch.from_numpy(E).to("cuda"), torch.from_numpy(H).to("cuda"))
        gm = {}
        solutions = {}

        def solve(tag):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ysol, info = op.solve(b, rtol=1e-4, maxit=args.maxit)
            torch.cuda.synchronize()
            r = {"seconds": time.perf_counter() - t0, "iters": info[0]["iters"],
                 "true_relres": info[0]["true_relres"], "converged": info[0]["converged"],
                 "precond_iters": info[0]["precond_iters"], "fallbacks": info[0]["fallbacks"]}
            log(f"GMRES {tag}: {r}")
            gm[tag] = r
            solutions[tag] = ysol.cpu().numpy()[0]

        solve("mixed" if fp32 else "fp64")
        if fp32 and not args.no_fp64_gmres:
            B.ifgf_set_precision(ih, B.IFGF_FP64)
            solve("fp64")
            B.ifgf_set_precision(ih, B.IFGF_FP32)
        nq = surf.nc * surf.nc
        dims = [8 * nq + 4, 256, 256, 8 * nq]
        nparams = sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(len(dims) - 1))
        op.set_preconditioner(np.zeros(nparams, np.float32), dims)
        solve("scaling_only" + ("_mixed" if fp32 else ""))
        op.set_preconditioner(None)

    learned = None
    if not args.no_gmres and not args.no_learned and os.path.exists(WEIGHTS):
        learned = learned_preconditioner(log)
    res = {
        "metric": METRIC, "value": value, "unit": "matvecs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": ("IFGF raw sums only: " if args.ifgf_only else "") +
                               f"N-Mueller forward map, dielectric sphere radius {args.radius} "
                               f"(eps_r 2.25 in vacuum, k_int = 3 pi, k_ext = 2 pi), 6x{args.npf}x{args.npf} "
                               f"patches x {args.nc}x{args.nc} Chebyshev nodes ({surf.n} points, {4 * surf.n} unknowns), "
                               f"IFGF tol {args.tol}, {args.nrhs} RHS per step, "
                               + ("mixed: FP32 IFGF, FP64 corrections/assembly/GMRES" if fp32 else "FP64"),
                   "Ps": st["Ps"], "Pa": st["Pa"], "D": st["D"], "plan_seconds": round(plan_s, 2),
                   "precision": args.precision},
        "fp64_form": fp64_form,
        "gmres_time_to_1e-4_s": (gm.get("mixed") or gm.get("fp64"))["seconds"] if gm else None,
        "gmres": gm,
        "learned_preconditioner": learned,
        "roofline": roof,
        "kernels_ms_per_step": {k: round(v["ms"] / args.steps, 4) for k, v in kern.items()},
    }
    if not args.no_batch and not args.ifgf_only:
        res["batching"] = batching(log)
    if args.bodies32:
        res["bodies32"] = bodies32(log)
    if not args.no_cpu and not args.ifgf_only:
        # the oracle (O1) on the nodes of args.oracle_patches patches, and the
        # Mie error of the mixed GMRES solution, in the oracle's own program
        mie_path = None
        if gm and "mixed" in solutions:
            import tempfile
            mie_path = os.path.join(tempfile.mkdtemp(), "y.npy")
            np.save(mie_path, solutions["mixed"])
        o1 = oracle_sample(args, args.oracle_patches, log, mie_solution=mie_path)
        rows = o1["rows"]

        def rel(a, b):
            return float(np.linalg.norm(a - b) / np.linalg.norm(b))

        err = {}
        for form, g in gpu_forms.items():
            sd = g["SD"][:, :, rows]
            err["mixed" if form == "fp32" else form] = {
                "S": max(rel(sd[q, :8], o1["SD"][q, :8]) for q in range(2)),
                "D": max(rel(sd[q, 8:], o1["SD"][q, 8:]) for q in range(2)),
                "Ay": rel(g["Ay"][:, rows], o1["Ay"])}
        err["rows"] = f"{rows.size} points of {len(o1['patches'])} patches drawn from seed 2 " \
                      f"({4 * rows.size} rows of A y); S, D: IFGF sums of densities from seed 3 vs " \
                      f"direct sums; A y: unknowns from seed 2 vs the oracle's forward map"
        err["within_tol"] = all(v[k] <= args.tol for v in err.values() if isinstance(v, dict) for k in v)
        res["err_vs_o1"] = err
        if "mie_rel_err" in o1:
            res["mie_err"] = {"mixed_solution": float(o1["mie_rel_err"]),
                              "points": f"1000 Fibonacci points at radius {0.7 * args.radius:g} (interior)"}
        log(f"errors vs O1: {err}; Mie {res.get('mie_err')}")
        t_rows = float(o1["seconds_forward"])
        per_matvec = t_rows * surf.n / rows.size
        o2s = o2_config1_seconds(st["Ps"], st["Pa"])
        res["cpu_baseline"] = {
            "value": 1.0 / per_matvec, "unit": "matvecs/s", "cores": int(o1["nproc"]), "kind": "oracle",
            "sample": f"oracle O1 forward map (direct regular sums, singular corrections, assembly) on "
                      f"{rows.size} of {surf.n} points ({4 * rows.size} rows) took {t_rows:.1f} s over "
                      f"{int(o1['nproc'])} worker processes (one BLAS thread each); extrapolated "
                      f"x{surf.n / rows.size:.0f} to one matvec",
            "cpu_model": cpu_model(), "nproc_host": os.cpu_count(),
            "o2_config1_seconds": o2s,
            "o2_note": f"reference IFGF (O2), one process, on the 1,536-point unit sphere at orders "
                       f"({st['Ps']}, {st['Pa']}); at this workload's size it would take hours"}
    print(json.dumps(res), flush=True)
    op.close()


if __name__ == "__main__":
    main()
