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


def flops_per_unit(name, npts, nk=2):
    """Algorithmic flops per work unit (FMA = 2 flops, transcendental = 1,
    real x complex multiply-add = 4) of one IFGF pass carrying nk kernels:
    2 (both, 16 complex columns) or 1 (one kernel per pass, 8 columns; the
    pass repeats the geometry)."""
    c = 8 * nk
    return {
        "near": 280.0,                                   # (target, source) pair, 2 wavenumbers
        "leaf": 160.0 if nk == 2 else 90.0,              # (interpolation point, source) pair
        "targets": 4.0 * npts * c + 4.0 * npts * 6 * nk + 10.0 * npts + 300.0,   # (target, cousin box)
        "propagate": 4.0 * npts * c + 2.0 * npts + 150.0,                       # (parent point, child box)
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
    # the 64 right-hand sides split over copies of the operator, one graph
    # branch per copy: the small applies run side by side
    ncopy = 8
    copies = [op] + [NMullerOperator(s, 1.0, 2.25, tol=1e-4, precision=B.IFGF_FP32, max_nrhs=64 // ncopy)
                     for _ in range(ncopy - 1)]
    per = 64 // ncopy
    gb = NMullerGraph(copies, [y[i * per:(i + 1) * per] for i in range(ncopy)],
                      [out[i * per:(i + 1) * per] for i in range(ncopy)])
    t_branch = clock(gb.launch)
    # the same split launched eagerly, one HIP stream per copy (default priority)
    streams = [torch.cuda.Stream() for _ in range(ncopy)]

    def eager_streams():
        torch.cuda.current_stream().synchronize()
        for i, (c, st) in enumerate(zip(copies, streams)):
            c.apply(y[i * per:(i + 1) * per], out[i * per:(i + 1) * per], stream=st.cuda_stream)
        for st in streams:
            st.synchronize()

    t_streams = clock(eager_streams)
    ref = torch.empty_like(out)
    for i in range(64):
        op.apply(y[i:i + 1], ref[i:i + 1])
    gb.launch()
    torch.cuda.synchronize()
    branch_dev = float(torch.linalg.norm(out - ref) / torch.linalg.norm(ref))
    res = {"workload": "config-1 sphere (1,536 points), 64 RHS, mixed form",
           "rhs_matvecs_per_s_looped": 64 / t_loop, "rhs_matvecs_per_s_batched": 64 / t_batch,
           "rhs_matvecs_per_s_graph": 64 / t_graph, "graph_nodes": g.nodes, "autotuned_columns": cols,
           "rhs_matvecs_per_s_graph_branches": 64 / t_branch, "graph_branches": ncopy,
           "graph_branches_vs_looped": t_loop / t_branch, "graph_branches_rel_dev": branch_dev,
           "rhs_matvecs_per_s_streams": 64 / t_streams, "streams_vs_looped": t_loop / t_streams,
           "ms_looped": t_loop * 1e3, "ms_batched": t_batch * 1e3, "ms_graph": t_graph * 1e3,
           "ms_graph_branches": t_branch * 1e3}
    gb.close()
    for c in copies[1:]:
        c.close()
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


def bodies32(log, reps=5, check=True):
    """Config 3b: 32 uneven ellipsoids (a, b, c ~ U[0.5, 3], eps_r ~ U[1.5, 4],
    seeds 1000 + i; patches per face ceil(sqrt(A / 1.5)) for surface area A, so
    a patch is about (0.5 wavelengths)^2; 10 x 10 nodes), mixed form: 32
    looped applies vs one graph launch in which every body is a branch of its
    own (the bodies share nothing, so they run side by side).  The graph's
    outputs are compared with the looped ones, and A y of the 4 smallest
    bodies with the oracle's O1 forward map on 3 random patches each."""
    import numpy as np
    import torch
    import synth
    from paper_2408_02274_amd import NMullerGraph, NMullerOperator
    from paper_2408_02274_amd import binding as B

    def area(a, b, c, p=1.6075):   # Knud Thomsen's approximation
        return 4 * math.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3) ** (1 / p)

    ops, ys, outs, npts, specs = [], [], [], [], []
    t0 = time.perf_counter()
    for i, (a, b, c, eps) in enumerate(synth.ellipsoid_batch(32, 1000)):
        npf = max(1, math.ceil(math.sqrt(area(a, b, c) / 1.5)))
        s = synth.ellipsoid(a, b, c, npf, 10)
        ops.append(NMullerOperator(s, 1.0, eps, tol=1e-4, precision=B.IFGF_FP32, fp32_workspaces=1))
        ys.append(torch.from_numpy(synth.complex_normal((1, 4, s.n), 100 + i)).to("cuda"))
        outs.append(torch.empty_like(ys[-1]))
        npts.append(s.n)
        specs.append((a, b, c, eps, npf))
    plan_s = time.perf_counter() - t0
    log(f"bodies32: {sum(npts)} points, plans {plan_s:.0f} s")

    def clock(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    t_loop = clock(lambda: [op.apply(y, o) for op, y, o in zip(ops, ys, outs)])
    looped = [o.clone() for o in outs]
    g = NMullerGraph(ops, ys, outs)
    t_graph = clock(g.launch)
    dev = max(float(torch.linalg.norm(o - r) / torch.linalg.norm(r)) for o, r in zip(outs, looped))
    res = {"workload": "32 ellipsoids, seeds 1000..1031, mixed form", "points_total": int(sum(npts)),
           "points_min": int(min(npts)), "points_max": int(max(npts)), "plan_seconds": plan_s,
           "ms_looped": t_loop * 1e3, "ms_graph": t_graph * 1e3, "batch_matvecs_per_s_graph": 1 / t_graph,
           "body_matvecs_per_s_graph": 32 / t_graph, "body_matvecs_per_s_looped": 32 / t_loop,
           "graph_vs_looped": t_loop / t_graph, "graph_branches": 32, "graph_nodes": g.nodes,
           "graph_vs_looped_rel_dev": dev,
           "note": "one graph launch with one branch per body (fork/join), not a persistent kernel"}
    g.close()
    if check:
        import tempfile
        import subprocess
        nproc = min(16, os.cpu_count() or 1)
        err = {}
        for i in sorted(range(32), key=lambda j: npts[j])[:4]:
            a, b, c, eps, npf = specs[i]
            o = os.path.join(tempfile.mkdtemp(), "o1.npz")
            cmd = [sys.executable, "-m", "oracle.sample", "--geometry", "ellipsoid",
                   "--axes", ",".join(repr(float(v)) for v in (a, b, c)), "--npf", str(npf), "--nc", "10",
                   "--eps-e", "1.0", "--eps-i", repr(float(eps)), "--npatch", "3", "--y-seed", str(100 + i),
                   "--nproc", str(min(nproc, 3)), "--out", o]
            subprocess.run(cmd, cwd=ROOT, check=True, timeout=1200)
            o1 = dict(np.load(o))
            g_ay = looped[i].cpu().numpy()[0][:, o1["rows"]]
            err[f"body {i} ({npts[i]} points)"] = float(np.linalg.norm(g_ay - o1["Ay"]) / np.linalg.norm(o1["Ay"]))
        res["err_vs_o1_Ay"] = err
        res["err_rows"] = "A y on the nodes of 3 random patches (seed 2) of each of the 4 smallest bodies"
    for op in ops:
        op.close()
    log(f"bodies32: {res}")
    return res


def one_kernel_per_pass(surf, eps, prec, tol, y, out_ref, value, steps, log):
    """Remark 3 on the same workload: the operator rebuilt with one kernel per
    IFGF pass (half the cone-buffer memory), its matvec rate against the
    default mode's, and the deviation of its A y from the default's."""
    import torch
    from paper_2408_02274_amd import NMullerOperator
    from paper_2408_02274_amd import binding as B
    t0 = time.perf_counter()
    op = NMullerOperator(surf, eps[0], eps[1], tol=tol, precision=prec, kernel_at_a_time=1)
    plan_s = time.perf_counter() - t0
    out = torch.empty_like(y)
    op.apply(y, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        op.apply(y, out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = B.ifgf_stats(op.ifgf_handle())
    dev = float(torch.linalg.norm(out - out_ref) / torch.linalg.norm(out_ref))
    op.close()
    both, one = st["cone_buffer_bytes_by_mode"]
    r = {"matvecs_per_s": steps / el, "ms_per_step": el / steps * 1e3,
         "slowdown_vs_both_kernels": value / (steps / el), "plan_seconds": round(plan_s, 2),
         "kernels_per_pass": st["kernels_per_pass"],
         "cone_buffer_bytes": {"both_kernels": both, "one_kernel": one},
         "rel_l2_vs_both_kernels": dev}
    log(f"one kernel per pass: {r}")
    return r


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
    out["note"] = ("the network is compared with M = D^-1 alone, its fixed part: a ratio above 1 means the "
                   "learned correction costs time")
    out["config5_status"] = ("partial: trained on operator pairs (e i.i.d., r = A e) of ellipsoids with semi-axes "
                             "U[0.5, 2] and 21,600 points, evaluated on 4 held-out bodies, instead of solver pairs "
                             "on U[1, 4] bodies of 38,400 points and 200 held-out bodies; it beats plain GMRES but "
                             "not M = D^-1 alone")
    log(f"learned preconditioner: {out}")
    return out


def waveguide(args, log):
    """The large workload shaped like the paper's waveguide example (Sec. IV):
    rounded rectangular box 40 x 1 x 0.5 wavelengths with edge radius 0.1,
    patches of about 0.087 wavelengths with 10 x 10 nodes (16,704 patches,
    1,670,400 points, 6,681,600 unknowns), eps 12.1 inside and 2.1 outside
    (k_int = 21.86, k_ext = 9.105), excited by an electric dipole y-polarised
    at the complex source point (-20.5, 0, 0) + i b x (b = k_ext w0^2 / 2,
    w0 = 0.4): a Gaussian beam launched into the end face x = -20.
    Timed: N-Mueller matvecs in the mixed form (FP32 IFGF with FP32-sized
    workspaces, FP64 near-field corrections built on the device, FP64
    assembly), and flexible GMRES(80) with M = D^-1 to a 1e-4 residual.  The
    residuals come from the mixed operator: beside 132 GiB of FP64
    corrections the FP64 IFGF form does not fit.  GMRES runs one restart cycle per call (the next call starts from
    the last iterate), which keeps progress lines coming and costs one extra
    residual matvec per cycle.  Checked: the IFGF sums and A y against the
    oracle's O1 forward map on the nodes of --oracle-patches-wg random
    patches; device memory."""
    import numpy as np
    import torch
    import synth
    from paper_2408_02274_amd import NMullerOperator
    from paper_2408_02274_amd import binding as B
    geo = {"half": (20.0, 0.5, 0.25), "edge": 0.1, "side": 0.087, "nc": 10}
    surf = synth.rounded_box(geo["half"], geo["edge"], geo["side"], geo["nc"])
    eps_e, eps_i = 2.1, 12.1
    omega = 2 * math.pi
    ke = omega * math.sqrt(eps_e)
    free0 = torch.cuda.mem_get_info()[0]
    t0 = time.perf_counter()
    op = NMullerOperator(surf, eps_e, eps_i, tol=args.tol, precision=B.IFGF_FP32, fp32_workspaces=1, verbose=1,
                         kernel_at_a_time=1 if args.wg_one_kernel else 0)
    plan_s = time.perf_counter() - t0
    free1 = torch.cuda.mem_get_info()[0]
    info = op.plan_info()
    ih = op.ifgf_handle()
    st0 = B.ifgf_stats(ih)
    log(f"waveguide plan: n = {surf.n}, {plan_s:.1f} s, {(free0 - free1) / 2**30:.1f} GiB on the device; "
        f"corrections {info}")
    stream = torch.cuda.current_stream()
    y = torch.from_numpy(synth.complex_normal((1, 4, surf.n), 2)).to("cuda")
    out = torch.empty_like(y)
    for _ in range(args.warmup):
        op.apply(y, out, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    B.ifgf_set_timing(ih, True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        op.apply(y, out, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = B.ifgf_stats(ih)
    B.ifgf_set_timing(ih, False)
    log(f"{args.steps} matvecs in {el:.2f} s")
    Ay = out.cpu().numpy()[0]
    phi = torch.from_numpy(synth.complex_normal((1, 8, surf.n), 3)).to("cuda")
    sd = torch.empty((1, 2, 14, surf.n), dtype=torch.complex128, device="cuda")
    B.ifgf_apply(ih, phi, 1, sd)
    torch.cuda.synchronize()
    SD = sd.cpu().numpy()[0]
    del phi, sd, y, out
    npts = st["Ps"] * st["Pa"] * st["Pa"]
    kern = kernel_table(st, args.steps, npts)
    dom = max(kern, key=lambda k: kern[k]["ms"])
    d = kern[dom]
    achieved = d["flop"] / (d["ms"] * 1e-3)
    roof = {"bound": "mfma", "kernel": dom, "achieved": achieved / 1e12, "peak": PEAK["fp32_mfma"] / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK["fp32_mfma"], "traffic": None,
            "avg_launch_ms": d["ms"] / d["launches"], "flop_per_launch": d["flop"] / d["launches"]}

    # excitation and GMRES
    pts = torch.from_numpy(np.ascontiguousarray(surf.x)).to("cuda")
    w0 = 0.4
    beam = (ke * w0 * w0 / 2, 0.0, 0.0)
    E, H = B.ifgf_dipole_field(pts, ke, eps_e, omega, (0.0, 1.0, 0.0), (-20.5, 0.0, 0.0), beam)
    b = op.rhs(E.unsqueeze(0), H.unsqueeze(0))
    del E, H, pts
    torch.cuda.empty_cache()           # the solver allocates its bases outside torch's cache
    # flexible GMRES with M = D^-1 (the identity part of eq. n_muller, which
    # differs by (eps_e + eps_i) / 2 = 7.1 between the two rows here)
    nq = 100
    dims = [8 * nq + 4, 256, 256, 8 * nq]
    op.set_preconditioner(np.zeros(sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(3)), np.float32), dims)
    restart = args.wg_restart
    ysol = torch.zeros_like(b)
    iters, t_gm, cycles, last = 0, 0.0, 0, None
    while iters < args.maxit:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ysol, inf = op.solve(b, y=ysol, rtol=1e-4, maxit=min(restart, args.maxit - iters), restart=restart)
        torch.cuda.synchronize()
        t_gm += time.perf_counter() - t0
        last = inf[0]
        iters += last["iters"]
        cycles += 1
        log(f"GMRES cycle {cycles}: {iters} iterations, residual {last['true_relres']:.3e}, {t_gm:.1f} s")
        if last["converged"] or last["iters"] == 0:
            break
    gm = {"seconds": t_gm, "iters": iters, "true_relres": last["true_relres"], "converged": last["converged"],
          "solver": f"flexible GMRES({restart}), M = D^-1", "cycles": cycles,
          "residual_fp64": last["residual_fp64"],
          "residual_form": "mixed operator (FP32 IFGF, FP64 corrections and assembly), FP64 arithmetic"}
    ynorm = float(torch.linalg.norm(ysol))
    del ysol, b
    peak_gib = (free0 - torch.cuda.mem_get_info()[0]) / 2**30
    op.close()
    res = {"metric": METRIC, "value": args.steps / el, "unit": "matvecs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": f"N-Mueller forward map, rounded box 40 x 1 x 0.5 wavelengths, edge radius 0.1, "
                                  f"{surf.P} patches x 10 x 10 nodes ({surf.n} points, {4 * surf.n} unknowns), "
                                  f"eps 12.1 inside / 2.1 outside (k_int = {omega * math.sqrt(eps_i):.3f}, "
                                  f"k_ext = {ke:.3f}), IFGF tol {args.tol}, complex-source-point dipole RHS; "
                                  f"mixed: FP32 IFGF with FP32-sized workspaces, FP64 corrections/assembly/GMRES",
                      "Ps": st["Ps"], "Pa": st["Pa"], "D": st["D"], "plan_seconds": round(plan_s, 1),
                      "corrections_seconds": round(info["corrections_seconds"], 2),
                      "corrections_on_device": info["corrections_on_device"],
                      "correction_pairs": info["correction_pairs"],
                      "correction_GiB": round(info["correction_bytes"] / 2**30, 2),
                      "ifgf_cone_buffer_GiB": round(st0.get("cone_buffer_bytes", 0) / 2**30, 2),
                      "ifgf_kernels_per_pass": st0.get("kernels_per_pass"),
                      "ifgf_target_result_GiB": round(st0.get("target_result_bytes", 0) / 2**30, 2),
                      "plan_device_GiB": round((free0 - free1) / 2**30, 2),
                      "peak_device_GiB": round(peak_gib, 2)},
           "gmres_time_to_1e-4_s": t_gm if last["converged"] else None,
           "gmres": gm, "solution_norm": ynorm,
           "roofline": roof,
           "kernels_ms_per_step": {k: round(v["ms"] / args.steps, 3) for k, v in kern.items()},
           "paper_context": "Table I row 5 (1,572,864 points): T_IFGF 50.14 s, forward map 58.14 s on 128 "
                            "EPYC 7763 cores"}
    if not args.no_cpu:
        import tempfile
        import subprocess
        nproc = min(16, os.cpu_count() or 1)
        o = os.path.join(tempfile.mkdtemp(), "o1.npz")
        cmd = [sys.executable, "-m", "oracle.sample", "--geometry", "rounded_box", "--nc", "10",
               "--half", ",".join(repr(v) for v in geo["half"]), "--edge", repr(geo["edge"]),
               "--side", repr(geo["side"]), "--eps-e", repr(eps_e), "--eps-i", repr(eps_i),
               "--npatch", str(args.oracle_patches_wg), "--nproc", str(nproc), "--out", o]
        t0 = time.perf_counter()
        subprocess.run(cmd, cwd=ROOT, check=True, timeout=1200)
        log(f"oracle sample ({args.oracle_patches_wg} patches) in {time.perf_counter() - t0:.1f} s")
        o1 = dict(np.load(o))
        rows = o1["rows"]

        def rel(a, b):
            return float(np.linalg.norm(a - b) / np.linalg.norm(b))

        gs = SD[:, :, rows]
        err = {"S": max(rel(gs[q, :8], o1["SD"][q, :8]) for q in range(2)),
               "D": max(rel(gs[q, 8:], o1["SD"][q, 8:]) for q in range(2)),
               "Ay": rel(Ay[:, rows], o1["Ay"]),
               "rows": f"{rows.size} points of {len(o1['patches'])} patches drawn from seed 2 ({4 * rows.size} "
                       f"rows of A y); S, D: IFGF sums of densities from seed 3 vs direct sums; A y: unknowns "
                       f"from seed 2 vs the oracle's forward map"}
        err["within_tol"] = all(err[k] <= args.tol for k in ("S", "D", "Ay"))
        res["err_vs_o1"] = err
        t_rows = float(o1["seconds_forward"])
        per_matvec = t_rows * surf.n / rows.size
        res["cpu_baseline"] = {
            "value": 1.0 / per_matvec, "unit": "matvecs/s", "cores": int(o1["nproc"]), "kind": "oracle",
            "sample": f"oracle O1 forward map (direct regular sums, singular corrections, assembly) on "
                      f"{rows.size} of {surf.n} points ({4 * rows.size} rows) took {t_rows:.1f} s over "
                      f"{int(o1['nproc'])} worker processes (one BLAS thread each); extrapolated "
                      f"x{surf.n / rows.size:.0f} to one matvec",
            "gmres_seconds_estimated": per_matvec * iters,
            "gmres_note": "estimated: O1 matvec time x the GPU's GMRES iteration count",
            "cpu_model": cpu_model(), "nproc_host": os.cpu_count()}
        log(f"waveguide errors vs O1: {err}")
    return res


def kernel_table(st, steps, npts):
    kern = {}
    nk = st.get("kernels_per_pass") or 2
    for name, t in st.get("timing", {}).items():
        kern[name] = {"launches": t["launches"], "ms": t["ms"],
                      "flop": flops_per_unit(name, npts, nk) * t["units"],
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
    ap.add_argument("--oracle-patches-wg", type=int, default=11,
                    help="patches of the waveguide sampled by the oracle (100 nodes each)")
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
                    help="the 1.67M-point rounded-box waveguide workload instead (N-Mueller matvecs and "
                         "GMRES with the dipole excitation; ~10 minutes)")
    ap.add_argument("--wg-one-kernel", action="store_true",
                    help="waveguide: one kernel per IFGF pass (half the cone buffers, room for a larger Krylov basis)")
    ap.add_argument("--wg-restart", type=int, default=80, help="waveguide: FGMRES restart length")
    ap.add_argument("--no-kat", action="store_true",
                    help="skip the one-kernel-per-pass (Remark 3) measurement")
    ap.add_argument("--no-bodies32", action="store_true",
                    help="skip the 32-ellipsoid batch (config 3b; its plans and oracle checks take ~2 minutes)")
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
    if not args.no_kat and not args.ifgf_only and args.nrhs == 1:
        res["one_kernel_per_pass"] = one_kernel_per_pass(surf, (eps_e, eps_i), prec, args.tol, y, out_main,
                                                         value, args.steps, log)
    if not args.no_batch and not args.ifgf_only:
        res["batching"] = batching(log)
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
    op.close()
    if not args.no_bodies32 and not args.ifgf_only:
        import torch
        torch.cuda.empty_cache()
        res["bodies32"] = bodies32(log, check=not args.no_cpu)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
