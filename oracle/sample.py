"""Oracle values of a large forward map on sampled rows, computed in a
process pool over the host cores (oracle; test infrastructure only).

Run as a separate program (python -m oracle.sample ...) so that its worker
processes never share a process with device work.  For a cube-sphere of
radius R (6 npf^2 patches of Nc x Nc nodes, the geometry of the paper's
sphere runs, Sec. IV), an ellipsoid of the uneven batch or the rounded box
of its waveguide example, it computes, on the nodes of `npatch` patches drawn from `seed`:

  * the direct regular sums S_q[phi_k], D_q[phi_k] of O1 (eq. ifgf_sum_em,
    self term excluded) for i.i.d. complex normal densities phi (seed
    `phi_seed`, shape [8, N]) and weights w = Fejer x Jacobian;
  * the forward map A y of eq. n_muller (O1: direct sums, singular
    corrections of Sec. III-D, operator assembly) for i.i.d. complex normal
    unknowns y (seed `y_seed`, shape [4, N]);
  * optionally, for a solution y read from a file, the interior field of the
    representation at 1000 Fibonacci points of radius 0.7 R against the Mie
    series (the paper's accuracy check, Sec. IV-B).

With --direct-rows K it computes only the direct regular sums S and D on K
random nodes (seed `seed`) of a sphere or of the rounded box of the paper's
waveguide example (Sec. IV), with constant weights and given wavenumbers.

Every worker rebuilds the surface from the generator arguments and handles
whole patches (the assembly differentiates per patch), one BLAS thread each.
Output: an .npz with rows, S/D [2, 14, rows], Ay [4, rows], timings.
"""
from __future__ import annotations

import argparse
import math
import os
import time

import numpy as np

_W = {}


def _surface(geom):
    import synth
    if geom["kind"] == "sphere":
        return synth.cube_sphere(geom["npf"], geom["nc"], geom["radius"])
    if geom["kind"] == "ellipsoid":
        return synth.ellipsoid(*geom["axes"], geom["npf"], geom["nc"])
    return synth.rounded_box(geom["half"], geom["edge"], geom["side"], geom["nc"])


def _init(geom, eps_e, eps_i, y_seed, phi_seed):
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass
    import synth
    from . import surface
    s = _surface(geom)
    _W["geo"] = s
    _W["surf"] = surface.PatchSurface(s.P, s.nc, s.x, s.du, s.dv)
    _W["eps"] = (eps_e, eps_i)
    _W["y"] = synth.complex_normal((4, s.n), y_seed)
    _W["phi"] = synth.complex_normal((8, s.n), phi_seed)


def _forward_rows(chunk):
    from . import direct, nmuller
    surf = _W["surf"]
    t0 = time.perf_counter()
    nm = nmuller.NMuller(surf, _W["eps"][0], _W["eps"][1], patches=list(chunk))
    ay = nm.apply(_W["y"])
    sd = direct.regular_sums(surf.x, surf.n, surf.w, _W["phi"], nm.kappas, targets=nm.rows)
    return nm.rows, ay, sd, time.perf_counter() - t0


def _direct_rows(args):
    from . import direct
    rows, w, ks = args
    s = _W["geo"]
    t0 = time.perf_counter()
    sd = direct.regular_sums(s.x, s.normal, np.full(s.n, w), _W["phi"], ks, targets=rows, block=16)
    return sd, time.perf_counter() - t0


def _field_points(args):
    from . import nmuller
    y, pts = args
    surf = _W["surf"]
    nm = nmuller.NMuller(surf, _W["eps"][0], _W["eps"][1], corrections={})
    E, _ = nmuller.interior_field(nm, y, pts)
    return E


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--geometry", default="sphere", choices=["sphere", "rounded_box", "ellipsoid"])
    ap.add_argument("--axes", default="1,1,1", help="ellipsoid: semi-axes a,b,c")
    ap.add_argument("--npf", type=int, default=0)
    ap.add_argument("--nc", type=int, required=True)
    ap.add_argument("--radius", type=float, default=1.0)
    ap.add_argument("--half", default="20,0.5,0.25", help="rounded box: outer half extents")
    ap.add_argument("--edge", type=float, default=0.1, help="rounded box: edge radius")
    ap.add_argument("--side", type=float, default=0.087, help="rounded box: patch side")
    ap.add_argument("--direct-rows", type=int, default=0, help="direct sums only, on this many random nodes")
    ap.add_argument("--weight", type=float, default=1.0, help="constant weight of the --direct-rows sums")
    ap.add_argument("--k-int", type=float, default=0.0)
    ap.add_argument("--k-ext", type=float, default=0.0)
    ap.add_argument("--eps-e", type=float, default=1.0)
    ap.add_argument("--eps-i", type=float, default=2.25)
    ap.add_argument("--npatch", type=int, default=11, help="patches sampled (0: Mie check only)")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--y-seed", type=int, default=2)
    ap.add_argument("--phi-seed", type=int, default=3)
    ap.add_argument("--nproc", type=int, default=os.cpu_count())
    ap.add_argument("--mie-solution", default=None, help=".npy [4, N] complex: solution y to check against Mie")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    from multiprocessing import get_context
    if a.geometry == "sphere":
        geom = {"kind": "sphere", "npf": a.npf, "nc": a.nc, "radius": a.radius}
    elif a.geometry == "ellipsoid":
        geom = {"kind": "ellipsoid", "axes": tuple(float(v) for v in a.axes.split(",")), "npf": a.npf, "nc": a.nc}
    else:
        geom = {"kind": "rounded_box", "half": tuple(float(v) for v in a.half.split(",")), "edge": a.edge,
                "side": a.side, "nc": a.nc}
    res = {}
    ctx = get_context("spawn")
    with ctx.Pool(a.nproc, initializer=_init,
                  initargs=(geom, a.eps_e, a.eps_i, a.y_seed, a.phi_seed)) as pool:
        if a.direct_rows > 0:
            n = _surface(geom).n
            rows = np.sort(np.random.default_rng(a.seed).choice(n, a.direct_rows, replace=False))
            ks = (a.k_int, a.k_ext)
            t0 = time.perf_counter()
            parts = pool.map(_direct_rows, [(c, a.weight, ks) for c in np.array_split(rows, 4 * a.nproc)])
            res["seconds_direct"] = time.perf_counter() - t0
            res["rows"] = rows
            res["SD"] = np.concatenate([p[0] for p in parts], axis=2)
            res["n"] = n
        elif a.npatch > 0:
            P = _surface(geom).P
            patches = np.sort(np.random.default_rng(a.seed).choice(P, a.npatch, replace=False))
            res["patches"] = patches
            t0 = time.perf_counter()
            parts = pool.map(_forward_rows, [[int(p)] for p in patches])
            res["seconds_forward"] = time.perf_counter() - t0
            res["rows"] = np.concatenate([p[0] for p in parts])
            res["Ay"] = np.concatenate([p[1] for p in parts], axis=1)
            res["SD"] = np.concatenate([p[2] for p in parts], axis=2)
            res["worker_seconds"] = np.array([p[3] for p in parts])
        if a.mie_solution:
            import synth
            from . import mie
            y = np.load(a.mie_solution)
            pts = synth.fibonacci_sphere(1000, 0.7 * a.radius)
            t0 = time.perf_counter()
            chunks = np.array_split(pts, a.nproc)
            E = np.concatenate(pool.map(_field_points, [(y, c) for c in chunks if len(c)]), axis=0)
            omega = 2 * math.pi
            Em, _ = mie.MieSphere(a.radius, omega * math.sqrt(a.eps_e), omega * math.sqrt(a.eps_i),
                                  omega).fields(pts, "int")
            res["mie_rel_err"] = float(np.linalg.norm(E - Em) / np.linalg.norm(Em))
            res["seconds_mie"] = time.perf_counter() - t0
    res["nproc"] = a.nproc
    np.savez(a.out, **res)


if __name__ == "__main__":
    main()
