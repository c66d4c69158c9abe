"""Learned FGMRES preconditioner: training data from solver trajectories,
training on the device, evaluation against plain GMRES (project addition;
the paper solves with plain GMRES, Sec. III-A).

Every numerical step runs in libifgf.so: trajectories (nmuller_solve_trajectory),
the (residual, error) pair layout (nmuller_precond_pairs), the network's
forward/backward/Adam (mlp_train_step) and FGMRES (nmuller_solve with a
preconditioner set).  This module only orchestrates them.

Workload (synthetic, seeded): ellipsoids with semi-axes a, b, c ~ U[0.5, 2]
and interior permittivity eps_r ~ U[2, 12] in vacuum, 6 x 6 x 6 patches of
10 x 10 nodes (21,600 points), one plane wave each with direction uniform on
the sphere and polarisation uniform in its tangent plane.  Training bodies
use seeds 6000 + i, held-out bodies 5000 + i.

    python -m paper_2408_02274_amd.precond train --bodies 6 --out params.npz
    python -m paper_2408_02274_amd.precond eval --params params.npz --bodies 4
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

HIDDEN = (256, 256)
TRAIN_SEED0 = 6000
HELDOUT_SEED0 = 5000


def dims_for(nc, hidden=HIDDEN):
    """Network widths: 8 Nc^2 residual values + 4 patch features in, 8 Nc^2 out."""
    return [8 * nc * nc + 4, *hidden, 8 * nc * nc]


def init_params(dims, seed, last_scale=0.1):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, the last layer
    scaled down so that the untrained preconditioner is close to D^-1."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(dims) - 1):
        W = rng.standard_normal((dims[i], dims[i + 1])) * math.sqrt(2.0 / dims[i])
        if i == len(dims) - 2:
            W *= last_scale
        parts += [W.ravel(), np.zeros(dims[i + 1])]
    return np.concatenate(parts).astype(np.float32)


AXES = (0.5, 2.0)
EPS = (2.0, 12.0)
NPF = 6


def body(seed, npf=NPF, nc=10, axes=AXES, eps_range=EPS):
    """(surface, eps_r, semi-axes) of the ellipsoid drawn from `seed`."""
    import synth
    (a, b, c, eps), = synth.ellipsoid_batch(1, seed, axes, eps_range)
    return synth.ellipsoid(a, b, c, npf, nc), eps, (a, b, c)


def plane_wave_rhs(op, surf, seed, omega=2 * math.pi):
    """b for E = p exp(i k_e d.x), H = (k_e / omega) d x p exp(i k_e d.x)."""
    import torch
    import synth
    d, p = synth.plane_wave_batch(1, seed)
    ke = omega
    ph = np.exp(1j * ke * (surf.x @ d[0]))
    E = (p[0][None, :] * ph[:, None])[None]
    H = ((ke / omega) * np.cross(d[0], p[0])[None, :] * ph[:, None])[None]
    return op.rhs(torch.from_numpy(E).to("cuda"), torch.from_numpy(H).to("cuda"))


def make_operator(surf, eps, tol=1e-4, precision=None):
    from . import binding as B
    from .binding import NMullerOperator
    prec = B.IFGF_FP32 if precision is None else precision
    return NMullerOperator(surf, 1.0, eps, tol=tol, precision=prec)


def collect_pairs(op, b, dims, maxit=300, stride=2, cap=150, rtol_star=1e-6, margin=30.0, log=None):
    """(X, T) training rows from one GMRES trajectory: the iterates x_k,
    their residuals r_k and the last iterate y*, error e_k = y* - x_k.  Only
    records whose residual is at least `margin` times the final one are kept,
    so that the error of y* stays small against e_k."""
    import torch
    n = op.n
    X = torch.empty((cap, 4, n), dtype=torch.complex128, device="cuda")
    R = torch.empty_like(X)
    y, cnt, info = op.solve_trajectory(b, X, R, rtol=rtol_star, maxit=maxit, stride=stride)
    rn = torch.linalg.norm(R[:cnt].reshape(cnt, -1), dim=1)
    final = info["true_relres"] * float(torch.linalg.norm(b))
    keep = int((rn >= margin * final).sum().item())
    if log:
        log(f"trajectory: {info['iters']} iterations to {info['true_relres']:.2e}, "
            f"{cnt} records, {keep} kept")
    cnt = keep
    if cnt == 0:
        return None, None, info
    E = y[None] - X[:cnt]
    op.set_preconditioner(np.zeros(int(sum(dims[i] * dims[i + 1] + dims[i + 1]
                                           for i in range(len(dims) - 1))), np.float32), dims)
    Xr, Tr = op.precond_pairs(R[:cnt].contiguous(), E.contiguous())
    op.set_preconditioner(None)
    del X, R, E
    return Xr, Tr, info


def collect_random_pairs(op, dims, npairs, seed, log=None):
    """(X, T) training rows from operator-generated pairs: errors e with
    i.i.d. complex normal entries and residuals r = A e (one matvec each).
    Per patch, regressing e on r this way approximates the local inverse of
    the operator, the part of A^-1 a patch-local map can represent."""
    import torch
    import synth
    n = op.n
    E = torch.from_numpy(synth.complex_normal((npairs, 4, n), seed)).to("cuda")
    R = torch.empty_like(E)
    for i in range(npairs):
        op.apply(E[i:i + 1], R[i:i + 1])
    op.set_preconditioner(np.zeros(int(sum(dims[i] * dims[i + 1] + dims[i + 1]
                                           for i in range(len(dims) - 1))), np.float32), dims)
    Xr, Tr = op.precond_pairs(R, E)
    op.set_preconditioner(None)
    if log:
        log(f"random pairs: {npairs}")
    del E, R
    return Xr, Tr


def collect_krylov_pairs(op, b, dims, iters=150, log=None):
    """(X, T) rows from solver-generated Krylov pairs: the residuals r_k of a
    GMRES trajectory taken as errors e_k, with r = A e_k (one matvec each).
    The inputs then have the statistics of the vectors FGMRES hands the
    preconditioner, and r = A e holds exactly."""
    import torch
    n = op.n
    X = torch.empty((iters, 4, n), dtype=torch.complex128, device="cuda")
    R = torch.empty_like(X)
    y, cnt, info = op.solve_trajectory(b, X, R, rtol=1e-12, maxit=iters, stride=1)
    del X
    E = R[:cnt]
    E /= torch.linalg.norm(E.reshape(cnt, -1), dim=1).reshape(cnt, 1, 1)
    AE = torch.empty_like(E)
    for i in range(cnt):
        op.apply(E[i:i + 1], AE[i:i + 1])
    op.set_preconditioner(np.zeros(int(sum(dims[i] * dims[i + 1] + dims[i + 1]
                                           for i in range(len(dims) - 1))), np.float32), dims)
    Xr, Tr = op.precond_pairs(AE, E.contiguous())
    op.set_preconditioner(None)
    if log:
        log(f"krylov pairs: {cnt} (trajectory residual {info['true_relres']:.2e})")
    del R, E, AE
    return Xr, Tr


def train(dims, X, T, epochs=30, batch=2048, lr=1e-3, seed=0, dtype=None, log=None):
    """Adam on the mean-squared error of the rows (X, T), cosine step decay.
    Returns (parameters, per-epoch mean losses)."""
    import torch
    from .binding import MLP, MLP_BF16
    net = MLP(dims, dtype=MLP_BF16 if dtype is None else dtype, max_batch=batch)
    net.set_params(init_params(dims, seed))
    N = X.shape[0]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    steps = max(1, N // batch)
    total = epochs * steps
    t = 0
    for ep in range(epochs):
        perm = torch.randperm(N, generator=gen, device="cuda").to(torch.int32)
        acc = torch.zeros(1, dtype=torch.float32, device="cuda")
        for s in range(steps):
            step_lr = lr * 0.5 * (1.0 + math.cos(math.pi * t / total))
            net.train_step(X, T, perm[s * batch:(s + 1) * batch], max(step_lr, 1e-3 * lr), loss)
            acc += loss
            t += 1
        hist.append(float(acc.item()) / steps)
        if log:
            log(f"epoch {ep}: mse {hist[-1]:.4e}")
    params = net.params()
    net.close()
    return params, hist


def evaluate(op, b, params, dims, rtol=1e-4, maxit=800, dtype=None):
    """Plain GMRES, FGMRES with M = D^-1 only, and learned FGMRES on one
    system; FP64 true residuals."""
    import torch
    from .binding import MLP_BF16
    out = {}
    op.set_preconditioner(None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y0, i0 = op.solve(b, rtol=rtol, maxit=maxit)
    torch.cuda.synchronize()
    out["plain"] = dict(i0[0], wall=time.perf_counter() - t0)
    # the network switched off (all parameters zero): M = D^-1 alone
    op.set_preconditioner(np.zeros_like(params), dims, MLP_BF16 if dtype is None else dtype)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    yd, idd = op.solve(b, rtol=rtol, maxit=maxit)
    torch.cuda.synchronize()
    out["scaling_only"] = dict(idd[0], wall=time.perf_counter() - t0)
    op.set_preconditioner(params, dims, MLP_BF16 if dtype is None else dtype)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y1, i1 = op.solve(b, rtol=rtol, maxit=maxit)
    torch.cuda.synchronize()
    out["learned"] = dict(i1[0], wall=time.perf_counter() - t0)
    op.set_preconditioner(None)
    return out


def _log(msg):
    print(f"[precond] {msg}", file=sys.stderr, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["train", "eval"])
    ap.add_argument("--bodies", type=int, default=4)
    ap.add_argument("--params", default=None, help="npz with the trained parameters (eval)")
    ap.add_argument("--out", default=None, help="where to write the trained parameters (train)")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--stride", type=int, default=2)
    ap.add_argument("--maxit", type=int, default=300)
    ap.add_argument("--pairs", choices=["mixed", "krylov", "random", "trajectory"], default="random",
                    help="krylov: GMRES residuals as errors e, r = A e; random: i.i.d. e, r = A e; "
                         "mixed: both; trajectory: e_k = y* - x_k, r_k = b - A x_k")
    ap.add_argument("--npairs", type=int, default=200, help="random pairs per body")
    ap.add_argument("--hidden", default="256,256",
                    help="hidden widths, comma separated, or 'none' for a single affine layer")
    args = ap.parse_args(argv)
    import torch

    if args.mode == "train":
        Xs, Ts, meta = [], [], []
        dims = None
        for i in range(args.bodies):
            seed = TRAIN_SEED0 + i
            surf, eps, axes = body(seed)
            hidden = () if args.hidden == "none" else tuple(int(h) for h in args.hidden.split(","))
            dims = dims_for(surf.nc, hidden)
            t0 = time.perf_counter()
            op = make_operator(surf, eps)
            _log(f"body {seed}: axes {np.round(axes, 2).tolist()} eps {eps:.2f}, plan {time.perf_counter() - t0:.1f} s")
            if args.pairs in ("random", "krylov", "mixed"):
                parts = []
                if args.pairs in ("krylov", "mixed"):
                    parts.append(collect_krylov_pairs(op, plane_wave_rhs(op, surf, seed), dims, log=_log))
                if args.pairs in ("random", "mixed"):
                    parts.append(collect_random_pairs(op, dims, args.npairs // (2 if args.pairs == "mixed" else 1),
                                                      seed, log=_log))
                X = torch.cat([p[0] for p in parts])
                T = torch.cat([p[1] for p in parts])
                del parts
                info = {"iters": 0}
            else:
                b = plane_wave_rhs(op, surf, seed)
                X, T, info = collect_pairs(op, b, dims, maxit=args.maxit, stride=args.stride, log=_log)
            if X is None:
                op.close()
                continue
            Xs.append(X)
            Ts.append(T)
            meta.append({"seed": seed, "eps": eps, "axes": list(axes), "trajectory_iters": info["iters"],
                         "pairs": int(X.shape[0] // surf.P)})
            op.close()
            torch.cuda.empty_cache()
        X = torch.cat(Xs)
        T = torch.cat(Ts)
        del Xs, Ts
        _log(f"training rows: {X.shape[0]} x {X.shape[1]}")
        t0 = time.perf_counter()
        params, hist = train(dims, X, T, epochs=args.epochs, batch=args.batch, lr=args.lr, log=_log)
        ttrain = time.perf_counter() - t0
        if args.out:
            np.savez(args.out, params=params, dims=np.array(dims), loss=np.array(hist))
        print(json.dumps({"mode": "train", "pairs": args.pairs, "bodies": meta, "rows": int(X.shape[0]), "dims": dims,
                          "loss_first": hist[0], "loss_last": hist[-1], "train_seconds": ttrain}), flush=True)
        return 0

    z = np.load(args.params)
    params, dims = z["params"], [int(d) for d in z["dims"]]
    res = []
    for i in range(args.bodies):
        seed = HELDOUT_SEED0 + i
        surf, eps, axes = body(seed)
        op = make_operator(surf, eps)
        b = plane_wave_rhs(op, surf, seed)
        r = evaluate(op, b, params, dims)
        r.update({"seed": seed, "eps": eps, "axes": list(axes)})
        _log(json.dumps(r))
        res.append(r)
        op.close()
    print(json.dumps({"mode": "eval", "results": res}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
