"""GPU checks of the learned-preconditioner network and its use in FGMRES.

Kernels against the oracle MLP (oracle/mlp.py):
 - FP32 operands: forward, parameter and input gradients to 1e-5 relative
   (FP32 accumulation over at most ~800 terms: ~sqrt(K) 2^-24 ~ 2e-6).
 - BF16 operands: the oracle rounds every matrix-product operand to bfloat16
   at the same points; the remaining differences are FP32 accumulation
   order and the rare operand whose rounding flips because the FP32 and FP64
   sums straddle a bfloat16 rounding boundary (one bf16 ulp, 2^-8, on a
   fraction ~sqrt(K) 2^-16 of the entries): bar 2e-3 relative L2.
"""
import math

import numpy as np
import pytest

import synth
from oracle import mlp as omlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _rel(a, b):
    a = np.asarray(a)
    if not np.iscomplexobj(a):
        a = a.astype(np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _net_case(dims, B, dtype, seed):
    from paper_2408_02274_amd import MLP
    theta = omlp.init_params(dims, seed).astype(np.float32)
    rng = np.random.default_rng(seed + 1)
    # non-zero biases so that the bias gradients and additions are exercised
    for i in range(len(dims) - 1):
        o = sum(dims[j] * dims[j + 1] + dims[j + 1] for j in range(i)) + dims[i] * dims[i + 1]
        theta[o:o + dims[i + 1]] = rng.uniform(-0.1, 0.1, dims[i + 1])
    X = rng.standard_normal((B, dims[0])).astype(np.float32)
    dY = rng.standard_normal((B, dims[-1])).astype(np.float32)
    net = MLP(dims, dtype=dtype, max_batch=max(B, 8))
    net.set_params(theta)
    Xd = torch.from_numpy(X).to("cuda")
    Y = net.forward(Xd).cpu().numpy()
    dX = torch.empty_like(Xd)
    net.backward(torch.from_numpy(dY).to("cuda"), dX)
    g = net.grad()
    dXh = dX.cpu().numpy()
    net.close()
    return theta.astype(np.float64), X.astype(np.float64), dY.astype(np.float64), Y, g, dXh


@pytest.mark.parametrize("dims,B", [([70, 96, 33, 50], 77), ([804, 256, 256, 800], 384)])
def test_fp32_forward_backward_match_oracle(dims, B):
    from paper_2408_02274_amd import MLP_FP32
    _say(f"[gpu] mlp fp32 dims={dims} B={B}")
    theta, X, dY, Y, g, dX = _net_case(dims, B, MLP_FP32, 11)
    Yo, cache = omlp.forward(theta, dims, X)
    go, dXo = omlp.backward(dims, cache, dY)
    assert _rel(Y, Yo) < 1e-5
    assert _rel(dX, dXo) < 1e-5
    o = 0
    for i in range(len(dims) - 1):
        nw = dims[i] * dims[i + 1]
        assert _rel(g[o:o + nw], go[o:o + nw]) < 1e-5, f"dW layer {i}"
        assert _rel(g[o + nw:o + nw + dims[i + 1]], go[o + nw:o + nw + dims[i + 1]]) < 1e-5, f"db layer {i}"
        o += nw + dims[i + 1]


@pytest.mark.parametrize("dims,B", [([70, 96, 33, 50], 77), ([804, 256, 256, 800], 384)])
def test_bf16_forward_backward_match_rounded_oracle(dims, B):
    from paper_2408_02274_amd import MLP_BF16
    _say(f"[gpu] mlp bf16 dims={dims} B={B}")
    theta, X, dY, Y, g, dX = _net_case(dims, B, MLP_BF16, 12)
    q = omlp.bf16_round
    Yo, cache = omlp.forward(theta, dims, X, quant=q)
    go, dXo = omlp.backward(dims, cache, dY, quant=q)
    assert _rel(Y, Yo) < 2e-3
    assert _rel(dX, dXo) < 2e-3
    assert _rel(g, go) < 2e-3
    # and the rounding matters: the unrounded FP64 network differs by more
    Yf, _ = omlp.forward(theta, dims, X)
    assert _rel(Y, Yf) > 1e-4


def test_train_step_matches_oracle_adam():
    from paper_2408_02274_amd import MLP, MLP_FP32
    dims, N, B, lr = [40, 64, 24], 300, 50, 1e-3
    rng = np.random.default_rng(13)
    theta = omlp.init_params(dims, 14).astype(np.float32)
    X = rng.standard_normal((N, dims[0])).astype(np.float32)
    T = rng.standard_normal((N, dims[-1])).astype(np.float32)
    idx = rng.choice(N, B, replace=False).astype(np.int32)
    _say("[gpu] mlp train step fp32")
    net = MLP(dims, dtype=MLP_FP32, max_batch=B)
    net.set_params(theta)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    Xd, Td, Id = (torch.from_numpy(a).to("cuda") for a in (X, T, idx))
    th = theta.astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for t in range(1, 4):
        net.train_step(Xd, Td, Id, lr, loss)
        torch.cuda.synchronize()
        Yo, cache = omlp.forward(th, dims, X[idx].astype(np.float64))
        lo, dYo = omlp.mse(Yo, T[idx].astype(np.float64))
        go, _ = omlp.backward(dims, cache, dYo)
        assert abs(float(loss.item()) - lo) < 1e-5 * lo
        th, m, v = omlp.adam_step(th, m, v, go, t, lr)
        p = net.params()
        big = np.abs(go) > 1e-4
        # Adam's step is lr g_hat / (sqrt(v_hat) + eps): exact up to FP32 rounding where g is not tiny
        assert np.max(np.abs(p - th)[big]) < 1e-3 * lr
        assert np.max(np.abs(p - th)) < 2.5 * lr
        th = p.astype(np.float64)   # continue from the device state
    net.close()


# ---------------------------------------------------------------------------
# the preconditioner inside the N-Mueller operator

def _small_op(precision=None):
    from paper_2408_02274_amd import NMullerOperator
    from paper_2408_02274_amd import binding as B
    s = synth.ellipsoid(1.0, 0.8, 1.2, 2, 6)     # 24 patches x 6 x 6
    kw = {"Ps": 5, "Pa": 5}
    if precision is not None:
        kw["precision"] = precision
    return s, NMullerOperator(s, 1.0, 3.0, tol=1e-3, **kw), B


def _pack(v, P, nq):
    """numpy version of the patch layout: v [4][n] complex -> [P][8 nq]."""
    out = np.zeros((P, 8 * nq))
    for c in range(4):
        blk = v[c].reshape(P, nq)
        out[:, (2 * c) * nq:(2 * c + 1) * nq] = blk.real
        out[:, (2 * c + 1) * nq:(2 * c + 2) * nq] = blk.imag
    return out


def _unpack(Y, P, nq):
    v = np.zeros((4, P * nq), complex)
    for c in range(4):
        v[c] = (Y[:, (2 * c) * nq:(2 * c + 1) * nq] + 1j * Y[:, (2 * c + 1) * nq:(2 * c + 2) * nq]).ravel()
    return v


def test_patch_features_from_geometry():
    s, op, B = _small_op()
    f = op.patch_features()
    nq = s.nc * s.nc
    ke, ki = 2 * math.pi, 2 * math.pi * math.sqrt(3.0)
    for p in range(s.P):
        x = s.x[p * nq:(p + 1) * nq]
        nr = s.normal[p * nq:(p + 1) * nq]
        d = np.linalg.norm(x.max(0) - x.min(0))
        mn = nr.sum(0) / np.linalg.norm(nr.sum(0))
        ang = np.max(np.arccos(np.clip(nr @ mn, -1, 1)))
        assert np.allclose(f[p], [ke * d / (2 * math.pi), ki * d / (2 * math.pi), 2 * ang, 0.3], rtol=1e-5)
    op.close()


def test_preconditioner_apply_matches_oracle_network():
    s, op, B = _small_op()
    nq = s.nc * s.nc
    dims = [8 * nq + 4, 40, 8 * nq]
    theta = omlp.init_params(dims, 21, last_scale=0.5).astype(np.float32)
    _say("[gpu] preconditioner apply fp32 vs oracle network")
    op.set_preconditioner(theta, dims, B.MLP_FP32)
    v = synth.complex_normal((2, 4, s.n), 22)
    z = op.precond_apply(torch.from_numpy(v).to("cuda")).cpu().numpy()
    feat = op.patch_features().astype(np.float64)
    dm, dj = 1.0, 2.0 / (1.0 + 3.0)
    for i in range(2):
        sc = np.sqrt(np.sum(np.abs(v[i]) ** 2) / v[i].size)
        X = np.concatenate([_pack(v[i] / sc, s.P, nq), feat], axis=1)
        Y, _ = omlp.forward(theta.astype(np.float64), dims, X.astype(np.float32).astype(np.float64))
        zo = np.concatenate([dm * v[i][:2], dj * v[i][2:]]) + sc * _unpack(Y, s.P, nq)
        assert _rel(z[i], zo) < 1e-5
    # zero weights: M = D^-1 exactly
    op.set_preconditioner(np.zeros_like(theta), dims, B.MLP_BF16)
    z0 = op.precond_apply(torch.from_numpy(v).to("cuda")).cpu().numpy()
    assert np.array_equal(z0[:, :2], dm * v[:, :2]) and np.allclose(z0[:, 2:], dj * v[:, 2:], rtol=1e-15)
    op.close()


def test_training_pairs_layout():
    s, op, B = _small_op()
    nq = s.nc * s.nc
    dims = [8 * nq + 4, 8, 8 * nq]
    op.set_preconditioner(np.zeros(omlp.n_params(dims), np.float32), dims)
    R = synth.complex_normal((3, 4, s.n), 31)
    E = synth.complex_normal((3, 4, s.n), 32)
    X, T = op.precond_pairs(torch.from_numpy(R).to("cuda"), torch.from_numpy(E).to("cuda"))
    X, T = X.cpu().numpy(), T.cpu().numpy()
    feat = op.patch_features()
    dj = 2.0 / 4.0
    for i in range(3):
        sc = np.sqrt(np.sum(np.abs(R[i]) ** 2) / R[i].size)
        rows = slice(i * s.P, (i + 1) * s.P)
        assert np.allclose(X[rows, :8 * nq], _pack(R[i] / sc, s.P, nq), rtol=1e-6, atol=1e-6)
        assert np.array_equal(X[rows, 8 * nq:], feat)
        tgt = (E[i] - np.concatenate([R[i][:2], dj * R[i][2:]])) / sc
        assert np.allclose(T[rows], _pack(tgt, s.P, nq), rtol=1e-6, atol=1e-6)
    op.close()


def _plane_wave_rhs(op, s, seed=3):
    d, p = synth.plane_wave_batch(1, seed)
    ke = 2 * math.pi
    ph = np.exp(1j * ke * (s.x @ d[0]))
    E = (p[0][None, :] * ph[:, None])[None]
    H = ((ke / (2 * math.pi)) * np.cross(d[0], p[0])[None, :] * ph[:, None])[None]
    return op.rhs(torch.from_numpy(E).to("cuda"), torch.from_numpy(H).to("cuda"))


def test_trajectory_residuals_are_true_residuals():
    s, op, B = _small_op()
    b = _plane_wave_rhs(op, s)
    cap = 20
    X = torch.empty((cap, 4, s.n), dtype=torch.complex128, device="cuda")
    R = torch.empty_like(X)
    _say("[gpu] trajectory")
    y, cnt, info = op.solve_trajectory(b, X, R, rtol=1e-6, maxit=200, stride=2)
    assert info["converged"] and cnt >= 3
    norms = []
    for j in range(cnt):
        r = b[0] - op.apply(X[j:j + 1])[0]
        assert float(torch.linalg.norm(r - R[j]) / torch.linalg.norm(r)) < 1e-8
        norms.append(float(torch.linalg.norm(R[j])))
    assert all(norms[j + 1] <= norms[j] * (1 + 1e-12) for j in range(len(norms) - 1))   # GMRES is monotone
    op.close()


def test_fgmres_with_scaling_preconditioner_and_fallbacks():
    s, op, B = _small_op()
    nq = s.nc * s.nc
    dims = [8 * nq + 4, 32, 8 * nq]
    b = _plane_wave_rhs(op, s)
    y0, i0 = op.solve(b, rtol=1e-5, maxit=300)
    # zero network: M = D^-1, a block scaling
    op.set_preconditioner(np.zeros(omlp.n_params(dims), np.float32), dims)
    y1, i1 = op.solve(b, rtol=1e-5, maxit=300)
    _say("[gpu] fgmres plain / scaled", i0, i1)
    for y, inf in ((y0, i0[0]), (y1, i1[0])):
        rel = float(torch.linalg.norm(b - op.apply(y)) / torch.linalg.norm(b))
        assert inf["converged"] and rel <= 1e-5 and abs(rel - inf["true_relres"]) < 1e-9
    # (D^-1 equalises the identity parts of the two rows of eq. n_muller and
    # by itself changes the iteration count)
    assert i1[0]["fallbacks"] == 0 and i1[0]["precond_iters"] == i1[0]["iters"]
    # non-finite network output: the first preconditioned column is dropped
    op.set_preconditioner(np.full(omlp.n_params(dims), np.nan, np.float32), dims)
    y2, i2 = op.solve(b, rtol=1e-5, maxit=300)
    _say("[gpu] fgmres nan network", i2)
    assert i2[0]["fallbacks"] == 1 and i2[0]["precond_iters"] == 0 and i2[0]["converged"]
    # ... and the solve goes on with M = D^-1 from the same start
    assert i2[0]["iters"] == i1[0]["iters"]
    # a large random network stalls and is abandoned
    theta = (omlp.init_params(dims, 41, last_scale=50.0)).astype(np.float32)
    op.set_preconditioner(theta, dims)
    y3, i3 = op.solve(b, rtol=1e-5, maxit=400)
    _say("[gpu] fgmres random network", i3)
    assert i3[0]["converged"]
    rel = float(torch.linalg.norm(b - op.apply(y3)) / torch.linalg.norm(b))
    assert rel <= 1e-5
    op.close()


@pytest.fixture(scope="module")
def held_out_solves():
    """The committed network (trained on operator-generated pairs of the
    ellipsoid family, seeds 6000+) on held-out body 5002: plain GMRES,
    flexible GMRES with M = D^-1 alone, and with the network, each to a 1e-4
    FP64 true residual."""
    import os
    from paper_2408_02274_amd import precond
    path = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_2408_02274_amd", "weights",
                        "precond_nc10.npz")
    z = np.load(path)
    params, dims = z["params"], [int(v) for v in z["dims"]]
    surf, eps, axes = precond.body(5002)
    _say(f"[gpu] trained preconditioner, body 5002: n = {surf.n}, eps {eps:.2f}")
    op = precond.make_operator(surf, eps)
    b = precond.plane_wave_rhs(op, surf, 5002)
    r = precond.evaluate(op, b, params, dims, rtol=1e-4, maxit=800)
    op.close()
    _say({k: (r[k]["iters"], round(r[k]["wall"], 2), r[k]["fallbacks"]) for k in ("plain", "scaling_only", "learned")})
    return r


def test_trained_preconditioner_converges_without_fallback(held_out_solves):
    r = held_out_solves
    for k in ("plain", "scaling_only", "learned"):
        assert r[k]["converged"] and r[k]["true_relres"] <= 1e-4
    assert r["learned"]["fallbacks"] == 0
    assert r["learned"]["iters"] < r["plain"]["iters"]


@pytest.mark.xfail(strict=False, reason="the learned correction does not beat its fixed part M = D^-1: on "
                                        "held-out body 5003 it took 229 iterations / 4.76 s against 199 / "
                                        "4.14 s for D^-1 alone (plain GMRES 311 / 6.36 s)")
def test_trained_preconditioner_beats_its_fixed_part(held_out_solves):
    r = held_out_solves
    assert r["learned"]["wall"] < r["scaling_only"]["wall"] < r["plain"]["wall"]
