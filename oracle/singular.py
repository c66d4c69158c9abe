"""Singular and near-singular quadrature and local corrections (oracle;
test infrastructure only).

Sec. III-B..III-D of the paper:
  * patch distance dist(x, Gamma_p) and the singular set S_l = {p : dist <= delta}
    (eq. dist, patch_sing);
  * closest point (u~, v~) = argmin |x_l - eta_p(u, v)| by golden-section
    search started from the nearest node, exact when x_l is a node of the
    patch (eq. dist_min);
  * Kress's sigmoidal map w(tau) with parameter d (eq. mk_cov_1, mk_cov_2)
    and the clustering maps xi_alpha of eq. cov;
  * moments beta_mn = sum_ij K(x_l, eta(u_i, v_j)) J T_m(u_i) T_n(v_j)
    mu_i mu_j w_i w_j on N_beta Fejer nodes mapped by xi (eq. int_moments_cov,
    int_moments_1), which with the Chebyshev expansion of the density
    (eq. phi_cheby, rp_exp) give nodal singular weights;
  * local correction (Sec. III-H): the regular sum already counts every node
    q != l with weight w_q K(x_l, x_q), so C_lq = W_lq - [q != l] w_q K(x_l, x_q).

Kernels K: G_k (single layer, S) and n_l . grad_x G_k (normal derivative, D,
principal value on the smooth surface), for both wavenumbers.

Readings:
  A10 delta_p = 1.0 x the diagonal of patch p's node bounding box;
  A11 N_beta = 6 Nc (even, so no Fejer node falls at tau = 0) and d = 4.  The
      paper chooses N_beta to match the IFGF accuracy; this product-map
      quadrature converges algebraically in N_beta (on the unit sphere with
      Nc = 8: N_beta = 24 gives 8e-4, 48 gives 5e-5, 96 gives 5e-6 relative
      error of S[Y_1^0]), so 6 Nc is the smallest multiple reaching ~1e-4;
  A12 golden section: bracket [u_{i*+1}, u_{i*-1}] x [v_{j*+1}, v_{j*-1}] around the
      nearest node, clipped to [-1, 1]; 4 alternating u/v sweeps of 40
      iterations; alpha within 1e-6 of +-1 snaps to +-1 (the paper's end-point
      cases of eq. cov);
  A13 between nodes the patch is the tensor Chebyshev interpolant of its node
      coordinates.
Pins: w and xi end-point values and vanishing derivatives; sphere eigenvalues
of S and D including these corrections (tests/test_oracle_singular.py).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import cheb

GOLD = (math.sqrt(5.0) - 1.0) / 2.0


class Params:
    def __init__(self, delta_factor=1.0, nbeta=None, d=4, sweeps=4, iters=40):
        self.delta_factor = delta_factor
        self.nbeta = nbeta
        self.d = d
        self.sweeps = sweeps
        self.iters = iters

    def nb(self, nc):
        if self.nbeta is not None:
            return self.nbeta
        return 6 * nc


# --- eq. mk_cov_1 / mk_cov_2 -------------------------------------------
def _nu(tau, d):
    return (1.0 / d - 0.5) * ((math.pi - tau) / math.pi) ** 3 + (1.0 / d) * ((tau - math.pi) / math.pi) + 0.5


def _dnu(tau, d):
    return -(3.0 / math.pi) * (1.0 / d - 0.5) * ((math.pi - tau) / math.pi) ** 2 + 1.0 / (d * math.pi)


def kress_w(tau, d):
    a = _nu(tau, d) ** d
    b = _nu(2 * math.pi - tau, d) ** d
    return 2 * math.pi * a / (a + b)


def kress_dw(tau, d):
    n1, n2 = _nu(tau, d), _nu(2 * math.pi - tau, d)
    a, b = n1 ** d, n2 ** d
    da = d * n1 ** (d - 1) * _dnu(tau, d)
    db = -d * n2 ** (d - 1) * _dnu(2 * math.pi - tau, d)
    return 2 * math.pi * (da * b - a * db) / (a + b) ** 2


# --- eq. cov ----------------------------------------------------------------
def xi(alpha, tau, d):
    """Clustering map xi_alpha(tau) and its derivative, alpha [B], tau [M] -> [B, M]."""
    al = np.asarray(alpha, dtype=np.float64)[:, None]
    t = np.asarray(tau, dtype=np.float64)[None, :]
    at = np.abs(t)
    sg = np.sign(t)
    u_mid = al + ((sg - al) / math.pi) * kress_w(math.pi * at, d)
    m_mid = (1.0 - al * sg) * kress_dw(math.pi * at, d)
    tp = np.abs((t - 1.0) / 2.0)
    u_p1 = al - ((1.0 + al) / math.pi) * kress_w(math.pi * tp, d)
    m_p1 = kress_dw(math.pi * (1.0 - t) / 2.0, d) * np.ones_like(al)
    tm = np.abs((t + 1.0) / 2.0)
    u_m1 = al + ((1.0 - al) / math.pi) * kress_w(math.pi * tm, d)
    m_m1 = kress_dw(math.pi * (1.0 + t) / 2.0, d) * np.ones_like(al)
    is_p = al == 1.0
    is_m = al == -1.0
    u = np.where(is_p, u_p1, np.where(is_m, u_m1, u_mid))
    mu = np.where(is_p, m_p1, np.where(is_m, m_m1, m_mid))
    return u, mu


# --- patch interpolant (reading A13) ----------------------------------------
def patch_coefficients(surf):
    """Tensor Chebyshev coefficients of node coordinates: [P, nc(m), nc(n), 3]."""
    g = surf.grid(surf.x)                                   # [P, i, j, 3]
    c = cheb.coefficients(g, axis=1)
    return cheb.coefficients(c, axis=2)


def eval_patch(A, U, V, deriv=False):
    """eta (and d_u eta, d_v eta) at tensor points: A [B, nc, nc, 3], U [B, Mu], V [B, Mv]."""
    nc = A.shape[1]
    Tu, Tv = cheb.T(nc, U), cheb.T(nc, V)
    X = np.einsum("bim,bmnc,bjn->bijc", Tu, A, Tv, optimize=True)
    if not deriv:
        return X
    dTu, dTv = cheb.dT(nc, U), cheb.dT(nc, V)
    Xu = np.einsum("bim,bmnc,bjn->bijc", dTu, A, Tv, optimize=True)
    Xv = np.einsum("bim,bmnc,bjn->bijc", Tu, A, dTv, optimize=True)
    return X, Xu, Xv


def _dist2(A, x, u, v):
    e = eval_patch(A, u[:, None], v[:, None])[:, 0, 0, :]
    d = x - e
    return np.sum(d * d, axis=1)


def _golden(f, lo, hi, iters):
    a, b = lo.copy(), hi.copy()
    c = b - GOLD * (b - a)
    dd = a + GOLD * (b - a)
    fc, fd = f(c), f(dd)
    for _ in range(iters):
        left = fc < fd
        nb_ = np.where(left, dd, b)
        na_ = np.where(left, a, c)
        nc_ = np.where(left, nb_ - GOLD * (nb_ - na_), dd)
        nd_ = np.where(left, c, na_ + GOLD * (nb_ - na_))
        fnew = f(np.where(left, nc_, nd_))
        fc, fd = np.where(left, fnew, fd), np.where(left, fc, fnew)
        a, b, c, dd = na_, nb_, nc_, nd_
    return 0.5 * (a + b)


def closest_points(surf, A, tgt, pat, prm: Params):
    """(u~, v~, dist) for target indices tgt [B] and patches pat [B] (eq. dist_min)."""
    nc = surf.nc
    t = cheb.nodes(nc)
    xg = surf.x[:surf.P * nc * nc].reshape(surf.P, nc, nc, 3)
    xl = surf.x[tgt]
    d2 = np.sum((xg[pat] - xl[:, None, None, :]) ** 2, axis=3).reshape(len(tgt), -1)
    k = np.argmin(d2, axis=1)
    i0, j0 = k // nc, k % nc
    u0, v0 = t[i0], t[j0]
    lo_u = np.where(i0 + 1 < nc, t[np.minimum(i0 + 1, nc - 1)], -1.0)
    hi_u = np.where(i0 > 0, t[np.maximum(i0 - 1, 0)], 1.0)
    lo_v = np.where(j0 + 1 < nc, t[np.minimum(j0 + 1, nc - 1)], -1.0)
    hi_v = np.where(j0 > 0, t[np.maximum(j0 - 1, 0)], 1.0)
    Ab = A[pat]
    u, v = u0.copy(), v0.copy()
    own = (tgt // (nc * nc)) == pat
    for _ in range(prm.sweeps):
        u = _golden(lambda uu: _dist2(Ab, xl, uu, v), lo_u, hi_u, prm.iters)
        v = _golden(lambda vv: _dist2(Ab, xl, u, vv), lo_v, hi_v, prm.iters)
    # a node of the patch itself: its own parameters exactly
    li = (tgt % (nc * nc)) // nc
    lj = tgt % nc
    u = np.where(own, t[li], u)
    v = np.where(own, t[lj], v)
    u = np.where(np.abs(1.0 - np.abs(u)) < 1e-6, np.sign(u), u)
    v = np.where(np.abs(1.0 - np.abs(v)) < 1e-6, np.sign(v), v)
    dist = np.sqrt(_dist2(Ab, xl, u, v))
    dist = np.where(own, 0.0, dist)
    return u, v, dist


def patch_diameters(surf):
    xg = surf.grid(surf.x).reshape(surf.P, -1, 3)
    ext = xg.max(axis=1) - xg.min(axis=1)
    return np.sqrt(np.sum(ext * ext, axis=1)), xg.min(axis=1), xg.max(axis=1)


def singular_pairs(surf, A, prm: Params, targets=None):
    """All (target l, patch p) with dist(x_l, Gamma_p) <= delta_p, plus (u~, v~)."""
    diam, lo, hi = patch_diameters(surf)
    delta = prm.delta_factor * diam
    tg = np.arange(surf.N) if targets is None else np.asarray(targets)
    X = surf.x[tg]
    # prefilter by the distance to the node bounding box (the patch bulges by
    # far less than delta beyond it)
    gap = np.maximum(0.0, np.maximum(lo[None] - X[:, None], X[:, None] - hi[None]))
    bd = np.sqrt(np.sum(gap * gap, axis=2))
    ti, pi = np.nonzero(bd <= 1.5 * delta[None, :])
    t_idx = tg[ti]
    u, v, dist = closest_points(surf, A, t_idx, pi, prm)
    keep = dist <= delta[pi]
    return t_idx[keep], pi[keep], u[keep], v[keep]


def corrections(surf, kappas, prm: Params | None = None, targets=None, batch=256):
    """Local-correction matrices C (CSR, [N, N]) keyed ('S', q) and ('D', q).

    Row l holds, for every node of every patch in S_l, the singular weight
    minus the regular (Fejer) weight times the kernel, so that
    regular sum + C @ phi is the corrected operator.
    """
    prm = prm or Params()
    nc = surf.nc
    nb = prm.nb(nc)
    A = patch_coefficients(surf)
    tl, pl, ul, vl = singular_pairs(surf, A, prm, targets)
    t = cheb.nodes(nb)
    wt = cheb.fejer_weights(nb)
    M = cheb.transform_matrix(nc)                           # [m, i']
    rows, cols = [], []
    vals = {("S", 0): [], ("S", 1): [], ("D", 0): [], ("D", 1): []}
    nodes_local = np.arange(nc * nc)
    for b0 in range(0, tl.size, batch):
        sl = slice(b0, b0 + batch)
        tg, pa, ua, va = tl[sl], pl[sl], ul[sl], vl[sl]
        B = tg.size
        U, MU = xi(ua, t, prm.d)
        V, MV = xi(va, t, prm.d)
        Ab = A[pa]
        Y, Yu, Yv = eval_patch(Ab, U, V, deriv=True)        # [B, nb, nb, 3]
        cr = np.cross(Yu, Yv)
        Jq = np.sqrt(np.sum(cr * cr, axis=3))
        dx = surf.x[tg][:, None, None, :] - Y
        r = np.sqrt(np.sum(dx * dx, axis=3))
        nd = np.sum(surf.n[tg][:, None, None, :] * dx, axis=3)
        wgt = Jq * (MU * wt[None, :])[:, :, None] * (MV * wt[None, :])[:, None, :]
        Tu, Tv = cheb.T(nc, U), cheb.T(nc, V)                # [B, nb, nc]
        # regular (Fejer) weights times kernel at the patch nodes
        qn = pa[:, None] * nc * nc + nodes_local[None, :]    # [B, nc^2] global node ids
        dq = surf.x[tg][:, None, :] - surf.x[qn]
        rq = np.sqrt(np.sum(dq * dq, axis=2))
        selfq = qn == tg[:, None]
        rq = np.where(selfq, 1.0, rq)
        ndq = np.sum(surf.n[tg][:, None, :] * dq, axis=2)
        for q, k in enumerate(kappas):
            G = np.exp(1j * k * r) / (4 * np.pi * r)
            KD = G * (1j * k - 1.0 / r) * nd / r
            Gq = np.where(selfq, 0.0, np.exp(1j * k * rq) / (4 * np.pi * rq))
            KDq = np.where(selfq, 0.0, Gq * (1j * k - 1.0 / rq) * ndq / rq)
            for name, F, Kq in (("S", G, Gq), ("D", KD, KDq)):
                beta = np.einsum("bim,bij,bjn->bmn", Tu, F * wgt, Tv, optimize=True)
                W = np.einsum("mi,bmn,nj->bij", M, beta, M, optimize=True).reshape(B, -1)
                vals[(name, q)].append(W - surf.w[qn] * Kq)
        rows.append(np.repeat(tg, nc * nc))
        cols.append(qn.ravel())
    r_ = np.concatenate(rows)
    c_ = np.concatenate(cols)
    out = {}
    for key, v in vals.items():
        out[key] = sp.csr_matrix((np.concatenate(v).ravel(), (r_, c_)), shape=(surf.N, surf.N))
    out["pairs"] = (tl, pl)
    return out
