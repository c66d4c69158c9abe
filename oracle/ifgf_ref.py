"""O2: the reference IFGF, step by step (oracle; test infrastructure only).

Follows Sec. III-E..III-I of the paper in its order and notation:

  * single box: factorisation G(x,y) = G(x,x_S) g_S(x,y) with the analytic
    factor g_S = |x-x_S|/|x-y| exp(i k (|x-y| - |x-x_S|))   (eq. ifgf_fact,
    ifgf_ana_factor), radial variable s = h/r with h = sqrt(3) H / 2 and
    box-centred spherical angles (eq. ifgf_cov);
  * cone domain E = [0, eta] x [0, pi] x [0, 2 pi), eta = sqrt(3)/3, split
    into n_s x n_a x 2 n_a cone segments (eq. cone_dom, box_cone_seg), each
    carrying a P_s x P_a x P_a tensor Chebyshev interpolant (Sec. III-F);
  * octree: level-1 cube containing all points, level d boxes of side
    H_d = H_1 / 2^(d-1), relevant (non-empty) boxes only, D the first level
    with H_D <= 0.25 lambda (eq. rele_boxes); neighbours and cousins
    (eq. box_neighbor, box_cousin); relevant cones defined recursively from
    level 3 (eq. rele_cone); cone counts per level (Remark 2);
  * the algorithm summary of Sec. III-G: direct near sums at level D, direct
    F^D at leaf-cone interpolation points, then for d = D..3 interpolation to
    cousin points times the centred factor and interpolation to the parent's
    interpolation points times the re-centring factor G(x,x_child)/G(x,x_parent);
  * IFGF_Vec (Sec. III-I): one traversal for 8 densities x 2 kernels,
    normal derivative of the single-layer sums for densities 0..5.

Readings where the text is silent or garbled:
  A1  leaf size uses the shorter wavelength 2 pi / max(k0, k1);
  A2  a_d uses max(k0, k1); A3 the cone rule counts from level D+1 down;
  A4  the radial and the angular cone counts both double (Remark 2 as written;
      refine_radial=False doubles only the angular count, an alternative whose
      radial interpolation error grows with kappa H on large boxes);
  A5  neighbours are the 27 boxes with ||j - k||_inf <= 1 (self included);
  A6  cone intervals half-open with the last closed: index = min(floor, n-1),
      phi = atan2(y, x) mapped to [0, 2 pi); the angular indices are decided
      against the boundary directions k pi / n_a (their C-library cos and
      sin): theta >= k pi / n_a  <=>  cos theta <= cos(k pi / n_a), and phi
      >= k pi / n_a  <=>  the point lies counter-clockwise of that boundary
      ray, tested by a cross product in its half plane -- no acos or atan2
      decides an index, so every implementation that forms the same
      products takes the same decision, also for points exactly on a
      boundary (which symmetric surfaces produce);
  A7  Chebyshev coefficients w_i = (2/n) c_i sum_j f(x_j) T_i(x_j), c_0 = 1/2,
      with n = P_s or P_a nodes on each cone interval;
  A8  normal derivative: the analytic derivative of the same interpolant by
      default (the h -> 0 limit of the paper's forward difference); the
      forward difference with h = 1e-6 is available as deriv="fd";
  A21 the level-1 side is the largest bounding-box extent times (1 + 1e-9),
      centred on the bounding box, so that every point lies in a half-open box.

Pins (tests/test_oracle_ifgf.py): counting-kernel exactness (G = 1 makes every
(target, source) pair count exactly once across the near field and all
levels), brute-force comparison with O1 at the paper's (P_s, P_a) = (3, 5),
error decreasing with the interpolation orders, disjoint and covering cone
partition, neighbour/cousin lists against an O(B^2) classification.
"""
from __future__ import annotations

import math

import numpy as np

from . import cheb

SQRT3 = math.sqrt(3.0)
ETA = SQRT3 / 3.0
TWO_PI = 2.0 * math.pi
NS, ND = 8, 6


class Params:
    def __init__(self, Ps=3, Pa=5, ns_init=1, na_init=2, leaf_wavelengths=0.25,
                 refine_radial=True, kernel="helmholtz", deriv="analytic", fd_h=1e-6):
        self.Ps, self.Pa = Ps, Pa
        self.ns_init, self.na_init = ns_init, na_init
        self.leaf_wavelengths = leaf_wavelengths
        self.refine_radial = refine_radial
        self.kernel = kernel          # "helmholtz" | "counting"
        self.deriv = deriv            # "analytic" | "fd"
        self.fd_h = fd_h


def morton_key(k: np.ndarray) -> np.ndarray:
    """Interleave the bits of integer box coordinates (x most significant)."""
    k = k.astype(np.int64)
    key = np.zeros(k.shape[0], dtype=np.int64)
    for b in range(20):
        key |= ((k[:, 0] >> b) & 1) << (3 * b + 2)
        key |= ((k[:, 1] >> b) & 1) << (3 * b + 1)
        key |= ((k[:, 2] >> b) & 1) << (3 * b)
    return key


# Interpolation points use the platform C library's sin/cos (Python's math
# module) and the continuous (theta, phi) of a point its acos/atan2; the cone
# index of a point is decided against tables of the boundary directions
# (reading A6), computed with the same library.
_acos = np.frompyfunc(math.acos, 1, 1)
_atan2 = np.frompyfunc(math.atan2, 2, 1)
_sin = np.frompyfunc(math.sin, 1, 1)
_cos = np.frompyfunc(math.cos, 1, 1)


def _f64(a):
    return np.asarray(a, dtype=object).astype(np.float64)


def spherical(dx, dy, dz):
    """r, theta = arccos(dz/r) and phi = atan2(dy, dx) mapped to [0, 2 pi)."""
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    ct = np.clip(dz / r, -1.0, 1.0)
    th = _f64(_acos(ct))
    ph = _f64(_atan2(dy, dx))
    ph = np.where(ph < 0.0, ph + TWO_PI, ph)
    return r, th, ph


def boundary_directions(na):
    """cos and sin of the cone boundary angles k pi / na, k = 0..na."""
    da = math.pi / na
    return (np.array([math.cos(k * da) for k in range(na + 1)]),
            np.array([math.sin(k * da) for k in range(na + 1)]))


def cone_of(dx, dy, dz, h, ns, na):
    """Cone segment index gamma = (i_s, i_theta, i_phi) flattened, plus (s, theta, phi).

    i_s = min(floor(s / ds), ns - 1); i_theta counts the boundaries k = 1..na-1
    with theta >= k pi / na, i.e. cos theta <= cos(k pi / na); i_phi counts
    the boundaries phi >= k pi / na: in the upper half plane (y > 0, or y = 0
    and x >= 0) those k = 1..na-1 whose boundary ray (cos, sin) has the
    point on or counter-clockwise of it (cos_k y - sin_k x >= 0), in the
    lower half the same test on the point turned by pi, plus na (reading A6).
    A point on the z axis (x = y = 0) has i_phi = 0."""
    r, th, ph = spherical(dx, dy, dz)
    s = h / r
    ds = ETA / ns
    i_s = np.minimum(np.floor(s / ds), ns - 1).astype(np.int64)
    ct = np.clip(dz / r, -1.0, 1.0)
    C, S = boundary_directions(na)
    Ck, Sk = C[None, 1:na], S[None, 1:na]
    i_t = np.sum(np.atleast_1d(ct)[:, None] <= Ck, axis=1).astype(np.int64)
    dx, dy = np.atleast_1d(dx), np.atleast_1d(dy)
    up = (dy > 0) | ((dy == 0) & (dx >= 0))
    px = np.where(up, dx, -dx)
    py = np.where(up, dy, -dy)
    i_p = np.sum(Ck * py[:, None] - Sk * px[:, None] >= 0, axis=1).astype(np.int64)
    i_p = np.where(up, i_p, i_p + na)
    i_p = np.where((dx == 0) & (dy == 0), 0, i_p)
    return (i_s * na + i_t) * (2 * na) + i_p, r, s, th, ph


class Level:
    pass


class Tree:
    """Box octree, cone structure and relevant-cone tables (algorithm step 1)."""

    def __init__(self, x, kappas, params: Params | None = None):
        self.p = p = params or Params()
        x = np.asarray(x, dtype=np.float64)
        self.N = N = x.shape[0]
        self.kappas = tuple(float(k) for k in kappas)
        kmax = max(self.kappas)
        lo, hi = x.min(axis=0), x.max(axis=0)
        self.center = 0.5 * (lo + hi)
        ext = float(np.max(hi - lo))
        self.H1 = ext * (1.0 + 1e-9) if ext > 0 else 1.0
        lam = TWO_PI / kmax
        D = 1
        while self.H1 * 2.0 ** (-(D - 1)) > p.leaf_wavelengths * lam:
            D += 1
        self.D = D
        self.origin = self.center - 0.5 * self.H1
        HD = math.ldexp(self.H1, -(D - 1))
        nmax = 1 << (D - 1)
        kD = np.floor((x - self.origin[None, :]) / HD).astype(np.int64)
        kD = np.clip(kD, 0, nmax - 1)
        keyD = morton_key(kD)
        self.perm = np.lexsort((np.arange(N), keyD))     # sorted position -> input index
        self.xs = x[self.perm]
        kD = kD[self.perm]
        keyD = keyD[self.perm]

        # cone counts (Remark 2, readings A2-A4)
        self.ns = {}
        self.na = {}
        ns, na = p.ns_init, p.na_init
        for d in range(D, 2, -1):
            Hd = math.ldexp(self.H1, -(d - 1))
            a = 2 if kmax * Hd > 0.5 else 1
            na *= a
            if p.refine_radial:
                ns *= a
            self.ns[d], self.na[d] = ns, na

        # boxes per level (linear octree in Morton order)
        self.levels = {}
        for d in range(1, D + 1):
            L = Level()
            L.d = d
            L.H = math.ldexp(self.H1, -(d - 1))
            L.h = SQRT3 / 2.0 * L.H
            key = keyD >> (3 * (D - d))
            starts = np.flatnonzero(np.r_[True, key[1:] != key[:-1]])
            L.start = starts
            L.end = np.r_[starts[1:], N]
            L.key = key[starts]
            L.coords = kD[starts] >> (D - d)
            L.centers = self.origin[None, :] + L.H * (L.coords + 0.5)
            L.nb = starts.size
            L.box_of_point = np.repeat(np.arange(L.nb), L.end - L.start)
            self.levels[d] = L
        for d in range(2, D + 1):
            L, P = self.levels[d], self.levels[d - 1]
            L.parent = np.searchsorted(P.key, L.key >> 3)
            P.child_start = np.searchsorted(L.parent, np.arange(P.nb), side="left")
            P.child_end = np.searchsorted(L.parent, np.arange(P.nb), side="right")
        for d in range(1, D + 1):
            self._neighbours(self.levels[d])
        for d in range(3, D + 1):
            self._cousins(self.levels[d], self.levels[d - 1])
        self._relevant_cones()

    # --- eq. box_neighbor / box_cousin ---------------------------------
    def _neighbours(self, L):
        lut = {tuple(c): i for i, c in enumerate(L.coords.tolist())}
        nbrs = []
        for c in L.coords.tolist():
            lst = []
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        j = lut.get((c[0] + dx, c[1] + dy, c[2] + dz))
                        if j is not None:
                            lst.append(j)
            nbrs.append(np.array(sorted(lst), dtype=np.int64))
        L.neighbours = nbrs

    def _cousins(self, L, P):
        cous = []
        for b in range(L.nb):
            mine = set(L.neighbours[b].tolist())
            lst = []
            for pn in P.neighbours[L.parent[b]]:
                for c in range(P.child_start[pn], P.child_end[pn]):
                    if c not in mine:
                        lst.append(c)
            cous.append(np.array(sorted(lst), dtype=np.int64))
        L.cousins = cous

    # --- cone segments --------------------------------------------------
    def ncones(self, d):
        return self.ns[d] * self.na[d] * 2 * self.na[d]

    def cone_nodes(self, d, cone_ids):
        """(s, theta, phi) interpolation nodes of the given cones: [n, Ps, Pa, Pa] each."""
        p = self.p
        ns, na = self.ns[d], self.na[d]
        i_p = cone_ids % (2 * na)
        i_t = (cone_ids // (2 * na)) % na
        i_s = cone_ids // (2 * na * na)
        ds, da = ETA / ns, math.pi / na
        xs, xa = cheb.nodes(p.Ps), cheb.nodes(p.Pa)
        s = (i_s[:, None] + 0.5) * ds + 0.5 * ds * xs[None, :]
        t = (i_t[:, None] + 0.5) * da + 0.5 * da * xa[None, :]
        f = (i_p[:, None] + 0.5) * da + 0.5 * da * xa[None, :]
        S = np.broadcast_to(s[:, :, None, None], (cone_ids.size, p.Ps, p.Pa, p.Pa))
        Th = np.broadcast_to(t[:, None, :, None], S.shape)
        Ph = np.broadcast_to(f[:, None, None, :], S.shape)
        return S, Th, Ph

    def cone_points(self, d, boxes, cone_ids):
        """Cartesian interpolation points X [n, Ps*Pa*Pa, 3] of cones (box, cone)."""
        L = self.levels[d]
        S, Th, Ph = self.cone_nodes(d, cone_ids)
        n = cone_ids.size
        rr = (L.h / S).reshape(n, -1)
        st, ct = _f64(_sin(Th)).reshape(n, -1), _f64(_cos(Th)).reshape(n, -1)
        sp, cp = _f64(_sin(Ph)).reshape(n, -1), _f64(_cos(Ph)).reshape(n, -1)
        c = L.centers[boxes]
        X = np.empty((n, rr.shape[1], 3))
        X[..., 0] = c[:, None, 0] + rr * (st * cp)
        X[..., 1] = c[:, None, 1] + rr * (st * sp)
        X[..., 2] = c[:, None, 2] + rr * ct
        return X

    def local_coords(self, d, cone_ids, s, th, ph):
        """Affine maps of (s, theta, phi) onto [-1, 1] within the cone intervals."""
        ns, na = self.ns[d], self.na[d]
        i_p = cone_ids % (2 * na)
        i_t = (cone_ids // (2 * na)) % na
        i_s = cone_ids // (2 * na * na)
        ds, da = ETA / ns, math.pi / na
        us = (s - (i_s + 0.5) * ds) / (0.5 * ds)
        ut = (th - (i_t + 0.5) * da) / (0.5 * da)
        up = (ph - (i_p + 0.5) * da) / (0.5 * da)
        return us, ut, up

    # --- eq. rele_cone: relevant cones, recursively from level 3 ------
    def _relevant_cones(self):
        self.tgt_pairs = {}     # level -> (target sorted idx, box, slot, cone)
        self.prop_pairs = {}    # level d (child) -> (parent slot, point k, child box, child slot, cone)
        for d in range(3, self.D + 1):
            L = self.levels[d]
            nc = self.ncones(d)
            # (1) cousin points
            bl, tl = [], []
            for b in range(L.nb):
                for c in L.cousins[b]:
                    pts = np.arange(L.start[c], L.end[c])
                    tl.append(pts)
                    bl.append(np.full(pts.size, b, dtype=np.int64))
            tb = np.concatenate(bl) if bl else np.zeros(0, np.int64)
            tt = np.concatenate(tl) if tl else np.zeros(0, np.int64)
            dlt = self.xs[tt] - L.centers[tb]
            tc = cone_of(dlt[:, 0], dlt[:, 1], dlt[:, 2], L.h, self.ns[d], self.na[d])[0]
            keys = [tb * nc + tc]
            # (2) interpolation points of relevant parent cones
            if d >= 4:
                P = self.levels[d - 1]
                X = self.cone_points(d - 1, P.slot_box, P.slot_cone)   # [nsP, npts, 3]
                npts = X.shape[1]
                ps_l, pk_l, cb_l, pj_l = [], [], [], []
                nch = P.child_end[P.slot_box] - P.child_start[P.slot_box]
                for j in range(8):
                    has = np.flatnonzero(nch > j)
                    if has.size == 0:
                        continue
                    cb = P.child_start[P.slot_box[has]] + j
                    ps_l.append(np.repeat(has, npts))
                    pk_l.append(np.tile(np.arange(npts), has.size))
                    cb_l.append(np.repeat(cb, npts))
                    pj_l.append(np.full(has.size * npts, j, dtype=np.int64))
                pj = np.concatenate(pj_l)
                pslot = np.concatenate(ps_l)
                pk = np.concatenate(pk_l)
                cbox = np.concatenate(cb_l)
                Xp = X[pslot, pk]
                dlt = Xp - L.centers[cbox]
                pc = cone_of(dlt[:, 0], dlt[:, 1], dlt[:, 2], L.h, self.ns[d], self.na[d])[0]
                keys.append(cbox * nc + pc)
            allk = np.unique(np.concatenate(keys))
            L.slot_key = allk
            L.slot_box = allk // nc
            L.slot_cone = allk % nc
            L.nslots = allk.size
            self.tgt_pairs[d] = (tt, tb, np.searchsorted(allk, tb * nc + tc), tc)
            if d >= 4:
                self.prop_pairs[d] = (pslot, pk, cbox,
                                      np.searchsorted(allk, cbox * nc + pc), pc, pj)

    def counts(self):
        """Plan unit counts used for algorithmic work estimates."""
        L = self.levels[self.D]
        near = sum(int(L.end[b] - L.start[b]) * int(sum(L.end[c] - L.start[c] for c in L.neighbours[b]))
                   for b in range(L.nb)) - self.N
        out = {"D": self.D, "near_pairs": near, "leaf_slots": int(L.nslots)}
        for d in range(3, self.D + 1):
            out[f"slots_{d}"] = int(self.levels[d].nslots)
            out[f"target_pairs_{d}"] = int(self.tgt_pairs[d][0].size)
            if d >= 4:
                out[f"prop_pairs_{d}"] = int(self.prop_pairs[d][0].size)
        return out


class ReferenceIFGF:
    """The IFGF_Vec forward evaluation of eq. ifgf_sum_em (algorithm steps 2-3)."""

    def __init__(self, x, normals, weights, kappas, params: Params | None = None):
        self.tree = Tree(x, kappas, params)
        t = self.tree
        self.p = t.p
        self.ns_ = np.asarray(normals, dtype=np.float64)[t.perm]
        self.w = np.asarray(weights, dtype=np.float64)[t.perm]
        Ps, Pa = self.p.Ps, self.p.Pa
        self.Ms = cheb.transform_matrix(Ps)
        self.Ma = cheb.transform_matrix(Pa)

    # kernel pieces -----------------------------------------------------
    def _counting(self):
        return self.p.kernel == "counting"

    def _analytic_factor(self, k, r_xy, r_xc):
        """g = |x - x_c| / |x - y| exp(i k (|x - y| - |x - x_c|))  (eq. ifgf_ana_factor)."""
        if self._counting():
            return np.ones(np.broadcast(r_xy, r_xc).shape, dtype=np.complex128)
        return (r_xc / r_xy) * np.exp(1j * k * (r_xy - r_xc))

    def _centred(self, k, r):
        """G(x, x_c) = exp(i k r) / (4 pi r)."""
        if self._counting():
            return np.ones(np.shape(r), dtype=np.complex128)
        return np.exp(1j * k * r) / (4.0 * np.pi * r)

    def _coefficients(self, vals):
        """Cone values [n, Ps, Pa, Pa, ...] -> Chebyshev coefficients (Sec. III-F)."""
        c = np.tensordot(self.Ms, vals, axes=(1, 1))          # [i, n, Pa, Pa, ...]
        c = np.tensordot(self.Ma, c, axes=(1, 2))             # [j, i, n, Pa, ...]
        c = np.tensordot(self.Ma, c, axes=(1, 3))             # [k, j, i, n, ...]
        return np.moveaxis(np.moveaxis(np.moveaxis(c, 3, 0), 3, 1), 3, 2)

    def _basis(self, us, ut, up, deriv):
        """Tensor Chebyshev basis rows [n, Ps*Pa*Pa] (and d/du-hat rows)."""
        Ps, Pa = self.p.Ps, self.p.Pa
        Ts, Tt, Tp = cheb.T(Ps, us), cheb.T(Pa, ut), cheb.T(Pa, up)
        B = (Ts[:, :, None, None] * Tt[:, None, :, None] * Tp[:, None, None, :]).reshape(us.size, -1)
        if not deriv:
            return B, None
        dTs, dTt, dTp = cheb.dT(Ps, us), cheb.dT(Pa, ut), cheb.dT(Pa, up)
        Bs = (dTs[:, :, None, None] * Tt[:, None, :, None] * Tp[:, None, None, :]).reshape(us.size, -1)
        Bt = (Ts[:, :, None, None] * dTt[:, None, :, None] * Tp[:, None, None, :]).reshape(us.size, -1)
        Bp = (Ts[:, :, None, None] * Tt[:, None, :, None] * dTp[:, None, None, :]).reshape(us.size, -1)
        return B, (Bs, Bt, Bp)

    def _basis_kind(self, us, ut, up, kind):
        """Value rows (kind 0) or d/ds-hat, d/dtheta-hat, d/dphi-hat rows (kind 1, 2, 3)."""
        Ps, Pa = self.p.Ps, self.p.Pa
        fs = cheb.dT if kind == 1 else cheb.T
        ft = cheb.dT if kind == 2 else cheb.T
        fp = cheb.dT if kind == 3 else cheb.T
        A, Bv, Cv = fs(Ps, us), ft(Pa, ut), fp(Pa, up)
        return (A[:, :, None, None] * Bv[:, None, :, None] * Cv[:, None, None, :]).reshape(us.size, -1)

    def _contract(self, slot, us, ut, up, C, kind=0, chunk=1 << 17):
        """F[p] = basis(p) . C[slot[p]] for every pair p, one BLAS product per cone.

        C: cone data [nslots, Ps*Pa*Pa, ncol] complex.  Returns [pairs, ncol].
        """
        npair = slot.size
        ncol = C.shape[-1]
        Cr = np.ascontiguousarray(C).view(np.float64)         # [nslots, npts, 2*ncol]
        out = np.empty((npair, 2 * ncol))
        order = np.argsort(slot, kind="stable")
        for c0 in range(0, npair, chunk):
            idx = order[c0:c0 + chunk]
            B = self._basis_kind(us[idx], ut[idx], up[idx], kind)
            ss = slot[idx]
            cuts = np.flatnonzero(np.r_[True, ss[1:] != ss[:-1], True])
            res = np.empty((idx.size, 2 * ncol))
            for g0, g1 in zip(cuts[:-1], cuts[1:]):
                res[g0:g1] = B[g0:g1] @ Cr[ss[g0]]
            out[idx] = res
        return out.view(np.complex128)

    @staticmethod
    def _scatter_add(dst, idx, val):
        """dst[idx[p]] += val[p] for 2D dst/val (duplicates in idx accumulate)."""
        order = np.argsort(idx, kind="stable")
        si = idx[order]
        cuts = np.flatnonzero(np.r_[True, si[1:] != si[:-1]])
        dst[si[cuts]] += np.add.reduceat(val[order], cuts, axis=0)

    # algorithm step 2a: direct sums on neighbour points at level D ----
    def _near(self, a, out):
        t = self.tree
        L = t.levels[t.D]
        for b in range(L.nb):
            tg = np.arange(L.start[b], L.end[b])
            src = np.concatenate([np.arange(L.start[c], L.end[c]) for c in L.neighbours[b]])
            d = t.xs[tg, None, :] - t.xs[None, src, :]
            r = np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2])
            self_mask = tg[:, None] == src[None, :]
            r = np.where(self_mask, 1.0, r)
            nd = np.sum(self.ns_[tg, None, :] * d, axis=-1)
            for q, k in enumerate(t.kappas):
                if self._counting():
                    g = np.where(self_mask, 0.0, 1.0 + 0j)
                    gd = np.zeros_like(g)
                else:
                    g = np.where(self_mask, 0.0, np.exp(1j * k * r) / (4.0 * np.pi * r))
                    gd = g * (1j * k - 1.0 / r) / r * nd
                out[q, :NS, tg] += (g @ a[:, src].T)
                out[q, NS:, tg] += (gd @ a[:ND, src].T)

    # algorithm step 2b: F^D at relevant leaf-cone interpolation points --
    def _leaf_values(self, a):
        t = self.tree
        d = t.D
        L = t.levels[d]
        Ps, Pa = self.p.Ps, self.p.Pa
        vals = np.zeros((L.nslots, Ps, Pa, Pa, 2, NS), dtype=np.complex128)
        X = t.cone_points(d, L.slot_box, L.slot_cone)            # [nslots, npts, 3]
        order = np.argsort(L.slot_box, kind="stable")
        bounds = np.searchsorted(L.slot_box[order], np.arange(L.nb + 1))
        for b in range(L.nb):
            sl = order[bounds[b]:bounds[b + 1]]
            if sl.size == 0:
                continue
            Xb = X[sl].reshape(-1, 3)
            src = np.arange(L.start[b], L.end[b])
            dxc = Xb - L.centers[b][None, :]
            r_xc = np.sqrt(dxc[:, 0] ** 2 + dxc[:, 1] ** 2 + dxc[:, 2] ** 2)
            dxy = Xb[:, None, :] - t.xs[None, src, :]
            r_xy = np.sqrt(dxy[..., 0] ** 2 + dxy[..., 1] ** 2 + dxy[..., 2] ** 2)
            for q, k in enumerate(t.kappas):
                g = self._analytic_factor(k, r_xy, r_xc[:, None])
                F = g @ a[:, src].T                              # [npts_all, 8]
                vals[sl, ..., q, :] = F.reshape(sl.size, Ps, Pa, Pa, NS)
        return vals

    # algorithm step 3a: interpolation onto cousin points ----------------
    def _targets(self, d, coef, out):
        t = self.tree
        L = t.levels[d]
        tt, tb, slot, cone = t.tgt_pairs[d]
        if tt.size == 0:
            return
        ns, na = t.ns[d], t.na[d]
        npts = self.p.Ps * self.p.Pa * self.p.Pa
        C = coef.reshape(L.nslots, npts, 2, NS)
        CD = np.ascontiguousarray(C[..., :ND]).reshape(L.nslots, npts, 2 * ND)
        C = C.reshape(L.nslots, npts, 2 * NS)
        fd = self.p.deriv == "fd" and not self._counting()
        ds_, da_ = ETA / ns, math.pi / na
        dlt = t.xs[tt] - L.centers[tb]
        _, r, s, th, ph = cone_of(dlt[:, 0], dlt[:, 1], dlt[:, 2], L.h, ns, na)
        us, ut, up = t.local_coords(d, cone, s, th, ph)
        F = self._contract(slot, us, ut, up, C).reshape(-1, 2, NS)
        nrm = self.ns_[tt]
        if fd:
            dl2 = dlt + self.p.fd_h * nrm
            _, r2, s2, th2, ph2 = cone_of(dl2[:, 0], dl2[:, 1], dl2[:, 2], L.h, ns, na)
            us2, ut2, up2 = t.local_coords(d, cone, s2, th2, ph2)   # same cone: may extrapolate
            F2 = self._contract(slot, us2, ut2, up2, CD).reshape(-1, 2, ND)
        elif not self._counting():
            Fs = self._contract(slot, us, ut, up, CD, 1).reshape(-1, 2, ND) * (2.0 / ds_)
            Ft = self._contract(slot, us, ut, up, CD, 2).reshape(-1, 2, ND) * (2.0 / da_)
            Fp = self._contract(slot, us, ut, up, CD, 3).reshape(-1, 2, ND) * (2.0 / da_)
            rhat = dlt / r[:, None]
            n_r = np.sum(nrm * rhat, axis=1)
            st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
            n_th = nrm[:, 0] * ct * cp + nrm[:, 1] * ct * sp - nrm[:, 2] * st
            n_ph = -nrm[:, 0] * sp + nrm[:, 1] * cp
            with np.errstate(divide="ignore", invalid="ignore"):
                c_ph = np.where(st > 0.0, n_ph / (r * st), 0.0)   # grad phi = phi-hat / (r sin theta)
            c_s = -(L.h / (r * r)) * n_r                          # grad s = -(h / r^2) r-hat
            c_t = n_th / r                                        # grad theta = theta-hat / r
        res = np.zeros((tt.size, 2, NS + ND), dtype=np.complex128)
        for q, k in enumerate(t.kappas):
            Gc = self._centred(k, r)
            res[:, q, :NS] = Gc[:, None] * F[:, q, :]
            if self._counting():
                continue
            if fd:
                Gc2 = self._centred(k, r2)
                res[:, q, NS:] = (Gc2[:, None] * F2[:, q, :] - Gc[:, None] * F[:, q, :ND]) / self.p.fd_h
            else:
                dG = (1j * k - 1.0 / r) * n_r                     # n . grad G(x, x_B) / G
                res[:, q, NS:] = Gc[:, None] * (dG[:, None] * F[:, q, :ND] + c_s[:, None] * Fs[:, q, :]
                                                + c_t[:, None] * Ft[:, q, :] + c_ph[:, None] * Fp[:, q, :])
        acc = np.zeros((t.N, 2 * (NS + ND)), dtype=np.complex128)
        self._scatter_add(acc, tt, res.reshape(tt.size, -1))
        out += acc.reshape(t.N, 2, NS + ND).transpose(1, 2, 0)

    # algorithm step 3b: interpolation onto parent interpolation points -
    def _propagate(self, d, coef):
        """Level-d coefficients -> level-(d-1) cone values with re-centring."""
        t = self.tree
        L, P = t.levels[d], t.levels[d - 1]
        Ps, Pa = self.p.Ps, self.p.Pa
        npts = Ps * Pa * Pa
        pslot, pk, cbox, cslot, cone, pj = t.prop_pairs[d]
        X = t.cone_points(d - 1, P.slot_box, P.slot_cone)
        Xp = X[pslot, pk]
        dlt = Xp - L.centers[cbox]
        _, r_c, s, th, ph = cone_of(dlt[:, 0], dlt[:, 1], dlt[:, 2], L.h, t.ns[d], t.na[d])
        dp = Xp - P.centers[P.slot_box[pslot]]
        r_p = np.sqrt(dp[:, 0] ** 2 + dp[:, 1] ** 2 + dp[:, 2] ** 2)
        us, ut, up = t.local_coords(d, cone, s, th, ph)
        C = coef.reshape(L.nslots, npts, 2 * NS)
        F = self._contract(cslot, us, ut, up, C).reshape(-1, 2, NS)
        for q, k in enumerate(t.kappas):
            # re-centring G(X, x_child) / G(X, x_parent) equals the analytic factor
            F[:, q, :] *= self._analytic_factor(k, r_c, r_p)[:, None]
        vals = np.zeros((P.nslots * npts, 2 * NS), dtype=np.complex128)
        F = F.reshape(-1, 2 * NS)
        dest = pslot * npts + pk
        for j in range(8):            # within one child ordinal every destination is unique
            m = pj == j
            vals[dest[m]] += F[m]
        return vals.reshape(P.nslots, Ps, Pa, Pa, 2, NS)

    def apply(self, phi):
        """phi [8, N] complex in input order -> out [2, 14, N] in input order."""
        t = self.tree
        phi = np.asarray(phi)
        a = phi[:, t.perm] * self.w[None, :]
        out = np.zeros((2, NS + ND, t.N), dtype=np.complex128)
        self._near(a, out)
        if t.D >= 3:
            vals = self._leaf_values(a)
            for d in range(t.D, 2, -1):
                coef = self._coefficients(vals)
                self._targets(d, coef, out)
                if d > 3:
                    vals = self._propagate(d, coef)
        res = np.empty_like(out)
        res[:, :, t.perm] = out
        return res
