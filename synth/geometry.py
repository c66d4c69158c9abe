"""Analytic parametrised surfaces sampled at open Chebyshev nodes.

A surface is a union of P quadrilateral patches eta_p : [-1,1]^2 -> R^3
(Sec. III-A of the paper).  Node l = j + Nc*i + p*Nc^2 sits at
eta_p(u_i, v_j) with u_k = cos((k + 1/2) pi / Nc) (the open Chebyshev grid
of the paper's eq. cheby_nodes).  For each node the generator returns the
exact point, the exact parametrisation derivatives d eta/du, d eta/dv and
the exact outward unit normal.  Every patch is oriented so that
d eta/du x d eta/dv points outward.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def open_cheb_nodes(nc: int) -> np.ndarray:
    """Open Chebyshev points cos((k + 1/2) pi / nc), k = 0..nc-1."""
    k = np.arange(nc, dtype=np.float64)
    return np.cos((k + 0.5) * np.pi / nc)


@dataclass
class Surface:
    """Nodes of a patch-parametrised surface in the paper's point order."""
    kind: str
    P: int                     # number of patches
    nc: int                    # nodes per patch and direction
    x: np.ndarray              # [N,3] points
    du: np.ndarray             # [N,3] d eta / du
    dv: np.ndarray             # [N,3] d eta / dv
    normal: np.ndarray         # [N,3] exact outward unit normal
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.x.shape[0]


def _pack(kind, patches, nc, params, outward):
    """Sample patch maps on the nc x nc open Chebyshev grid.

    patches: list of callables f(U, V) -> (X, XU, XV) on arrays of (u, v).
    outward: callable X -> unit outward normal, used to fix orientation.
    """
    t = open_cheb_nodes(nc)
    U, V = np.meshgrid(t, t, indexing="ij")          # U[i,j] = u_i, V[i,j] = v_j
    U = U.ravel()
    V = V.ravel()
    xs, dus, dvs = [], [], []
    for f in patches:
        X, XU, XV = f(U, V)
        # orientation check at the patch's nodes (mean sign)
        nrm = outward(X)
        sgn = np.sum(np.cross(XU, XV) * nrm)
        if sgn < 0:
            # reverse u: eta'(u,v) = eta(-u,v); nodes are symmetric under u->-u
            X, XU, XV = f(-U, V)
            XU = -XU
        xs.append(X)
        dus.append(XU)
        dvs.append(XV)
    x = np.concatenate(xs)
    du = np.concatenate(dus)
    dv = np.concatenate(dvs)
    return Surface(kind, len(patches), nc, x, du, dv, outward(x), params)


def _face_frames():
    """(e_n, e_a, e_b) with e_a x e_b = e_n for the six cube faces."""
    ex, ey, ez = np.eye(3)
    return [(ex, ey, ez), (-ex, ez, ey), (ey, ez, ex),
            (-ey, ex, ez), (ez, ex, ey), (-ez, ey, ex)]


def _cube_sphere_patches(npf: int, scale=(1.0, 1.0, 1.0)):
    """Equiangular cube-sphere: each face split into npf x npf patches."""
    S = np.asarray(scale, dtype=np.float64)
    out = []
    edges = np.linspace(-np.pi / 4, np.pi / 4, npf + 1)
    for (en, ea, eb) in _face_frames():
        for a in range(npf):
            for b in range(npf):
                a0, a1 = edges[a], edges[a + 1]
                b0, b1 = edges[b], edges[b + 1]

                def f(U, V, en=en, ea=ea, eb=eb, a0=a0, a1=a1, b0=b0, b1=b1):
                    al = 0.5 * (a0 + a1) + 0.5 * (a1 - a0) * U
                    be = 0.5 * (b0 + b1) + 0.5 * (b1 - b0) * V
                    ta, tb = np.tan(al), np.tan(be)
                    p = en[None, :] + ta[:, None] * ea[None, :] + tb[:, None] * eb[None, :]
                    rn = np.sqrt(np.sum(p * p, axis=1))
                    ph = p / rn[:, None]
                    dpa = (1.0 / np.cos(al) ** 2)[:, None] * ea[None, :] * (0.5 * (a1 - a0))
                    dpb = (1.0 / np.cos(be) ** 2)[:, None] * eb[None, :] * (0.5 * (b1 - b0))

                    def dnorm(dp):
                        return (dp - ph * np.sum(ph * dp, axis=1)[:, None]) / rn[:, None]
                    return ph * S, dnorm(dpa) * S, dnorm(dpb) * S
                out.append(f)
    return out


def cube_sphere(npf: int, nc: int, radius: float = 1.0,
                center=(0.0, 0.0, 0.0)) -> Surface:
    """Sphere of the given radius: 6*npf^2 patches of nc x nc nodes."""
    c = np.asarray(center, dtype=np.float64)
    pats = _cube_sphere_patches(npf, (radius, radius, radius))
    shifted = [(lambda U, V, f=f: _shift(f(U, V), c)) for f in pats]

    def outward(X):
        d = X - c[None, :]
        return d / np.sqrt(np.sum(d * d, axis=1))[:, None]
    return _pack("sphere", shifted, nc,
                 {"radius": radius, "npf": npf, "center": c.tolist()}, outward)


def _shift(t, c):
    X, XU, XV = t
    return X + c[None, :], XU, XV


def ellipsoid(a: float, b: float, c: float, npf: int, nc: int) -> Surface:
    """Ellipsoid x^2/a^2 + y^2/b^2 + z^2/c^2 = 1 as a scaled cube-sphere."""
    pats = _cube_sphere_patches(npf, (a, b, c))
    inv2 = np.array([1.0 / a ** 2, 1.0 / b ** 2, 1.0 / c ** 2])

    def outward(X):
        g = X * inv2[None, :]
        return g / np.sqrt(np.sum(g * g, axis=1))[:, None]
    return _pack("ellipsoid", pats, nc, {"axes": [a, b, c], "npf": npf}, outward)


def _bilinear_sphere_patch(c00, c10, c01, c11, center, r):
    """Patch of a sphere: bilinear blend of 4 corner directions, normalised."""
    c00, c10, c01, c11 = (np.asarray(v, dtype=np.float64) for v in (c00, c10, c01, c11))

    def f(U, V):
        su, sv = 0.5 * (1 + U), 0.5 * (1 + V)
        p = ((1 - su)[:, None] * (1 - sv)[:, None] * c00 + su[:, None] * (1 - sv)[:, None] * c10
             + (1 - su)[:, None] * sv[:, None] * c01 + su[:, None] * sv[:, None] * c11)
        pu = 0.5 * ((1 - sv)[:, None] * (c10 - c00) + sv[:, None] * (c11 - c01))
        pv = 0.5 * ((1 - su)[:, None] * (c01 - c00) + su[:, None] * (c11 - c10))
        rn = np.sqrt(np.sum(p * p, axis=1))
        ph = p / rn[:, None]

        def dn(dp):
            return (dp - ph * np.sum(ph * dp, axis=1)[:, None]) / rn[:, None]
        return center[None, :] + r * ph, r * dn(pu), r * dn(pv)
    return f


def rounded_box(half_outer, radius: float, side: float, nc: int) -> Surface:
    """Rounded rectangular box: the Minkowski sum of an inner box with a ball.

    half_outer: outer half-extents (Lx, Ly, Lz); radius: edge radius; side:
    target patch side.  Patch seams sit on the curvature seams: 6 flat faces,
    12 quarter cylinders and 8 sphere octants (each octant split into 3 quads).
    """
    r = float(radius)
    L = np.asarray(half_outer, dtype=np.float64) - r          # inner half extents
    pats = []

    def nsplit(length):
        return max(1, int(math.ceil(length / side)))

    # flat faces: axis k at +/- (L_k + r), spanning the other two axes
    for k in range(3):
        i1, i2 = [a for a in range(3) if a != k]
        n1, n2 = nsplit(2 * L[i1]), nsplit(2 * L[i2])
        for sgn in (1.0, -1.0):
            for a in range(n1):
                for b in range(n2):
                    lo1 = -L[i1] + 2 * L[i1] * a / n1
                    hi1 = -L[i1] + 2 * L[i1] * (a + 1) / n1
                    lo2 = -L[i2] + 2 * L[i2] * b / n2
                    hi2 = -L[i2] + 2 * L[i2] * (b + 1) / n2

                    def f(U, V, k=k, i1=i1, i2=i2, sgn=sgn, lo1=lo1, hi1=hi1, lo2=lo2, hi2=hi2):
                        X = np.zeros((U.size, 3))
                        X[:, k] = sgn * (L[k] + r)
                        X[:, i1] = 0.5 * (lo1 + hi1) + 0.5 * (hi1 - lo1) * U
                        X[:, i2] = 0.5 * (lo2 + hi2) + 0.5 * (hi2 - lo2) * V
                        XU = np.zeros_like(X)
                        XV = np.zeros_like(X)
                        XU[:, i1] = 0.5 * (hi1 - lo1)
                        XV[:, i2] = 0.5 * (hi2 - lo2)
                        return X, XU, XV
                    pats.append(f)
    # quarter cylinders along axis k, at corner signs (s1, s2) of the other axes
    arc = 0.5 * np.pi * r
    for k in range(3):
        i1, i2 = [a for a in range(3) if a != k]
        nk, nt = nsplit(2 * L[k]), nsplit(arc)
        for s1 in (1.0, -1.0):
            for s2 in (1.0, -1.0):
                for a in range(nk):
                    for b in range(nt):
                        lo = -L[k] + 2 * L[k] * a / nk
                        hi = -L[k] + 2 * L[k] * (a + 1) / nk
                        t0 = 0.5 * np.pi * b / nt
                        t1 = 0.5 * np.pi * (b + 1) / nt

                        def f(U, V, k=k, i1=i1, i2=i2, s1=s1, s2=s2, lo=lo, hi=hi, t0=t0, t1=t1):
                            t = 0.5 * (t0 + t1) + 0.5 * (t1 - t0) * V
                            X = np.zeros((U.size, 3))
                            X[:, k] = 0.5 * (lo + hi) + 0.5 * (hi - lo) * U
                            X[:, i1] = s1 * (L[i1] + r * np.cos(t))
                            X[:, i2] = s2 * (L[i2] + r * np.sin(t))
                            XU = np.zeros_like(X)
                            XU[:, k] = 0.5 * (hi - lo)
                            XV = np.zeros_like(X)
                            XV[:, i1] = -s1 * r * np.sin(t) * 0.5 * (t1 - t0)
                            XV[:, i2] = s2 * r * np.cos(t) * 0.5 * (t1 - t0)
                            return X, XU, XV
                        pats.append(f)
    # sphere octants: each split into 3 quads around the octant centroid
    for sx in (1.0, -1.0):
        for sy in (1.0, -1.0):
            for sz in (1.0, -1.0):
                s = np.array([sx, sy, sz])
                cen = s * L
                e = [s[0] * np.array([1.0, 0, 0]), s[1] * np.array([0, 1.0, 0]),
                     s[2] * np.array([0, 0, 1.0])]
                g = (e[0] + e[1] + e[2]) / 3.0
                for q in range(3):
                    a_, b_, c_ = e[q], e[(q + 1) % 3], e[(q + 2) % 3]
                    mab = 0.5 * (a_ + b_)
                    mac = 0.5 * (a_ + c_)
                    pats.append(_bilinear_sphere_patch(a_, mab, mac, g, cen, r))

    def outward(X):
        d = X - np.clip(X, -L[None, :], L[None, :])
        return d / np.sqrt(np.sum(d * d, axis=1))[:, None]
    return _pack("rounded_box", pats, nc,
                 {"half_outer": list(map(float, half_outer)), "radius": r, "side": side},
                 outward)


def fibonacci_sphere(n: int, radius: float) -> np.ndarray:
    """n nearly uniform points on a sphere (Fibonacci lattice)."""
    k = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * k / n
    rho = np.sqrt(1.0 - z * z)
    phi = np.pi * (3.0 - np.sqrt(5.0)) * k
    return radius * np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)
