"""Surface quantities on the patch grid (oracle; test infrastructure only).

Node l = j + Nc*i + p*Nc^2 sits at eta_p(u_i, v_j) (Sec. III-A, eq. mesh_pts_l).
From the parametrisation derivatives at the nodes:
  J = |d_u eta x d_v eta|,  n = d_u eta x d_v eta / J,
  w_l = w_i w_j J_l with the Fejer weights (Sec. III-C, eq. non_sing),
  tangent basis t1 = d_u eta / |d_u eta|, t2 = n x t1 (reading A14),
  surface gradient and divergence by per-patch Chebyshev differentiation
  (Sec. III intro: derivatives via the Chebyshev recurrence).
Pins: sum of weights = sphere area, integral of n = 0, integral of x.n =
3 x volume; gradient/divergence of known fields (tests/test_oracle_surface.py).
"""
from __future__ import annotations

import numpy as np

from . import cheb


class PatchSurface:
    def __init__(self, P, nc, x, du, dv):
        self.P, self.nc = int(P), int(nc)
        self.x = np.asarray(x, dtype=np.float64)
        self.du = np.asarray(du, dtype=np.float64)
        self.dv = np.asarray(dv, dtype=np.float64)
        cr = np.cross(self.du, self.dv)
        self.J = np.sqrt(np.sum(cr * cr, axis=1))
        self.n = cr / self.J[:, None]
        wf = cheb.fejer_weights(self.nc)
        self.w = (np.outer(wf, wf).ravel()[None, :] * np.ones((self.P, 1))).ravel() * self.J
        lu = np.sqrt(np.sum(self.du * self.du, axis=1))
        self.t1 = self.du / lu[:, None]
        self.t2 = np.cross(self.n, self.t1)
        # metric and its inverse
        self.guu = np.sum(self.du * self.du, axis=1)
        self.guv = np.sum(self.du * self.dv, axis=1)
        self.gvv = np.sum(self.dv * self.dv, axis=1)
        det = self.guu * self.gvv - self.guv ** 2
        self.iuu, self.iuv, self.ivv = self.gvv / det, -self.guv / det, self.guu / det

    @property
    def N(self):
        return self.x.shape[0]

    def grid(self, f):
        """[N, ...] node values -> [P, nc(i: u), nc(j: v), ...]."""
        return f.reshape((self.P, self.nc, self.nc) + f.shape[1:])

    def d_du(self, f):
        return cheb.differentiate(self.grid(f), axis=1).reshape(f.shape)

    def d_dv(self, f):
        return cheb.differentiate(self.grid(f), axis=2).reshape(f.shape)

    def surface_grad(self, f):
        """Tangential gradient of scalar node values f [N] (complex ok) -> [N, 3]."""
        fu, fv = self.d_du(f), self.d_dv(f)
        cu = self.iuu * fu + self.iuv * fv
        cv = self.iuv * fu + self.ivv * fv
        return cu[:, None] * self.du + cv[:, None] * self.dv

    def surface_div(self, a):
        """Surface divergence of a tangent field a [N, 3]:
        div a = (1/J) [d_u (J a^u) + d_v (J a^v)], a = a^u d_u eta + a^v d_v eta."""
        bu = np.sum(a * self.du, axis=1)
        bv = np.sum(a * self.dv, axis=1)
        au = self.iuu * bu + self.iuv * bv
        av = self.iuv * bu + self.ivv * bv
        return (self.d_du(self.J * au) + self.d_dv(self.J * av)) / self.J
