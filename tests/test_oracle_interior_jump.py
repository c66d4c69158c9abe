"""The oracle's interior field (reading A15) against its on-surface operator
through the jump relations, just inside Gamma.

For a tangential density a, n x curl S_k[a] tends to K_k[a] - a/2 from the
interior (the principal-value K of eq. n_muller and its jump).  interior_field
evaluates E_i = -omega mu_i curl S_i[m] (j = 0) and H_i = -omega eps_i
curl S_i[j] (m = 0) by plain quadrature at points x - h n; their limits as
h -> 0 (polynomial extrapolation from h = 0.08 .. 0.28, where the plain
quadrature is accurate) must match the on-surface K_i computed with the
singular corrections.  The opposite jump (K + a/2) is far off, so a sign or
factor error in either piece fails.  Unit sphere, 3 x 3 patches per face of
12 x 12 nodes, k_i = 3 pi; rows of one patch.
"""
import math

import numpy as np

import synth
from oracle import nmuller, surface


def _limits():
    s = synth.cube_sphere(3, 12, 1.0)
    surf = surface.PatchSurface(s.P, s.nc, s.x, s.du, s.dv)
    nm = nmuller.NMuller(surf, 1.0, 2.25, patches=[5])
    c = np.array([0.3, -0.5, 0.8])
    d = np.array([0.2, 0.1, -0.4])
    a = c[None, :] - surf.n * (surf.n @ c)[:, None]
    a = a * np.exp(1j * (surf.x @ d))[:, None]
    at = np.stack([np.sum(a * surf.t1, 1), np.sum(a * surf.t2, 1)])
    zero = np.zeros_like(at)
    rows = nm.rows[[0, 17, 40, 77, 100, 143]]
    hs = np.array([0.08, 0.12, 0.16, 0.2, 0.24, 0.28])
    out = []
    for which in ("m", "j"):
        y = np.concatenate([at, zero]) if which == "m" else np.concatenate([zero, at])
        phi = nm.densities(y)
        SD = nm.layer_sums(phi)
        K, _, _ = nm._KRT(SD, 0, 0, 6) if which == "m" else nm._KRT(SD, 0, 3, 7)
        vals = []
        for h in hs:
            X = surf.x[rows] - h * surf.n[rows]
            E, H = nmuller.interior_field(nm, y, X)
            F = E / (-nm.omega * nm.mu_i) if which == "m" else H / (-nm.omega * nm.eps_i)
            vals.append(np.cross(surf.n[rows], F))
        vals = np.array(vals)
        coef = np.linalg.lstsq(np.vander(hs, 5), vals.reshape(len(hs), -1), rcond=None)[0]
        lim = coef[-1].reshape(len(rows), 3)
        out.append((lim, K[rows], a[rows]))
    return out


def test_interior_field_limits_on_gamma_follow_the_jump_relations():
    for lim, K, a in _limits():
        want = K - 0.5 * a
        err = np.linalg.norm(lim - want) / np.linalg.norm(want)
        wrong = np.linalg.norm(lim - (K + 0.5 * a)) / np.linalg.norm(want)
        print(f"interior limit vs K - a/2: {err:.3e}; vs K + a/2: {wrong:.3e}")
        assert err < 0.1
        assert wrong > 0.5
