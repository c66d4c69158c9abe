"""CPU checks of the library's N-Mueller plan tables against the oracle."""
import math

import numpy as np
import pytest

import synth
from oracle import singular, surface

B = pytest.importorskip("paper_2408_02274_amd.binding")


@pytest.mark.parametrize("geom", ["sphere", "ellipsoid"])
def test_surface_and_corrections_equal_oracle(geom):
    s = synth.cube_sphere(1, 6, 1.0) if geom == "sphere" else synth.ellipsoid(1.0, 0.7, 1.3, 1, 6)
    surf = surface.PatchSurface(s.P, s.nc, s.x, s.du, s.dv)
    nm = B.NMullerOperator(s, 1.0, 2.25, tol=1e-3, host_only=1)
    try:
        for which, ref in [(0, surf.n), (1, surf.w), (2, surf.t1), (3, surf.t2), (4, surf.J)]:
            assert np.array_equal(nm.geometry(which), ref)
        ro, pp, vals = nm.corrections()
        C = singular.corrections(surf, (3 * math.pi, 2 * math.pi))
        tl, pl = C["pairs"]
        lib_pairs = np.stack([np.repeat(np.arange(surf.N), np.diff(ro)), pp])
        assert np.array_equal(lib_pairs, np.stack([tl, pl]))
        nq = s.nc * s.nc
        for k, key in enumerate([("S", 0), ("S", 1), ("D", 0), ("D", 1)]):
            Do = C[key].toarray()
            Dl = np.zeros_like(Do)
            for e, (l, p) in enumerate(zip(lib_pairs[0], lib_pairs[1])):
                Dl[l, p * nq:(p + 1) * nq] += vals[e, k]
            scale = np.max(np.abs(Do))
            # S: rounding only.  D: the n.(x - y) cancellation next to the
            # singular point makes FP64 results order-dependent at ~1e-8.
            tol = 1e-11 if key[0] == "S" else 1e-7
            assert np.max(np.abs(Dl - Do)) < tol * scale, key
    finally:
        nm.close()
