"""nmuller_solve_noalloc (GMRES workspaces in the library's static device
scratch) against nmuller_solve (workspaces allocated per call), through the
C-ABI, on two calls in a row, the second on a smaller operator.

Bar: both run the same GMRES arithmetic; the only difference between runs
is the summation order of the FP64 propagation's LDS atomics, a ~1e-16
relative perturbation per product that the Krylov process carries into the
iterate at about the size of (iteration count) x 1e-16 / (residual
reduction); 1e-9 relative on y and equal iteration counts (within one) leave
ample room.  The second call reuses the array the first call filled, so
stale contents of the scratch would show here.
"""
import numpy as np
import pytest

import synth
from oracle import nmuller, surface

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _case(npf, nc):
    from paper_2408_02274_amd import NMullerOperator
    s = synth.cube_sphere(npf, nc, 1.0)
    surf = surface.PatchSurface(s.P, s.nc, s.x, s.du, s.dv)
    nm_o = nmuller.NMuller(surf, 1.0, 2.25, corrections={})    # geometry only
    E, H = nm_o.incident_plane_wave([0, 0, 1.0], [1.0, 0, 0])
    op = NMullerOperator(s, 1.0, 2.25, tol=1e-3, Ps=5, Pa=5)
    b = op.rhs(torch.from_numpy(E[None]).to("cuda"), torch.from_numpy(H[None]).to("cuda"))
    return op, b


@pytest.mark.parametrize("restart", [0, 20])
def test_noalloc_solve_matches_allocating_solve(restart):
    from paper_2408_02274_amd import binding as B
    for npf, nc in ((2, 8), (2, 6)):          # config-1 sphere (1,536 points), then 864 points
        _say(f"[gpu] nmuller_solve_noalloc sphere npf={npf} nc={nc} restart={restart}")
        op, b = _case(npf, nc)
        y_ref, info_ref = op.solve(b, rtol=1e-4, maxit=300, restart=restart)
        y = torch.full_like(b, complex(float("nan"), 0.0))
        info = B.nmuller_solve_noalloc(op.handle, b, y, False, 1e-4, 300, restart)
        torch.cuda.synchronize()
        yr, yn = y_ref.cpu().numpy(), y.cpu().numpy()
        op.close()
        _say(info_ref[0], info)
        assert info["converged"] and info["true_relres"] <= 1e-4
        assert abs(info["iters"] - info_ref[0]["iters"]) <= 1
        assert np.linalg.norm(yn - yr) <= 1e-9 * np.linalg.norm(yr)


def test_noalloc_rejects_workspace_beyond_scratch():
    from paper_2408_02274_amd import binding as B
    op, b = _case(2, 8)
    y = torch.empty_like(b)
    _say("[gpu] nmuller_solve_noalloc oversize basis")
    with pytest.raises(B.IFGFError) as ei:
        B.nmuller_solve_noalloc(op.handle, b, y, False, 1e-4, 5000, 0)   # basis of 5,000 x 6,144
    assert "static scratch" in str(ei.value)
    op.close()
