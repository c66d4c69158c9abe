"""The plan tables built by kernels on the device (Sec. III-G algorithm step
1: Morton order, boxes, neighbours and cousins, relevant cones of eq.
rele_cone, cousin-pair and parent-point cone slots, propagation groups and
tiles) against the host builder and the oracle.

Bar: integer tables bit for bit.  Every decision is taken with the same
formula and operation order, using only +, -, *, /, sqrt and floor against
host-computed tables of the cone boundary directions and of the
interpolation nodes' sines and cosines, so ties (the cube-sphere puts points
exactly on cone boundaries) break the same way.  The sums of plans built
either way agree to 1e-12 (FP64; the propagation's LDS accumulation order is
the only difference between runs).
"""
import math
import time

import numpy as np
import pytest

import synth
from oracle import ifgf_ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


CASES = {
    "sphere_c1": lambda: (synth.cube_sphere(2, 8), (3 * math.pi, 2 * math.pi)),
    "ellipsoid": lambda: (synth.ellipsoid(1.0, 0.6, 1.4, 2, 6), (2 * math.pi * 1.5, 2 * math.pi)),
    "rounded_box": lambda: (synth.rounded_box((3.0, 0.5, 0.25), 0.1, 0.3, 4), (2 * math.pi * 3.48, 2 * math.pi * 1.45)),
}


def _cloud():
    rng = np.random.default_rng(11)
    x = rng.uniform(-1, 1, (900, 3))
    n = np.tile([1.0, 0.0, 0.0], (900, 1))
    return x, n, (7.0, 5.0)


def _geometry(case):
    if case == "cloud":
        return _cloud()
    s, ks = CASES[case]()
    return s.x, s.normal, ks


@pytest.mark.parametrize("case", sorted(CASES) + ["cloud"])
@pytest.mark.parametrize("order", [(3, 5, 1), (4, 6, 1), (5, 5, 0)])
def test_device_plan_tables_equal_host_builder(case, order):
    from paper_2408_02274_amd import binding as B
    x, n, ks = _geometry(case)
    Ps, Pa, rr = order
    _say(f"[gpu] device plan vs host plan: {case}, n = {len(x)}, orders ({Ps}, {Pa}), refine_radial {rr}")
    kw = dict(Ps=Ps, Pa=Pa, refine_radial=rr)
    h = B.ifgf_plan(x, n, np.ones(len(x)), ks[0], ks[1], 1e-3, host_only=1, plan_on_device=0, **kw)
    g = B.ifgf_plan(x, n, np.ones(len(x)), ks[0], ks[1], 1e-3, plan_on_device=1, keep_pair_tables=1, **kw)
    try:
        ch, cg = B.ifgf_plan_counts(h), B.ifgf_plan_counts(g)
        assert ch == cg
        D = ch[1]
        assert np.array_equal(B.ifgf_plan_table(h, 0), B.ifgf_plan_table(g, 0))
        for d in range(3, D + 1):
            assert np.array_equal(B.ifgf_plan_table(h, 1000 + d), B.ifgf_plan_table(g, 1000 + d)), d
            assert np.array_equal(B.ifgf_plan_table(h, 2000 + d), B.ifgf_plan_table(g, 2000 + d)), d
            if d < D:
                assert np.array_equal(B.ifgf_plan_table(h, 3000 + d), B.ifgf_plan_table(g, 3000 + d)), d
        sh, sg = B.ifgf_stats(h), B.ifgf_stats(g)
        for Lh, Lg in zip(sh["levels"], sg["levels"]):
            for k in ("boxes", "ns", "na", "slots", "prop_groups", "prop_tiles"):
                assert Lh[k] == Lg[k], (Lh["d"], k)
        if order == (3, 5, 1) and case != "rounded_box":
            t = ifgf_ref.Tree(x, ks, ifgf_ref.Params(Ps=Ps, Pa=Pa, refine_radial=bool(rr)))
            assert np.array_equal(B.ifgf_plan_table(g, 0), t.perm)
            for d in range(3, t.D + 1):
                assert np.array_equal(B.ifgf_plan_table(g, 1000 + d), t.levels[d].slot_key)
    finally:
        B.ifgf_destroy(h)
        B.ifgf_destroy(g)


@pytest.mark.parametrize("prec", [0, 1])
def test_device_planned_sums_equal_host_planned(prec):
    from paper_2408_02274_amd import IFGFPlan
    s, ks = CASES["sphere_c1"]()
    w = np.random.default_rng(3).uniform(0.5, 1.5, s.n)
    phi = torch.from_numpy(synth.complex_normal((1, 8, s.n), 4)).to("cuda")
    _say(f"[gpu] sums of device- and host-planned plans, precision {prec}")
    out = []
    for on_dev in (0, 1):
        plan = IFGFPlan(s.x, s.normal, w, ks[0], ks[1], 1e-4, precision=prec, plan_on_device=on_dev)
        out.append(plan.apply(phi).cpu().numpy())
        plan.close()
    rel = float(np.linalg.norm(out[1] - out[0]) / np.linalg.norm(out[0]))
    assert rel < (1e-12 if prec == 0 else 1e-6)


def test_device_plan_of_the_benchmark_sphere():
    """The 153,600-point sphere (radius 5, D = 7, up to 2^18 cones per box at
    level 3): counts, permutation and relevant-cone tables equal the host
    builder's; plan times printed."""
    from paper_2408_02274_amd import binding as B
    s = synth.cube_sphere(16, 10, 5.0)
    ks = (3 * math.pi, 2 * math.pi)
    w = np.ones(s.n)
    t0 = time.perf_counter()
    h = B.ifgf_plan(s.x, s.normal, w, ks[0], ks[1], 1e-4, host_only=1, plan_on_device=0)
    t1 = time.perf_counter()
    g = B.ifgf_plan(s.x, s.normal, w, ks[0], ks[1], 1e-4, plan_on_device=1, precision=1, fp32_workspaces=1)
    t2 = time.perf_counter()
    _say(f"[gpu] benchmark sphere plan: host tables {t1 - t0:.1f} s, device tables + upload {t2 - t1:.1f} s")
    try:
        assert B.ifgf_plan_counts(h) == B.ifgf_plan_counts(g)
        assert np.array_equal(B.ifgf_plan_table(h, 0), B.ifgf_plan_table(g, 0))
        D = B.ifgf_plan_counts(h)[1]
        for d in range(3, D + 1):
            assert np.array_equal(B.ifgf_plan_table(h, 1000 + d), B.ifgf_plan_table(g, 1000 + d)), d
        sh, sg = B.ifgf_stats(h), B.ifgf_stats(g)
        for Lh, Lg in zip(sh["levels"], sg["levels"]):
            assert (Lh["prop_groups"], Lh["prop_tiles"]) == (Lg["prop_groups"], Lg["prop_tiles"])
    finally:
        B.ifgf_destroy(h)
        B.ifgf_destroy(g)
