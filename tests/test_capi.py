"""CPU checks of the C-ABI: the library loads, exports every declared symbol,
validates arguments and builds host plan tables equal to the oracle's."""
import ctypes
import math

import numpy as np
import pytest

import synth

P = pytest.importorskip("paper_2408_02274_amd")
from paper_2408_02274_amd import binding  # noqa: E402
from oracle import ifgf_ref  # noqa: E402


def test_library_exports_every_declared_symbol():
    names = binding.exported_symbols()
    assert "ifgf_plan" in names and "ifgf_apply" in names
    L = binding.lib()
    for nm in names:
        assert hasattr(L, nm), nm
        assert ctypes.cast(getattr(L, nm), ctypes.c_void_p).value


@pytest.mark.parametrize("kw,msg", [
    (dict(k_int=-1.0), "wavenumbers"),
    (dict(tol=1.0), "tol"),
    (dict(weights_bad=True), "weight"),
    (dict(normal_bad=True), "unit"),
    (dict(dup=True), "duplicate"),
])
def test_plan_rejects_invalid_input(kw, msg):
    s = synth.cube_sphere(1, 4)
    x, n, w = s.x.copy(), s.normal.copy(), np.ones(s.n)
    if kw.get("weights_bad"):
        w[3] = 0.0
    if kw.get("normal_bad"):
        n[2] *= 1.1
    if kw.get("dup"):
        x[7] = x[5]
    with pytest.raises(binding.IFGFError, match=msg):
        binding.ifgf_plan(x, n, w, kw.get("k_int", 3.0), 2.0, kw.get("tol", 1e-3), host_only=1)


@pytest.mark.parametrize("case", ["sphere_c1", "ellipsoid", "cloud"])
def test_host_tables_equal_oracle(case):
    if case == "sphere_c1":
        s = synth.cube_sphere(2, 8)
        x, n, ks = s.x, s.normal, (3 * math.pi, 2 * math.pi)
    elif case == "ellipsoid":
        s = synth.ellipsoid(1.0, 0.6, 1.4, 2, 6)
        x, n, ks = s.x, s.normal, (2 * math.pi * 1.5, 2 * math.pi)
    else:
        rng = np.random.default_rng(11)
        x = rng.uniform(-1, 1, (900, 3))
        n = np.tile([1.0, 0.0, 0.0], (900, 1))
        ks = (7.0, 5.0)
    for Ps, Pa in [(3, 5), (5, 5)]:
        h = binding.ifgf_plan(x, n, np.ones(len(x)), ks[0], ks[1], 1e-3, Ps=Ps, Pa=Pa, host_only=1)
        try:
            t = ifgf_ref.Tree(x, ks, ifgf_ref.Params(Ps=Ps, Pa=Pa))
            assert np.array_equal(binding.ifgf_plan_table(h, 0), t.perm)
            c = binding.ifgf_plan_counts(h)
            assert c[1] == t.D
            oc = t.counts()
            assert c[4] == oc["near_pairs"]
            for i, d in enumerate(range(3, t.D + 1)):
                assert np.array_equal(binding.ifgf_plan_table(h, 1000 + d), t.levels[d].slot_key)
                assert c[7 + 4 * i + 1] == oc[f"target_pairs_{d}"]
                if d >= 4:
                    assert c[7 + 4 * i + 2] == oc[f"prop_pairs_{d}"]
        finally:
            binding.ifgf_destroy(h)


def test_host_only_plan_refuses_apply():
    s = synth.cube_sphere(1, 4)
    h = binding.ifgf_plan(s.x, s.normal, np.ones(s.n), 3.0, 2.0, 1e-3, host_only=1)
    L = binding.lib()
    rc = L.ifgf_apply(h, 1, 1, 1, None)
    assert rc == -4
    binding.ifgf_destroy(h)


def _oracle_target_slots_in_library_order(t, d):
    L = t.levels[d]
    tt, tb, slot, _ = t.tgt_pairs[d]
    key = tt * L.nb + tb
    order = np.argsort(key)
    ks, ss = key[order], slot[order]
    want = []
    for i in range(t.N):
        cs = L.cousins[L.box_of_point[i]]
        want.append(ss[np.searchsorted(ks, i * L.nb + cs)])
    return np.concatenate(want) if want else np.zeros(0, np.int64)


@pytest.mark.parametrize("case", ["sphere_c1", "ellipsoid"])
def test_pair_tables_equal_oracle(case):
    # every (target, cousin box) and (parent point, child box) pair must be
    # served by the same cone in the library plan as in the oracle
    if case == "sphere_c1":
        s, ks = synth.cube_sphere(2, 8), (3 * math.pi, 2 * math.pi)
    else:
        s, ks = synth.ellipsoid(1.0, 0.6, 1.4, 2, 6), (3 * math.pi, 2 * math.pi)
    h = binding.ifgf_plan(s.x, s.normal, np.ones(s.n), ks[0], ks[1], 1e-3, Ps=3, Pa=5, host_only=1)
    try:
        t = ifgf_ref.Tree(s.x, ks, ifgf_ref.Params(Ps=3, Pa=5))
        for d in range(3, t.D + 1):
            assert np.array_equal(binding.ifgf_plan_table(h, 2000 + d),
                                  _oracle_target_slots_in_library_order(t, d))
            if d >= 4:
                pslot, pk, cbox, cslot, pcone, pj = t.prop_pairs[d]
                Pl = t.levels[d - 1]
                npts = 75
                nch = Pl.child_end[Pl.slot_box] - Pl.child_start[Pl.slot_box]
                off = np.r_[0, np.cumsum(nch * npts)]
                want = np.empty(off[-1], dtype=np.int64)
                want[off[pslot] + pj * npts + pk] = cslot
                assert np.array_equal(binding.ifgf_plan_table(h, 3000 + d - 1), want)
    finally:
        binding.ifgf_destroy(h)


def test_binding_fails_loudly_without_the_library(tmp_path, monkeypatch):
    """No CPU fallback: a missing libifgf.so is an ImportError, not a
    silent switch to another implementation."""
    import paper_2408_02274_amd.binding as B
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "libifgf.so"))
    with pytest.raises(ImportError):
        B.lib()


def test_literal_radial_refinement_tables_equal_oracle():
    """refine_radial = 1 (both cone counts doubled per level, the literal
    rule of Remark 2): cone counts per level and relevant-cone tables equal
    the oracle's, and the radial count really grows."""
    s = synth.cube_sphere(2, 6)
    ks = (1.5 * math.pi, math.pi)
    h = binding.ifgf_plan(s.x, s.normal, np.ones(s.n), ks[0], ks[1], 1e-3, Ps=3, Pa=5,
                          refine_radial=1, host_only=1)
    try:
        t = ifgf_ref.Tree(s.x, ks, ifgf_ref.Params(Ps=3, Pa=5, refine_radial=True))
        c = binding.ifgf_plan_counts(h)
        assert c[1] == t.D
        grew = False
        for i, d in enumerate(range(3, t.D + 1)):
            nsna = c[7 + 4 * i + 3]
            assert (nsna >> 16, nsna & 0xFFFF) == (t.ns[d], t.na[d])
            grew |= t.ns[d] > 1
            assert np.array_equal(binding.ifgf_plan_table(h, 1000 + d), t.levels[d].slot_key)
        assert grew
    finally:
        binding.ifgf_destroy(h)


def test_plan_refuses_more_cones_per_box_than_32_bit_indices_hold():
    """Remark 2's doubling from level D up: a cloud 1,600 wavelengths across
    has D = 14 and 2^11 x 2^12 x 2^13 cones per box at level 3; cone indices
    are 32-bit, so the plan is refused before any table is built."""
    rng = np.random.default_rng(4)
    x = rng.uniform(-800.0, 800.0, (50, 3))
    n = np.tile([0.0, 0.0, 1.0], (50, 1))
    with pytest.raises(binding.IFGFError, match="2\\^31 cones"):
        binding.ifgf_plan(x, n, np.ones(50), 2 * math.pi, 2 * math.pi, 1e-3, host_only=1)


@pytest.mark.parametrize("orders", [(4, 6), (4, 5), (3, 5)])
def test_one_kernel_per_pass_halves_the_cone_buffers(orders):
    """Remark 3: the interpolation data of one kernel at a time take half the
    memory of both kernels' (up to the padding of a cone's k-steps to a
    multiple of 4 instead of 2), computed from the relevant cone counts
    before any device memory is touched."""
    s = synth.cube_sphere(2, 8)
    Ps, Pa = orders
    h = binding.ifgf_plan(s.x, s.normal, np.ones(s.n), 3 * math.pi, 2 * math.pi, 1e-3,
                          Ps=Ps, Pa=Pa, host_only=1, plan_on_device=0)
    try:
        st = binding.ifgf_stats(h)
        both, one = st["cone_buffer_bytes_by_mode"]
        D = st["D"]
        slots = [max([L["slots"] for L in st["levels"] if (D - L["d"]) % 2 == b] or [0]) for b in (0, 1)]
        nab = Ps * Pa
        ks = nab + ((Pa - 4) * nab + 3) // 4
        rows_both, rows_one = 4 * (ks + ks % 2), 4 * ((ks + 3) // 4 * 4)
        assert both == sum(8 * max(sl, 1) * rows_both * 32 for sl in slots)
        assert one == sum(8 * max(sl, 1) * rows_one * 16 for sl in slots)
        assert one * 2 * rows_both == both * rows_one
        assert st["kernels_per_pass"] == 0          # host-only plans hold no buffers
    finally:
        binding.ifgf_destroy(h)


@pytest.mark.parametrize("kw,msg", [(dict(kernel_at_a_time=2), "kernel_at_a_time"),
                                    (dict(cone_memory_budget=-1), "cone_memory_budget")])
def test_plan_rejects_bad_kernel_mode_options(kw, msg):
    s = synth.cube_sphere(1, 4)
    with pytest.raises(binding.IFGFError, match=msg):
        binding.ifgf_plan(s.x, s.normal, np.ones(s.n), 3.0, 2.0, 1e-3, host_only=1, **kw)
