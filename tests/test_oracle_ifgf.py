"""Pins for the reference IFGF (O2): bookkeeping, tables and accuracy."""
import math

import numpy as np
import pytest

import synth
from oracle import direct, ifgf_ref


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def small_case():
    s = synth.cube_sphere(2, 6, 1.0)                  # 864 points
    rng = np.random.default_rng(5)
    w = rng.uniform(0.5, 1.5, s.n)
    phi = synth.complex_normal((8, s.n), 6)
    ks = (1.5 * math.pi, 1.0 * math.pi)
    return s, w, phi, ks


def test_counting_kernel_counts_every_pair_once(small_case):
    # With G = 1 all factors are 1 and Chebyshev interpolation reproduces the
    # constant box sums exactly, so O2 must return sum_{m != l} a_m.
    s, w, phi, ks = small_case
    ref = ifgf_ref.ReferenceIFGF(s.x, s.normal, w, ks, ifgf_ref.Params(kernel="counting"))
    assert ref.tree.D >= 4
    out = ref.apply(phi)
    a = phi * w
    exact = a.sum(axis=1)[:, None] - a
    for q in range(2):
        assert np.max(np.abs(out[q, :8] - exact)) < 1e-12 * np.max(np.abs(exact))


def test_counting_kernel_volume_cloud():
    # points filling a cube (not a surface): more neighbours and cousins per box
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, (700, 3))
    n = np.tile([0.0, 0.0, 1.0], (700, 1))
    w = np.ones(700)
    phi = synth.complex_normal((8, 700), 8)
    ref = ifgf_ref.ReferenceIFGF(x, n, w, (6.0, 4.0), ifgf_ref.Params(kernel="counting"))
    assert ref.tree.D >= 4
    out = ref.apply(phi)
    exact = phi.sum(axis=1)[:, None] - phi
    assert np.max(np.abs(out[0, :8] - exact)) < 1e-11


def test_accuracy_against_direct_sum_improves_with_order(small_case):
    # cone rule of Remark 2 (radial and angular counts doubled): the S and D
    # errors fall by at least 5x from (3, 5) to (4, 6) to (5, 7); measured
    # 4.6e-5 / 4.4e-4, 2.9e-6 / 4.3e-5, 2.3e-7 / 6.5e-6
    s, w, phi, ks = small_case
    o1 = direct.regular_sums(s.x, s.normal, w, phi, ks)
    errs = {}
    for Ps, Pa in [(3, 5), (4, 6), (5, 7)]:
        o2 = ifgf_ref.ReferenceIFGF(s.x, s.normal, w, ks, ifgf_ref.Params(Ps=Ps, Pa=Pa)).apply(phi)
        errs[(Ps, Pa)] = (max(_rel(o2[q, :8], o1[q, :8]) for q in range(2)),
                          max(_rel(o2[q, 8:], o1[q, 8:]) for q in range(2)))
    assert errs[(3, 5)][0] < 1e-3 and errs[(3, 5)][1] < 1e-3
    assert errs[(4, 6)][0] < 1e-4 and errs[(4, 6)][1] < 1e-4
    assert errs[(5, 7)][0] < 1e-5 and errs[(5, 7)][1] < 1e-5
    for k in range(2):
        assert errs[(4, 6)][k] < errs[(3, 5)][k] / 5
        assert errs[(5, 7)][k] < errs[(4, 6)][k] / 5


def test_angular_only_cones_lose_radial_accuracy(small_case):
    # doubling only the angular cone count leaves the radial interpolation
    # coarser: worse single-layer sums than the rule as written at (5, 5)
    s, w, phi, ks = small_case
    o1 = direct.regular_sums(s.x, s.normal, w, phi, ks)
    e = {}
    for rr in (True, False):
        o2 = ifgf_ref.ReferenceIFGF(s.x, s.normal, w, ks,
                                    ifgf_ref.Params(Ps=3, Pa=5, refine_radial=rr)).apply(phi)
        e[rr] = max(_rel(o2[q, :8], o1[q, :8]) for q in range(2))
    assert e[True] < e[False] / 3


def test_fd_derivative_close_to_analytic(small_case):
    # the paper's forward difference (h = 1e-6) approaches the analytic derivative
    s, w, phi, ks = small_case
    pa = ifgf_ref.ReferenceIFGF(s.x, s.normal, w, ks, ifgf_ref.Params(Ps=5, Pa=5)).apply(phi)
    pf = ifgf_ref.ReferenceIFGF(s.x, s.normal, w, ks, ifgf_ref.Params(Ps=5, Pa=5, deriv="fd")).apply(phi)
    assert _rel(pf[:, :8], pa[:, :8]) < 1e-14
    assert _rel(pf[:, 8:], pa[:, 8:]) < 1e-4


def test_neighbours_and_cousins_brute_force(small_case):
    s, w, phi, ks = small_case
    t = ifgf_ref.Tree(s.x, ks)
    for d in range(1, t.D + 1):
        L = t.levels[d]
        C = L.coords
        for b in range(L.nb):
            cheb = np.max(np.abs(C - C[b]), axis=1)
            assert np.array_equal(np.flatnonzero(cheb <= 1), L.neighbours[b])
            if d >= 3:
                P = t.levels[d - 1]
                pc = P.coords[L.parent]                        # parent coords of every box
                par_nb = np.max(np.abs(pc - P.coords[L.parent[b]]), axis=1) <= 1
                expect = np.flatnonzero(par_nb & (cheb > 1))
                assert np.array_equal(expect, L.cousins[b])
    # level-1 box is relevant and every point is inside its leaf box (half-open)
    L = t.levels[t.D]
    lo = t.origin + L.H * L.coords[L.box_of_point]
    assert np.all(t.xs >= lo) and np.all(t.xs < lo + L.H)


def test_cone_partition_disjoint_and_covering():
    # random (s, theta, phi) in E plus the interval end points: the index
    # function picks the unique cone whose (half-open, last closed) intervals hold it
    rng = np.random.default_rng(3)
    ns, na = 2, 4
    eta = math.sqrt(3) / 3
    s = np.r_[rng.uniform(0, eta, 2000), 0.0, eta, eta / 2]
    th = np.r_[rng.uniform(0, math.pi, 2000), 0.0, math.pi, math.pi / 2]
    ph = np.r_[rng.uniform(0, 2 * math.pi, 2000), 0.0, 2 * math.pi - 1e-15, math.pi]
    h = 1.0
    r = h / np.maximum(s, 1e-100)
    dx, dy, dz = r * np.sin(th) * np.cos(ph), r * np.sin(th) * np.sin(ph), r * np.cos(th)
    cone, _, s2, th2, ph2 = ifgf_ref.cone_of(dx, dy, dz, h, ns, na)
    i_p = cone % (2 * na)
    i_t = (cone // (2 * na)) % na
    i_s = cone // (2 * na * na)
    assert np.all((0 <= i_s) & (i_s < ns) & (0 <= i_t) & (i_t < na) & (0 <= i_p) & (i_p < 2 * na))
    ds, da = eta / ns, math.pi / na
    tol = 1e-12
    assert np.all(s2 >= i_s * ds - tol) and np.all(s2 <= (i_s + 1) * ds + tol)
    assert np.all(th2 >= i_t * da - tol) and np.all(th2 <= (i_t + 1) * da + tol)
    assert np.all(ph2 >= i_p * da - tol) and np.all(ph2 <= (i_p + 1) * da + tol)


def test_relevant_cone_invariants(small_case):
    s, w, phi, ks = small_case
    t = ifgf_ref.Tree(s.x, ks)
    eta = math.sqrt(3) / 3
    for d in range(3, t.D + 1):
        L = t.levels[d]
        nc = t.ncones(d)
        tt, tb, slot, cone = t.tgt_pairs[d]
        # every cousin target lands in a relevant cone with s <= eta
        assert np.array_equal(L.slot_key[slot], tb * nc + cone)
        dl = t.xs[tt] - L.centers[tb]
        r = np.sqrt(np.sum(dl * dl, axis=1))
        assert np.all(L.h / r <= eta * (1 + 1e-12))
        if d >= 4:
            pslot, pk, cbox, cslot, pcone, pj = t.prop_pairs[d]
            assert np.array_equal(L.slot_key[cslot], cbox * nc + pcone)
            P = t.levels[d - 1]
            X = t.cone_points(d - 1, P.slot_box, P.slot_cone)[pslot, pk]
            rc = np.sqrt(np.sum((X - L.centers[cbox]) ** 2, axis=1))
            # parent interpolation points lie at s_child <= sqrt(3)/2 / (3 - sqrt(3)/2)
            assert np.all(L.h / rc <= (math.sqrt(3) / 2) / (3 - math.sqrt(3) / 2) + 1e-12)


def test_vectorised_sums_equal_single_density_runs(small_case):
    """IFGF_Vec (all 16 density x kernel columns through one cone structure,
    Sec. III-I) equals one run per density with the others zero (IFGF_Seq)."""
    s, w, phi, ks = small_case
    ref = ifgf_ref.ReferenceIFGF(s.x, s.normal, w, ks, ifgf_ref.Params())
    full = ref.apply(phi)
    for c in range(8):
        one = np.zeros_like(phi)
        one[c] = phi[c]
        out = ref.apply(one)
        scale = np.max(np.abs(full[:, c]))
        assert np.max(np.abs(out[:, c] - full[:, c])) < 1e-13 * scale
        if c < 6:
            assert np.max(np.abs(out[:, 8 + c] - full[:, 8 + c])) < 1e-13 * np.max(np.abs(full[:, 8 + c]))
        others = [k for k in range(8) if k != c]
        assert np.max(np.abs(out[:, others])) == 0.0
