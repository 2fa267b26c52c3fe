"""GPU parity: tree, cell records, interaction lists and FP64 forces of the HIP
path against the CPU oracle on the same seeded inputs.

Bar: permutation, split axes, node masses, centres of mass, sizes s and h_max
bit-identical; quadrupoles within 1e-14 of M s^2; far and near lists identical
(the same cells for every sink); FP64 accelerations within 1e-12 of the oracle's
FMM (max_i |da_i| / max(|a_i|, 1e-3 rms|a|)); momentum statistics within
1e-12 of sum|F|."""
import numpy as np
import pytest

from paper_2502_01496_amd import workloads as W
from paper_2502_01496_amd import fmm as F
from tests.gpu_util import force_err, gpu_run, say, to_dev

pytestmark = pytest.mark.gpu


def sorted_by_sink(off, src):
    seg = np.repeat(np.arange(len(off) - 1), np.diff(off))
    return src[np.lexsort((src, seg))]


def _grid_ties(n, seed, grid=8):
    rng = np.random.default_rng(seed)
    x = np.round(rng.random((n, 3)) * grid) / grid      # many tied coordinates
    x += 1e-9 * rng.standard_normal((n, 3)) * (rng.random((n, 1)) < 0.5)
    return x, np.full(n, 1.0 / n), np.full(n, 0.02)


def _case(name):
    if name == "plummer_4096":
        x, m, h = W.plummer(4096, 1)
        return x, m, h, 0.5, 8
    if name == "plummer_65536":
        x, m, h = W.plummer(65536, 11)
        return x, m, h, 0.5, 8
    if name == "plummer_100003_ragged":
        x, m, h = W.plummer(100003, 12)
        return x, m, h, 0.5, 8
    if name == "binary_2x8192":
        x, m, h = W.polytrope_binary(8192, 2, cache=False)
        return x, m, h, 0.5, 8
    if name == "binary_2x4096_theta0.3":
        x, m, h = W.polytrope_binary(4096, 2, cache=False)
        return x, m, h, 0.3, 8
    if name == "binary_2x4096_theta0.7":
        x, m, h = W.polytrope_binary(4096, 2, cache=False)
        return x, m, h, 0.7, 8
    if name == "clumpy_20000_lognormal":
        x, m, h = W.clumpy_cube(20000, 3, cache=False)
        return x, m, h, 0.5, 8
    if name == "plummer_5000_leaf3":
        x, m, h = W.plummer(5000, 4)
        return x, m, h, 0.5, 3
    if name == "plummer_3001_leaf10_theta1":
        x, m, h = W.plummer(3001, 5)
        return x, m, h, 1.0, 10
    if name == "plummer_777_leaf1":
        x, m, h = W.plummer(777, 6)
        return x, m, h, 0.6, 1
    if name == "ties_3000":
        x, m, h = _grid_ties(3000, 7)
        return x, m, h, 0.5, 8
    if name == "ties_short_20000":
        # about ten particles per grid value of each axis: runs of equal high
        # key halves of a few entries, across the sort's block and tile edges
        x, m, h = _grid_ties(20000, 13, grid=2048)
        return x, m, h, 0.5, 8
    if name == "tiny_1":
        return np.array([[0.1, 0.2, 0.3]]), np.array([2.0]), np.array([0.1]), 0.5, 8
    if name == "tiny_7":
        x, m, h = W.plummer(7, 8)
        return x, m, h, 0.5, 8
    if name == "tiny_9":
        x, m, h = W.plummer(9, 9)
        return x, m, h, 0.5, 8
    if name == "theta0_2048":
        x, m, h = W.plummer(2048, 10)
        return x, m, h, 0.0, 8
    raise KeyError(name)


CASES = ["tiny_1", "tiny_7", "tiny_9", "plummer_4096", "plummer_5000_leaf3",
         "plummer_3001_leaf10_theta1", "plummer_777_leaf1", "ties_3000", "ties_short_20000",
         "theta0_2048",
         "binary_2x4096_theta0.3", "binary_2x4096_theta0.7", "binary_2x8192",
         "clumpy_20000_lognormal", "plummer_65536", "plummer_100003_ragged"]


@pytest.mark.parametrize("name", CASES)
def test_fp64_parity(orc, name):
    x, m, h, theta, leaf = _case(name)
    say(f"[gpu parity] case={name} n={len(m)} theta={theta} leaf={leaf}")
    a, ex, info = gpu_run(x, m, h, theta=theta, leaf=leaf)
    ref = orc.fmm(x, m, h, theta=theta, leaf_size=leaf)
    t, mom, lists = ref.tree, ref.mom, ref.lists
    # tree
    assert info["nodes"] == t.nnodes
    np.testing.assert_array_equal(ex["first"], t.first)
    np.testing.assert_array_equal(ex["count"], t.count)
    np.testing.assert_array_equal(ex["left"], t.left)
    np.testing.assert_array_equal(ex["right"], t.right)
    np.testing.assert_array_equal(ex["perm"], t.perm)
    np.testing.assert_array_equal(ex["axis"], t.axis)
    # cell records: bit-identical M, c, s, h_max
    rec = ex["rec"]
    np.testing.assert_array_equal(rec[:, 0], mom.M)
    np.testing.assert_array_equal(rec[:, 1:4], mom.c)
    np.testing.assert_array_equal(rec[:, 4], mom.s)
    np.testing.assert_array_equal(rec[:, 5], mom.hmax)
    scale = (mom.M * mom.s ** 2)[:, None]
    assert (np.abs(rec[:, 6:12] - mom.Q) <= 1e-14 * scale + 1e-300).all()
    # interaction lists: the same set of cells for every sink (the order in
    # which a list is emitted is free)
    for off_k, src_k, ref_off, ref_src in (("far_off", "far_src", lists.far_off, lists.far_src),
                                           ("near_off", "near_src", lists.near_off,
                                            lists.near_src)):
        np.testing.assert_array_equal(ex[off_k], ref_off)
        np.testing.assert_array_equal(sorted_by_sink(ex[off_k], ex[src_k]),
                                      sorted_by_sink(ref_off, ref_src))
    # forces
    err = force_err(a, ref.a)
    say(f"    max rel force error vs oracle FMM: {err:.3e}")
    assert err <= 1e-12


def test_stats_parity(orc):
    import torch

    from paper_2502_01496_amd import fmm as F
    from tests.gpu_util import to_dev

    x, m, h = W.plummer(4096, 1)
    say("[gpu parity] momentum stats, plummer_4096")
    a, _, _ = gpu_run(x, m, h, export=False)
    v = W.cotangent(4096, 21) * 0.1
    X, V, Mt, A = to_dev(x, v, m, a)
    st = F.fmm_momentum_stats(X, V, Mt, A)
    ref = orc.stats(x, v, m, a)
    assert np.abs(st["sumF"] - ref["sumF"]).max() <= 1e-12 * ref["sumAbsF"]
    assert st["sumAbsF"] == pytest.approx(ref["sumAbsF"], rel=1e-13)
    assert st["mass"] == pytest.approx(ref["mass"], rel=1e-14)
    np.testing.assert_allclose(st["xcom"], ref["xcom"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(st["P"], ref["P"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(st["L"], ref["L"], rtol=0, atol=1e-13)
    # float accelerations are accumulated in FP64 too
    st32 = F.fmm_momentum_stats(X, None, Mt, A.float())
    ref32 = orc.stats(x, None, m, a.astype(np.float32).astype(np.float64))
    assert np.abs(st32["sumF"] - ref32["sumF"]).max() <= 1e-12 * ref32["sumAbsF"]
    assert (st32["P"] == 0).all()


def test_deterministic(orc):
    x, m, h = W.polytrope_binary(8192, 2, cache=False)
    say("[gpu parity] determinism, binary_2x8192, two runs")
    a1, _, _ = gpu_run(x, m, h, export=False)
    a2, _, _ = gpu_run(x, m, h, export=False)
    assert np.array_equal(a1, a2)


def _check_lists_and_forces(orc, x, m, h, theta, leaf):
    a, ex, info = gpu_run(x, m, h, theta=theta, leaf=leaf)
    ref = orc.fmm(x, m, h, theta=theta, leaf_size=leaf)
    lists = ref.lists
    for off_k, src_k, ref_off, ref_src in (("far_off", "far_src", lists.far_off, lists.far_src),
                                           ("near_off", "near_src", lists.near_off,
                                            lists.near_src)):
        np.testing.assert_array_equal(ex[off_k], ref_off)
        np.testing.assert_array_equal(sorted_by_sink(ex[off_k], ex[src_k]),
                                      sorted_by_sink(ref_off, ref_src))
    assert force_err(a, ref.a) <= 1e-12
    return ex


def test_list_slots_regrow(orc):
    # theta = 0.3 on 2 x 16384 gives far lists longer than the initial slots
    x, m, h = W.polytrope_binary(16384, 2, cache=False)
    say("[gpu parity] list slot regrowth, binary_2x16384 theta=0.3")
    ex = _check_lists_and_forces(orc, x, m, h, 0.3, 8)
    assert np.diff(ex["far_off"]).max() > 512


def test_narrow_stack_fallback(orc, monkeypatch):
    # a tiny stack limit for the wide walk: most leaves are redone by the
    # exact narrow-stack walk, and the lists must not change
    monkeypatch.setenv("FMM_MI355_WIDE_STACK", "8")
    x, m, h = W.plummer(20000, 13)
    say("[gpu parity] narrow-stack walk fallback, plummer_20000")
    _check_lists_and_forces(orc, x, m, h, 0.5, 8)


@pytest.mark.parametrize("budget", [1, 3])
@pytest.mark.parametrize("name", ["plummer_4096", "plummer_777_leaf1", "theta0_2048",
                                  "plummer_3001_leaf10_theta1", "plummer_100003_ragged"])
def test_workgroup_walk(orc, monkeypatch, name, budget):
    # a step budget of 1 sends every leaf group to the workgroup walk, 3 only
    # some of them: the lists are the oracle's, and the forces too
    monkeypatch.setenv("FMM_MI355_WALK_BUDGET", str(budget))
    test_fp64_parity(orc, name)


def test_workgroup_walk_deterministic(monkeypatch):
    monkeypatch.setenv("FMM_MI355_WALK_BUDGET", "2")
    x, m, h = W.plummer(50000, 14)
    say("[gpu parity] workgroup walk determinism, plummer_50000, two runs")
    a1, _, _ = gpu_run(x, m, h, export=False)
    a2, _, _ = gpu_run(x, m, h, export=False)
    assert np.array_equal(a1, a2)


def test_workgroup_walk_stack_fallback(orc, monkeypatch):
    # the workgroup walk's own stack overflow sends its leaves to the narrow
    # walk (a wide stack of 8 entries overflows on the first pushes)
    monkeypatch.setenv("FMM_MI355_WALK_BUDGET", "1")
    monkeypatch.setenv("FMM_MI355_WIDE_STACK", "8")
    x, m, h = W.plummer(20000, 13)
    say("[gpu parity] workgroup walk + narrow-stack fallback, plummer_20000")
    _check_lists_and_forces(orc, x, m, h, 0.5, 8)


@pytest.mark.parametrize("name", ["plummer_4096", "ties_3000", "ties_short_20000",
                                  "clumpy_20000_lognormal", "plummer_100003_ragged"])
def test_full_key_morton_sort(orc, monkeypatch, name):
    # the Morton order by all eight key digits (used once a tree has met
    # concentrated data) gives the same (key, position) order as the sort by
    # halves: tree, records, lists and forces as in the parity test
    monkeypatch.setenv("FMM_MI355_MORTON_FULL", "1")
    test_fp64_parity(orc, name)


def test_morton_sort_switch_keeps_the_tree():
    # a Plummer sphere whose halo sets the bounding box: most Morton keys of
    # the core share their high half, the first forces call switches the
    # tree to the full-key sort, and the rebuilt tree is the same
    import torch

    x, m, h = W.plummer(1 << 18, 21)
    say("[gpu parity] Morton sort switch on concentrated data, plummer_2^18")
    X, Mt, H = to_dev(x, m, h)
    A = torch.empty((len(m), 3), dtype=torch.float64, device="cuda")
    t = F.fmm_build_tree(X, F.default_params())
    try:
        exs = []
        for _ in range(2):
            t = F.fmm_build_tree(X, F.default_params(), tree=t)
            F.fmm_moments(t, X, Mt, H)
            F.fmm_forces(t, A, F.FMM_REWALK)
            torch.cuda.synchronize()
            exs.append(F.fmm_debug_export(t, lists=False))
    finally:
        F.fmm_tree_free(t)
    for k in ("perm", "first", "count", "left", "right", "axis"):
        assert np.array_equal(exs[0][k], exs[1][k]), k


@pytest.mark.parametrize("bad", ["nan_position", "zero_mass", "negative_h"])
def test_bad_input_data_reported(orc, bad):
    # data errors are found on the device and reported by fmm_forces
    # (FMM_ERR_INVALID with the reason); the same tree then takes good data
    import torch

    x, m, h = W.plummer(4096, 1)
    xb, mb, hb = x.copy(), m.copy(), h.copy()
    if bad == "nan_position":
        xb[17, 1] = np.nan
        why = "non-finite positions"
    elif bad == "zero_mass":
        mb[100] = 0.0
        why = "masses not positive"
    else:
        hb[5] = -0.01
        why = "smoothing lengths not positive"
    say(f"[gpu parity] bad input reported: {bad}")
    A = torch.empty((len(m), 3), dtype=torch.float64, device="cuda")
    X, Mt, H = to_dev(xb, mb, hb)
    t = F.fmm_build_tree(X, F.default_params())
    try:
        F.fmm_moments(t, X, Mt, H)
        with pytest.raises(F.FmmError) as ei:
            F.fmm_forces(t, A)
        assert why in str(ei.value)
        X, Mt, H = to_dev(x, m, h)
        t = F.fmm_build_tree(X, F.default_params(), tree=t)
        F.fmm_moments(t, X, Mt, H)
        F.fmm_forces(t, A)
        torch.cuda.synchronize()
        a = A.cpu().numpy()
    finally:
        F.fmm_tree_free(t)
    assert force_err(a, orc.fmm(x, m, h).a) <= 1e-12

