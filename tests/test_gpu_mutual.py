"""GPU parity of the mutual (symmetric) walk of Sec. 7 against the oracle.

Bar: far lists (sinks of every level) and near lists identical as sets per
sink; FP64 accelerations within 1e-12 of the oracle's mutual FMM (M2L, L2L
down the tree, L2P, near field); |sum F| / sum |F| at round-off (every cell
pair acts in both directions, so the total force cancels); bitwise
reproducible although the pairs are appended in a run-dependent order."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_01496_amd import fmm as F
from paper_2502_01496_amd import workloads as W
from tests.gpu_util import eta, force_err, gpu_run, gpu_vjp, say, to_dev
from tests.test_gpu_parity import _case, sorted_by_sink

pytestmark = pytest.mark.gpu

CASES = ["tiny_1", "tiny_7", "tiny_9", "plummer_4096", "plummer_5000_leaf3",
         "plummer_3001_leaf10_theta1", "plummer_777_leaf1", "ties_3000", "theta0_2048",
         "binary_2x4096_theta0.3", "binary_2x8192", "clumpy_20000_lognormal",
         "plummer_100003_ragged"]


def _stats_ratio(x, m, a):
    X, Mt, A = to_dev(x, m, a)
    return F.fmm_momentum_stats(X, None, Mt, A)["ratio"]


def _check_lists(ex, lists):
    for off_k, src_k, ref_off, ref_src in (("far_off", "far_src", lists.far_off, lists.far_src),
                                           ("near_off", "near_src", lists.near_off,
                                            lists.near_src)):
        np.testing.assert_array_equal(ex[off_k], ref_off)
        np.testing.assert_array_equal(sorted_by_sink(ex[off_k], ex[src_k]),
                                      sorted_by_sink(ref_off, ref_src))


@pytest.mark.parametrize("name", CASES)
def test_mutual_fp64_parity(orc, name):
    x, m, h, theta, leaf = _case(name)
    say(f"[gpu mutual] case={name} n={len(m)} theta={theta} leaf={leaf}")
    a, ex, info = gpu_run(x, m, h, theta=theta, leaf=leaf, walk=F.FMM_WALK_MUTUAL, local=True)
    ref = orc.fmm(x, m, h, theta=theta, leaf_size=leaf, policy=O.MUTUAL)
    _check_lists(ex, ref.lists)
    assert info["sinks"] == ref.tree.nnodes
    # local expansions of the leaves after L2L (scale: the largest |L| of each order)
    leaves = ref.tree.left < 0
    for lo, hi in ((0, 3), (3, 9), (9, 19)):
        got, want = ex["local"][leaves, lo:hi], ref.L[leaves, lo:hi]
        scale = max(np.abs(want).max(), 1e-300)
        assert np.abs(got - want).max() <= 1e-12 * scale
    err = force_err(a, ref.a)
    ratio = _stats_ratio(x, m, a)
    say(f"    max rel force error vs oracle mutual FMM: {err:.3e}; |sumF|/sum|F| = {ratio:.3e}")
    assert err <= 1e-12
    if len(m) > 1:
        assert ratio <= 1e-13
    else:
        assert (a == 0).all()  # a lone particle feels no force (the ratio is 0/0)


def test_mutual_conserves_where_leaf_walk_does_not(orc):
    x, m, h = W.polytrope_binary(8192, 2, cache=False)
    say("[gpu mutual] momentum: leaf<-cell vs mutual, binary_2x8192")
    a_p, _, _ = gpu_run(x, m, h, export=False)
    a_m, _, _ = gpu_run(x, m, h, export=False, walk=F.FMM_WALK_MUTUAL)
    r_p, r_m = _stats_ratio(x, m, a_p), _stats_ratio(x, m, a_m)
    d = orc.direct_sinks(x, m, h, np.arange(0, len(m), 37))
    e_m = eta(a_m[::37], d)
    say(f"    ratio leaf<-cell {r_p:.3e}, mutual {r_m:.3e}; mutual eta vs direct {e_m:.3e}")
    assert r_p > 1e-8 and r_m < 1e-13
    assert e_m < 1e-2


def test_mutual_fp32(orc):
    x, m, h = W.polytrope_binary(8192, 2, cache=False)
    say("[gpu mutual] FP32 form, binary_2x8192")
    a, _, _ = gpu_run(x, m, h, precision=F.FMM_FP32, export=False, walk=F.FMM_WALK_MUTUAL)
    ref = orc.fmm(x, m, h, policy=O.MUTUAL)
    e = eta(a, ref.a)
    ratio = _stats_ratio(x, m, a)
    say(f"    eta vs FP64 oracle mutual FMM {e:.3e}; |sumF|/sum|F| = {ratio:.3e}")
    assert e <= 1e-5
    assert ratio <= 1e-6


def test_mutual_deterministic():
    x, m, h = W.clumpy_cube(20000, 3, cache=False)
    say("[gpu mutual] determinism, clumpy_20000, two runs")
    a1, _, _ = gpu_run(x, m, h, export=False, walk=F.FMM_WALK_MUTUAL)
    a2, _, _ = gpu_run(x, m, h, export=False, walk=F.FMM_WALK_MUTUAL)
    assert np.array_equal(a1, a2)


def test_mutual_lists_ascending(orc):
    # every far and near list holds distinct source ids in ascending order
    x, m, h = W.clumpy_cube(20000, 3, cache=False)
    say("[gpu mutual] list order, clumpy_20000")
    _, ex, _ = gpu_run(x, m, h, walk=F.FMM_WALK_MUTUAL)
    for off, src in (("far_off", "far_src"), ("near_off", "near_src")):
        o, sv = ex[off], ex[src]
        for v in range(len(o) - 1):
            seg = sv[o[v]:o[v + 1]]
            assert (np.diff(seg) > 0).all(), (off, v)


def test_mutual_buffer_regrowth(orc, monkeypatch):
    # first capacities of 256 entries: frontier, far and near buffers all
    # overflow and are grown over several walks; the lists must not change
    monkeypatch.setenv("FMM_MI355_MW_CAP", "256")
    x, m, h = W.plummer(4096, 1)
    say("[gpu mutual] buffer regrowth, plummer_4096, first capacity 256")
    a, ex, _ = gpu_run(x, m, h, walk=F.FMM_WALK_MUTUAL)
    ref = orc.fmm(x, m, h, policy=O.MUTUAL)
    _check_lists(ex, ref.lists)
    assert force_err(a, ref.a) <= 1e-12


def test_policy_switch_on_one_tree(orc):
    import torch

    x, m, h = W.plummer(4096, 1)
    say("[gpu mutual] leaf<-cell -> mutual -> leaf<-cell -> mutual on one tree, with VJPs")
    X, Mt, H = to_dev(x, m, h)
    A = torch.empty((len(m), 3), dtype=torch.float64, device="cuda")
    AB = torch.from_numpy(W.cotangent(len(m), 38)).to("cuda")
    XB = torch.empty_like(A)
    MB = torch.empty_like(Mt)
    t = F.fmm_build_tree(X, F.default_params())
    walks = (F.FMM_WALK_PHANTOM, F.FMM_WALK_MUTUAL, F.FMM_WALK_PHANTOM, F.FMM_WALK_MUTUAL)
    try:
        out, vjp = [], []
        for walk in walks:
            t = F.fmm_build_tree(X, F.default_params(walk=walk), tree=t)
            F.fmm_moments(t, X, Mt, H)
            F.fmm_forces(t, A)
            F.fmm_forces_vjp(t, AB, XB, MB)
            torch.cuda.synchronize()
            out.append(A.cpu().numpy().copy())
            vjp.append((XB.cpu().numpy().copy(), MB.cpu().numpy().copy()))
        # frozen lists: forces again without a walk
        F.fmm_forces(t, A)
        torch.cuda.synchronize()
        out.append(A.cpu().numpy().copy())
    finally:
        F.fmm_tree_free(t)
    ref_p = orc.fmm(x, m, h).a
    ref_m = orc.fmm(x, m, h, policy=O.MUTUAL).a
    assert force_err(out[0], ref_p) <= 1e-12
    assert force_err(out[1], ref_m) <= 1e-12
    assert np.array_equal(out[0], out[2]) and np.array_equal(out[1], out[3])
    assert np.array_equal(out[3], out[4])
    # the reverse pass on a reused tree equals that on a fresh one, per walk
    for k, walk in enumerate(walks):
        _, [(xf, mf)] = gpu_vjp(x, m, h, W.cotangent(len(m), 38), walk=walk)
        assert np.array_equal(vjp[k][0], xf) and np.array_equal(vjp[k][1], mf)
