"""Combinations of the options on the GPU against the oracle: tree shape x
expansion form x walk x precision, the VJP of the FP32 form with the second
expansion form, the census on a mutual walk over the centre-of-mass tree, and
the smallest trees.  Bars as in the single-option tests: FP64 forces within
1e-12 of the oracle's FMM of the same options, FP32 eta <= 1e-5, VJP within
1e-6 of central finite differences."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_01496_amd import fmm as F
from paper_2502_01496_amd import workloads as W
from tests.gpu_util import eta, force_err, gpu_run, gpu_vjp, say, to_dev
from tests.test_gpu_vjp import fd_check

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [F.FMM_TREE_MEDIAN, F.FMM_TREE_COM])
@pytest.mark.parametrize("form", [F.FMM_EXPANSION_PHANTOM, F.FMM_EXPANSION_DEHNEN])
@pytest.mark.parametrize("walk", [F.FMM_WALK_PHANTOM, F.FMM_WALK_MUTUAL])
def test_option_grid_fp64_and_fp32(orc, shape, form, walk):
    x, m, h = W.clumpy_cube(12000, 31, cache=False)
    leaf = 10 if shape == F.FMM_TREE_COM else 8
    say(f"[gpu combos] shape={shape} form={form} walk={walk} clumpy_12000")
    ref = orc.fmm(x, m, h, leaf_size=leaf, policy=walk, form=form, tree_kind=shape)
    a, _, _ = gpu_run(x, m, h, leaf=leaf, walk=walk, expansion=form, tree_shape=shape,
                      export=False)
    a32, _, _ = gpu_run(x, m, h, leaf=leaf, walk=walk, expansion=form, tree_shape=shape,
                        precision=F.FMM_FP32, export=False)
    err, e32 = force_err(a, ref.a), eta(a32, ref.a)
    say(f"    FP64 max rel err {err:.2e}; FP32 eta {e32:.2e}")
    assert err <= 1e-12
    assert e32 <= 1e-5


def test_fp32_form_vjp_with_second_expansion(orc):
    x, m, h = W.plummer(3000, 32)
    abar = W.cotangent(len(m), 36)
    say("[gpu combos] FP32-form VJP, second expansion form, plummer_3000")
    _, [(xb, mb)] = gpu_vjp(x, m, h, abar, precision=F.FMM_FP32,
                            expansion=F.FMM_EXPANSION_DEHNEN)
    worst = fd_check(orc, x, m, h, abar, xb, mb, 0.5, 8, form=O.DEHNEN_FORM)
    say(f"    worst directional error {worst:.2e}")
    assert worst <= 1e-5  # outputs rounded to FP32


@pytest.mark.parametrize("n,leaf", [(2, 1), (3, 1), (11, 10), (64, 1)])
def test_smallest_com_trees(orc, n, leaf):
    rng = np.random.default_rng(n)
    x = rng.random((n, 3))
    if n == 3:
        x[1] = x[0]  # two particles at one point
    m = rng.random(n) + 0.5
    h = np.full(n, 0.05)
    say(f"[gpu combos] centre-of-mass tree n={n} leaf={leaf}")
    for walk in (F.FMM_WALK_PHANTOM, F.FMM_WALK_MUTUAL):
        a, ex, _ = gpu_run(x, m, h, leaf=leaf, walk=walk, tree_shape=F.FMM_TREE_COM,
                           theta=0.9)
        ref = orc.fmm(x, m, h, theta=0.9, leaf_size=leaf, policy=walk, tree_kind=O.COM_TREE)
        np.testing.assert_array_equal(ex["perm"], ref.tree.perm)
        np.testing.assert_array_equal(ex["left"], ref.tree.left)
        assert force_err(a, ref.a) <= 1e-12


def test_census_on_mutual_com_tree():
    import torch

    x, m, h = W.plummer(5000, 33)
    say("[gpu combos] census of a mutual walk over the centre-of-mass tree")
    X, Mt, H = to_dev(x, m, h)
    t = F.fmm_build_tree(X, F.default_params(leaf_size=10, tree=F.FMM_TREE_COM,
                                             walk=F.FMM_WALK_MUTUAL), m=Mt)
    try:
        F.fmm_moments(t, X, Mt, H)
        A = torch.empty((len(m), 3), dtype=torch.float64, device="cuda")
        F.fmm_forces(t, A)
        got = F.fmm_asymmetry_estimate(t)
    finally:
        F.fmm_tree_free(t)
    assert got == {"F33": 0.0, "F46": 0.0, "n_asym": 0, "n_asym_super": 0}
