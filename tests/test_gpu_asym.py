"""GPU census of asymmetric cell pairs and the total-force estimates eq. (33)
and eq. (46) against the oracle.

Bar: pair counts identical; both sums within 1e-12 (relative) of the oracle's
(the per-pair terms are the same IEEE operations, only the summation order
differs); all four zero on the mutual walk's lists; bitwise reproducible."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_01496_amd import fmm as F
from paper_2502_01496_amd import workloads as W
from tests.gpu_util import say, to_dev
from tests.test_gpu_parity import _case

pytestmark = pytest.mark.gpu


def gpu_estimate(x, m, h, theta=0.5, leaf=8, walk=F.FMM_WALK_PHANTOM, m_leaf=0.0, repeat=1):
    import torch

    X, Mt, H = to_dev(x, m, h)
    p = F.default_params(theta=theta, leaf_size=leaf, walk=walk)
    t = F.fmm_build_tree(X, p)
    try:
        F.fmm_moments(t, X, Mt, H)
        A = torch.empty((len(m), 3), dtype=torch.float64, device="cuda")
        F.fmm_forces(t, A)
        out = [F.fmm_asymmetry_estimate(t, m_leaf) for _ in range(repeat)]
        st = F.fmm_momentum_stats(X, None, Mt, A)
    finally:
        F.fmm_tree_free(t)
    return out, st


@pytest.mark.parametrize("name", ["tiny_1", "tiny_9", "plummer_4096", "plummer_777_leaf1",
                                  "binary_2x4096_theta0.7", "binary_2x8192",
                                  "clumpy_20000_lognormal", "plummer_100003_ragged"])
def test_asym_parity(orc, name):
    x, m, h, theta, leaf = _case(name)
    say(f"[gpu asym] case={name} n={len(m)} theta={theta} leaf={leaf}")
    (got,), st = gpu_estimate(x, m, h, theta, leaf)
    ref = orc.fmm(x, m, h, theta=theta, leaf_size=leaf)
    want = orc.asym_estimate(ref.tree, ref.mom, ref.lists)
    say(f"    {got}; |sumF| = {np.linalg.norm(st['sumF']):.3e}")
    assert got["n_asym"] == want["n_asym"] and got["n_asym_super"] == want["n_asym_super"]
    for k in ("F33", "F46"):
        assert got[k] == pytest.approx(want[k], rel=1e-12, abs=1e-300)


def test_asym_explicit_leaf_mass_and_determinism(orc):
    x, m, h = W.polytrope_binary(8192, 2, cache=False)
    say("[gpu asym] explicit m_leaf, two calls, binary_2x8192")
    ml = 10.0 / len(m)
    out, _ = gpu_estimate(x, m, h, m_leaf=ml, repeat=2)
    assert out[0] == out[1]
    ref = orc.fmm(x, m, h)
    want = orc.asym_estimate(ref.tree, ref.mom, ref.lists, m_leaf=ml)
    assert out[0]["F46"] == pytest.approx(want["F46"], rel=1e-12)


@pytest.mark.parametrize("name", ["plummer_4096", "clumpy_20000_lognormal"])
def test_mutual_lists_have_no_asymmetric_pair(name):
    x, m, h, theta, leaf = _case(name)
    say(f"[gpu asym] mutual lists, case={name}")
    (got,), _ = gpu_estimate(x, m, h, theta, leaf, walk=F.FMM_WALK_MUTUAL)
    assert got == {"F33": 0.0, "F46": 0.0, "n_asym": 0, "n_asym_super": 0}
