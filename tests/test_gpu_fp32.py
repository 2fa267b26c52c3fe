"""GPU precision form: FP64 tree, moments, walk and reductions; FP32 M2L, L2P and
P2P with FP32 accumulation on leaf-relative offsets.

Bar (the FP32 rounding of ~10^3-term sums): normalised RMS error against the
oracle's FP64 FMM eta <= 1e-5 and the 99th percentile of the per-particle
relative error <= 1e-4; the interaction lists are the FP64 ones; against the
FP64 direct sum the FP32 form keeps the FMM's own accuracy (eta within 1% of
the FP64 FMM's)."""
import numpy as np
import pytest

from paper_2502_01496_amd import fmm as F
from paper_2502_01496_amd import workloads as W
from tests.gpu_util import eta, gpu_run, say

pytestmark = pytest.mark.gpu


def _pp_rel(a, ref):
    nr = np.linalg.norm(ref, axis=1)
    return np.linalg.norm(a - ref, axis=1) / np.maximum(nr, 1e-3 * np.sqrt((nr ** 2).mean()))


@pytest.mark.parametrize("name", ["plummer_4096", "binary_2x8192", "clumpy_20000", "leaf10_5000"])
def test_fp32_against_oracle(orc, name):
    leaf = 8
    if name == "plummer_4096":
        x, m, h = W.plummer(4096, 1)
    elif name == "binary_2x8192":
        x, m, h = W.polytrope_binary(8192, 2, cache=False)
    elif name == "clumpy_20000":
        x, m, h = W.clumpy_cube(20000, 3, cache=False)
    else:
        x, m, h = W.plummer(5000, 14)
        leaf = 10
    say(f"[gpu fp32] case={name} n={len(m)}")
    a32, ex32, _ = gpu_run(x, m, h, leaf=leaf, precision=F.FMM_FP32)
    ref = orc.fmm(x, m, h, leaf_size=leaf)
    e = eta(a32, ref.a)
    p99 = np.percentile(_pp_rel(a32, ref.a), 99)
    say(f"    eta vs FP64 oracle FMM {e:.2e}, p99 {p99:.2e}")
    assert e <= 1e-5 and p99 <= 1e-4
    np.testing.assert_array_equal(ex32["perm"], ref.tree.perm)
    np.testing.assert_array_equal(ex32["far_off"], ref.lists.far_off)
    np.testing.assert_array_equal(ex32["near_off"], ref.lists.near_off)
    st32 = orc.stats(x, None, m, a32)
    st64 = orc.stats(x, None, m, ref.a)
    say(f"    |sumF|/sum|F|: fp32 {st32['ratio']:.3e}, fp64 {st64['ratio']:.3e}")
    assert abs(st32["ratio"] - st64["ratio"]) <= 2e-6 + 0.1 * st64["ratio"]


def test_fp32_accuracy_vs_direct(orc):
    x, m, h = W.polytrope_binary(4096, 2, cache=False)
    say("[gpu fp32] accuracy vs direct sum, binary_2x4096")
    a32, _, _ = gpu_run(x, m, h, precision=F.FMM_FP32, export=False)
    a64, _, _ = gpu_run(x, m, h, export=False)
    d = orc.direct(x, m, h)
    e32, e64 = eta(a32, d), eta(a64, d)
    say(f"    eta vs direct: fp32 {e32:.3e}, fp64 {e64:.3e}")
    assert e32 <= 1.01 * e64 + 1e-6


def test_fp32_leaf10_page_aligned_binary():
    # Regression: with leaf size 10 every leaf has a second source block, empty
    # for leaves of at most 8 particles; the last leaf's empty block starts one
    # past the last particle, which for n = 2^19 is the first byte after the
    # page-aligned FP32 particle arrays.  The FP32 form must not read there
    # and must agree with the FP64 form.
    x, m, h = W.polytrope_binary(1 << 18, 2)
    say("[gpu fp32] binary 2 x 2^18, leaf 10: FP32 form against FP64 on the GPU")
    a32, _, _ = gpu_run(x, m, h, leaf=10, precision=F.FMM_FP32, export=False)
    a64, _, _ = gpu_run(x, m, h, leaf=10, export=False)
    e = eta(a32, a64)
    say(f"    eta FP32 vs FP64 {e:.2e}")
    assert e <= 1e-5
