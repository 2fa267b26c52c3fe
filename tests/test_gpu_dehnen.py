"""GPU parity of the second expansion form (Sec. 4, eqs. (25)-(26) with p = 3)
against the oracle.

Bar: FP64 accelerations and leaf local expansions within 1e-12 of the
oracle's FMM of the same form, for the leaf <- cell and the mutual walk;
FP32 form within eta 1e-5; |sum F| / sum |F| at round-off for the mutual walk
and well above it for the leaf <- cell walk (the asymmetry of Sec. 4 does not
depend on the expansion form); VJP of the form within 1e-6 of central finite
differences of the oracle's frozen-tree FMM of the same form."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_01496_amd import fmm as F
from paper_2502_01496_amd import workloads as W
from tests.gpu_util import eta, force_err, gpu_run, gpu_vjp, say, to_dev
from tests.test_gpu_parity import _case
from tests.test_gpu_vjp import fd_check

pytestmark = pytest.mark.gpu

DEH = F.FMM_EXPANSION_DEHNEN


def _ratio(x, m, a):
    X, Mt, A = to_dev(x, m, a)
    return F.fmm_momentum_stats(X, None, Mt, A)["ratio"]


@pytest.mark.parametrize("walk", [F.FMM_WALK_PHANTOM, F.FMM_WALK_MUTUAL])
@pytest.mark.parametrize("name", ["plummer_4096", "plummer_777_leaf1", "binary_2x4096_theta0.3",
                                  "clumpy_20000_lognormal", "plummer_100003_ragged"])
def test_dehnen_fp64_parity(orc, name, walk):
    x, m, h, theta, leaf = _case(name)
    say(f"[gpu dehnen] case={name} walk={walk} n={len(m)}")
    a, ex, _ = gpu_run(x, m, h, theta=theta, leaf=leaf, walk=walk, expansion=DEH, local=True)
    ref = orc.fmm(x, m, h, theta=theta, leaf_size=leaf, policy=walk, form=O.DEHNEN_FORM)
    leaves = ref.tree.left < 0
    for lo, hi in ((0, 3), (3, 9), (9, 19)):
        got, want = ex["local"][leaves, lo:hi], ref.L[leaves, lo:hi]
        scale = max(np.abs(want).max(), 1e-300)
        assert np.abs(got - want).max() <= 1e-12 * scale
    err = force_err(a, ref.a)
    ratio = _ratio(x, m, a)
    say(f"    max rel force error {err:.3e}; |sumF|/sum|F| = {ratio:.3e}")
    assert err <= 1e-12
    if walk == F.FMM_WALK_MUTUAL:
        assert ratio <= 1e-13


def test_dehnen_fp32(orc):
    x, m, h = W.polytrope_binary(8192, 2, cache=False)
    say("[gpu dehnen] FP32 form, binary_2x8192, both walks")
    for walk in (F.FMM_WALK_PHANTOM, F.FMM_WALK_MUTUAL):
        a, _, _ = gpu_run(x, m, h, precision=F.FMM_FP32, export=False, walk=walk, expansion=DEH)
        ref = orc.fmm(x, m, h, policy=walk, form=O.DEHNEN_FORM)
        e = eta(a, ref.a)
        say(f"    walk={walk}: eta vs FP64 oracle {e:.3e}")
        assert e <= 1e-5


def test_asymmetry_persists_with_dehnen_form(orc):
    x, m, h = W.polytrope_binary(8192, 2, cache=False)
    say("[gpu dehnen] momentum and accuracy of the two forms, binary_2x8192")
    d = orc.direct_sinks(x, m, h, np.arange(0, len(m), 29))
    out = {}
    for form in (F.FMM_EXPANSION_PHANTOM, DEH):
        for walk in (F.FMM_WALK_PHANTOM, F.FMM_WALK_MUTUAL):
            a, _, _ = gpu_run(x, m, h, export=False, walk=walk, expansion=form)
            out[form, walk] = (_ratio(x, m, a), eta(a[::29], d))
            say(f"    form={form} walk={walk}: ratio {out[form, walk][0]:.3e}, "
                f"eta vs direct {out[form, walk][1]:.3e}")
    for form in (F.FMM_EXPANSION_PHANTOM, DEH):
        assert out[form, F.FMM_WALK_PHANTOM][0] > 1e-8
        assert out[form, F.FMM_WALK_MUTUAL][0] < 1e-13
        assert out[form, F.FMM_WALK_PHANTOM][1] < 1e-2
    assert 0.5 < out[DEH, F.FMM_WALK_PHANTOM][1] / out[F.FMM_EXPANSION_PHANTOM,
                                                     F.FMM_WALK_PHANTOM][1] < 2.0


@pytest.mark.parametrize("name", ["plummer_4096", "binary_2x2048"])
def test_dehnen_vjp_matches_finite_differences(orc, name):
    if name == "plummer_4096":
        x, m, h = W.plummer(4096, 1)
    else:
        x, m, h = W.polytrope_binary(2048, 2, cache=False)
    abar = W.cotangent(len(m), 33)
    say(f"[gpu dehnen] VJP finite differences, case={name}")
    _, [(xb, mb)] = gpu_vjp(x, m, h, abar, expansion=DEH)
    worst = fd_check(orc, x, m, h, abar, xb, mb, 0.5, 8, form=O.DEHNEN_FORM)
    say(f"    worst directional error {worst:.2e}")
    assert worst <= 1e-6
