"""GPU vector-Jacobian product of the FMM accelerations (tree membership and
interaction lists held fixed) against the CPU oracle.

Checks: central finite differences (eps = 1e-4, FP64) of <abar, a(x, m)> computed
by the oracle's frozen-tree FMM along normalised random directions, within 1e-6
of |xbar| |e| (resp. |mbar| |e|); at theta = 0 the FMM is the direct sum, so the
VJP must equal the oracle's analytic direct-sum adjoint to 1e-12; at theta = 0.5
it differs from that adjoint only by the FMM truncation (at most ten times the
forward error eta of the same configuration); bitwise reproducible.  The same
for the lists of the mutual walk (Sec. 7), whose total force vanishes for any
x and m: with abar_i = m_i e the VJP must give xbar = 0 and mbar_j = -e . a_j
up to rounding, which the leaf <- cell walk does not."""
import numpy as np
import pytest

from paper_2502_01496_amd import fmm as F
from paper_2502_01496_amd import workloads as W
from tests.gpu_util import gpu_vjp, say

pytestmark = pytest.mark.gpu


def fd_check(orc, x, m, h, abar, xb, mb, theta, leaf, ndir=4, eps=1e-4, seed=0, form=0,
             tree_kind=0, policy=0):
    ref = orc.fmm(x, m, h, theta=theta, leaf_size=leaf, form=form, tree_kind=tree_kind,
                  policy=policy)
    tree, lists = ref.tree, ref.lists
    phi = lambda xx, mm: float((orc.fmm_frozen(xx, mm, h, tree, lists, form=form,
                                               policy=policy) * abar).sum())
    rng = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(ndir):
        e = rng.standard_normal(x.shape)
        e /= np.linalg.norm(e)
        fd = (phi(x + eps * e, m) - phi(x - eps * e, m)) / (2 * eps)
        err = abs((xb * e).sum() - fd) / np.linalg.norm(xb)
        worst = max(worst, err)
        em = rng.standard_normal(m.shape)
        em /= np.linalg.norm(em)
        epm = eps * m.mean()
        fd = (phi(x, m + epm * em) - phi(x, m - epm * em)) / (2 * epm)
        err = abs((mb * em).sum() - fd) / np.linalg.norm(mb)
        worst = max(worst, err)
    return worst


@pytest.mark.parametrize("name", ["plummer_4096", "binary_2x2048", "leaf10_3000", "clumpy_6000"])
def test_vjp_matches_finite_differences(orc, name):
    leaf, theta = 8, 0.5
    if name == "plummer_4096":
        x, m, h = W.plummer(4096, 1)
    elif name == "binary_2x2048":
        x, m, h = W.polytrope_binary(2048, 2, cache=False)
    elif name == "leaf10_3000":
        x, m, h = W.plummer(3000, 15)
        leaf = 10
    else:
        x, m, h = W.clumpy_cube(6000, 3, cache=False)
    abar = W.cotangent(len(m), 31)
    say(f"[gpu vjp] finite differences, case={name} n={len(m)}")
    _, [(xb, mb)] = gpu_vjp(x, m, h, abar, theta=theta, leaf=leaf)
    worst = fd_check(orc, x, m, h, abar, xb, mb, theta, leaf)
    say(f"    worst directional error {worst:.2e}")
    assert worst <= 1e-6


def test_vjp_theta0_is_direct_adjoint(orc):
    x, m, h = W.plummer(2048, 16)
    h = h * 5.0  # many softened pairs
    abar = W.cotangent(len(m), 32)
    say("[gpu vjp] theta = 0 against the direct-sum adjoint, plummer_2048")
    _, [(xb, mb)] = gpu_vjp(x, m, h, abar, theta=0.0)
    xr, mr = orc.direct_vjp(x, m, h, abar)
    assert np.abs(xb - xr).max() <= 1e-12 * np.abs(xr).max()
    assert np.abs(mb - mr).max() <= 1e-12 * np.abs(mr).max()


@pytest.mark.parametrize("name", ["plummer_4096", "binary_2x4096"])
def test_vjp_close_to_direct_adjoint(orc, name):
    # the FMM adjoint differs from the direct-sum adjoint by the FMM's own
    # truncation; derivatives of a truncated expansion carry a larger relative
    # error than the forces, so the bound is ten times the forward error eta
    # (it guards against a wrong term, which would give an O(1) difference;
    # exactness is pinned by the finite-difference test)
    if name == "plummer_4096":
        x, m, h = W.plummer(4096, 1)
    else:
        x, m, h = W.polytrope_binary(4096, 2, cache=False)
    abar = W.cotangent(len(m), 33)
    say(f"[gpu vjp] theta = 0.5 against the direct-sum adjoint, {name}")
    a, [(xb, mb)] = gpu_vjp(x, m, h, abar, theta=0.5)
    d = orc.direct(x, m, h)
    eta_fwd = np.sqrt(((a - d) ** 2).sum() / (d ** 2).sum())
    xr, mr = orc.direct_vjp(x, m, h, abar)
    ex = np.linalg.norm(xb - xr) / np.linalg.norm(xr)
    em = np.linalg.norm(mb - mr) / np.linalg.norm(mr)
    say(f"    forward eta {eta_fwd:.2e}; relative difference: xbar {ex:.2e}, mbar {em:.2e}")
    assert ex <= 10 * eta_fwd and em <= 10 * eta_fwd


def test_vjp_deterministic_and_fp32(orc):
    x, m, h = W.polytrope_binary(4096, 2, cache=False)
    abar = W.cotangent(len(m), 34)
    say("[gpu vjp] determinism and FP32 form, binary_2x4096")
    _, [(x1, m1), (x2, m2)] = gpu_vjp(x, m, h, abar, repeat=2)
    assert np.array_equal(x1, x2) and np.array_equal(m1, m2)
    _, [(x3, m3)] = gpu_vjp(x, m, h, abar, precision=F.FMM_FP32)
    assert np.linalg.norm(x3 - x1) <= 1e-5 * np.linalg.norm(x1)
    assert np.linalg.norm(m3 - m1) <= 1e-5 * np.linalg.norm(m1)


@pytest.mark.parametrize("name,form,shape", [("plummer_4096", 0, 0), ("binary_2x2048", 0, 0),
                                             ("plummer_4096_dehnen", 1, 0),
                                             ("clumpy_6000_com", 0, 1), ("leaf10_3000", 0, 0)])
def test_mutual_vjp_matches_finite_differences(orc, name, form, shape):
    leaf, theta = 8, 0.5
    if name.startswith("plummer_4096"):
        x, m, h = W.plummer(4096, 1)
    elif name == "binary_2x2048":
        x, m, h = W.polytrope_binary(2048, 2, cache=False)
    elif name == "leaf10_3000":
        x, m, h = W.plummer(3000, 15)
        leaf = 10
    else:
        x, m, h = W.clumpy_cube(6000, 3, cache=False)
    abar = W.cotangent(len(m), 35)
    say(f"[gpu vjp] mutual walk, finite differences, case={name} n={len(m)}")
    _, [(xb, mb)] = gpu_vjp(x, m, h, abar, theta=theta, leaf=leaf, expansion=form,
                            tree_shape=shape, walk=F.FMM_WALK_MUTUAL)
    worst = fd_check(orc, x, m, h, abar, xb, mb, theta, leaf, form=form, tree_kind=shape,
                     policy=orc.MUTUAL)
    say(f"    worst directional error {worst:.2e}")
    assert worst <= 1e-6


def test_mutual_vjp_theta0_is_direct_adjoint(orc):
    # theta = 0: no pair is well separated, every leaf pair is near
    x, m, h = W.plummer(2048, 16)
    abar = W.cotangent(len(m), 36)
    say("[gpu vjp] mutual walk, theta = 0 against the direct-sum adjoint, plummer_2048")
    _, [(xb, mb)] = gpu_vjp(x, m, h, abar, theta=0.0, walk=F.FMM_WALK_MUTUAL)
    xr, mr = orc.direct_vjp(x, m, h, abar)
    assert np.abs(xb - xr).max() <= 1e-12 * np.abs(xr).max()
    assert np.abs(mb - mr).max() <= 1e-12 * np.abs(mr).max()


@pytest.mark.parametrize("name,form,prec", [("plummer_8192", 0, F.FMM_FP64),
                                            ("binary_2x4096", 0, F.FMM_FP64),
                                            ("binary_2x4096_dehnen", 1, F.FMM_FP64),
                                            ("plummer_8192_fp32", 0, F.FMM_FP32)])
def test_mutual_vjp_momentum_identity(name, form, prec):
    # sum_i m_i a_i = 0 identically for the mutual lists, so for abar_i = m_i e:
    # xbar = d(e . sum F)/dx = 0 and mbar_j = -e . a_j
    if name.startswith("plummer"):
        x, m, h = W.plummer(8192, 5)
    else:
        x, m, h = W.polytrope_binary(4096, 2, cache=False)
    rng = np.random.default_rng(7)
    e = np.array([0.75, -0.5, 0.25])  # dyadic: m_i e is exact in FP32 too (m = 2^-k here)
    ab_id = m[:, None] * e[None, :]
    ab_rnd = ab_id * rng.choice([-1.0, 1.0], size=(len(m), 1))  # no cancellation
    say(f"[gpu vjp] mutual walk, momentum identity, case={name} n={len(m)}")
    res = {}
    for walk in (F.FMM_WALK_MUTUAL, F.FMM_WALK_PHANTOM):
        a, [(xb, mb)] = gpu_vjp(x, m, h, ab_id, expansion=form, precision=prec, walk=walk)
        _, [(xr, _)] = gpu_vjp(x, m, h, ab_rnd, expansion=form, precision=prec, walk=walk)
        res[walk] = (np.abs(xb).max() / np.abs(xr).max(),
                     np.abs(mb + a @ e).max() / np.abs(a @ e).max())
    say(f"    mutual: |xbar| {res[1][0]:.1e}, |mbar + e.a| {res[1][1]:.1e}; "
        f"leaf <- cell: {res[0][0]:.1e}, {res[0][1]:.1e}")
    # FP32 trees: the forward a is FP32, the reverse pass FP64
    tol_m = 1e-12 if prec == F.FMM_FP64 else 1e-5
    assert res[F.FMM_WALK_MUTUAL][0] <= 1e-12 and res[F.FMM_WALK_MUTUAL][1] <= tol_m
    assert res[F.FMM_WALK_PHANTOM][0] >= 1e-6


def test_mutual_vjp_deterministic_and_fp32(orc):
    x, m, h = W.polytrope_binary(4096, 2, cache=False)
    abar = W.cotangent(len(m), 37)
    say("[gpu vjp] mutual walk, determinism and FP32 form, binary_2x4096")
    _, [(x1, m1), (x2, m2)] = gpu_vjp(x, m, h, abar, repeat=2, walk=F.FMM_WALK_MUTUAL)
    assert np.array_equal(x1, x2) and np.array_equal(m1, m2)
    _, [(x3, m3)] = gpu_vjp(x, m, h, abar, precision=F.FMM_FP32, walk=F.FMM_WALK_MUTUAL)
    assert np.linalg.norm(x3 - x1) <= 1e-5 * np.linalg.norm(x1)
    assert np.linalg.norm(m3 - m1) <= 1e-5 * np.linalg.norm(m1)


@pytest.mark.parametrize("precision", [F.FMM_FP64, F.FMM_FP32])
@pytest.mark.parametrize("walk", [F.FMM_WALK_PHANTOM, F.FMM_WALK_MUTUAL])
def test_vjp_only_preparation_equals_full_forces(orc, precision, walk):
    # FMM_VJP_ONLY walks the tree (and forms an FP64 tree's far-field
    # expansions) without evaluating the forces: the reverse pass that follows
    # is the one after a full forces call, bit for bit
    import torch

    x, m, h = W.polytrope_binary(3000, 6, cache=False)
    abar = W.cotangent(len(m), 35)
    say(f"[gpu vjp] FMM_VJP_ONLY preparation, precision {precision}, walk {walk}")
    X = torch.from_numpy(x).cuda()
    Mt = torch.from_numpy(m).cuda()
    H = torch.from_numpy(h).cuda()
    dt = torch.float32 if precision == F.FMM_FP32 else torch.float64
    AB = torch.from_numpy(abar).cuda().to(dt)
    outs = []
    for flags in (F.FMM_REWALK, F.FMM_REWALK | F.FMM_VJP_ONLY):
        t = F.fmm_build_tree(X, F.default_params(precision=precision, walk=walk))
        try:
            F.fmm_moments(t, X, Mt, H)
            A = None if flags & F.FMM_VJP_ONLY else torch.empty((len(m), 3), dtype=dt,
                                                                 device="cuda")
            F.fmm_forces(t, A, flags)
            XB = torch.empty((len(m), 3), dtype=dt, device="cuda")
            MB = torch.empty(len(m), dtype=dt, device="cuda")
            F.fmm_forces_vjp(t, AB, XB, MB)
            torch.cuda.synchronize()
            outs.append((XB.cpu().numpy(), MB.cpu().numpy()))
            if flags & F.FMM_VJP_ONLY:
                with pytest.raises(F.FmmError):
                    F.fmm_forces(t, A, F.FMM_VJP_ONLY | 8)  # an unknown flag bit
        finally:
            F.fmm_tree_free(t)
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
