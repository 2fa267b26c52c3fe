"""Checkpointed backpropagation through KDK leapfrog steps, and the autograd
Function around the FMM forces.

The reference is the oracle: KDK steps with the frozen-tree FMM, each step
holding the tree and lists the unperturbed trajectory had at that step, and
central finite differences (eps = 1e-4) of a random linear functional
J = <w, x_T> + <u, v_T> along normalised directions in x_0 and m."""
import numpy as np
import pytest
import torch

from paper_2502_01496_amd import fmm as F
from paper_2502_01496_amd import leapfrog as LF
from paper_2502_01496_amd import workloads as W
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def oracle_kdk(orc, x0, v0, m, h, dt, steps, structs=None, theta=0.5, policy=0):
    """KDK with the oracle; records (tree, lists) per visited position unless
    given, in which case they are held fixed."""
    rec = [] if structs is None else None

    def force(x, k):
        if structs is None:
            r = orc.fmm(x, m, h, theta=theta, policy=policy)
            rec.append((r.tree, r.lists))
            return r.a
        return orc.fmm_frozen(x, m, h, *structs[k], policy=policy)

    x, v = x0.copy(), v0.copy()
    a = force(x, 0)
    for k in range(steps):
        v = v + 0.5 * dt * a
        x = x + dt * v
        a = force(x, k + 1)
        v = v + 0.5 * dt * a
    return x, v, rec


@pytest.mark.parametrize("walk", [F.FMM_WALK_PHANTOM, F.FMM_WALK_MUTUAL])
def test_leapfrog_adjoint_matches_finite_differences(orc, walk):
    x0, m, h = W.polytrope_binary(1024, 2, cache=False)
    n = len(m)
    rng = np.random.default_rng(5)
    v0 = 0.1 * rng.standard_normal((n, 3))
    dt, steps = 1e-3, 4
    w = rng.standard_normal((n, 3))
    u = rng.standard_normal((n, 3))
    say(f"[gpu leapfrog] adjoint vs frozen-structure finite differences, n={n}, steps={steps}, "
        f"walk={walk}")
    field = LF.ForceField(theta=0.5, walk=walk)
    X0, V0, Mt, H = to_dev(x0, v0, m, h)
    try:
        xT, vT, ckpt = LF.kdk_forward(X0, V0, Mt, H, dt, steps, field)
        xbar, vbar, mbar = LF.kdk_backward(ckpt, Mt, H, dt, field, *to_dev(w, u))
    finally:
        field.free()
    xbar, vbar, mbar = (t.cpu().numpy() for t in (xbar, vbar, mbar))
    # the GPU trajectory equals the oracle's
    xr, vr, structs = oracle_kdk(orc, x0, v0, m, h, dt, steps, policy=walk)
    assert np.abs(xT.cpu().numpy() - xr).max() < 1e-12

    def J(xx, vv, mm):
        xt, vt, _ = oracle_kdk(orc, xx, vv, mm, h, dt, steps, structs, policy=walk)
        return float((w * xt).sum() + (u * vt).sum())

    eps = 1e-4
    for _ in range(3):
        e = rng.standard_normal((n, 3))
        e /= np.linalg.norm(e)
        fd = (J(x0 + eps * e, v0, m) - J(x0 - eps * e, v0, m)) / (2 * eps)
        assert abs((xbar * e).sum() - fd) <= 1e-6 * np.linalg.norm(xbar)
        fd = (J(x0, v0 + eps * e, m) - J(x0, v0 - eps * e, m)) / (2 * eps)
        assert abs((vbar * e).sum() - fd) <= 1e-6 * np.linalg.norm(vbar)
        em = rng.standard_normal(n)
        em /= np.linalg.norm(em)
        ep = eps * m.mean()
        fd = (J(x0, v0, m + ep * em) - J(x0, v0, m - ep * em)) / (2 * ep)
        assert abs((mbar * em).sum() - fd) <= 1e-6 * np.linalg.norm(mbar)


def test_com_drift_gradient_runs_and_is_consistent():
    x0, m, h = W.polytrope_binary(2048, 2, cache=False)
    say("[gpu leapfrog] centre-of-mass drift loss and gradient, binary_2x2048, 5 steps")
    X0, Mt, H = to_dev(x0, m, h)
    field = LF.ForceField(theta=0.5)
    try:
        L, gx, gm, gv = LF.com_drift_gradient(X0, torch.zeros_like(X0), Mt, H, 1e-3, 5, field)
    finally:
        field.free()
    assert L > 0.0 and np.isfinite(L)
    assert torch.isfinite(gx).all() and torch.isfinite(gm).all()


def test_com_drift_gradient_closed_form_with_mutual_walk():
    # With the mutual walk sum_i m_i a_i = 0 for any x and m, so KDK moves the
    # centre of mass at constant velocity: D = X_T - X_0 = T dt V, V = sum m v_0 / M,
    # and L = |D|^2 has dL/dx_0 = 0, dL/dv_0,j = 2 T dt m_j D / M and
    # dL/dm_j = 2 T dt D . (v_0,j - V) / M.  The checkpointed reverse sweep must
    # give these through the force VJPs; the leaf <- cell walk moves the
    # centre of mass through its force asymmetry and does not.
    x0, m, h = W.polytrope_binary(2048, 2, cache=False)
    rng = np.random.default_rng(9)
    n = len(m)
    m = m * (0.5 + rng.random(n))  # unequal masses
    v0 = 0.1 * rng.standard_normal((n, 3)) + np.array([0.3, -0.2, 0.1])
    dt, steps = 1e-2, 5
    M = m.sum()
    V = (m[:, None] * v0).sum(0) / M
    D = steps * dt * V
    gv_ref = 2 * steps * dt * m[:, None] * D[None, :] / M
    gm_ref = 2 * steps * dt * ((v0 - V) @ D) / M
    say(f"[gpu leapfrog] centre-of-mass drift gradient in closed form, mutual walk, n={n}")
    out = {}
    for walk in (F.FMM_WALK_MUTUAL, F.FMM_WALK_PHANTOM):
        X0, V0, Mt, H = to_dev(x0, v0, m, h)
        field = LF.ForceField(theta=0.5, walk=walk)
        try:
            L, gx, gm, gv = LF.com_drift_gradient(X0, V0, Mt, H, dt, steps, field)
        finally:
            field.free()
        out[walk] = (L, gx.cpu().numpy(), gm.cpu().numpy(), gv.cpu().numpy())
    L, gx, gm, gv = out[F.FMM_WALK_MUTUAL]
    scale_x = np.abs(gv_ref).max() / (steps * dt)  # |dL/dx_T|
    rx = np.abs(gx).max() / scale_x
    rx_leaf = np.abs(out[F.FMM_WALK_PHANTOM][1]).max() / scale_x
    say(f"    mutual: |gx| / |dL/dx_T| {rx:.1e}; leaf <- cell {rx_leaf:.1e}")
    assert L == pytest.approx(float(D @ D), rel=1e-12)
    assert rx <= 1e-12 and rx_leaf >= 1e3 * max(rx, 1e-16)
    assert np.abs(gv - gv_ref).max() <= 1e-12 * np.abs(gv_ref).max()
    assert np.abs(gm - gm_ref).max() <= 1e-10 * np.abs(gm_ref).max()


def test_autograd_function_matches_vjp_and_rebuilds():
    x, m, h = W.plummer(3000, 17)
    abar = W.cotangent(3000, 18)
    say("[gpu leapfrog] autograd Function, plummer_3000")
    X, Mt, H, AB = to_dev(x, m, h, abar)
    field = LF.ForceField(theta=0.5)
    try:
        Xr = X.clone().requires_grad_(True)
        Mr = Mt.clone().requires_grad_(True)
        a = LF.FmmForce.apply(Xr, Mr, H, field)
        ref_xb, ref_mb = field.vjp(AB)          # VJP right after the forward
        ref_xb, ref_mb = ref_xb.clone(), ref_mb.clone()
        field.forces(X + 0.01, Mt, H)            # another evaluation in between
        gx, gm = torch.autograd.grad((a * AB).sum(), (Xr, Mr))
    finally:
        field.free()
    assert torch.equal(gx, ref_xb) and torch.equal(gm, ref_mb)


@pytest.mark.parametrize("adt", [torch.float64, torch.float32])
def test_momentum_stats_async_equals_sync(adt):
    """The device-output statistics equal the synchronous ones bit for bit,
    on two calls in a row on one stream (the second with other inputs)."""
    rng = np.random.default_rng(11)
    out = torch.zeros((2, 16), dtype=torch.float64, device="cuda")
    ref = []
    for k, n in enumerate((5000, 1777)):
        x = torch.tensor(rng.normal(size=(n, 3)), device="cuda")
        v = torch.tensor(rng.normal(size=(n, 3)), device="cuda")
        m = torch.tensor(rng.uniform(0.5, 1.5, size=n), device="cuda")
        a = torch.tensor(rng.normal(size=(n, 3)), device="cuda").to(adt)
        say(f"stats async vs sync: n={n} a={adt}")
        F.fmm_momentum_stats_async(x, v, m, a, out[k])
        ref.append(F.fmm_momentum_stats(x, v, m, a))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for k, st in enumerate(ref):
        want = np.concatenate([st["sumF"], [st["sumAbsF"], st["ratio"], st["mass"]], st["xcom"],
                               st["P"], st["L"]])
        np.testing.assert_array_equal(got[k, :15], want)
