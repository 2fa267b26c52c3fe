"""GPU checks at the full sizes of the paper-derived workloads, in the launch
configuration the benchmark times (one tree per call sequence, default
capacities, leaf size 8).

* binary 2 x 2^18, theta in {0.3, 0.5, 0.7}: tree, cell records and lists
  bit-identical to the oracle, FP64 forces within 1e-12 of the oracle FMM;
  100 KDK steps whose per-step momentum statistics satisfy the exact KDK
  identities of the centre of mass;
* clumpy cube 2^22: FP64 against the oracle FMM on every particle, FP32
  against FP64, both against the direct sum on sampled sinks;
* Plummer 2^20: FP32 forward with the tree fixed, VJP against central finite
  differences of the FP64 frozen-list forces; its first 4096 particles as
  their own system against the oracle's direct-sum adjoint;
* binary 2 x 2^23: FP32 forward through 10 KDK steps and the checkpointed
  backward pass of |x_com(T) - x_com(0)|^2, against central finite
  differences with every step's tree and lists held at the forward pass's;
  its step-0 FP64 forward against the oracle: tree and cell records
  bit-identical, list lengths and forces of 2048 sampled sink leaves from
  the oracle's per-leaf evaluation on its own tree;
* binary 2 x 2^18, the first 10 KDK steps (theta = 0.5) against the oracle:
  every step's forces on every particle, the KDK update, and the oracle's own
  trajectory (positions and total force per step)."""
import time

import numpy as np
import pytest
import torch

from paper_2502_01496_amd import fmm as F
from paper_2502_01496_amd import leapfrog as LF
from paper_2502_01496_amd import workloads as W
from tests.gpu_util import eta, force_err, gpu_run, gpu_vjp, oracle_fmm_threaded, say, to_dev
from tests.test_gpu_parity import sorted_by_sink

pytestmark = pytest.mark.gpu


def _rel_rows(a, ref):
    return np.linalg.norm(a - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-300)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("theta", [0.3, 0.5, 0.7])
def test_binary_2x2e18_full_parity(orc, theta):
    x, m, h = W.polytrope_binary(1 << 18, 2)
    say(f"[gpu full] binary 2x2^18 theta={theta}: GPU FP64 vs oracle FMM, all particles")
    a, ex, info = gpu_run(x, m, h, theta=theta)
    ref = orc.fmm(x, m, h, theta=theta)
    t, mom, lists = ref.tree, ref.mom, ref.lists
    np.testing.assert_array_equal(ex["perm"], t.perm)
    np.testing.assert_array_equal(ex["axis"], t.axis)
    rec = ex["rec"]
    np.testing.assert_array_equal(rec[:, 0], mom.M)
    np.testing.assert_array_equal(rec[:, 1:4], mom.c)
    np.testing.assert_array_equal(rec[:, 4], mom.s)
    np.testing.assert_array_equal(rec[:, 5], mom.hmax)
    for off_k, src_k, ro, rs in (("far_off", "far_src", lists.far_off, lists.far_src),
                                 ("near_off", "near_src", lists.near_off, lists.near_src)):
        np.testing.assert_array_equal(ex[off_k], ro)
        np.testing.assert_array_equal(sorted_by_sink(ex[off_k], ex[src_k]), sorted_by_sink(ro, rs))
    err = force_err(a, ref.a)
    st = orc.stats(x, None, m, a)
    st_ref = orc.stats(x, None, m, ref.a)
    say(f"    far {info['n_far']} near {info['n_near']}; max rel force error {err:.3e}; "
        f"|sumF|/sum|F| GPU {st['ratio']:.4e} oracle {st_ref['ratio']:.4e}")
    assert err <= 1e-12
    assert np.abs(st["sumF"] - st_ref["sumF"]).max() <= 1e-12 * st_ref["sumAbsF"]


@pytest.mark.timeout(600)
def test_binary_2x2e18_kdk_100_steps_com_identities():
    x0, m, h = W.polytrope_binary(1 << 18, 2)
    n, dt, steps = len(m), 1e-3, 100
    say(f"[gpu full] binary 2x2^18: {steps} KDK steps, dt={dt}, per-step momentum statistics")
    X, Mt, H = to_dev(x0, m, h)
    V = torch.zeros_like(X)
    g = F.GravityFMM(theta=0.5)
    A = torch.empty_like(X)
    try:
        g.forces(X, Mt, H, out=A)
        st = [F.fmm_momentum_stats(X, V, Mt, A)]
        for _ in range(steps):
            F.fmm_kick_drift(X, V, A, 0.5 * dt, dt)
            g.forces(X, Mt, H, out=A)
            F.fmm_kick_drift(X, V, A, 0.5 * dt, 0.0)
            st.append(F.fmm_momentum_stats(X, V, Mt, A))
    finally:
        g.free()
    M = st[0]["mass"]
    for k in range(steps):
        s0, s1 = st[k], st[k + 1]
        F0, F1 = s0["sumF"], s1["sumF"]
        V0, V1 = s0["P"] / M, s1["P"] / M
        dV = dt / (2 * M) * (F0 + F1)
        dX = dt * V0 + dt * dt / (2 * M) * F0
        scale_v = dt / M * max(s0["sumAbsF"], s1["sumAbsF"])
        assert np.abs((V1 - V0) - dV).max() <= 1e-9 * scale_v + 1e-15
        assert np.abs((s1["xcom"] - s0["xcom"]) - dX).max() <= 1e-12 * (1 + np.abs(dX).max())
    drift = np.linalg.norm(st[-1]["xcom"] - st[0]["xcom"])
    ratios = np.array([s["ratio"] for s in st])
    say(f"    |sumF|/sum|F|: first {ratios[0]:.3e} mean {ratios.mean():.3e} last {ratios[-1]:.3e}; "
        f"centre-of-mass drift after {steps} steps {drift:.3e}")
    assert (ratios > 0).all() and (ratios < 1e-4).all()


@pytest.mark.timeout(900)
def test_clumpy_2e22_precision_forms(orc):
    x, m, h = W.clumpy_cube(1 << 22, 3)
    n = len(m)
    say(f"[gpu full] clumpy 2^22: FP64 and FP32 forms, oracle FMM and sampled direct sum")
    a64, _, _ = gpu_run(x, m, h, export=False)
    a32, _, _ = gpu_run(x, m, h, precision=F.FMM_FP32, export=False)
    ref = orc.fmm(x, m, h)
    err64 = force_err(a64, ref.a)
    rel32 = _rel_rows(a32, ref.a)
    e32 = eta(a32, ref.a)
    sinks = np.random.default_rng(9).choice(n, 512, replace=False)
    d = orc.direct_sinks(x, m, h, sinks)
    e64d, e32d, eod = eta(a64[sinks], d), eta(a32[sinks], d), eta(ref.a[sinks], d)
    r64, r32, rref = (orc.stats(x, None, m, a)["ratio"] for a in (a64, a32, ref.a))
    say(f"    FP64 vs oracle FMM: max rel {err64:.3e}")
    say(f"    FP32 vs FP64 oracle FMM: eta {e32:.3e}, median {np.median(rel32):.3e}, "
        f"p99 {np.percentile(rel32, 99):.3e}, max {rel32.max():.3e}")
    say(f"    vs direct (512 sinks): eta FP64 {e64d:.3e}, FP32 {e32d:.3e}, oracle FMM {eod:.3e}")
    say(f"    |sumF|/sum|F|: FP64 {r64:.4e}, FP32 {r32:.4e}, oracle {rref:.4e}")
    assert err64 <= 1e-12
    assert e32 <= 1e-5 and np.percentile(rel32, 99) <= 1e-4
    # the error against the direct sum is the method's: the GPU's equals the
    # oracle FMM's on the same sinks (FP64 to round-off, FP32 to its own error)
    assert abs(e64d - eod) <= 1e-9 * eod and abs(e32d - eod) <= 1e-4 * eod + 1e-7
    assert abs(r64 - rref) <= 1e-10 and abs(r32 - rref) <= 1e-3 * rref + 1e-8


def _frozen_forces(tree, X, Mt, H, out):
    F.fmm_moments(tree, X, Mt, H)
    F.fmm_forces(tree, out, 0)
    return out


@pytest.mark.timeout(600)
def test_plummer_2e20_vjp_fp32_forward():
    x, m, h = W.plummer(1 << 20, 4)
    n = len(m)
    abar = W.cotangent(n, 41)
    say(f"[gpu full] Plummer 2^20: FP32 forward, VJP vs FP64 frozen-list finite differences")
    X, Mt, H, AB = to_dev(x, m, h, abar)
    p32 = F.default_params(precision=F.FMM_FP32)
    t32 = F.fmm_build_tree(X, p32)
    t64 = F.fmm_build_tree(X, F.default_params())
    try:
        F.fmm_moments(t32, X, Mt, H)
        A32 = torch.empty((n, 3), dtype=torch.float32, device="cuda")
        F.fmm_forces(t32, A32)
        XB = torch.empty((n, 3), dtype=torch.float32, device="cuda")
        MB = torch.empty(n, dtype=torch.float32, device="cuda")
        F.fmm_forces_vjp(t32, AB.float(), XB, MB)
        xb, mb = XB.double(), MB.double()
        A64 = torch.empty((n, 3), dtype=torch.float64, device="cuda")
        F.fmm_moments(t64, X, Mt, H)
        F.fmm_forces(t64, A64)           # lists of the unperturbed positions
        rng = np.random.default_rng(43)
        eps = 1e-4
        worst = 0.0
        for k in range(4):
            e = torch.from_numpy(rng.standard_normal((n, 3))).cuda()
            e /= torch.linalg.norm(e)
            jp = float((AB * _frozen_forces(t64, X + eps * e, Mt, H, A64)).sum())
            jm = float((AB * _frozen_forces(t64, X - eps * e, Mt, H, A64)).sum())
            fd, an = (jp - jm) / (2 * eps), float((xb * e).sum())
            worst = max(worst, abs(fd - an) / float(torch.linalg.norm(xb)))
            em = torch.from_numpy(rng.standard_normal(n)).cuda()
            em /= torch.linalg.norm(em)
            ep = eps * float(Mt.mean())
            jp = float((AB * _frozen_forces(t64, X, Mt + ep * em, H, A64)).sum())
            jm = float((AB * _frozen_forces(t64, X, Mt - ep * em, H, A64)).sum())
            fd, an = (jp - jm) / (2 * ep), float((mb * em).sum())
            worst = max(worst, abs(fd - an) / float(torch.linalg.norm(mb)))
    finally:
        F.fmm_tree_free(t32)
        F.fmm_tree_free(t64)
    say(f"    worst |FD - VJP| / |grad| over 4 x and 4 m directions: {worst:.3e}")
    assert worst <= 1e-5


def test_plummer_2e20_subset_direct_adjoint(orc):
    # the first 4096 particles of the Plummer 2^20 set as their own system
    # (m = 1/4096): the VJP of the FP32-forward tree against the oracle's
    # direct-sum adjoint, which it matches up to the FMM truncation (at most
    # ten times the forward error eta of the same tree)
    x, _, h = W.plummer(1 << 20, 4)
    x, h = x[:4096].copy(), h[:4096].copy()
    m = np.full(4096, 1.0 / 4096)
    abar = W.cotangent(1 << 20, 41)[:4096].copy()
    say("[gpu full] Plummer 2^20, first 4096 particles: VJP vs the direct-sum adjoint")
    a, [(xb, mb)] = gpu_vjp(x, m, h, abar, precision=F.FMM_FP32)
    d = orc.direct(x, m, h)
    eta_fwd = eta(a, d)
    xr, mr = orc.direct_vjp(x, m, h, abar)
    ex = np.linalg.norm(xb - xr) / np.linalg.norm(xr)
    em = np.linalg.norm(mb - mr) / np.linalg.norm(mr)
    say(f"    forward eta {eta_fwd:.2e}; relative difference: xbar {ex:.2e}, mbar {em:.2e}")
    assert ex <= 10 * eta_fwd and em <= 10 * eta_fwd


@pytest.mark.timeout(900)
def test_binary_2x2e23_backward_through_10_steps():
    x0, m, h = W.polytrope_binary(1 << 23, 5)
    n, dt, steps = len(m), 1e-3, 10
    say(f"[gpu full] binary 2x2^23: FP32 forward + checkpointed backward, {steps} KDK steps")
    X0, Mt, H = to_dev(x0, m, h)
    V0 = torch.zeros_like(X0)
    u = torch.from_numpy(np.random.default_rng(47).standard_normal((n, 3))).cuda()
    field = LF.ForceField(theta=0.5, precision=F.FMM_FP32)
    try:
        # warm-up pass (allocations, list capacities), then the timed pass
        LF.kdk_forward(X0, V0, Mt, H, dt, 1, field, keep=False)
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        t0 = time.perf_counter()
        xT, vT, ckpt = LF.kdk_forward(X0, V0, Mt, H, dt, steps, field)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L, gxT, gx0, gm = LF.com_drift_loss_grad(X0, xT, Mt)
        xbar, _, mbar = LF.kdk_backward(ckpt, Mt, H, dt, field, gxT, torch.zeros_like(vT))
        grad_x0 = xbar + gx0
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        peak = torch.cuda.max_memory_allocated() + F.fmm_tree_device_bytes(field.g.tree)
        say(f"    forward {t1 - t0:.3f} s, backward {t2 - t1:.3f} s: "
            f"{n * steps / (t2 - t0):.4e} particle-forces/s (forward + backward)")
        # adjoint of J = <u, v_T> (no identity part: a pure force-Jacobian check)
        xu, _, _ = LF.kdk_backward(ckpt, Mt, H, dt, field, torch.zeros_like(xT), u)
    finally:
        field.free()
    assert torch.isfinite(grad_x0).all() and torch.isfinite(mbar).all()
    # finite differences of J with every step's tree and lists held at the
    # forward pass's (FP64 frozen-list forces, trees built on the checkpoints)
    t = None
    A = torch.empty_like(X0)

    def J(xs):
        nonlocal t
        x, v = xs.clone(), torch.zeros_like(xs)
        for k in range(steps + 1):
            t = F.fmm_build_tree(ckpt[k], F.default_params(), tree=t)
            F.fmm_moments(t, ckpt[k], Mt, H)
            F.fmm_forces(t, A, F.FMM_REWALK)
            a = _frozen_forces(t, x, Mt, H, A)
            if k > 0:
                v += 0.5 * dt * a
            if k < steps:
                v += 0.5 * dt * a
                x += dt * v
        return float((u * v).sum())

    rng = np.random.default_rng(53)
    try:
        worst = 0.0
        for _ in range(2):
            e = torch.from_numpy(rng.standard_normal((n, 3))).cuda()
            e /= torch.linalg.norm(e)
            eps = 1e-3
            fd = (J(X0 + eps * e) - J(X0 - eps * e)) / (2 * eps)
            an = float((xu * e).sum())
            worst = max(worst, abs(an - fd) / float(torch.linalg.norm(xu)))
            say(f"    d<u, v_T>/dx_0 along e: backward {an:.6e}, FD {fd:.6e}")
    finally:
        if t is not None:
            F.fmm_tree_free(t)
    say(f"    loss |x_com(T)-x_com(0)|^2 = {L:.4e}; |dL/dx_0| = {float(torch.linalg.norm(grad_x0)):.3e}; "
        f"peak HBM (torch + library) {peak / 2**30:.2f} GiB; worst rel FD mismatch {worst:.3e}")
    assert worst <= 1e-5


def _check_tree_records(ex, tree, mom):
    np.testing.assert_array_equal(ex["perm"], tree.perm)
    for k in ("first", "count", "left", "right", "axis"):
        np.testing.assert_array_equal(ex[k], getattr(tree, k))
    rec = ex["rec"]
    np.testing.assert_array_equal(rec[:, 0], mom.M)
    np.testing.assert_array_equal(rec[:, 1:4], mom.c)
    np.testing.assert_array_equal(rec[:, 4], mom.s)
    np.testing.assert_array_equal(rec[:, 5], mom.hmax)
    scale = (mom.M * mom.s ** 2)[:, None]
    assert (np.abs(rec[:, 6:12] - mom.Q) <= 1e-14 * scale + 1e-300).all()


def test_tied_grid_2e20_tree_against_oracle(orc):
    # 2^20 particles on a 64^3 grid, half of them moved by 1e-9: cells of this
    # size take their sides by rank at every level, and ties of the split
    # coordinate are decided by Morton rank exactly as the oracle decides them
    rng = np.random.default_rng(61)
    n = 1 << 20
    x = np.round(rng.random((n, 3)) * 64) / 64
    x += 1e-9 * rng.standard_normal((n, 3)) * (rng.random((n, 1)) < 0.5)
    m, h = np.full(n, 1.0 / n), np.full(n, 0.02)
    say(f"[gpu full] tied grid 2^20: tree and records bit-exact against the oracle")
    X, Mt, H = to_dev(x, m, h)
    t = F.fmm_build_tree(X, F.default_params())
    try:
        F.fmm_moments(t, X, Mt, H)
        torch.cuda.synchronize()
        ex = F.fmm_debug_export(t, lists=False)
    finally:
        F.fmm_tree_free(t)
    tree = orc.build_tree(x, 8)
    mom = orc.moments(x, m, h, tree)
    _check_tree_records(ex, tree, mom)


@pytest.mark.timeout(900)
def test_binary_2x2e23_step0_against_oracle(orc):
    x, m, h = W.polytrope_binary(1 << 23, 5)
    n = len(m)
    say(f"[gpu full] binary 2x2^23 step 0, FP64: tree bit-exact, 2048 sampled leaves vs oracle")
    X, Mt, H = to_dev(x, m, h)
    t = F.fmm_build_tree(X, F.default_params())
    try:
        F.fmm_moments(t, X, Mt, H)
        A = torch.empty_like(X)
        F.fmm_forces(t, A)
        torch.cuda.synchronize()
        ex = F.fmm_debug_export(t, lists="offsets")
        a = A.cpu().numpy()
    finally:
        F.fmm_tree_free(t)
    del X, Mt, H, A
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    tree = orc.build_tree(x, 8)
    mom = orc.moments(x, m, h, tree)
    say(f"    oracle tree and moments of {n} particles: {time.perf_counter() - t0:.1f} s")
    _check_tree_records(ex, tree, mom)
    leaves = np.flatnonzero(tree.left < 0)
    sel = np.sort(np.random.default_rng(59).choice(leaves, 2048, replace=False))
    ao, cnt = orc.fmm_leaves(x, m, h, tree, mom, sel, counts=True)
    np.testing.assert_array_equal(np.diff(ex["far_off"])[sel], cnt[:, 0])
    np.testing.assert_array_equal(np.diff(ex["near_off"])[sel], cnt[:, 1])
    rows = np.concatenate([tree.perm[tree.first[v]:tree.first[v] + tree.count[v]] for v in sel])
    err = force_err(a[rows], ao[rows])
    say(f"    {len(rows)} particles of {len(sel)} leaves ({cnt[:, 0].mean():.0f} far, "
        f"{cnt[:, 1].mean():.0f} near cells per leaf): max rel force error {err:.3e}")
    assert err <= 1e-12


@pytest.mark.timeout(900)
def test_binary_2x2e18_first_10_kdk_steps_against_oracle(orc):
    x0, m, h = W.polytrope_binary(1 << 18, 2)
    n, dt, steps = len(m), 1e-3, 10
    say(f"[gpu full] binary 2x2^18: {steps} KDK steps, theta 0.5, every step against the oracle")
    X, Mt, H = to_dev(x0, m, h)
    V = torch.zeros_like(X)
    A = torch.empty_like(X)
    g = F.GravityFMM(theta=0.5)
    xs, vs, as_ = [], [], []
    try:
        g.forces(X, Mt, H, out=A)
        xs.append(X.cpu().numpy()), vs.append(V.cpu().numpy()), as_.append(A.cpu().numpy())
        for _ in range(steps):
            F.fmm_kick_drift(X, V, A, 0.5 * dt, dt)
            g.forces(X, Mt, H, out=A)
            F.fmm_kick_drift(X, V, A, 0.5 * dt, 0.0)
            xs.append(X.cpu().numpy()), vs.append(V.cpu().numpy()), as_.append(A.cpu().numpy())
    finally:
        g.free()
    # (1) every step: the oracle's forces at the GPU's positions, and the KDK
    # update of the GPU's state repeated on the host (same two operations per
    # component, so bit for bit)
    worst = 0.0
    for k in range(steps + 1):
        ao, _, _ = oracle_fmm_threaded(orc, xs[k], m, h, theta=0.5)
        err = force_err(as_[k], ao)
        sg, so = orc.stats(xs[k], None, m, as_[k]), orc.stats(xs[k], None, m, ao)
        worst = max(worst, err)
        assert err <= 1e-12, (k, err)
        assert np.abs(sg["sumF"] - so["sumF"]).max() <= 1e-12 * so["sumAbsF"], k
        if k < steps:
            vh = vs[k] + (0.5 * dt) * as_[k]
            np.testing.assert_array_equal(xs[k + 1], xs[k] + dt * vh)
            np.testing.assert_array_equal(vs[k + 1], vh + (0.5 * dt) * as_[k + 1])
    # (2) the oracle's own trajectory from the same start
    xo, vo = x0.copy(), np.zeros_like(x0)
    ao, _, _ = oracle_fmm_threaded(orc, xo, m, h, theta=0.5)
    dx_max = dF_max = 0.0
    for k in range(steps):
        vo = vo + (0.5 * dt) * ao
        xo = xo + dt * vo
        ao, _, _ = oracle_fmm_threaded(orc, xo, m, h, theta=0.5)
        vo = vo + (0.5 * dt) * ao
        dx = np.abs(xo - xs[k + 1]).max() / np.abs(xo).max()
        so, sg = orc.stats(xo, vo, m, ao), orc.stats(xs[k + 1], vs[k + 1], m, as_[k + 1])
        dF = np.abs(so["sumF"] - sg["sumF"]).max() / so["sumAbsF"]
        dx_max, dF_max = max(dx_max, dx), max(dF_max, dF)
        assert dx <= 1e-12 and dF <= 1e-12, (k, dx, dF)
    say(f"    forces at the GPU's positions: worst max rel error {worst:.2e}; oracle's own "
        f"trajectory: positions {dx_max:.2e}, sum F {dF_max:.2e} of sum |F|")
