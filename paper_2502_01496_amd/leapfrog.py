"""Kick-drift-kick leapfrog over the FMM forces, its checkpointed adjoint, and
a torch.autograd.Function for one force evaluation.

Forward step (fixed dt), with a(x) the FMM accelerations:
    v <- v + dt/2 a(x);   x <- x + dt v;   v <- v + dt/2 a(x)
The adjoint of T steps needs a(x) and its VJP at every visited position
x_0..x_T and nothing else (the forces depend on x only), so the forward keeps
the positions as checkpoints and the reverse sweep rebuilds the tree at each
checkpoint (the build is deterministic, so the tree and the interaction lists
are those of the forward pass) and walks it without evaluating the forces
again.  The two half kicks that act at x_k (the last
of step k-1 and the first of step k) carry the same cotangent, so one VJP per
checkpoint suffices:

    xbar, vbar <- dL/dx_T, dL/dv_T;   (xbar, mbar) += VJP(x_T; dt/2 vbar)
    for k = T-1 .. 0:
        vbar <- vbar + dt xbar                       (drift)
        (xbar, mbar) += VJP(x_k; c vbar),  c = dt (k > 0), dt/2 (k = 0)

The force evaluations and VJPs run in the library's kernels; the O(N) adjoint
updates are elementwise tensor operations.
"""
from __future__ import annotations

import torch

from . import fmm as F


class ForceField:
    """One tree reused for every evaluation at a fixed particle count."""

    def __init__(self, theta=0.5, leaf_size=8, G=1.0, precision=F.FMM_FP64, r_kern=2.0,
                 walk=F.FMM_WALK_PHANTOM, expansion=F.FMM_EXPANSION_PHANTOM,
                 tree_shape=F.FMM_TREE_MEDIAN):
        self.g = F.GravityFMM(theta=theta, leaf_size=leaf_size, G=G, precision=precision,
                              r_kern=r_kern, walk=walk, expansion=expansion,
                              tree_shape=tree_shape)
        self.generation = 0          # bumped by every build
        self.dtype = torch.float32 if precision == F.FMM_FP32 else torch.float64

    def forces(self, x, m, h, out=None):
        """Build the tree at x, then moments, walk and forces."""
        self.g.build(x, m=m)
        self.generation += 1
        F.fmm_moments(self.g.tree, x, m, h)
        if out is None:
            out = torch.empty((x.shape[0], 3), dtype=self.dtype, device=x.device)
        F.fmm_forces(self.g.tree, out, F.FMM_REWALK)
        return out

    def prepare_vjp(self, x, m, h):
        """Build the tree at x, then moments and walk: the state the reverse
        pass needs, without evaluating the forces (they are known from the
        forward sweep)."""
        self.g.build(x, m=m)
        self.generation += 1
        F.fmm_moments(self.g.tree, x, m, h)
        F.fmm_forces(self.g.tree, None, F.FMM_REWALK | F.FMM_VJP_ONLY)

    def vjp(self, abar):
        """VJP of the last forces() call: (xbar, mbar) in the force dtype."""
        n = abar.shape[0]
        xb = torch.empty((n, 3), dtype=self.dtype, device=abar.device)
        mb = torch.empty(n, dtype=self.dtype, device=abar.device)
        F.fmm_forces_vjp(self.g.tree, abar.to(self.dtype).contiguous(), xb, mb)
        return xb, mb

    def free(self):
        self.g.free()


class FmmForce(torch.autograd.Function):
    """a = FMM accelerations of (x, m) with smoothing lengths h.

    The backward pass is the library VJP with the tree and interaction lists
    of this forward call held fixed.  If the ForceField evaluated other
    positions in between, the tree is rebuilt at the saved positions first
    (deterministic, so the lists are the same)."""

    @staticmethod
    def forward(ctx, x, m, h, field: ForceField):
        a = field.forces(x.detach(), m.detach(), h.detach())
        ctx.field = field
        ctx.gen = field.generation
        ctx.save_for_backward(x.detach(), m.detach(), h.detach())
        return a

    @staticmethod
    def backward(ctx, abar):
        field = ctx.field
        x, m, h = ctx.saved_tensors
        if field.generation != ctx.gen:
            field.forces(x, m, h)
        xb, mb = field.vjp(abar.contiguous())
        return xb.to(x.dtype), mb.to(m.dtype), None, None


def kdk_forward(x0, v0, m, h, dt, steps, field: ForceField, keep=True, on_step=None):
    """Run KDK steps; returns (x_T, v_T, checkpoints [x_0..x_T] or None)."""
    x = x0.clone()
    v = v0.clone()
    a = field.forces(x, m, h)
    ckpt = [x.clone()] if keep else None
    for k in range(steps):
        F.fmm_kick_drift(x, v, a, 0.5 * dt, dt)
        field.forces(x, m, h, out=a)
        F.fmm_kick_drift(x, v, a, 0.5 * dt, 0.0)
        if keep:
            ckpt.append(x.clone())
        if on_step is not None:
            on_step(k, x, v, a)
    return x, v, ckpt


def kdk_backward(ckpt, m, h, dt, field: ForceField, xbar_T, vbar_T):
    """Reverse sweep over the checkpoints; returns (xbar_0, vbar_0, mbar)."""
    T = len(ckpt) - 1
    xbar = xbar_T.to(torch.float64).clone()
    vbar = vbar_T.to(torch.float64).clone()
    mbar = torch.zeros_like(m, dtype=torch.float64)
    field.prepare_vjp(ckpt[T], m, h)
    xb, mb = field.vjp(0.5 * dt * vbar)
    xbar += xb.double()
    mbar += mb.double()
    for k in range(T - 1, -1, -1):
        vbar += dt * xbar
        field.prepare_vjp(ckpt[k], m, h)
        c = dt if k > 0 else 0.5 * dt
        xb, mb = field.vjp(c * vbar)
        xbar += xb.double()
        mbar += mb.double()
    return xbar, vbar, mbar


def com_drift_loss_grad(x0, xT, m):
    """L = |X_T - X_0|^2 with X the centre of mass; returns (L, dL/dx_T,
    dL/dx_0 (direct part), dL/dm (direct part))."""
    M = m.sum()
    X0 = (m[:, None] * x0).sum(0) / M
    XT = (m[:, None] * xT).sum(0) / M
    D = XT - X0
    L = float((D * D).sum())
    gxT = (2.0 / M) * m[:, None] * D[None, :]
    gx0 = -gxT
    # elementwise product and row sum (a matrix-vector call fails for very
    # tall matrices in the BLAS library)
    gm = (2.0 / M) * (((xT - XT) - (x0 - X0)) * D[None, :]).sum(1)
    return L, gxT, gx0, gm


def com_drift_gradient(x0, v0, m, h, dt, steps, field: ForceField):
    """Loss |X_T - X_0|^2 after `steps` KDK steps and its gradient with respect
    to the initial positions and the masses (forward with per-step position
    checkpoints, then the reverse sweep)."""
    xT, vT, ckpt = kdk_forward(x0, v0, m, h, dt, steps, field)
    L, gxT, gx0, gm = com_drift_loss_grad(x0, xT, m)
    xbar, vbar, mbar = kdk_backward(ckpt, m, h, dt, field, gxT, torch.zeros_like(vT))
    return L, xbar + gx0, mbar + gm, vbar
