"""Long interaction lists split into pieces (several wavefronts per sink
leaf, partial sums folded in piece order): for a given piece size the forces
and the reverse pass are bit-identical to those of whole lists summed piece
by piece, and match the oracle FMM to 1e-12; the split is taken after a walk
that found long lists, so the second call of a tree uses it.  Small pieces
(the FMM_MI355_PIECE hook) make ordinary trees split."""
import os

import numpy as np
import pytest
import torch

from paper_2502_01496_amd import fmm as F
from paper_2502_01496_amd import workloads as W
from tests.gpu_util import force_err, say, to_dev

pytestmark = pytest.mark.gpu


def _forces_twice(x, m, h, piece=None, **kw):
    """Forces of a fresh tree, then again after a rewalk (when a split
    predicted by the first walk applies), then on the kept lists."""
    old = os.environ.get("FMM_MI355_PIECE")
    if piece is not None:
        os.environ["FMM_MI355_PIECE"] = str(piece)
    try:
        X, Mt, H = to_dev(x, m, h)
        p = F.default_params(**kw)
        t = F.fmm_build_tree(X, p)
    finally:
        if piece is not None:
            if old is None:
                del os.environ["FMM_MI355_PIECE"]
            else:
                os.environ["FMM_MI355_PIECE"] = old
    dt = torch.float32 if p.precision == F.FMM_FP32 else torch.float64
    out = []
    AB = torch.from_numpy(W.cotangent(len(m), 5)).cuda().to(dt)

    def vjp():
        XB = torch.empty((len(m), 3), dtype=dt, device="cuda")
        MB = torch.empty(len(m), dtype=dt, device="cuda")
        F.fmm_forces_vjp(t, AB, XB, MB)
        torch.cuda.synchronize()
        return XB.cpu().numpy(), MB.cpu().numpy()

    try:
        F.fmm_moments(t, X, Mt, H)
        for flags in (0, F.FMM_REWALK, 0):
            A = torch.empty((len(m), 3), dtype=dt, device="cuda")
            F.fmm_forces(t, A, flags)
            torch.cuda.synchronize()
            out.append(A.cpu().numpy())
            if len(out) == 1:
                # after the first walk the sink side of the reverse pass still
                # takes whole lists (summed piece by piece)
                first_vjp = vjp()
        out.append(vjp())
        out.append(first_vjp)
    finally:
        F.fmm_tree_free(t)
    return out


@pytest.mark.parametrize("precision", [F.FMM_FP64, F.FMM_FP32])
@pytest.mark.parametrize("expansion", [F.FMM_EXPANSION_PHANTOM, F.FMM_EXPANSION_DEHNEN])
@pytest.mark.parametrize("piece", [1, 3, 7])
def test_split_lists_bit_identical(orc, precision, expansion, piece):
    x, m, h = W.clumpy_cube(20000, 41, n_clumps=5, cache=False)
    say(f"[gpu pieces] clumpy 20000, precision {precision}, form {expansion}, pieces of {piece}")
    whole = _forces_twice(x, m, h, precision=precision, expansion=expansion)
    split = _forces_twice(x, m, h, piece=piece, precision=precision, expansion=expansion)
    # with one piece size, the first call (whole lists, summed piece by piece)
    # and the later calls (pieces on separate wavefronts, then folded) agree
    # bit for bit
    np.testing.assert_array_equal(split[1], split[0])
    np.testing.assert_array_equal(split[2], split[0])
    # the reverse pass too: whole lists and split lists, one piece size
    for k in range(2):
        np.testing.assert_array_equal(split[3][k], split[4][k])
    # other piece sizes only re-associate the sums
    tol = 1e-12 if precision == F.FMM_FP64 else 1e-5
    assert force_err(split[1], whole[1]) <= tol
    for k in range(2):
        d = np.abs(split[3][k] - whole[3][k]).max() / np.abs(whole[3][k]).max()
        assert d <= tol
    if precision == F.FMM_FP64:
        ref = orc.fmm(x, m, h, form=expansion)
        assert force_err(split[1], ref.a) <= 1e-12
        assert force_err(whole[1], ref.a) <= 1e-12


def test_plummer_long_lists_split_by_default(orc):
    # the untruncated Plummer sphere: halo leaves with very long lists
    x, m, h = W.plummer(1 << 17, 42)
    say("[gpu pieces] Plummer 2^17: lists long enough to split without the hook")
    X, Mt, H = to_dev(x, m, h)
    t = F.fmm_build_tree(X, F.default_params())
    try:
        F.fmm_moments(t, X, Mt, H)
        A = torch.empty_like(X)
        F.fmm_forces(t, A)
        ex = F.fmm_debug_export(t, lists="offsets")
        a1 = A.cpu().numpy()
        F.fmm_forces(t, A, F.FMM_REWALK)
        torch.cuda.synchronize()
        a2 = A.cpu().numpy()
    finally:
        F.fmm_tree_free(t)
    longest = max(np.diff(ex["near_off"]).max(), np.diff(ex["far_off"]).max() // 2)
    say(f"    longest near list {np.diff(ex['near_off']).max()}, far {np.diff(ex['far_off']).max()}")
    assert longest > 512
    np.testing.assert_array_equal(a1, a2)
    ref = orc.fmm(x, m, h)
    assert force_err(a2, ref.a) <= 1e-12
