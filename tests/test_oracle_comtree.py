"""Pins for the oracle's kd-tree cut through the centre of mass (Sec. 2 as
written): an exact big-integer Python re-implementation of the cut rule on
small inputs (identical trees), the cut lying at the FP64 centre of mass to
within the quantisation, the longest-axis choice, leaf sizes, coincident
particles, and the FMM on it (theta = 0 is the direct sum; the leaf <- cell
walk leaves a total force, the mutual walk does not)."""
import numpy as np
import pytest

from paper_2502_01496_amd import workloads as W


def py_comtree(x, m, leaf):
    """Big-integer restatement of the cut rule (ties, grid and weights as in
    the oracle's header)."""
    n = len(x)
    lo = x.min(0)
    ext = float((x.max(0) - lo).max()) or 1.0
    scale = 4294967296.0 / ext
    q = np.floor((x - lo) * scale)
    q = np.where(q >= 4294967295.0, 4294967295.0, q).astype(np.int64)
    if m is None:
        w = np.ones(n, np.int64)
    else:
        v = np.floor(m / m.max() * 16777216.0)
        w = np.clip(v, 1, 16777216).astype(np.int64)
    # root order: Morton rank (the oracle's own key sort is pinned elsewhere)
    from oracle import oracle as O

    _, order = O.morton(x)
    order = [int(i) for i in order]
    first, count, left, right, axis = [], [], [], [], []

    def node(lo_, cnt):
        vid = len(first)
        first.append(lo_)
        count.append(cnt)
        left.append(-1)
        right.append(-1)
        axis.append(-1)
        if cnt <= leaf:
            return vid
        idx = order[lo_:lo_ + cnt]
        ext_q = [int(q[idx, d].max()) - int(q[idx, d].min()) for d in range(3)]
        ax = max(range(3), key=lambda d: (ext_q[d], -d))
        axis[vid] = ax
        if ext_q[ax] == 0:
            nl = (cnt + 1) // 2
        else:
            sw = sum(int(w[i]) for i in idx)
            swq = sum(int(w[i]) * int(q[i, ax]) for i in idx)
            L = [i for i in idx if int(q[i, ax]) * sw < swq]
            R = [i for i in idx if not int(q[i, ax]) * sw < swq]
            order[lo_:lo_ + cnt] = L + R
            nl = len(L)
        lch = node(lo_, nl)
        rch = node(lo_ + nl, cnt - nl)
        left[vid], right[vid] = lch, rch
        return vid

    node(0, n)
    return (np.array(order), np.array(first), np.array(count), np.array(left), np.array(right),
            np.array(axis))


@pytest.mark.parametrize("case", ["plummer_300_leaf10", "plummer_257_leaf1", "clumpy_400_mass",
                                  "grid_ties_200", "coincident_40"])
def test_matches_big_integer_restatement(orc, case):
    rng = np.random.default_rng(41)
    m = None
    leaf = 10
    if case == "plummer_300_leaf10":
        x, _, _ = W.plummer(300, 3)
    elif case == "plummer_257_leaf1":
        x, _, _ = W.plummer(257, 4)
        leaf = 1
    elif case == "clumpy_400_mass":
        x = rng.random((400, 3))
        x[:200] = 0.5 + 0.01 * rng.standard_normal((200, 3))
        m = np.exp(rng.standard_normal(400))
        leaf = 4
    elif case == "grid_ties_200":
        x = np.round(rng.random((200, 3)) * 4) / 4.0
        leaf = 3
    else:
        x = np.tile(np.array([[0.3, 0.3, 0.3]]), (40, 1))
        x[:5] += 1e-3 * rng.random((5, 3))
        leaf = 2
    t = orc.build_tree_com(x, m, leaf)
    got = (t.perm, t.first, t.count, t.left, t.right, t.axis)
    want = py_comtree(x, m, leaf)
    for g, w_ in zip(got, want):
        np.testing.assert_array_equal(g, w_)


def test_cut_is_at_the_centre_of_mass(orc):
    x, m, _ = W.plummer(5000, 8)
    rng = np.random.default_rng(3)
    for masses in (None, m * np.exp(0.5 * rng.standard_normal(len(m)))):
        t = orc.build_tree_com(x, masses, 10)
        mm = np.ones(len(x)) if masses is None else masses
        ext = (x.max(0) - x.min(0)).max()
        grid = ext / 2.0 ** 32
        slack_w = 0.0 if masses is None else 2.0 ** -23  # relative weight rounding
        for v in np.nonzero(t.left >= 0)[0]:
            idx = t.perm[t.first[v]:t.first[v] + t.count[v]]
            d = t.axis[v]
            xd = x[idx, d]
            ext_v = xd.max() - xd.min()
            # longest axis (up to the grid)
            assert ext_v >= (x[idx].max(0) - x[idx].min(0)).max() - 2 * grid
            c = (mm[idx] * xd).sum() / mm[idx].sum()
            tol = 2 * grid + slack_w * ext_v + 1e-12 * abs(c)
            li = t.perm[t.first[t.left[v]]:t.first[t.left[v]] + t.count[t.left[v]]]
            ri = t.perm[t.first[t.right[v]]:t.first[t.right[v]] + t.count[t.right[v]]]
            assert len(li) > 0 and len(ri) > 0
            assert x[li, d].max() < c + tol
            assert x[ri, d].min() > c - tol
        assert (t.count[t.left < 0] <= 10).all()
        assert (t.count[t.left < 0] >= 1).all()


def test_fmm_on_the_com_tree(orc):
    x, m, h = W.plummer(3000, 9)
    d = orc.direct(x, m, h)
    a0 = orc.fmm(x, m, h, theta=0.0, leaf_size=10, tree_kind=orc.COM_TREE).a
    np.testing.assert_allclose(a0, d, rtol=1e-11, atol=1e-12 * np.abs(d).max())
    r_leaf = orc.fmm(x, m, h, leaf_size=10, tree_kind=orc.COM_TREE)
    r_mut = orc.fmm(x, m, h, leaf_size=10, tree_kind=orc.COM_TREE, policy=orc.MUTUAL)
    assert orc.stats(x, None, m, r_leaf.a)["ratio"] > 1e-9
    assert orc.stats(x, None, m, r_mut.a)["ratio"] < 1e-13
    eta = np.sqrt(((r_leaf.a - d) ** 2).sum() / (d ** 2).sum())
    assert eta < 3e-2
