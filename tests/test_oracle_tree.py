"""Pins for the oracle's Morton order, kd-tree, cell properties and walks."""
import numpy as np
import pytest

from paper_2502_01496_amd import workloads as W


def ordkey(v):
    b = np.frombuffer(np.float64(v).tobytes(), np.uint64)[0]
    return int(~b & 0xFFFFFFFFFFFFFFFF) if b >> 63 else int(b | (1 << 63))


def test_morton_brute_force(orc):
    rng = np.random.default_rng(11)
    x = rng.standard_normal((500, 3))
    x[7] = x[3]  # a tie
    key, order = orc.morton(x)
    lo = x.min(0)
    ext = (x.max(0) - lo).max()
    for i in range(len(x)):
        q = [min(2 ** 21 - 1, int(np.floor((x[i, d] - lo[d]) * (2 ** 21 / ext)))) for d in range(3)]
        k = 0
        for b in range(21):
            for d in range(3):
                k |= ((q[d] >> b) & 1) << (3 * b + d)
        assert int(key[i]) == k
    ref = sorted(range(len(x)), key=lambda i: (int(key[i]), i))
    assert list(order) == ref


def check_tree(x, tree, leaf_size):
    n = len(x)
    rank = np.empty(n, int)
    _, order = __import__("oracle.oracle", fromlist=["morton"]).morton(x)
    rank[order] = np.arange(n)
    assert sorted(tree.perm) == list(range(n))
    assert tree.first[0] == 0 and tree.count[0] == n
    leaves = np.flatnonzero(tree.is_leaf)
    # leaves partition [0, n) left to right
    pos = 0
    for v in leaves:
        assert tree.first[v] == pos and 1 <= tree.count[v] <= leaf_size
        pos += tree.count[v]
    assert pos == n
    for v in np.flatnonzero(~tree.is_leaf):
        f, c = tree.first[v], tree.count[v]
        l, r = tree.left[v], tree.right[v]
        assert c > leaf_size
        assert l == v + 1  # pre-order
        assert tree.first[l] == f and tree.count[l] == (c + 1) // 2
        assert tree.first[r] == f + tree.count[l] and tree.count[r] == c // 2
        idx = tree.perm[f:f + c]
        ext = x[idx].max(0) - x[idx].min(0)
        d = tree.axis[v]
        assert d == int(np.argmax(ext))  # first maximum: ties -> lowest axis
        kl = [(ordkey(x[i, d]), rank[i]) for i in tree.perm[f:f + tree.count[l]]]
        kr = [(ordkey(x[i, d]), rank[i]) for i in tree.perm[tree.first[r]:f + c]]
        assert max(kl) < min(kr)
    for v in leaves:
        idx = tree.perm[tree.first[v]:tree.first[v] + tree.count[v]]
        assert (np.diff(rank[idx]) > 0).all()  # ascending Morton rank inside a leaf


@pytest.mark.parametrize("n,leaf", [(1, 8), (8, 8), (9, 8), (100, 8), (1000, 8), (777, 3), (4096, 10)])
def test_tree_invariants(orc, n, leaf):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, 3)) * np.array([1.0, 0.5, 2.0])
    check_tree(x, orc.build_tree(x, leaf), leaf)


def test_tree_ties_and_degenerate(orc):
    rng = np.random.default_rng(2)
    x = np.round(rng.random((300, 3)) * 4) / 4  # many tied coordinates
    check_tree(x, orc.build_tree(x, 8), 8)
    x = np.zeros((50, 3))
    t = orc.build_tree(x, 8)
    check_tree(x, t, 8)
    assert list(t.perm) == list(range(50))


def test_balanced_tree_shape(orc):
    x, m, h = W.plummer(4096, 1)
    t = orc.build_tree(x, 8)
    assert t.nnodes == 1023 and (t.count[t.is_leaf] == 8).all()


def test_moments_against_direct_p2m(orc):
    x, m, h = W.plummer(1000, 3)
    m = m * (1 + np.random.default_rng(0).random(1000))
    t = orc.build_tree(x, 8)
    mom = orc.moments(x, m, h, t)
    for v in range(t.nnodes):
        idx = t.perm[t.first[v]:t.first[v] + t.count[v]]
        M, c, Q = orc.p2m(x[idx], m[idx])
        assert mom.M[v] == pytest.approx(M, rel=1e-14)
        np.testing.assert_allclose(mom.c[v], c, rtol=0, atol=1e-13 * (1 + np.abs(c).max()))
        sref = np.sqrt(((x[idx] - mom.c[v]) ** 2).sum(1).max())
        assert mom.s[v] == pytest.approx(sref, rel=1e-15)
        assert mom.hmax[v] == h[idx].max()
        scale = M * sref ** 2
        np.testing.assert_allclose(mom.Q[v], Q, rtol=0, atol=1e-12 * scale)


def accept(mom, a, b, theta, r_kern):
    d = mom.c[a] - mom.c[b]
    r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    open4 = mom.s[b] ** 2 > theta ** 2 * r2
    t = (mom.s[a] + mom.s[b]) + r_kern * max(mom.hmax[a], mom.hmax[b])
    return not (open4 or r2 < t * t)


def ancestors(tree, v):
    par = {}
    for u in range(tree.nnodes):
        if tree.left[u] >= 0:
            par[tree.left[u]] = u
            par[tree.right[u]] = u
    out = []
    while v in par:
        v = par[v]
        out.append(v)
    return out


@pytest.mark.parametrize("n,theta", [(64, 0.5), (64, 1.0), (60, 0.3), (200, 0.7)])
def test_phantom_walk_brute_force(orc, n, theta):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, 3))
    m = rng.random(n) + 0.5
    h = rng.random(n) * 0.05 + 0.01
    t = orc.build_tree(x, 4)
    mom = orc.moments(x, m, h, t)
    L = orc.walk(t, mom, theta, 2.0, orc.PHANTOM)
    anc = {v: ancestors(t, v) for v in range(t.nnodes)}
    for a in range(t.nnodes):
        if not t.is_leaf[a]:
            assert len(L.far(a)) == 0 and len(L.near(a)) == 0
            continue
        far_ref = [b for b in range(t.nnodes)
                   if accept(mom, a, b, theta, 2.0)
                   and all(not accept(mom, a, u, theta, 2.0) for u in anc[b])]
        near_ref = [b for b in range(t.nnodes) if t.is_leaf[b]
                    and not accept(mom, a, b, theta, 2.0)
                    and all(not accept(mom, a, u, theta, 2.0) for u in anc[b])]
        assert list(L.far(a)) == sorted(far_ref, key=lambda b: t.first[b])
        assert list(L.near(a)) == sorted(near_ref, key=lambda b: t.first[b])
        assert a in L.near(a)
        covered = np.zeros(n, int)
        for b in list(L.far(a)) + list(L.near(a)):
            covered[t.first[b]:t.first[b] + t.count[b]] += 1
        assert (covered == 1).all()  # far + near partition all particles


def test_mutual_walk_is_symmetric_and_covers_all_pairs(orc):
    rng = np.random.default_rng(5)
    n = 300
    x = rng.standard_normal((n, 3))
    m = rng.random(n) + 0.5
    h = np.full(n, 0.02)
    t = orc.build_tree(x, 8)
    mom = orc.moments(x, m, h, t)
    L = orc.walk(t, mom, 0.6, 2.0, orc.MUTUAL)
    for a in range(t.nnodes):
        for b in L.far(a):
            assert a in L.far(b)
            d = mom.c[a] - mom.c[b]
            r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
            assert 0.36 * r2 >= (mom.s[a] + mom.s[b]) ** 2
        for b in L.near(a):
            assert a in L.near(b) and t.is_leaf[a] and t.is_leaf[b]
    # every particle pair (i, j), i != j, is covered exactly once from i's side
    anc = {v: [v] + ancestors(t, v) for v in range(t.nnodes)}
    pos_leaf = np.empty(n, int)
    for v in np.flatnonzero(t.is_leaf):
        pos_leaf[t.first[v]:t.first[v] + t.count[v]] = v
    cnt = np.zeros((n, n), int)
    for p in range(n):
        for s in anc[pos_leaf[p]]:
            for b in list(L.far(s)) + ([] if s != pos_leaf[p] else list(L.near(s))):
                cnt[p, t.first[b]:t.first[b] + t.count[b]] += 1
    assert (cnt == 1).all()


def test_power_of_two_scaling_bit_identical(orc):
    x, m, h = W.plummer(2000, 9)
    a1 = orc.fmm(x, m, h).a
    a2 = orc.fmm(2 * x, 4 * m, 2 * h).a
    assert np.array_equal(a1, a2)


def test_permutation_invariance(orc):
    x, m, h = W.plummer(4096, 1)
    r1 = orc.fmm(x, m, h)
    p = np.random.default_rng(3).permutation(len(m))
    r2 = orc.fmm(x[p], m[p], h[p])
    assert np.array_equal(r2.a, r1.a[p])
