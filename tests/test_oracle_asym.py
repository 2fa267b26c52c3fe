"""Pins for the oracle's asymmetric-pair census and the total-force estimates
of Sec. 4 (eq. (33)) and Sec. 6 (eq. (46)): the two-leaf super-cell of Sec. 4
(eq. (33) reduces to the bound eq. (32), tests/golden/paper_sec4_eq31.json),
equal masses cancelling it, a brute-force Python evaluation of both sums on
small trees, and the lists of the two walks (every mutual pair has its
reverse; with the leaf <- cell lists every pair with a super-cell source is
asymmetric)."""
import json
import os

import numpy as np
import pytest

from paper_2502_01496_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def three_cell(orc, Ma, M1, M2, x, r):
    """root -> (alpha leaf, beta -> (beta1 leaf, beta2 leaf)), pre-order ids;
    lists: alpha <- beta, beta1 <- alpha, beta2 <- alpha (the leaf <- cell
    pattern of Sec. 4)."""
    left = np.array([1, -1, 3, -1, -1], np.int32)
    right = np.array([2, -1, 4, -1, -1], np.int32)
    Mb = M1 + M2
    M = np.array([Ma + Mb, Ma, Mb, M1, M2])
    ca = np.array([r, 0.0, 0.0])
    c1, c2 = x, -x * M1 / M2
    c = np.array([(Ma * ca) / (Ma + Mb), ca, np.zeros(3), c1, c2])
    s = np.array([r, 0.0, max(np.linalg.norm(c1), np.linalg.norm(c2)), 0.0, 0.0])
    far_off = np.array([0, 0, 1, 1, 2, 3], np.int32)
    far_src = np.array([2, 1, 1], np.int32)
    tree = orc.Tree(np.zeros(3, np.int32), np.zeros(5, np.int32), np.ones(5, np.int32), left,
                    right, np.full(5, -1, np.int32))
    mom = orc.Moments(M, c, s, np.zeros(5), np.zeros((5, 6)))
    lists = orc.Lists(far_off, far_src, np.zeros(6, np.int32), np.zeros(0, np.int32))
    return orc.asym_estimate(tree, mom, lists, m_leaf=1.0)


def test_two_leaf_supercell_is_the_bound_eq32(orc):
    g = json.load(open(os.path.join(GOLD, "paper_sec4_eq31.json")))
    Ma, M1, M2 = 1.3, 0.4, 1.1
    x = np.array([0.7, 0.45, 0.0])
    for r in (20.0, 80.0):
        est = three_cell(orc, Ma, M1, M2, x, r)
        l = np.linalg.norm(x)
        bound = g["bound_eq32"]["coefficient"] * l ** 3 * Ma * (M1 + M2) * (M1 / M2) * (
            1 - M1 / M2) / r ** 5
        assert est["F33"] == pytest.approx(bound, rel=1e-14)
        assert est["n_asym"] == 3 and est["n_asym_super"] == 1
        # eq. (46) for the same cells: N_beta = 2 leaves gives (N - 2) = 0
        assert est["F46"] == 0.0


def test_equal_masses_cancel(orc):
    est = three_cell(orc, 1.0, 0.7, 0.7, np.array([0.3, -0.2, 0.1]), 30.0)
    assert est["F33"] == 0.0


def _brute(tree, mom, lists, m_leaf):
    nn = tree.nnodes
    kids = {v: (int(tree.left[v]), int(tree.right[v])) for v in range(nn)}

    def leaves(v):
        if kids[v][0] < 0:
            return [v]
        return leaves(kids[v][0]) + leaves(kids[v][1])

    pairs = set()
    for a in range(nn):
        for b in lists.far(a):
            pairs.add((a, int(b)))
    T, U, N = {}, {}, {}
    for v in range(nn):
        lv = leaves(v)
        N[v] = len(lv)
        if len(lv) < 2:
            T[v] = U[v] = 0.0
            continue
        m1 = min(mom.M[u] for u in lv)
        l = max(np.linalg.norm(mom.c[u] - mom.c[v]) for u in lv if mom.M[u] == m1)
        rest = mom.M[v] - m1
        T[v] = m1 * l ** 3 / rest * (1 - m1 / rest)
        U[v] = mom.s[v] ** 3 * (N[v] - 2) / (N[v] - 1) ** 2
    f33 = f46 = 0.0
    nasym = nsuper = 0
    for a, b in sorted(pairs):
        if (b, a) in pairs:
            continue
        nasym += 1
        nsuper += int(N[a] >= 2 or N[b] >= 2)
        r = np.linalg.norm(mom.c[a] - mom.c[b])
        f33 += 4 * mom.M[a] * mom.M[b] / r ** 5 * (T[a] + T[b])
        f46 += 4 * m_leaf ** 2 * N[a] * N[b] / r ** 5 * (U[a] + U[b])
    return f33, f46, nasym, nsuper


@pytest.mark.parametrize("n,leaf,theta,seed", [(600, 8, 0.5, 1), (900, 3, 0.7, 2),
                                               (1024, 8, 0.4, 3)])
def test_matches_brute_force(orc, n, leaf, theta, seed):
    x, m, h = W.plummer(n, seed)
    rng = np.random.default_rng(seed)
    m = m * (0.5 + rng.random(n))  # unequal masses: the lightest leaf is unique
    tree = orc.build_tree(x, leaf)
    mom = orc.moments(x, m, h, tree)
    lists = orc.walk(tree, mom, theta)
    m_leaf = float(mom.M[0]) / int(tree.is_leaf.sum())
    est = orc.asym_estimate(tree, mom, lists)
    f33, f46, nasym, nsuper = _brute(tree, mom, lists, m_leaf)
    assert est["n_asym"] == nasym and est["n_asym_super"] == nsuper
    assert est["F33"] == pytest.approx(f33, rel=1e-12)
    assert est["F46"] == pytest.approx(f46, rel=1e-12)
    assert f33 > 0 and f46 != 0


def test_walk_lists(orc):
    x, m, h = W.plummer(3000, 7)
    tree = orc.build_tree(x, 8)
    mom = orc.moments(x, m, h, tree)
    mut = orc.asym_estimate(tree, mom, orc.walk(tree, mom, 0.5, policy=orc.MUTUAL))
    assert mut == {"F33": 0.0, "F46": 0.0, "n_asym": 0, "n_asym_super": 0}
    lists = orc.walk(tree, mom, 0.5)
    est = orc.asym_estimate(tree, mom, lists)
    internal_src = sum(int((tree.left[lists.far(a)] >= 0).sum()) for a in range(tree.nnodes))
    assert est["n_asym_super"] == internal_src
    assert est["n_asym"] >= internal_src
    assert est["F33"] > 0
