"""Pins for the oracle's second expansion form (Sec. 4, eqs. (25)-(26) with
p = 3): the sink and source offsets are expanded together and every term of
combined order above 2 is dropped.  Pinned against the point-mass field
(sympy), the double Taylor series of an explicit particle cluster, the
relation to eq. (6) stated in Sec. 4 (the extra index pairs (n, m) = (1, 2),
(2, 1), (2, 2)), the per-pair third law, the truncation order, and the
momentum behaviour of the two walks."""
import itertools
import math

import numpy as np
import pytest
import sympy as sp

from paper_2502_01496_amd import workloads as W

S2 = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}
S3 = {k: n for n, k in enumerate(
    [(0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1), (1, 1, 2),
     (1, 2, 2), (2, 2, 2)])}


def s2(i, j):
    return S2[tuple(sorted((i, j)))]


def s3(i, j, k):
    return S3[tuple(sorted((i, j, k)))]


@pytest.fixture(scope="module")
def green():
    """Derivative tensors of G(r) = -1/|r| up to order 5, from sympy."""
    r = sp.symbols("r0 r1 r2", real=True)
    G = -1 / sp.sqrt(r[0] ** 2 + r[1] ** 2 + r[2] ** 2)
    funcs = {}
    for order in range(6):
        for idx in itertools.combinations_with_replacement(range(3), order):
            e = G
            for a in idx:
                e = sp.diff(e, r[a])
            funcs[idx] = sp.lambdify(r, e, "numpy")

    def tensors(rv):
        out = []
        for order in range(6):
            T = np.empty((3,) * order) if order else np.empty(())
            for idx in itertools.product(range(3), repeat=order):
                T[idx] = funcs[tuple(sorted(idx))](*rv)
            out.append(T)
        return out

    return tensors


def cluster(rng, n, scale):
    y = rng.standard_normal((n, 3)) * scale
    m = rng.random(n) + 0.5
    y -= (m[:, None] * y).sum(0) / m.sum()  # offsets about the centre of mass
    return y, m


def series_field(D, x, y, m, pairs):
    """a_i(r, x) = -sum_{(k, l) in pairs} 1/(k! l!) sum_p m_p
    D^(1+k+l)_{i, x..x, (-y_p)..(-y_p)}: the double Taylor series of
    sum_p m_p grad G(r + x - y_p) over the index pairs given."""
    a = np.zeros(3)
    for k, l in pairs:
        T = D[1 + k + l]
        for _ in range(k):
            T = T @ x
        acc = np.zeros(3)
        for yp, mp in zip(y, m):
            t = T
            for _ in range(l):
                t = t @ (-yp)
            acc += mp * t
        a -= acc / (math.factorial(k) * math.factorial(l))
    return a


def test_dehnen_l1_is_eq6_and_l2_l3_are_point_mass_derivatives(orc):
    r1, r2, r3 = sp.symbols("r1 r2 r3", real=True)
    M = sp.Symbol("M")
    rv = sp.Matrix([r1, r2, r3])
    rn = sp.sqrt(r1 ** 2 + r2 ** 2 + r3 ** 2)
    mono = [-M * rv[i] / rn ** 3 for i in range(3)]  # field of a point mass
    d1 = [[sp.lambdify((r1, r2, r3, M), sp.diff(mono[i], v)) for v in (r1, r2, r3)]
          for i in range(3)]
    d2 = [[[sp.lambdify((r1, r2, r3, M), sp.diff(mono[i], v, w)) for w in (r1, r2, r3)]
           for v in (r1, r2, r3)] for i in range(3)]
    rng = np.random.default_rng(21)
    for _ in range(10):
        r = rng.standard_normal(3) * 3
        Mv = rng.random() + 0.2
        A = rng.standard_normal((3, 3))
        A = A + A.T
        A -= np.trace(A) / 3 * np.eye(3)
        Q = np.array([A[0, 0], A[0, 1], A[0, 2], A[1, 1], A[1, 2], A[2, 2]])
        Ld = orc.m2l(r, Mv, Q, orc.DEHNEN_FORM)
        Lp = orc.m2l(r, Mv, Q, orc.PHANTOM_FORM)
        np.testing.assert_array_equal(Ld[:3], Lp[:3])
        for i, j in itertools.product(range(3), repeat=2):
            want = d1[i][j](*r, Mv)
            assert Ld[3 + s2(i, j)] == pytest.approx(want, rel=1e-12, abs=1e-14 * abs(Mv))
        for i, j, k in itertools.product(range(3), repeat=3):
            want = d2[i][j][k](*r, Mv)
            assert Ld[9 + s3(i, j, k)] == pytest.approx(want, rel=1e-12, abs=1e-14 * abs(Mv))


def test_dehnen_is_the_truncated_double_series_of_a_cluster(orc, green):
    # eqs. (25)-(26), p = 3: all (n, m) with |n| + |m| <= 2; the moments are
    # those of explicit particles (raw second moments, not the traceless Q)
    rng = np.random.default_rng(22)
    dehnen = [(k, l) for k in range(3) for l in range(3) if k + l <= 2]
    phantom = dehnen + [(1, 2), (2, 1), (2, 2)]  # the index pairs added in Sec. 4
    for t in range(8):
        y, m = cluster(rng, 6 + t, 0.25)
        M, c, Q = orc.p2m(y, m)
        r = rng.standard_normal(3) * 2 + np.array([3.0, 0.0, 0.0])
        D = green(r)
        for _ in range(3):
            x = rng.standard_normal(3) * 0.2
            for form, pairs in ((orc.DEHNEN_FORM, dehnen), (orc.PHANTOM_FORM, phantom)):
                got = orc.l2p(orc.m2l(r, M, Q, form), x)
                want = series_field(D, x, y - c, m, pairs)
                np.testing.assert_allclose(got, want, rtol=1e-11,
                                           atol=1e-13 * np.abs(want).max())


def test_forms_differ_by_the_extra_index_pairs(orc, green):
    rng = np.random.default_rng(23)
    y, m = cluster(rng, 9, 0.3)
    M, c, Q = orc.p2m(y, m)
    r = np.array([2.5, -1.0, 0.7])
    D = green(r)
    x = np.array([0.15, 0.1, -0.2])
    diff = orc.l2p(orc.m2l(r, M, Q, orc.PHANTOM_FORM), x) - orc.l2p(
        orc.m2l(r, M, Q, orc.DEHNEN_FORM), x)
    extra = series_field(D, x, y - c, m, [(1, 2), (2, 1), (2, 2)])
    assert np.abs(extra).max() > 1e-6  # the pairs are not negligible here
    np.testing.assert_allclose(diff, extra, rtol=1e-10, atol=1e-14)


def _pair_force(orc, xa, ma, xb, mb, form):
    Ma, ca, Qa = orc.p2m(xa, ma)
    Mb, cb, Qb = orc.p2m(xb, mb)
    L = orc.m2l(ca - cb, Mb, Qb, form)
    return sum(mi * orc.l2p(L, xi - ca) for xi, mi in zip(xa, ma))


def test_dehnen_third_law_per_mutual_pair(orc):
    rng = np.random.default_rng(24)
    for t in range(20):
        xa, ma = cluster(rng, 4 + t % 6, 0.2)
        xb, mb = cluster(rng, 3 + t % 5, 0.3)
        xb = xb + rng.standard_normal(3) * 2 + np.array([4.0, 0, 0])
        Fab = _pair_force(orc, xa, ma, xb, mb, orc.DEHNEN_FORM)
        Fba = _pair_force(orc, xb, mb, xa, ma, orc.DEHNEN_FORM)
        assert np.linalg.norm(Fab + Fba) <= 1e-14 * np.linalg.norm(Fab)


def test_dehnen_truncation_is_third_order(orc):
    # shrinking the source cluster and the sink offset together by 2 divides
    # the relative error by ~2^3 (the first dropped terms have order 3)
    rng = np.random.default_rng(25)
    y0, m = cluster(rng, 12, 1.0)
    x0 = np.array([0.6, -0.4, 0.5])
    r = np.array([10.0, 3.0, -2.0])
    errs = []
    for s in (0.8, 0.4, 0.2, 0.1):
        y = y0 * s
        M, c, Q = orc.p2m(y, m)
        got = orc.l2p(orc.m2l(r, M, Q, orc.DEHNEN_FORM), x0 * s)
        d = (c + r + x0 * s) - y
        exact = -(m[:, None] * d / np.linalg.norm(d, axis=1)[:, None] ** 3).sum(0)
        errs.append(np.linalg.norm(got - exact) / np.linalg.norm(exact))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert (ratios > 6.0).all() and (ratios < 11.0).all(), errs


def test_dehnen_momentum_mutual_conserves_leaf_walk_does_not(orc):
    # Sec. 4: with the leaf <- cell lists the total force stays non-zero for
    # this form too; the mutual walk cancels it to round-off
    x, m, h = W.plummer(3000, 7)
    for policy, lo, hi in ((orc.PHANTOM, 1e-9, 1.0), (orc.MUTUAL, 0.0, 1e-13)):
        res = orc.fmm(x, m, h, policy=policy, form=orc.DEHNEN_FORM)
        ratio = orc.stats(x, None, m, res.a)["ratio"]
        assert lo < ratio < hi, (policy, ratio)
    # both forms truncate at the same order: comparable accuracy against the
    # direct sum (the one-sided criterion (4) dominates the error here)
    d = orc.direct(x, m, h)
    eta = {}
    for form in (orc.PHANTOM_FORM, orc.DEHNEN_FORM):
        a = orc.fmm(x, m, h, form=form).a
        eta[form] = np.sqrt(((a - d) ** 2).sum() / (d ** 2).sum())
    assert eta[orc.DEHNEN_FORM] < 3e-2
    assert 0.7 < eta[orc.DEHNEN_FORM] / eta[orc.PHANTOM_FORM] < 1.5
