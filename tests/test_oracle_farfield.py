"""Pins for the oracle's multipole arithmetic: P2M (eq. (7)), M2L (eq. (6) and its
r-derivatives), L2P (eq. (8)), L2L, the per-pair Newton's third law of Sec. 3,
and the three-cell example of Sec. 4 (eq. (31))."""
import itertools
import json
import os

import numpy as np
import pytest
import sympy as sp

GOLD = os.path.join(os.path.dirname(__file__), "golden")

S2 = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}


def s2(i, j):
    return S2[tuple(sorted((i, j)))]


S3 = {k: n for n, k in enumerate(
    [(0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1), (1, 1, 2),
     (1, 2, 2), (2, 2, 2)])}


def s3(i, j, k):
    return S3[tuple(sorted((i, j, k)))]


def cluster(rng, n, scale=0.1):
    x = rng.standard_normal((n, 3)) * scale
    m = rng.random(n) + 0.5
    return x, m


def newton_field(src_x, src_m, at):
    d = at - src_x
    r = np.linalg.norm(d, axis=1)
    return -(src_m[:, None] * d / r[:, None] ** 3).sum(0)


# ---------------------------------------------------------------- eq. (6) itself
@pytest.fixture(scope="module")
def sym_eq6():
    r1, r2, r3 = sp.symbols("r1 r2 r3", real=True)
    M = sp.Symbol("M")
    qxx, qxy, qxz, qyy, qyz = sp.symbols("qxx qxy qxz qyy qyz")
    Q = sp.Matrix([[qxx, qxy, qxz], [qxy, qyy, qyz], [qxz, qyz, -qxx - qyy]])
    rv = sp.Matrix([r1, r2, r3])
    r = sp.sqrt(r1 ** 2 + r2 ** 2 + r3 ** 2)
    rh = rv / r
    rQr = (rh.T * Q * rh)[0]
    # eq. (6) typed from the paper: attraction towards the source, r from source to sink
    a = [-M / r ** 2 * rh[i] + (sum(rh[k] * Q[i, k] for k in range(3)) - sp.Rational(5, 2) * rh[i] * rQr) / r ** 4
         for i in range(3)]
    syms = (r1, r2, r3, M, qxx, qxy, qxz, qyy, qyz)
    fa = sp.lambdify(syms, a, "numpy")
    d1 = [[sp.diff(a[i], v) for v in (r1, r2, r3)] for i in range(3)]
    d2 = [[[sp.diff(d1[i][j], v) for v in (r1, r2, r3)] for j in range(3)] for i in range(3)]
    return syms, fa, sp.lambdify(syms, d1, "numpy"), sp.lambdify(syms, d2, "numpy")


def traceless(rng):
    A = rng.standard_normal((3, 3))
    A = A + A.T
    A -= np.trace(A) / 3 * np.eye(3)
    return np.array([A[0, 0], A[0, 1], A[0, 2], A[1, 1], A[1, 2], A[2, 2]])


def test_m2l_matches_symbolic_derivatives_of_eq6(orc, sym_eq6):
    _, fa, fd1, fd2 = sym_eq6
    rng = np.random.default_rng(3)
    for _ in range(20):
        r = rng.standard_normal(3) * 3
        M = rng.random() + 0.1
        Q = traceless(rng) * 0.3
        args = (*r, M, Q[0], Q[1], Q[2], Q[3], Q[4])
        L = orc.m2l(r, M, Q)
        a = np.array(fa(*args), dtype=float)
        d1 = np.array(fd1(*args), dtype=float)
        d2 = np.array(fd2(*args), dtype=float)
        np.testing.assert_allclose(L[:3], a, rtol=1e-13, atol=1e-15 * np.abs(a).max())
        for i, j in itertools.product(range(3), repeat=2):
            assert L[3 + s2(i, j)] == pytest.approx(d1[i][j], rel=1e-12, abs=1e-14 * np.abs(d1).max())
        for i, j, k in itertools.product(range(3), repeat=3):
            assert L[9 + s3(i, j, k)] == pytest.approx(d2[i][j][k], rel=1e-12, abs=1e-14 * np.abs(d2).max())


def test_m2l_tensors_symmetric_and_traceless(orc):
    rng = np.random.default_rng(4)
    for _ in range(10):
        L = orc.m2l(rng.standard_normal(3) * 2, 1.3, traceless(rng))
        assert abs(L[3] + L[6] + L[8]) < 1e-13 * np.abs(L[3:9]).max()
        for k in range(3):  # contraction L3_iik = 0
            tr = sum(L[9 + s3(i, i, k)] for i in range(3))
            assert abs(tr) < 1e-13 * np.abs(L[9:]).max()


def test_m2l_l2p_converge_to_direct_cluster_field(orc):
    # truncation error of a quadrupole-order expansion falls as (size/r)^3
    rng = np.random.default_rng(1)
    xs, ms = cluster(rng, 10)
    M, c, Q = orc.p2m(xs, ms)
    y = np.array([0.05, -0.03, 0.02])
    errs = []
    for R in (2.0, 4.0, 8.0, 16.0):
        sink = c + np.array([R, 0.3 * R, -0.2 * R])
        L = orc.m2l(sink - c, M, Q)
        exact = newton_field(xs, ms, sink + y)
        errs.append(np.abs(orc.l2p(L, y) - exact).max() / np.abs(exact).max())
    errs = np.array(errs)
    assert errs[0] < 1e-3
    ratios = errs[:-1] / errs[1:]
    assert (ratios > 6.0).all() and (ratios < 11.0).all(), errs   # ~2^3 per doubling


def test_p2m_monopole_dipole_and_quadrupole_definition(orc):
    rng = np.random.default_rng(5)
    xs, ms = cluster(rng, 13, 0.5)
    M, c, Q = orc.p2m(xs, ms)
    assert M == pytest.approx(ms.sum(), rel=1e-15)
    np.testing.assert_allclose(ms @ (xs - c), 0.0, atol=1e-14)
    # far potential of the cluster: -M/r - 1/2 Q_ij r_i r_j / r^5 (+ O(r^-4))
    for R in (50.0, 100.0):
        p = c + R * np.array([0.6, 0.0, 0.8])
        phi = -(ms / np.linalg.norm(p - xs, axis=1)).sum()
        d = p - c
        Qf = np.array([[Q[s2(i, j)] for j in range(3)] for i in range(3)])
        approx = -M / R - 0.5 * d @ Qf @ d / R ** 5
        assert abs(phi - approx) < 3 * ms.sum() * 0.5 ** 3 * 3 / R ** 4


def test_l2l_is_exact_reexpansion(orc):
    rng = np.random.default_rng(6)
    L = orc.m2l(rng.standard_normal(3) * 3, 0.7, traceless(rng))
    for _ in range(10):
        delta = rng.standard_normal(3) * 0.2
        y = rng.standard_normal(3) * 0.2
        a0 = orc.l2p(L, y)
        a1 = orc.l2p(orc.l2l(L, delta), y - delta)
        np.testing.assert_allclose(a1, a0, rtol=1e-13, atol=1e-15 * np.abs(a0).max())


def pair_force(orc, xa, ma, xb, mb):
    """F_{b->a} = sum_{i in a} m_i L2P(M2L(b -> a), y_i)."""
    Ma, ca, Qa = orc.p2m(xa, ma)
    Mb, cb, Qb = orc.p2m(xb, mb)
    L = orc.m2l(ca - cb, Mb, Qb)
    return sum(mi * orc.l2p(L, xi - ca) for xi, mi in zip(xa, ma)), (Ma, ca, Qa), (Mb, cb, Qb), L


def test_newton_third_law_per_mutual_pair(orc):
    # Sec. 3: for the form (6)+(8) the force of cell b on cell a and of a on b
    # cancel to round-off for every well-separated pair.
    rng = np.random.default_rng(8)
    for t in range(25):
        xa, ma = cluster(rng, 5 + t % 7, 0.2)
        xb, mb = cluster(rng, 3 + t % 5, 0.3)
        xb += rng.standard_normal(3) * 2 + np.array([4.0, 0, 0])
        Fab, *_ = pair_force(orc, xa, ma, xb, mb)
        Fba, *_ = pair_force(orc, xb, mb, xa, ma)
        assert np.linalg.norm(Fab + Fba) <= 1e-14 * np.linalg.norm(Fab)


def test_pair_force_closed_form(orc):
    # With sum m y = 0 and harmonic a: F_{b->a} = M_a a_b(r) + 1/6 Q^a_jk d_j d_k a_b(r)
    rng = np.random.default_rng(9)
    for _ in range(10):
        xa, ma = cluster(rng, 9, 0.2)
        xb, mb = cluster(rng, 7, 0.2)
        xb += np.array([3.0, 1.0, -0.5])
        F, (Ma, ca, Qa), _, L = pair_force(orc, xa, ma, xb, mb)
        closed = Ma * L[:3] + np.array([
            sum(L[9 + s3(i, j, k)] * Qa[s2(j, k)] for j in range(3) for k in range(3))
            for i in range(3)]) / 6.0
        np.testing.assert_allclose(F, closed, rtol=1e-13, atol=1e-15 * np.abs(F).max())


def test_three_cell_example_eq31(orc):
    g = json.load(open(os.path.join(GOLD, "paper_sec4_eq31.json")))
    Ma, M1, M2 = 1.3, 0.4, 1.1
    x = np.array([0.7, 0.45, 0.0])
    Mb = M1 + M2
    K = Ma * Mb * (M1 / M2) * (1 - M1 / M2)
    prev = None
    for r in (20.0, 80.0, 320.0, 1280.0):
        cb = np.zeros(3)
        xa = np.array([[r, 0.0, 0.0]])
        xb = np.array([x, -x * M1 / M2])
        # beta -> alpha through the super-cell's multipoles, alpha -> beta1, beta2 leaf by leaf
        F_ba, *_ = pair_force(orc, xa, np.array([Ma]), xb, np.array([M1, M2]))
        F_a1, *_ = pair_force(orc, xb[:1], np.array([M1]), xa, np.array([Ma]))
        F_a2, *_ = pair_force(orc, xb[1:], np.array([M2]), xa, np.array([Ma]))
        F = F_ba + F_a1 + F_a2
        t1 = g["F1"]["terms"]
        t2 = g["F2"]["terms"]
        e1 = g["F1"]["coefficient"] * K / r ** 5 * (t1["x1^3"] * x[0] ** 3 + t1["x1*x2^2"] * x[0] * x[1] ** 2)
        e2 = g["F2"]["coefficient"] * K / r ** 5 * (t2["x2^3"] * x[1] ** 3 + t2["x1^2*x2"] * x[0] ** 2 * x[1])
        rat = np.array([F[0] / e1, F[1] / e2])
        assert abs(F[2]) < 1e-12 * abs(F[0])
        dev = np.abs(rat - 1).max()
        assert dev < 2.0 * np.linalg.norm(x) / r + 1e-6, (r, rat)
        if prev is not None:
            assert dev < prev
        prev = dev
        bound = g["bound_eq32"]["coefficient"] * np.linalg.norm(x) ** 3 * K / r ** 5
        assert np.linalg.norm(F) <= bound * (1 + 2 * np.linalg.norm(x) / r)
