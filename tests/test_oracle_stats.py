"""Pins for the oracle's momentum diagnostics (Secs. 5-6): the total force
sum F_i, its modulus sum sum |F_i| (the denominator of |sum F| / sum |F|), the
mass, the centre of mass, the momentum P = sum m v and the angular momentum
L = sum m x cross v, with F_i = m_i a_i.  Each value is fixed by hand-computed
cases or by a closed form, so that a dropped mass, a wrong sign or a wrong
component of the cross product fails here, not only in a comparison of the
GPU against the same oracle."""
import numpy as np
import pytest


def st(orc, x, v, m, a):
    return orc.stats(np.asarray(x, float), None if v is None else np.asarray(v, float),
                     np.asarray(m, float), np.asarray(a, float))


def test_single_particle_momenta(orc):
    # one particle at (1, 0, 0) moving along +y with m = 2: P = (0, 2, 0),
    # L = m x cross v = (0, 0, 2)
    s = st(orc, [[1.0, 0, 0]], [[0, 1.0, 0]], [2.0], [[0.0, 0, 0]])
    np.testing.assert_array_equal(s["P"], [0, 2, 0])
    np.testing.assert_array_equal(s["L"], [0, 0, 2])
    np.testing.assert_array_equal(s["xcom"], [1, 0, 0])
    assert s["mass"] == 2.0


@pytest.mark.parametrize("x,v,m,L", [
    # each component of the cross product, with both signs of its two terms
    ([0, 1.0, 0], [0, 0, 3.0], 0.5, [1.5, 0, 0]),      # y vz
    ([0, 0, 1.0], [0, 4.0, 0], 0.25, [-1.0, 0, 0]),    # -z vy
    ([0, 0, 2.0], [5.0, 0, 0], 1.0, [0, 10.0, 0]),     # z vx
    ([3.0, 0, 0], [0, 0, 1.0], 2.0, [0, -6.0, 0]),     # -x vz
    ([2.0, 0, 0], [0, 7.0, 0], 1.5, [0, 0, 21.0]),     # x vy
    ([0, 1.0, 0], [2.0, 0, 0], 3.0, [0, 0, -6.0]),     # -y vx
])
def test_angular_momentum_components(orc, x, v, m, L):
    s = st(orc, [x], [v], [m], [[0.0, 0, 0]])
    np.testing.assert_array_equal(s["L"], L)


def test_rigid_rotation_inertia_tensor(orc):
    # v = w e_z cross x for every particle: L = I w with the inertia tensor,
    # L_z = w sum m (x^2 + y^2), L_x = -w sum m x z, L_y = -w sum m y z
    rng = np.random.default_rng(11)
    x = rng.standard_normal((257, 3))
    m = rng.random(257) + 0.1
    w = 0.7
    v = np.stack([-w * x[:, 1], w * x[:, 0], np.zeros(257)], axis=1)
    s = st(orc, x, v, m, np.zeros_like(x))
    ref = w * np.array([-(m * x[:, 0] * x[:, 2]).sum(), -(m * x[:, 1] * x[:, 2]).sum(),
                        (m * (x[:, 0] ** 2 + x[:, 1] ** 2)).sum()])
    np.testing.assert_allclose(s["L"], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    np.testing.assert_allclose(s["P"], (m[:, None] * v).sum(0), rtol=1e-13, atol=1e-13)


def test_force_sums_hand_values(orc):
    # F_1 = 2 (3, 4, 0) = (6, 8, 0), |F_1| = 10; F_2 = 0.5 (0, 0, -1), |F_2| = 0.5
    s = st(orc, [[0.0, 0, 0], [1.0, 0, 0]], None, [2.0, 0.5], [[3.0, 4.0, 0], [0, 0, -1.0]])
    np.testing.assert_array_equal(s["sumF"], [6.0, 8.0, -0.5])
    assert s["sumAbsF"] == 10.5
    assert s["ratio"] == pytest.approx(np.sqrt(100.25) / 10.5, rel=1e-15)
    np.testing.assert_array_equal(s["P"], [0, 0, 0])
    np.testing.assert_array_equal(s["L"], [0, 0, 0])
    assert s["mass"] == 2.5
    np.testing.assert_allclose(s["xcom"], [0.2, 0, 0], rtol=1e-15)


def test_newtonian_pair_sum_abs_force(orc):
    # two point masses beyond the softening support: |F| = G m1 m2 / r^2 on
    # each, so sum |F| = 2 G m1 m2 / r^2 and sum F = 0 (Newton's third law)
    m1, m2, r, G = 0.3, 1.7, 2.5, 1.3
    x = np.array([[0.1, -0.2, 0.4], [0.1 + r * 0.6, -0.2, 0.4 + r * 0.8]])
    a = np.array([[0.6, 0, 0.8], [-0.6, 0, -0.8]]) * G / r ** 2 * np.array([[m2], [m1]])
    s = st(orc, x, None, [m1, m2], a)
    assert s["sumAbsF"] == pytest.approx(2 * G * m1 * m2 / r ** 2, rel=1e-15)
    assert np.abs(s["sumF"]).max() <= 1e-16
    # the oracle's own direct sum gives the same pair forces (softening 2h < r)
    ad = orc.direct(x, np.array([m1, m2]), np.array([0.1, 0.2]), G=G)
    np.testing.assert_allclose(ad, a, rtol=1e-14, atol=1e-16)


def test_sum_abs_force_weights_each_mass(orc):
    # scaling one particle's mass scales only its own |F| term: a dropped m_i
    # or a shared mass would fail
    rng = np.random.default_rng(5)
    x = rng.standard_normal((5, 3))
    a = rng.standard_normal((5, 3))
    m = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    base = st(orc, x, None, m, a)["sumAbsF"]
    for k in range(5):
        m2 = m.copy()
        m2[k] *= 3.0
        got = st(orc, x, None, m2, a)["sumAbsF"]
        assert got - base == pytest.approx(2.0 * m[k] * np.linalg.norm(a[k]), rel=1e-12)
