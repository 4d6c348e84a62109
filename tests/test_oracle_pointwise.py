"""Pins of the oracle's pointwise definitions against what the paper prints and
what the mathematics fixes (CPU only)."""
import os

import numpy as np
import pytest

from oracle import d2q9, feq_sfc, guo, heaviside, solid_stress

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CS2 = 1.0 / 3.0


def _table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "d2q9_table.txt"))
            if l.strip() and not l.startswith("#")]
    a = np.array(rows, dtype=float)
    return a[:, 1].astype(int), a[:, 2].astype(int), a[:, 3] / a[:, 4]


def test_d2q9_matches_printed_table():
    cx, cy, w = d2q9()
    tx, ty, tw = _table()
    assert np.array_equal(cx, tx) and np.array_equal(cy, ty)
    assert np.allclose(w, tw, rtol=0, atol=1e-17)
    # lattice isotropy the weights must satisfy
    assert abs(w.sum() - 1) < 1e-15
    assert abs((w * cx * cx).sum() - CS2) < 1e-15
    assert abs((w * cx * cy).sum()) < 1e-15


def _moments(f):
    cx, cy, _ = d2q9()
    return (f.sum(), np.array([(cx * f).sum(), (cy * f).sum()]),
            np.array([[(cx * cx * f).sum(), (cx * cy * f).sum()],
                      [(cy * cx * f).sum(), (cy * cy * f).sum()]]))


@pytest.mark.parametrize("seed", range(5))
def test_feq_sfc_moments(seed):
    # Eq. (2_3_feq_sfc): mass rho, momentum rho u; the SFC term only lowers the
    # isotropic pressure part of the second moment to c_s^2 (rho - drho)
    rng = np.random.default_rng(seed)
    rho = 1 + 0.2 * rng.standard_normal()
    u = 0.08 * rng.standard_normal(2)
    drho = 0.3 * rng.standard_normal()
    m0, m1, m2 = _moments(feq_sfc(rho, u[0], u[1], drho))
    assert abs(m0 - rho) < 1e-15
    assert np.allclose(m1, rho * u, rtol=0, atol=1e-16)
    expect = CS2 * (rho - drho) * np.eye(2) + rho * np.outer(u, u)
    assert np.allclose(m2, expect, rtol=0, atol=1e-15)


def test_feq_matches_expanded_form_of_sec_3_4():
    # the nine expanded equilibria printed in Sec. 3.4, Eq. (3_4_feq)
    rng = np.random.default_rng(7)
    for _ in range(20):
        rho, u, v, dr = 1 + 0.1 * rng.standard_normal(), *(0.1 * rng.standard_normal(2)), \
            0.2 * rng.standard_normal()
        s = u * u + v * v
        printed = np.array([
            2 * rho / 9 * (2 - 3 * s) + 5 / 9 * dr,
            rho / 18 * (2 + 6 * u + 9 * u * u - 3 * s) - dr / 9,
            rho / 18 * (2 + 6 * v + 9 * v * v - 3 * s) - dr / 9,
            rho / 18 * (2 - 6 * u + 9 * u * u - 3 * s) - dr / 9,
            rho / 18 * (2 - 6 * v + 9 * v * v - 3 * s) - dr / 9,
            rho / 36 * (1 + 3 * (u + v) + 9 * u * v + 3 * s) - dr / 36,
            rho / 36 * (1 - 3 * (u - v) - 9 * u * v + 3 * s) - dr / 36,
            rho / 36 * (1 - 3 * (u + v) + 9 * u * v + 3 * s) - dr / 36,
            rho / 36 * (1 + 3 * (u - v) - 9 * u * v + 3 * s) - dr / 36,
        ])
        assert np.allclose(feq_sfc(rho, u, v, dr), printed, rtol=0, atol=1e-15)


def test_sfc_correction_conserves_mass_and_momentum():
    # App. C, Eq. (a_3_cfi): f^c_0 = 4 (w1 + w2) drho, f^c_i = -w_i drho, and
    # sum f^c = 0, sum c f^c = 0
    _, _, w = d2q9()
    for dr in (-0.4, 0.1, 0.75):
        fc = feq_sfc(1.1, 0.03, -0.02, dr) - feq_sfc(1.1, 0.03, -0.02, 0.0)
        assert abs(fc[0] - 4 * (w[1] + w[5]) * dr) < 1e-15
        assert np.allclose(fc[1:], -w[1:] * dr, rtol=0, atol=1e-16)
        m0, m1, _ = _moments(fc)
        assert abs(m0) < 1e-15 and np.allclose(m1, 0, atol=1e-16)


@pytest.mark.parametrize("seed", range(5))
def test_guo_moments(seed):
    # Eq. (2_2_Fi) carries the force density F in the first moment and the
    # symmetric u F + F u in the second (forcing scheme of Guo et al.)
    rng = np.random.default_rng(100 + seed)
    u = 0.1 * rng.standard_normal(2)
    F = 1e-3 * rng.standard_normal(2)
    m0, m1, m2 = _moments(guo(u[0], u[1], F[0], F[1]))
    assert abs(m0) < 1e-18
    assert np.allclose(m1, F, rtol=0, atol=1e-18)
    assert np.allclose(m2, np.outer(u, F) + np.outer(F, u), rtol=0, atol=1e-18)


def test_guo_expanded_form_reading():
    # Eq. (3_4_Fi) printed: F_2 and F_4 carry 9 v F_x, which makes the forcing
    # create mass (sum F_i = 2 v (F_x - F_y)); with 9 v F_y (and F per unit
    # volume, no rho prefactor) the printed forms agree with Eq. (2_2_Fi).
    u, v, Fx, Fy = 0.04, -0.07, 2e-3, -1e-3

    def printed(fix):
        f2y = Fy if fix else Fx
        return np.array([
            4 / 9 * (-3 * u * Fx - 3 * v * Fy),
            1 / 9 * (3 * (1 - u) * Fx - 3 * v * Fy + 9 * u * Fx),
            1 / 9 * (-3 * u * Fx + 3 * (1 - v) * Fy + 9 * v * f2y),
            1 / 9 * (3 * (-1 - u) * Fx - 3 * v * Fy + 9 * u * Fx),
            1 / 9 * (-3 * u * Fx + 3 * (-1 - v) * Fy + 9 * v * f2y),
            1 / 36 * (3 * (1 - u) * Fx + 3 * (1 - v) * Fy + 9 * (u + v) * Fx + 9 * (u + v) * Fy),
            1 / 36 * (3 * (-1 - u) * Fx + 3 * (1 - v) * Fy + 9 * (u - v) * Fx + 9 * (-u + v) * Fy),
            1 / 36 * (3 * (-1 - u) * Fx + 3 * (-1 - v) * Fy + 9 * (u + v) * Fx + 9 * (u + v) * Fy),
            1 / 36 * (3 * (1 - u) * Fx + 3 * (-1 - v) * Fy + 9 * (u - v) * Fx + 9 * (-u + v) * Fy),
        ])
    assert np.allclose(guo(u, v, Fx, Fy), printed(True), rtol=0, atol=1e-18)
    m0, _, _ = _moments(printed(False))
    assert abs(m0 - 2 * v * (Fx - Fy)) < 1e-18 and abs(m0) > 1e-5


def test_heaviside_properties():
    # Eq. (2_3_heaviside)
    eps = 1.5
    assert heaviside(-eps, eps) == 0.0 and heaviside(eps, eps) == 1.0
    assert heaviside(-10, eps) == 0.0 and heaviside(10, eps) == 1.0
    assert abs(heaviside(0.0, eps) - 0.5) < 1e-16
    x = np.linspace(-eps, eps, 301)
    H = np.array([heaviside(t, eps) for t in x])
    assert np.all(np.diff(H) >= 0)
    assert np.allclose(H + np.array([heaviside(-t, eps) for t in x]), 1.0, atol=1e-15)
    # slope 1/eps at the interface, zero slope at both ends (C^1 blend)
    h = 1e-6
    assert abs((heaviside(h, eps) - heaviside(-h, eps)) / (2 * h) - 1 / eps) < 1e-8
    assert (heaviside(eps, eps) - heaviside(eps - h, eps)) / h < 1e-6
    assert (heaviside(-eps + h, eps) - heaviside(-eps, eps)) / h < 1e-6


def _J_of_map(A):
    """grad xi for the linear map xi = A x: J = A."""
    return np.asarray(A, float).reshape(4)


def test_stress_zero_when_undeformed_and_under_rotation():
    # Eq. (3_3_solid_stress): the "+1" of plane strain makes tau vanish at F = I
    ok, tau = solid_stress(_J_of_map(np.eye(2)), 0.3)
    assert ok and np.allclose(tau, 0, atol=1e-16)
    for th in (0.3, 1.2, -2.0):
        R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        ok, tau = solid_stress(_J_of_map(R.T), 0.7)  # xi = R^T x is a rigid rotation
        assert ok and np.allclose(tau, 0, atol=1e-15)


@pytest.mark.parametrize("gam", [0.05, 0.3, -0.8])
def test_stress_simple_shear_closed_form(gam):
    # xi = (x - gam y, y): F = [[1, gam], [0, 1]], tau = G [[2g^2/3, g], [g, -g^2/3]]
    G = 0.02
    ok, tau = solid_stress(_J_of_map([[1, -gam], [0, 1]]), G)
    assert ok
    assert np.allclose(tau, G * np.array([2 * gam ** 2 / 3, gam, -gam ** 2 / 3]), atol=1e-16)


@pytest.mark.parametrize("s", [0.8, 1.0, 1.25])
def test_stress_stretch_closed_form(s):
    # xi = (x / s, y): F = diag(s, 1), tau = G (diag(s^2, 1) - (s^2 + 2)/3 I)
    G = 0.5
    ok, tau = solid_stress(_J_of_map([[1 / s, 0], [0, 1]]), G)
    assert ok
    t = (s * s + 2) / 3
    assert np.allclose(tau, G * np.array([s * s - t, 0.0, 1 - t]), atol=1e-15)


def test_stress_singular_jacobian_is_dropped():
    ok, tau = solid_stress(_J_of_map([[1, 2], [0.5, 1]]), 1.0)  # det = 0
    assert not ok and np.all(tau == 0)
    ok, tau = solid_stress(_J_of_map([[0, 1], [1, 0]]), 1.0)  # det = -1 (inverted)
    assert not ok
