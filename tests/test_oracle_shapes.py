"""Pins of the oracle's reference level set phi0 for the two solid shapes
(CPU only).

The disc's phi0 is the signed distance |X - c| - R.  For an ellipse the paper
gives no formula (it only needs phi0 < 0 inside, = 0 on the boundary, and a
smooth blur band); the oracle's reading is the radial form
|X - c| (1 - 1/q), q = sqrt((x'/a)^2 + (y'/b)^2) in the body frame rotated by
theta.  The pins below fix what that reading means without retyping it: it is
the distance along the ray from the centre beyond the boundary point on that
ray (whose radius follows from the ellipse's polar equation), it vanishes on
the parametric boundary, it is the disc's when a = b (up to rounding), it is the
signed distance along both principal axes, and the nodes it marks as solid are
the lattice points inside the ellipse."""
import math

import numpy as np
import pytest

import workloads
from oracle import Oracle
from oracle.oracle import phi0

ELL = dict(cx=31.3, cy=27.9, R=11.0, G=0.01, rho_s=1.0, shape="ellipse", b=6.5, theta=0.61)


def test_equal_axes_give_the_disc():
    rng = np.random.default_rng(1)
    disc = dict(ELL, shape="disc")
    for theta in (0.0, 0.3, 2.0):
        circ = dict(ELL, b=ELL["R"], theta=theta)
        for X, Y in rng.uniform(10, 50, size=(200, 2)):
            assert abs(phi0(circ, X, Y) - phi0(disc, X, Y)) < 1e-13 * math.hypot(X, Y)


def test_zero_on_the_parametric_boundary_and_sign():
    a, b, th = ELL["R"], ELL["b"], ELL["theta"]
    c, s = math.cos(th), math.sin(th)
    for t in np.linspace(0, 2 * math.pi, 97):
        for scale, sign in ((1.0, 0), (0.8, -1), (1.25, 1)):
            x, y = scale * a * math.cos(t), scale * b * math.sin(t)
            X, Y = ELL["cx"] + c * x - s * y, ELL["cy"] + s * x + c * y
            v = phi0(ELL, X, Y)
            if sign == 0:
                assert abs(v) < 1e-13
            else:
                assert np.sign(v) == sign


def test_radial_distance_beyond_the_polar_radius():
    # polar equation of an ellipse about its centre:
    # r(psi) = a b / sqrt((b cos psi)^2 + (a sin psi)^2), psi from the a axis
    a, b, th = ELL["R"], ELL["b"], ELL["theta"]
    rng = np.random.default_rng(2)
    for _ in range(300):
        d, ang = rng.uniform(0.2, 30.0), rng.uniform(0, 2 * math.pi)
        psi = ang - th
        r = a * b / math.hypot(b * math.cos(psi), a * math.sin(psi))
        X, Y = ELL["cx"] + d * math.cos(ang), ELL["cy"] + d * math.sin(ang)
        assert abs(phi0(ELL, X, Y) - (d - r)) < 1e-12 * max(1.0, d)


def test_signed_distance_along_the_principal_axes_and_rotation():
    a, b, th = ELL["R"], ELL["b"], ELL["theta"]
    for t in (0.5, 3.0, 9.0, 14.0):
        for ang, r in ((th, a), (th + math.pi, a), (th + math.pi / 2, b), (th - math.pi / 2, b)):
            X, Y = ELL["cx"] + t * math.cos(ang), ELL["cy"] + t * math.sin(ang)
            assert abs(phi0(ELL, X, Y) - (t - r)) < 1e-12
    # a quarter turn swaps the roles of the axes
    swapped = dict(ELL, R=ELL["b"], b=ELL["R"], theta=ELL["theta"] + math.pi / 2)
    rng = np.random.default_rng(3)
    for X, Y in rng.uniform(10, 50, size=(100, 2)):
        assert abs(phi0(swapped, X, Y) - phi0(ELL, X, Y)) < 1e-12
    # the centre takes the smaller semi-axis
    assert phi0(ELL, ELL["cx"], ELL["cy"]) == -ELL["b"]


def test_initial_solid_nodes_are_the_lattice_points_inside():
    n = 64
    o = Oracle(**workloads.make(nx=n, ny=n, tau=0.8, solid=ELL)).init()
    _, _, phi = o.refmap()
    y, x = np.mgrid[0:n, 0:n] + 0.5
    c, s = math.cos(ELL["theta"]), math.sin(ELL["theta"])
    dx, dy = x - ELL["cx"], y - ELL["cy"]
    q2 = ((c * dx + s * dy) / ELL["R"]) ** 2 + ((-s * dx + c * dy) / ELL["b"]) ** 2
    inside = q2 < 1.0
    assert np.array_equal(np.nan_to_num(phi, nan=1.0) < 0.0, inside)
    assert abs(inside.sum() - math.pi * ELL["R"] * ELL["b"]) < 0.05 * math.pi * ELL["R"] * ELL["b"]


@pytest.mark.parametrize("bad", [dict(shape="square"), dict(b=0.0), dict(b=-1.0)])
def test_bad_shapes_are_rejected(bad):
    with pytest.raises(ValueError):
        Oracle(**workloads.make(nx=32, ny=32, tau=0.8, solid=dict(ELL, cx=16, cy=16, **bad)))
