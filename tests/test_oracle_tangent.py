"""Pins of the tangent-linear oracle (the FP64 oracle's source compiled with
dual numbers), which the GPU discrete adjoint is checked against.

* Its values are the plain oracle's, bit for bit, after whole steps of the
  one-solid cavity, the heavy periodic ellipse and two solids in contact: the
  dual build takes the same discrete decisions and does the same arithmetic.
* Pointwise derivatives against hand-derived closed forms: the smoothed
  Heaviside of Eq. (2_3_heaviside), the disc and ellipse reference level sets,
  the neo-Hookean stress of Eq. (2_4_neo-Hookean) through F = (grad xi)^-1,
  the smooth-flux-correction equilibrium and the Guo term.
* Whole-step tangents (centroid and mean displacement after several steps)
  against central differences of the plain oracle, for seeds in the shear
  modulus, the solid density, the ellipse's semi-axis and angle, gravity, the
  relaxation time, the lid speed and the initial velocity; and the contact
  force of two overlapping solids (Sec. 3.6) against differences in the
  position of one of them.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import Oracle
from oracle import oracle as plain
from oracle import tangent as tl
from oracle.tangent import TangentOracle

KEYS = ("centroid_x", "centroid_y", "disp_x", "disp_y")

CAVITY = workloads.make(nx=48, ny=48, tau=0.8, lid_ux=0.08,
                        solid=dict(cx=24.0, cy=28.0, R=9.0, G=0.01, rho_s=1.0))
HEAVY = workloads.make(nx=56, ny=48, tau=0.8, lid_ux=0.06, periodic_x=True,
                       gravity=(0.0, -2e-4),
                       solid=dict(cx=28.0, cy=26.0, R=11.0, G=0.01, rho_s=1.4,
                                  shape="ellipse", b=7.0, theta=0.5))


def _stream(nx, ny):
    return (workloads.uniform_velocity(nx, ny, 0.02, 0.01) +
            np.random.default_rng(5).normal(0.0, 1e-3, size=(2, ny, nx)))


def _overlap_cfg():
    # the second disc is off the mirror position of the first: with the centres
    # at 24 and 37 the nodes on x = 30.5 are equidistant from both, the contact
    # factor min(f(phi_p), f(phi_q)) sits on its kink there and rounding picks
    # the branch node by node (the map is not differentiable at that placement)
    return workloads.make(nx=64, ny=64, tau=0.8, periodic_x=True, periodic_y=True, eta=1.0,
                          solids=[dict(cx=24.0, cy=32.0, R=8.0, G=0.01, rho_s=1.0),
                                  dict(cx=37.3, cy=32.0, R=8.0, G=0.02, rho_s=1.0)])


# ------------------------------------------------------------ same values

@pytest.mark.parametrize("name,cfg,steps", [("cavity", CAVITY, 8), ("heavy", HEAVY, 8),
                                            ("contact", None, 3)])
def test_values_equal_the_plain_oracle_bitwise(name, cfg, steps):
    cfg = cfg or _overlap_cfg()
    u0 = _stream(cfg["nx"], cfg["ny"])
    a = Oracle(**cfg).init(u0).step(steps)
    b = TangentOracle(**cfg, dparams={"tau": 1.0}).init(u0, 0.5 * u0).step(steps)
    fv, fd = b.populations()
    assert np.array_equal(a.populations(), fv)
    assert np.any(fd != 0.0)
    (bx, by), _ = b.force()
    ax, ay = a.force()
    assert np.array_equal(ax, bx) and np.array_equal(ay, by)
    for body in range(len(cfg.get("solids") or [cfg["solid"]])):
        (X, Y, P), _ = b.refmap(body)
        X0, Y0, P0 = a.refmap(body)
        assert np.array_equal(np.isnan(X0), np.isnan(X))
        m = ~np.isnan(X0)
        assert np.array_equal(X0[m], X[m]) and np.array_equal(Y0[m], Y[m])
        assert np.array_equal(P0[m], P[m])
    dv, _ = b.diag()
    assert dv == a.diag()


def test_zero_seed_gives_zero_tangents():
    b = TangentOracle(**HEAVY).init(_stream(56, 48)).step(4)
    _, fd = b.populations()
    assert not np.any(fd)
    _, d = b.diag()
    assert all(v == 0.0 for v in d.values())


# ------------------------------------------------------------ pointwise

@pytest.mark.parametrize("phi", [-2.0, -1.2, -0.4, 0.0, 0.3, 1.1, 1.49, 2.5])
def test_heaviside_derivative(phi):
    eps = 1.5
    v, d = tl.heaviside(phi, 1.0, eps)
    assert v == plain.heaviside(phi, eps)
    inside = abs(phi) < eps
    want = (1.0 + math.cos(math.pi * phi / eps)) / (2.0 * eps) if inside else 0.0
    assert abs(d - want) <= 1e-15
    # with respect to the blur half-width: dH/deps = -phi/eps * dH/dphi
    _, de = tl.heaviside(phi, 0.0, eps, 1.0)
    assert abs(de - (-phi / eps) * want) <= 1e-15


def test_disc_level_set_gradient_is_the_unit_radial_vector():
    s = dict(cx=3.0, cy=-1.0, R=2.5, G=0.01, rho_s=1.0)
    for X, Y in ((5.0, 2.0), (-1.0, -1.5), (3.2, 0.4)):
        r = math.hypot(X - 3.0, Y + 1.0)
        _, gx = tl.phi0(s, X, Y, 1.0, 0.0)
        _, gy = tl.phi0(s, X, Y, 0.0, 1.0)
        assert abs(gx - (X - 3.0) / r) <= 1e-15 and abs(gy - (Y + 1.0) / r) <= 1e-15
        _, dR = tl.phi0(s, X, Y, dsolid={"R": 1.0})
        assert dR == -1.0


def test_ellipse_level_set_gradient():
    # phi = d (1 - 1/q), d = |X - c|, q^2 = (x'/a)^2 + (y'/b)^2 with (x', y')
    # the body-frame coordinates; by the chain rule
    # grad phi = (1 - 1/q) (X - c)/d + (d / q^3) R^T (x'/a^2, y'/b^2)
    a, b, th, cx, cy = 5.0, 2.0, 0.7, 1.0, 2.0
    s = dict(cx=cx, cy=cy, R=a, G=0.01, rho_s=1.0, shape="ellipse", b=b, theta=th)
    c, sn = math.cos(th), math.sin(th)
    for X, Y in ((4.0, 5.0), (0.2, 1.1), (-3.0, 2.5), (1.5, 2.0)):
        dx, dy = X - cx, Y - cy
        d = math.hypot(dx, dy)
        xp, yp = c * dx + sn * dy, -sn * dx + c * dy
        q = math.sqrt((xp / a) ** 2 + (yp / b) ** 2)
        px, py = xp / a ** 2, yp / b ** 2
        wx = (1 - 1 / q) * dx / d + d / q ** 3 * (c * px - sn * py)
        wy = (1 - 1 / q) * dy / d + d / q ** 3 * (sn * px + c * py)
        v, gx = tl.phi0(s, X, Y, 1.0, 0.0)
        _, gy = tl.phi0(s, X, Y, 0.0, 1.0)
        assert v == plain.phi0(s, X, Y)
        assert abs(gx - wx) <= 1e-14 * max(1.0, abs(wx))
        assert abs(gy - wy) <= 1e-14 * max(1.0, abs(wy))


def test_stress_derivatives():
    J = np.array([[0.93, 0.08], [-0.05, 1.04]])
    dJ = np.array([[0.3, -0.7], [0.2, 0.5]])
    G = 0.013
    ok, tau = plain.solid_stress(J, G)
    ok2, v, dG = tl.solid_stress(J, np.zeros(4), G, 1.0)
    assert ok and ok2 and np.array_equal(v, tau)
    assert np.max(np.abs(dG - tau / G)) <= 1e-15
    # F = J^-1: dF = -F dJ F, dB = dF F^T + F dF^T, dtau = G (dB - tr(dB)/3 I)
    F = np.linalg.inv(J)
    dF = -F @ dJ @ F
    dB = dF @ F.T + F @ dF.T
    want = G * np.array([dB[0, 0] - np.trace(dB) / 3, dB[0, 1], dB[1, 1] - np.trace(dB) / 3])
    _, _, dt = tl.solid_stress(J, dJ, G)
    assert np.max(np.abs(dt - want)) <= 1e-15


def test_equilibrium_and_forcing_derivatives():
    cx, cy, w = plain.d2q9()
    rho, ux, uy, dr = 1.03, 0.04, -0.02, 0.17
    v, d = tl.feq_sfc(rho, ux, uy, dr, (0.0, 1.0, 0.0, 0.0))
    assert np.array_equal(v, plain.feq_sfc(rho, ux, uy, dr))
    vc = cx * ux + cy * uy
    # d/dux of w rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 |u|^2)
    assert np.max(np.abs(d - w * rho * (3 * cx + 9 * vc * cx - 3 * ux))) <= 1e-15
    _, d = tl.feq_sfc(rho, ux, uy, dr, (0.0, 0.0, 0.0, 1.0))
    want = -w.copy()
    want[0] = np.sum(w[1:])
    assert np.max(np.abs(d - want)) <= 1e-15
    _, d = tl.feq_sfc(rho, ux, uy, dr, (1.0, 0.0, 0.0, 0.0))
    assert np.max(np.abs(d - w * (1 + 3 * vc + 4.5 * vc * vc - 1.5 * (ux * ux + uy * uy)))) <= 1e-15
    fx, fy = 2e-4, -3e-4
    # the Guo term is linear in F, and d/dux = w (-fx/cs^2 + cx (cx fx + cy fy)/cs^4)
    _, d = tl.guo(ux, uy, fx, fy, (0.0, 0.0, 1.0, 0.0))
    assert np.max(np.abs(d - plain.guo(ux, uy, 1.0, 0.0))) <= 1e-15
    _, d = tl.guo(ux, uy, fx, fy, (1.0, 0.0, 0.0, 0.0))
    assert np.max(np.abs(d - w * (-3 * fx + 9 * cx * (cx * fx + cy * fy)))) <= 1e-16


# ------------------------------------------------------------ whole steps

def _with(cfg, key, x):
    out = dict(cfg)
    if key.startswith("solid."):
        out["solid"] = dict(cfg["solid"], **{key[6:]: x})
    elif key == "gy":
        out["gravity"] = (cfg["gravity"][0], x)
    else:
        out[key] = x
    return out


def _base(cfg, key):
    if key.startswith("solid."):
        return cfg["solid"][key[6:]]
    return cfg["gravity"][1] if key == "gy" else cfg[key]


@pytest.mark.parametrize("cfg_name,key,h,steps", [
    ("cavity", "solid.G", 1e-4, 6),
    ("cavity", "lid_ux", 1e-5, 60),
    ("heavy", "solid.G", 1e-4, 6),
    ("heavy", "solid.rho_s", 1e-5, 6),
    ("heavy", "solid.b", 1e-4, 6),
    ("heavy", "solid.theta", 1e-5, 6),
    ("heavy", "gy", 1e-5, 6),
    ("heavy", "tau", 1e-4, 6),
])
def test_step_tangent_matches_central_differences(cfg_name, key, h, steps):
    cfg = {"cavity": CAVITY, "heavy": HEAVY}[cfg_name]
    u0 = _stream(cfg["nx"], cfg["ny"])
    x0 = _base(cfg, key)
    if key.startswith("solid."):
        seed = dict(dsolids=[{key[6:]: 1.0}])
    else:
        seed = dict(dparams={key: 1.0})
    _, t = TangentOracle(**cfg, **seed).init(u0).step(steps).diag()
    p = Oracle(**_with(cfg, key, x0 + h)).init(u0).step(steps).diag()
    m = Oracle(**_with(cfg, key, x0 - h)).init(u0).step(steps).diag()
    for k in KEYS:
        fd = (p[k] - m[k]) / (2 * h)
        print(key, k, "tangent", t[k], "central difference", fd)
        assert abs(t[k] - fd) <= 1e-5 * abs(t[k])


def test_step_tangent_in_the_initial_velocity():
    cfg, steps, h = HEAVY, 6, 1e-6
    u0 = _stream(56, 48)
    v = np.random.default_rng(17).normal(0.0, 1.0, size=u0.shape)
    _, t = TangentOracle(**cfg).init(u0, v).step(steps).diag()
    p = Oracle(**cfg).init(u0 + h * v).step(steps).diag()
    m = Oracle(**cfg).init(u0 - h * v).step(steps).diag()
    for k in KEYS:
        fd = (p[k] - m[k]) / (2 * h)
        assert abs(t[k] - fd) <= 1e-5 * abs(t[k])


def test_contact_force_tangent_in_a_solid_position():
    # two overlapping discs at rest: after one step the force is the contact
    # stress divergence; move the second disc along x
    cfg, h = _overlap_cfg(), 1e-5
    (fx, fy), (dfx, dfy) = TangentOracle(**cfg, dsolids=[{}, {"cx": 1.0}]).init().step(1).force()

    def moved(x):
        s = [dict(cfg["solids"][0]), dict(cfg["solids"][1], cx=x)]
        return Oracle(**dict(cfg, solids=s)).init().step(1).force()

    (px, py), (mx, my) = moved(37.3 + h), moved(37.3 - h)
    assert np.max(np.abs(dfx)) > 1e-4
    for d, p, m in ((dfx, px, mx), (dfy, py, my)):
        assert np.max(np.abs(d - (p - m) / (2 * h))) <= 1e-6 * np.max(np.abs(dfx))
