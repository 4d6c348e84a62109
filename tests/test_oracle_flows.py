"""Pins of the oracle's full step on flows with known answers: Couette and
Poiseuille profiles, Taylor-Green decay, exact conservation, the rest state
with a density contrast, an undeformed solid at rest and a rigidly translating
solid (CPU only)."""
import numpy as np
import pytest

import workloads
from oracle import Oracle


def test_couette_profile_is_exact():
    # periodic x, resting bottom wall, lid on top: u(y) = U y / H with halfway
    # bounce-back (Sec. 3.5) and the moving-wall term (y = j + 1/2)
    U, ny = 0.05, 16
    o = Oracle(**workloads.make(nx=4, ny=ny, tau=0.8, lid_ux=U, periodic_x=True)).init()
    o.step(20000)
    _, ux, uy = o.macro()
    y = np.arange(ny) + 0.5
    assert np.max(np.abs(ux - U * y[:, None] / ny)) < 1e-12
    assert np.max(np.abs(uy)) < 1e-12 * U


def test_poiseuille_profile():
    # body-force driven channel: u(y) = F / (2 nu) y (H - y).  BGK halfway
    # bounce-back puts the wall exactly halfway when (tau - 1/2)^2 = 3/16; at any
    # tau the bulk curvature is exactly -F / nu.
    F, ny = 1e-6, 16
    y = np.arange(ny) + 0.5
    tau = 0.5 + np.sqrt(3.0 / 16.0)
    nu = (tau - 0.5) / 3.0
    o = Oracle(**workloads.make(nx=4, ny=ny, tau=tau, periodic_x=True, fext=(F, 0.0))).init()
    o.step(40000)
    _, ux, uy = o.macro()
    exact = F / (2 * nu) * y * (ny - y)
    assert np.max(np.abs(ux[:, 0] - exact)) < 1e-9 * exact.max()
    o2 = Oracle(**workloads.make(nx=4, ny=ny, tau=0.8, periodic_x=True, fext=(F, 0.0))).init()
    o2.step(40000)
    _, u2, _ = o2.macro()
    curv = u2[2:, 0] - 2 * u2[1:-1, 0] + u2[:-2, 0]
    assert np.allclose(curv, -F / 0.1, rtol=1e-8)


def _tg_rate(n, tau=0.8, t0=50, t1=250):
    u0 = 1e-4
    o = Oracle(**workloads.make(nx=n, ny=n, tau=tau, periodic_x=True, periodic_y=True))
    U0 = workloads.taylor_green_velocity(n, u0)
    o.init(U0)
    amp = []
    for t in (t0, t1):
        o.step(t - o.step_count)
        _, ux, uy = o.macro()
        amp.append((ux * U0[0] + uy * U0[1]).sum() / (U0 ** 2).sum())
    rate = np.log(amp[0] / amp[1]) / (t1 - t0)
    k = 2 * np.pi / n
    return rate, 2 * (tau - 0.5) / 3 * k * k


def test_taylor_green_decay_second_order():
    # periodic Taylor-Green vortex decays as exp(-2 nu k^2 t); the LB rate
    # converges to it at second order in k
    errs = []
    for n in (16, 32, 64):
        r, exact = _tg_rate(n)
        errs.append(abs(r / exact - 1))
    assert errs[-1] < 2e-3
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(order - 2) < 0.15), order


@pytest.mark.parametrize("rho_s", [1.0, 1.4, 0.8])
def test_mass_conserved_in_cavity_with_solid(rho_s):
    # halfway bounce-back with the lid (corners included), the SFC and the
    # Guo forcing all conserve mass exactly
    cfg = workloads.cavity_disc_64()
    cfg["solid"]["rho_s"] = rho_s
    o = Oracle(**cfg).init()
    m0 = o.diag()["mass"]
    o.step(500)
    m1 = o.diag()["mass"]
    assert abs(m1 - m0) / m0 < 1e-13


def test_momentum_budget_with_uniform_force():
    # periodic box, uniform force density: sum_i c_i f_i grows by exactly F per
    # node and step (collision conserves momentum up to the Guo term)
    n, F = 24, np.array([1e-5, -2e-5])
    o = Oracle(**workloads.make(nx=n, ny=n, tau=0.7, periodic_x=True, periodic_y=True,
                                fext=tuple(F)))
    o.init(workloads.gaussian_velocity(n, n, 1e-3, seed=3))
    o.step(1)
    p1 = np.array([o.diag()["mom_x"], o.diag()["mom_y"]])
    o.step(200)
    p2 = np.array([o.diag()["mom_x"], o.diag()["mom_y"]])
    assert np.allclose(p2 - p1, 200 * n * n * F, rtol=1e-10, atol=1e-14)


def test_rest_state_with_density_contrast_is_fixed_point():
    # f = f^eq_SFC(rho_t, 0, drho): moving populations are all w_i rho_f, so the
    # density contrast of Eq. (2_3_drho) is kept exactly and nothing moves
    cfg = workloads.make(nx=48, ny=40, tau=0.9,
                         solid=dict(cx=22.0, cy=19.0, R=9.0, G=0.02, rho_s=1.5))
    o = Oracle(**cfg).init()
    f0 = o.populations()
    X0, Y0, _ = o.refmap()
    o.step(300)
    # rounding only: the zone map is re-fitted every step and feeds drho
    assert np.max(np.abs(o.populations() - f0)) < 1e-13
    X, Y, _ = o.refmap()
    m = ~np.isnan(X0)
    assert np.array_equal(m, ~np.isnan(X))
    tol = 1e-13 * np.max(np.abs(X0[m]))
    assert np.max(np.abs(X[m] - X0[m])) < tol and np.max(np.abs(Y[m] - Y0[m])) < tol
    rho, ux, uy = o.macro()
    assert rho.max() > 1.49 and np.max(np.abs(ux)) < 1e-13


def test_undeformed_solid_at_rest_keeps_xi_equal_x():
    cfg = workloads.cavity_disc_64()
    cfg["lid_ux"] = 0.0
    o = Oracle(**cfg).init().step(400)
    X, Y, _ = o.refmap()
    y, x = np.mgrid[0:64, 0:64] + 0.5
    m = ~np.isnan(X)
    assert m.sum() > 1000
    # solid nodes are not advected (u = 0 exactly); zone nodes are re-fitted
    # each step from exact solid values: rounding does not accumulate
    tol = 1e-13 * 64
    assert np.max(np.abs(X[m] - x[m])) < tol and np.max(np.abs(Y[m] - y[m])) < tol


@pytest.mark.parametrize("shape", [dict(), dict(shape="ellipse", b=5.0, theta=0.7)])
def test_rigid_translation(shape):
    # uniform flow through a periodic box with a neutrally buoyant disc or
    # ellipse: grad xi stays the identity (no stress, no force), the flow stays
    # uniform and xi(x, t) = x - u t exactly
    n, u = 64, np.array([0.05, 0.02])
    cfg = workloads.make(nx=n, ny=n, tau=0.7, periodic_x=True, periodic_y=True,
                         solid=dict(cx=24.0, cy=28.0, R=8.0, G=0.01, rho_s=1.0, **shape))
    o = Oracle(**cfg).init(workloads.uniform_velocity(n, n, *u))
    steps = 200
    o.step(steps)
    X, Y, _ = o.refmap()
    y, x = np.mgrid[0:n, 0:n] + 0.5
    m = ~np.isnan(X)
    assert m.sum() > 500
    assert np.max(np.abs(X[m] - (x[m] - steps * u[0]))) < 1e-11
    assert np.max(np.abs(Y[m] - (y[m] - steps * u[1]))) < 1e-11
    _, ux, uy = o.macro()
    assert np.max(np.abs(ux - u[0])) < 1e-13 and np.max(np.abs(uy - u[1])) < 1e-13
    d = o.diag()
    assert abs(d["centroid_x"] - (24.0 + steps * u[0])) < 0.05
    assert abs(d["centroid_y"] - (28.0 + steps * u[1])) < 0.05


def test_lid_with_fluid_density_conserves_mass_and_differs_only_where_rho_does():
    # lid_rho_mode 1: the moving-lid term uses rho_f instead of the
    # node's density.  Both lid links of a top node still cancel (mass is
    # exact); a flow whose top-row density stays rho_f is unchanged, and a
    # compressible cavity flow is not.
    base = workloads.cavity_disc_64()
    base["solid"]["rho_s"] = 1.3
    base["gravity"] = (0.0, -1e-4)
    o0 = Oracle(**base).init()
    o1 = Oracle(**dict(base, lid_rho_mode=1)).init()
    m0 = o1.diag()["mass"]
    o0.step(300)
    o1.step(300)
    assert abs(o1.diag()["mass"] - m0) < 1e-12 * m0
    r0, u0, _ = o0.macro()
    r1, u1, _ = o1.macro()
    assert np.max(np.abs(r0[-1] - 1.0)) > 1e-5
    assert np.max(np.abs(u1 - u0)) > 1e-9
    # the steady Couette profile, whose density is uniform, is still exact
    U, ny = 0.05, 16
    c1 = Oracle(**workloads.make(nx=4, ny=ny, tau=0.8, lid_ux=U, periodic_x=True,
                                 lid_rho_mode=1)).init()
    c1.step(20000)
    _, ux, uy = c1.macro()
    y = np.arange(ny) + 0.5
    assert np.max(np.abs(ux - U * y[:, None] / ny)) < 1e-12
    assert np.max(np.abs(uy)) < 1e-12 * U
    with pytest.raises(ValueError):
        Oracle(**dict(base, lid_rho_mode=2))
