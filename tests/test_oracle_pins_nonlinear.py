"""Pins of the oracle's reference-map phases on NON-linear inputs (CPU only).

Linear maps are reproduced by any consistent difference and by any weighting
of the least-squares fit, so the pins here use curved maps and a solid under
gravity, where a plausible slip (a first-order difference, other weights, a
missing normal factor, the wrong buoyancy) changes the result:

* Eq. (3_1_eno): the one-sided three-point difference is exact on quadratics,
  so one advection step of a quadratic map equals xi - u dxi/dx - v dxi/dy with
  the analytic derivatives, for every sign combination of (u, v).
* Sec. 3.2 / Eq. (3_2_extrap_weight): every extrapolated value equals the
  intercept of a weighted least-squares fit computed here independently
  (numpy lstsq on sqrt(w)-scaled rows), with the valid set, the scan-window
  growth and the weights written from the paper's steps (i)-(iii).
* The solid fraction of a half-edge (1 - H at the mean level set
  of its two nodes), through the node stress of a uniform shear.
* The buoyancy of a heavy solid ((1 - H)(rho_s - rho_f) g per node), through
  the force and the first step's momentum change in a periodic box.
"""
import numpy as np
import pytest

import workloads
from oracle import Oracle


def _H(phi, eps):
    """H_eps of Eq. (2_3_heaviside), written out here for the pins."""
    phi = np.asarray(phi, dtype=np.float64)
    mid = 0.5 * (1.0 + phi / eps + np.sin(np.pi * phi / eps) / np.pi)
    return np.where(phi < -eps, 0.0, np.where(phi > eps, 1.0, mid))


def _padded_coords(nx, ny):
    x = np.arange(-2, nx + 2) + 0.5
    y = np.arange(-2, ny + 2) + 0.5
    return np.meshgrid(x, y)


CX, CY, R = 24.0, 22.0, 8.0


def _disc_oracle(nx=48, ny=44, **kw):
    cfg = workloads.make(nx=nx, ny=ny, tau=0.8,
                         solid=dict(cx=CX, cy=CY, R=R, G=0.01, rho_s=1.0), **kw)
    return Oracle(**cfg).init(), cfg


# ------------------------------------------------------------ advection

# xi = x + quadratic: constant second derivatives, non-zero in both axes
QX = dict(a=0.004, b=-0.003, c=0.002, d=0.05, e=-0.02)
QY = dict(a=-0.002, b=0.0035, c=0.003, d=-0.04, e=0.03)


def _quad(q, x, y):
    u, v = x - CX, y - CY
    return q["a"] * u * u + q["b"] * u * v + q["c"] * v * v + q["d"] * u + q["e"] * v


def _quad_grad(q, x, y):
    u, v = x - CX, y - CY
    return 2 * q["a"] * u + q["b"] * v + q["d"], q["b"] * u + 2 * q["c"] * v + q["e"]


@pytest.mark.parametrize("vel", [(0.031, 0.017), (-0.023, 0.029), (0.027, -0.033),
                                 (-0.019, -0.021), (0.0, 0.025), (-0.03, 0.0)])
def test_advection_is_exact_on_quadratic_maps(vel):
    o, cfg = _disc_oracle()
    nx, ny = cfg["nx"], cfg["ny"]
    Xg, Yg = _padded_coords(nx, ny)
    X0 = Xg + _quad(QX, Xg, Yg)
    Y0 = Yg + _quad(QY, Xg, Yg)
    o.set_refmap_padded(X0, Y0)
    u, v = vel
    o.set_moments(np.ones((ny, nx)), np.full((ny, nx), u), np.full((ny, nx), v))
    _, _, phin = o.refmap_padded()
    solid = np.zeros_like(phin, dtype=bool)
    solid[2:-2, 2:-2] = phin[2:-2, 2:-2] < 0
    assert solid.sum() > 150
    o.phase("advect")
    o.phase("relabel")          # no extrapolation: only the advected nodes hold values
    X1, Y1, _ = o.refmap_padded()
    assert np.array_equal(np.isfinite(X1), solid)
    gxx, gxy = _quad_grad(QX, Xg, Yg)
    gyx, gyy = _quad_grad(QY, Xg, Yg)
    eX = X0 - (u * (1.0 + gxx) + v * gxy)
    eY = Y0 - (u * gyx + v * (1.0 + gyy))
    scale = np.max(np.abs(eX[solid]))
    assert np.max(np.abs(X1[solid] - eX[solid])) < 1e-13 * scale
    assert np.max(np.abs(Y1[solid] - eY[solid])) < 1e-13 * scale
    # a first-order upwind difference would be off by |u| xi_xx / 2 + |v| xi_yy / 2
    first_order_gap = 0.5 * (abs(u) * 2 * abs(QX["a"]) + abs(v) * 2 * abs(QX["c"]))
    assert first_order_gap > 1e3 * 1e-13 * scale


# ------------------------------------------------------------ extrapolation

def _nonlinear_map(Xg, Yg):
    X = Xg + 0.004 * (Yg - CY) ** 2 + 0.3 * np.sin(0.3 * Yg) + 0.002 * (Xg - CX) * (Yg - CY)
    Y = Yg - 0.003 * (Xg - CX) * (Yg - CY) + 0.2 * np.cos(0.25 * Xg) + 0.003 * (Xg - CX) ** 2
    return X, Y


def _wls_intercept(lay, Xv, Yv, phin, jt, it, l, r_max, det_rel):
    """Sec. 3.2 for target (jt, it) of layer l on padded arrays: grow the
    square scan window from half-width 2 until it holds at least three valid
    nodes (solid, or set in an earlier layer) and the weighted normal matrix
    is well posed; weights 2^-(|di| + |dj|), times the positive
    part of the cosine between d = x_t - x_k and the level-set normal for
    layers 1 and 2; the value at the target is the intercept of
    xi ~ A dx + B dy + C in target-centred coordinates."""
    ny, nx = lay.shape
    nrm = None
    if l <= 2:
        nb = [(jt, it + 1), (jt, it - 1), (jt + 1, it), (jt - 1, it)]
        if all(0 <= a < ny and 0 <= b < nx and np.isfinite(phin[a, b]) for a, b in nb):
            g = np.array([phin[jt, it + 1] - phin[jt, it - 1],
                          phin[jt + 1, it] - phin[jt - 1, it]]) / 2.0
            if np.hypot(*g) > 0:
                nrm = g / np.hypot(*g)
    for r in range(2, r_max + 1):
        rows, wts, vx, vy = [], [], [], []
        for dj in range(-r, r + 1):
            for di in range(-r, r + 1):
                j, i = jt + dj, it + di
                if not (0 <= j < ny and 0 <= i < nx):
                    continue
                lk = lay[j, i]
                if not (lk == 0 or (0 < lk < l and np.isfinite(Xv[j, i]))):
                    continue
                w = 2.0 ** (-(abs(di) + abs(dj)))
                if nrm is not None:
                    d = np.array([-di, -dj], dtype=np.float64)       # x_t - x_k
                    w *= max(0.0, float(d @ nrm) / np.hypot(*d))
                rows.append([di, dj, 1.0])
                wts.append(w)
                vx.append(Xv[j, i])
                vy.append(Yv[j, i])
        if len(rows) < 3:
            continue
        A = np.array(rows)
        w = np.array(wts)
        M = A.T @ (w[:, None] * A)
        if not np.linalg.det(M) > det_rel * w.sum() ** 3:
            continue
        sw = np.sqrt(w)[:, None]
        cx = np.linalg.lstsq(sw * A, sw[:, 0] * np.array(vx), rcond=None)[0]
        cy = np.linalg.lstsq(sw * A, sw[:, 0] * np.array(vy), rcond=None)[0]
        return cx[2], cy[2], r
    return np.nan, np.nan, r_max + 1


def _brute_layers(solid, L):
    ny, nx = solid.shape
    js, is_ = np.nonzero(solid)
    jj, ii = np.mgrid[0:ny, 0:nx]
    d = np.full((ny, nx), 10 ** 6)
    for a, b in zip(js, is_):
        d = np.minimum(d, np.abs(jj - a) + np.abs(ii - b))
    out = np.where(d <= L, d, -1)
    out[solid] = 0
    return out


@pytest.mark.parametrize("case", ["disc", "ellipse"])
def test_extrapolation_matches_independent_weighted_least_squares(case):
    kw = {}
    if case == "ellipse":
        solid = dict(cx=CX, cy=CY, R=10.0, b=5.0, theta=0.6, shape="ellipse", G=0.01,
                     rho_s=1.0)
    else:
        solid = dict(cx=CX, cy=CY, R=R, G=0.01, rho_s=1.0)
    cfg = workloads.make(nx=48, ny=44, tau=0.8, solid=solid, **kw)
    o = Oracle(**cfg).init()
    nx, ny = cfg["nx"], cfg["ny"]
    Xg, Yg = _padded_coords(nx, ny)
    X0, Y0 = _nonlinear_map(Xg, Yg)
    o.set_refmap_padded(X0, Y0)
    o.set_moments(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))
    _, _, phin = o.refmap_padded()
    o.phase("advect")           # u = 0: the solid values stay as planted
    o.phase("extrapolate")
    lay = o.layers_padded()
    o.phase("relabel")
    X1, Y1, _ = o.refmap_padded()
    solid_set = np.zeros(lay.shape, dtype=bool)
    solid_set[2:-2, 2:-2] = phin[2:-2, 2:-2] < 0
    assert np.array_equal(lay, _brute_layers(solid_set, cfg["layers"]))
    assert np.array_equal(X1[solid_set], X0[solid_set])
    checked = {1: 0, 2: 0, 3: 0}
    grown = 0
    worst = 0.0
    for l in range(1, cfg["layers"] + 1):
        for jt, it in zip(*np.nonzero(lay == l)):
            ex, ey, r = _wls_intercept(lay, X1, Y1, phin, jt, it, l, cfg["r_max"],
                                       cfg["det_rel"])
            assert np.isfinite(ex), (l, jt, it)
            worst = max(worst, abs(X1[jt, it] - ex), abs(Y1[jt, it] - ey))
            checked[min(l, 3)] += 1
            grown += r > 2
    assert min(checked.values()) > 40, checked
    # the fits are 3x3 normal equations solved by Cramer's rule in the oracle
    # and an SVD least-squares solve here: agreement to rounding of |xi| ~ 50
    print("worst", worst, checked, grown)
    assert worst < 5e-12, worst


def test_extrapolation_weights_matter_on_the_nonlinear_map():
    """Guard of the pin above: on this map, other weightings (uniform,
    2^-max(|di|, |dj|), or no normal factor) give layer-1 values that differ
    by far more than the pin's tolerance, so the pin can tell them apart."""
    nx, ny = 48, 44
    Xg, Yg = _padded_coords(nx, ny)
    X0, _ = _nonlinear_map(Xg, Yg)
    # a layer-1-like target just outside the disc, east side, valid nodes west
    jt, it = int(CY) + 2, int(CX + R) + 3
    pts = [(dj, di) for dj in range(-2, 3) for di in range(-2, 3) if di <= -1]

    def fit(wfun):
        A = np.array([[di, dj, 1.0] for dj, di in pts])
        w = np.array([wfun(di, dj) for dj, di in pts])
        v = np.array([X0[jt + dj, it + di] for dj, di in pts])
        sw = np.sqrt(w)[:, None]
        return np.linalg.lstsq(sw * A, sw[:, 0] * v, rcond=None)[0][2]

    base = fit(lambda di, dj: 2.0 ** (-(abs(di) + abs(dj))))
    for other in (lambda di, dj: 1.0, lambda di, dj: 2.0 ** (-max(abs(di), abs(dj)))):
        assert abs(fit(other) - base) > 1e-6


# ------------------------------------------------------------ edge fraction

@pytest.mark.parametrize("gam", [0.15, -0.2])
def test_half_edge_solid_fraction_is_taken_at_the_mean_level_set(gam):
    # uniform shear xi = (x - gam y, y): tau is the same closed form on every
    # half-edge, so the node stress (average of its four half-edges) is
    # tau * mean over the four edges of 1 - H((phi_a + phi_b) / 2)
    nx = ny = 40
    G, eps = 0.05, 1.5
    cfg = workloads.make(nx=nx, ny=ny, tau=0.8,
                         solid=dict(cx=20.0, cy=20.0, R=10.0, G=G, rho_s=1.0))
    o = Oracle(**cfg).init()
    Xg, Yg = _padded_coords(nx, ny)
    X, Y = Xg - gam * Yg, Yg.copy()
    o.set_refmap_padded(X, Y)
    o.phase("force")
    sxx, sxy, syy = o.stress()
    phi = np.hypot(X - 20.0, Y - 20.0) - 10.0     # disc level set at the map
    c = slice(2, -2)
    lamL = 1 - _H(0.5 * (phi[c, 1:-3] + phi[c, c]), eps)
    lamR = 1 - _H(0.5 * (phi[c, c] + phi[c, 3:-1]), eps)
    lamB = 1 - _H(0.5 * (phi[1:-3, c] + phi[c, c]), eps)
    lamT = 1 - _H(0.5 * (phi[c, c] + phi[3:-1, c]), eps)
    frac = 0.25 * (lamL + lamR + lamB + lamT)
    assert np.max(np.abs(sxy - G * gam * frac)) < 1e-15
    assert np.max(np.abs(sxx - G * 2 * gam * gam / 3 * frac)) < 1e-15
    assert np.max(np.abs(syy + G * gam * gam / 3 * frac)) < 1e-15
    # the other reading (mean of the two node fractions) differs here
    lam = 1 - _H(phi, eps)
    alt = 0.25 * (0.5 * (lam[c, 1:-3] + lam[c, c]) + 0.5 * (lam[c, c] + lam[c, 3:-1]) +
                  0.5 * (lam[1:-3, c] + lam[c, c]) + 0.5 * (lam[c, c] + lam[3:-1, c]))
    assert np.max(np.abs(alt - frac)) > 1e-3


# ------------------------------------------------------------ buoyancy

@pytest.mark.parametrize("rho_s,g", [(1.6, (0.0, -1e-4)), (0.7, (3e-5, 8e-5))])
def test_buoyancy_force_and_first_step_momentum(rho_s, g):
    # periodic box, solid at rest with xi = x: the stress vanishes (J = I up
    # to the rounding of the extrapolated zone values), so the force density is
    # the buoyancy (1 - H(phi0(x)))(rho_s - rho_f) g alone.  With tau = 1 the
    # BGK-Guo step adds exactly the summed force to the momentum
    # sum_nodes (sum_i c_i f_i + F / 2).
    n, eps = 48, 1.5
    cfg = workloads.make(nx=n, ny=n, tau=1.0, periodic_x=True, periodic_y=True, gravity=g,
                         solid=dict(cx=23.3, cy=25.1, R=9.0, G=0.02, rho_s=rho_s))
    o = Oracle(**cfg).init()
    d0 = o.diag()
    assert abs(d0["mom_x"]) < 1e-15 and abs(d0["mom_y"]) < 1e-15
    o.step(1)
    fx, fy = o.force()
    x = np.arange(n) + 0.5
    Xn, Yn = np.meshgrid(x, x)
    phi = np.hypot(Xn - 23.3, Yn - 25.1) - 9.0
    bx = (1 - _H(phi, eps)) * (rho_s - 1.0) * g[0]
    by = (1 - _H(phi, eps)) * (rho_s - 1.0) * g[1]
    G = cfg["solid"]["G"]
    assert np.max(np.abs(fx - bx)) < 1e-12 * G and np.max(np.abs(fy - by)) < 1e-12 * G
    gn = np.hypot(*g)
    assert abs(fx.sum() - bx.sum()) < 1e-12 * gn and abs(fy.sum() - by.sum()) < 1e-12 * gn
    # momentum sums run over 9 N populations of order 0.1: rounding ~ 1e-13
    d1 = o.diag()
    assert abs(d1["mom_x"] - bx.sum()) < 1e-12
    assert abs(d1["mom_y"] - by.sum()) < 1e-12
    # the pin separates the buoyancy from rho_s g or a flipped sign
    assert np.hypot(bx.sum(), by.sum()) > 10.0 * gn


def test_buoyancy_momentum_over_steps_general_tau():
    # R5 (Alg. 1 literal): u^n carries F^{n-1}/2, the collision of step n uses
    # F^n, so P^{n+1} - P^n = F^{n-1} (1/(2 tau) - 1/2) + F^n (3/2 - 1/(2 tau)),
    # summed over the nodes; checked each step with the oracle's own forces
    n, tau = 40, 0.7
    cfg = workloads.make(nx=n, ny=n, tau=tau, periodic_x=True, periodic_y=True,
                         gravity=(0.0, -2e-4),
                         solid=dict(cx=19.6, cy=21.2, R=8.0, G=0.02, rho_s=1.5))
    o = Oracle(**cfg).init()
    P = np.array([o.diag()["mom_x"], o.diag()["mom_y"]])
    Fprev = np.zeros(2)
    for _ in range(6):
        o.step(1)
        fx, fy = o.force()
        F = np.array([fx.sum(), fy.sum()])
        d = o.diag()
        P1 = np.array([d["mom_x"], d["mom_y"]])
        expect = Fprev * (0.5 / tau - 0.5) + F * (1.5 - 0.5 / tau)
        assert np.allclose(P1 - P, expect, rtol=1e-10, atol=1e-12), (P1 - P, expect)
        P, Fprev = P1, F
    assert abs(F[1]) > 1e-3
