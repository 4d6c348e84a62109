"""Pins of the oracle's reference-map phases (Secs. 3.1-3.3): layers against a
brute-force distance, exactness of the extrapolation and the advection on
linear maps, order independence, and the force closed forms (CPU only)."""
import numpy as np
import pytest

import workloads
from oracle import Oracle, layers_mask


def _brute_layers(solid, L):
    ny, nx = solid.shape
    js, is_ = np.nonzero(solid)
    out = np.full((ny, nx), -1, np.int32)
    for j in range(ny):
        for i in range(nx):
            if solid[j, i]:
                out[j, i] = 0
            elif len(is_):
                d = np.min(np.abs(is_ - i) + np.abs(js - j))
                if d <= L:
                    out[j, i] = d
    return out


@pytest.mark.parametrize("seed", range(4))
def test_layers_equal_manhattan_distance(seed):
    # Sec. 3.2: layer 1 = 4-neighbours of the solid, layer l = 4-neighbours of
    # layer l-1; on a rectangle this is the Manhattan distance to the solid
    rng = np.random.default_rng(seed)
    solid = np.zeros((30, 37), np.uint8)
    for _ in range(3):
        cx, cy, r = rng.uniform(5, 32), rng.uniform(5, 25), rng.uniform(1, 5)
        y, x = np.mgrid[0:30, 0:37]
        solid |= ((x - cx) ** 2 + (y - cy) ** 2 < r * r).astype(np.uint8)
    solid |= (rng.random(solid.shape) < 0.01).astype(np.uint8)
    L = 6
    assert np.array_equal(layers_mask(solid, L), _brute_layers(solid, L))


A_LIN = np.array([[1.03, -0.06], [0.04, 0.98]])
B_LIN = np.array([0.7, -1.1])


def _plant_linear(o, nx, ny):
    x = np.arange(-2, nx + 2) + 0.5
    y = np.arange(-2, ny + 2) + 0.5
    Xg, Yg = np.meshgrid(x, y)
    X = A_LIN[0, 0] * Xg + A_LIN[0, 1] * Yg + B_LIN[0]
    Y = A_LIN[1, 0] * Xg + A_LIN[1, 1] * Yg + B_LIN[1]
    o.set_refmap_padded(X, Y)
    return Xg, Yg


def _disc_sim(nx=48, ny=44, reverse=False):
    cfg = workloads.make(nx=nx, ny=ny, tau=0.8, reverse_order=reverse,
                         solid=dict(cx=24.0, cy=22.0, R=8.0, G=0.01, rho_s=1.0))
    o = Oracle(**cfg).init()
    return o, cfg


def test_extrapolation_reproduces_linear_map_and_layers():
    o, cfg = _disc_sim()
    nx, ny = cfg["nx"], cfg["ny"]
    Xg, Yg = _plant_linear(o, nx, ny)
    o.set_moments(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)))
    X0, Y0, phi0 = o.refmap_padded()
    o.phase("advect")
    o.phase("extrapolate")
    lay = o.layers_padded()
    o.phase("relabel")
    X, Y, _ = o.refmap_padded()
    # layers = Manhattan distance to the interior solid set, capped at 11
    solid = np.zeros_like(lay, dtype=np.uint8)
    solid[2:-2, 2:-2] = phi0[2:-2, 2:-2] < 0
    assert np.array_equal(lay, _brute_layers(solid, cfg["layers"]))
    zone = lay > 0
    assert zone.sum() > 500
    ex = A_LIN[0, 0] * Xg + A_LIN[0, 1] * Yg + B_LIN[0]
    ey = A_LIN[1, 0] * Xg + A_LIN[1, 1] * Yg + B_LIN[1]
    assert np.all(np.isfinite(X[zone]))
    # exact up to rounding that accumulates over the 11 layers (relative 1e-13)
    tol = 1e-13 * np.max(np.abs(ex[zone]))
    assert np.max(np.abs(X[zone] - ex[zone])) < tol
    assert np.max(np.abs(Y[zone] - ey[zone])) < tol
    assert np.all(np.isnan(X[lay < 0]))
    assert o.counters()[1] == 0


def test_extrapolation_independent_of_target_order():
    runs = []
    for rev in (False, True):
        cfg = workloads.cavity_disc_64()
        cfg["reverse_order"] = rev
        o = Oracle(**cfg).init().step(60)
        runs.append(o.refmap_padded())
    for a, b in zip(*runs):
        assert np.array_equal(np.nan_to_num(a, nan=-7.0), np.nan_to_num(b, nan=-7.0))


def test_advection_translates_linear_map_exactly():
    # Eqs. (3_1_refmap_adv), (3_1_eno): the one-sided 3-point differences are
    # exact on linear maps, so xi^{n+1} = xi - A u at every solid node
    o, cfg = _disc_sim()
    nx, ny = cfg["nx"], cfg["ny"]
    Xg, Yg = _plant_linear(o, nx, ny)
    u = np.array([0.031, -0.017])
    o.set_moments(np.ones((ny, nx)), np.full((ny, nx), u[0]), np.full((ny, nx), u[1]))
    _, _, phi0 = o.refmap_padded()
    o.phase("advect")
    o.phase("extrapolate")
    o.phase("relabel")
    X, Y, _ = o.refmap_padded()
    shift = A_LIN @ u
    ex = A_LIN[0, 0] * Xg + A_LIN[0, 1] * Yg + B_LIN[0] - shift[0]
    ey = A_LIN[1, 0] * Xg + A_LIN[1, 1] * Yg + B_LIN[1] - shift[1]
    m = np.isfinite(X)
    assert m.sum() > 500
    tol = 1e-13 * np.max(np.abs(ex[m]))
    assert np.max(np.abs(X[m] - ex[m])) < tol and np.max(np.abs(Y[m] - ey[m])) < tol


def _planted_force(nx, ny, periodic, Xf, Yf, G=0.05):
    cfg = workloads.make(nx=nx, ny=ny, tau=0.8, periodic_x=periodic, periodic_y=periodic,
                         solid=dict(cx=nx / 2, cy=ny / 2, R=10.0, G=G, rho_s=1.0))
    o = Oracle(**cfg).init()
    x = np.arange(-2, nx + 2) + 0.5
    y = np.arange(-2, ny + 2) + 0.5
    Xg, Yg = np.meshgrid(x, y)
    X, Y = Xf(Xg, Yg), Yf(Xg, Yg)
    if periodic:
        X[:2, :] = X[-2:, :] = X[:, :2] = X[:, -2:] = np.nan
    o.set_refmap_padded(X, Y)
    o.phase("force")
    return o, cfg


@pytest.mark.parametrize("gam", [0.1, -0.25])
def test_uniform_shear_gives_closed_form_stress_and_zero_interior_force(gam):
    # a uniform deformation has the same half-edge stress everywhere, so the
    # divergence vanishes wherever all four edges are fully solid, and the node
    # stress equals G [[2g^2/3, g], [g, -g^2/3]] (Eq. (3_3_solid_stress))
    G = 0.05
    o, cfg = _planted_force(40, 40, False, lambda x, y: x - gam * y, lambda x, y: y, G)
    fx, fy = o.force()
    sxx, sxy, syy = o.stress()
    _, _, phi = o.refmap()
    deep = phi < -(cfg["eps"] + 2.0)
    assert deep.sum() > 50
    assert np.max(np.abs(fx[deep])) < 1e-15 and np.max(np.abs(fy[deep])) < 1e-15
    assert np.allclose(sxx[deep], G * 2 * gam ** 2 / 3, atol=1e-15)
    assert np.allclose(sxy[deep], G * gam, atol=1e-15)
    assert np.allclose(syy[deep], -G * gam ** 2 / 3, atol=1e-15)
    # the blur zone does feel a force
    assert np.max(np.hypot(fx, fy)) > 1e-4 * G


def test_force_divergence_telescopes_on_periodic_grid():
    # flux form with the solid fraction taken at the half-edges: the sum of the
    # divergence over a periodic grid is zero
    n = 40
    k = 2 * np.pi / n
    o, _ = _planted_force(n, n, True, lambda x, y: x + 0.4 * np.sin(k * y) / k * 0.1,
                          lambda x, y: y - 0.3 * np.sin(k * x) / k * 0.1)
    fx, fy = o.force()
    assert np.max(np.abs(fx)) > 1e-4
    assert abs(fx.sum()) < 1e-15 * fx.size and abs(fy.sum()) < 1e-15 * fy.size
