"""Pins of the oracle's several-solid step (Sec. 3.6) on the CPU: symmetry
under relabelling the solids, rigid translation of several solids across a
periodic boundary (each map in its own unwrapped frame), exact mass
conservation, contact forces that are internal (zero net force) and push the
solids apart, linear in eta and G, zero for eta = 0, and the normalised
mixture density where solids overlap."""
import numpy as np
import pytest

import workloads
from oracle import Oracle

D1 = dict(cx=20.0, cy=32.0, R=8.0, G=0.01, rho_s=1.0)
D2 = dict(cx=44.0, cy=30.0, R=6.0, G=0.02, rho_s=1.0, shape="ellipse", b=9.0, theta=0.4)


def _fields(o):
    out = list(o.macro())
    for b in range(o.nsolid):
        out += list(o.refmap(b))
    return out


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(np.nan_to_num(x, nan=-9.0), np.nan_to_num(y, nan=-9.0))


def test_solid_order_does_not_matter():
    # two heavy solids close enough to touch under a lid-driven flow
    s1 = dict(D1, rho_s=1.3, cx=28.0)
    s2 = dict(D2, rho_s=1.6, cx=41.0)
    cfg = workloads.make(nx=64, ny=64, tau=0.8, lid_ux=0.08, gravity=(0.0, -1e-5),
                         solids=[s1, s2])
    a = Oracle(**cfg).init().step(60)
    b = Oracle(**dict(cfg, solids=[s2, s1])).init().step(60)
    fa, fb = _fields(a), _fields(b)
    _same(fa[:3], fb[:3])
    _same(fa[3:6], fb[6:9])
    _same(fa[6:9], fb[3:6])


def test_one_solid_in_a_list_is_the_single_solid_path():
    cfg = workloads.make(nx=48, ny=40, tau=0.8, lid_ux=0.05, solid=dict(D1, cx=24.0, cy=20.0))
    a = Oracle(**cfg).init().step(40)
    b = Oracle(**dict(cfg, solid=None, solids=[cfg["solid"]])).init().step(40)
    _same(_fields(a), _fields(b))


def test_rigid_translation_across_the_periodic_boundary():
    # uniform flow through a periodic box: grad xi stays the identity for
    # every solid, so there is no stress and no contact; each map obeys
    # xi(x, t) = x - u t in its own unwrapped frame (nearest image of the
    # reference centre), including the solid that crosses the boundary
    n, u = 64, np.array([0.05, -0.04])
    s1 = dict(D1, cx=58.0, cy=10.0)          # crosses x = n and y = 0
    s2 = dict(D2, cx=26.0, cy=40.0)
    cfg = workloads.make(nx=n, ny=n, tau=0.7, periodic_x=True, periodic_y=True,
                         solids=[s1, s2])
    o = Oracle(**cfg).init(workloads.uniform_velocity(n, n, *u))
    steps = 150
    o.step(steps)
    y, x = np.mgrid[0:n, 0:n] + 0.5
    for b, s in enumerate((s1, s2)):
        X, Y, _ = o.refmap(b)
        xu = s["cx"] + (x - s["cx"] + n / 2) % n - n / 2
        yu = s["cy"] + (y - s["cy"] + n / 2) % n - n / 2
        m = ~np.isnan(X)
        assert m.sum() > 300
        assert np.max(np.abs(X[m] - (xu[m] - steps * u[0]))) < 1e-11
        assert np.max(np.abs(Y[m] - (yu[m] - steps * u[1]))) < 1e-11
        d = o.diag_body(b)
        assert abs(d["disp_x"] - steps * u[0]) < 1e-9 and abs(d["disp_y"] - steps * u[1]) < 1e-9
    _, ux, uy = o.macro()
    assert np.max(np.abs(ux - u[0])) < 1e-13 and np.max(np.abs(uy - u[1])) < 1e-13


def test_mass_is_conserved_with_several_heavy_solids():
    cfg = workloads.make(nx=64, ny=64, tau=0.8, lid_ux=0.06, gravity=(0.0, -2e-5),
                         solids=[dict(D1, rho_s=1.5, cx=28.0), dict(D2, rho_s=1.2, cx=42.0)])
    o = Oracle(**cfg).init()
    m0 = o.diag()["mass"]
    o.step(200)
    assert abs(o.diag()["mass"] - m0) < 1e-10 * m0


def _overlap(eta=1.0, G=(0.01, 0.02), gap=-3.0, rho=(1.0, 1.0)):
    # two undeformed discs at rest on one row, their solid regions overlapping
    # by -gap nodes: the elastic stress is zero (grad xi = I) and, with equal
    # densities, so is every force other than the contact stress
    n = 64
    c1, r = 24.0, 8.0
    c2 = c1 + 2 * r + gap
    cfg = workloads.make(nx=n, ny=n, tau=0.8, periodic_x=True, periodic_y=True, eta=eta,
                         solids=[dict(cx=c1, cy=32.0, R=r, G=G[0], rho_s=rho[0]),
                                 dict(cx=c2, cy=32.0, R=r, G=G[1], rho_s=rho[1])])
    o = Oracle(**cfg).init()
    o.step(1)
    return o, 0.5 * (c1 + c2)


def test_contact_force_is_internal_and_repulsive():
    o, xm = _overlap()
    fx, fy = o.force()
    assert np.max(np.abs(fx)) > 1e-4
    # Newton's third law: the contact stress is a divergence on a periodic grid
    assert abs(fx.sum()) < 1e-14 and abs(fy.sum()) < 1e-14
    x = np.arange(64) + 0.5
    left, right = fx[:, x < xm].sum(), fx[:, x > xm].sum()
    assert left < -1e-4 and right > 1e-4
    # mirror symmetry about the row through both centres
    assert np.allclose(fx[32 - 5:32], fx[32:32 + 5][::-1], rtol=0, atol=1e-13)


def test_contact_force_scales_with_eta_and_moduli_and_vanishes_without_overlap():
    # the extrapolated zone reproduces xi = x up to rounding only, so the
    # elastic stress is a rounding residue (~1e-17) beside the contact stress
    f1 = _overlap(eta=1.0)[0].force()[0]
    scale = np.max(np.abs(f1))
    assert scale > 1e-4
    f2 = _overlap(eta=2.0)[0].force()[0]
    assert np.max(np.abs(2.0 * f1 - f2)) < 1e-11 * scale
    fg = _overlap(G=(0.02, 0.04))[0].force()[0]
    assert np.max(np.abs(2.0 * f1 - fg)) < 1e-11 * scale
    assert np.max(np.abs(_overlap(eta=0.0)[0].force()[0])) < 1e-13
    # blur zones apart (gap > 2 eps): no contact even though the extrapolation
    # zones overlap
    assert np.max(np.abs(_overlap(gap=3.2)[0].force()[0])) < 1e-13


def test_mixture_density_is_normalised_where_solids_overlap():
    o2 = Oracle(**workloads.make(nx=64, ny=64, tau=0.8, periodic_x=True, periodic_y=True,
                                 solids=[dict(cx=24.0, cy=32.0, R=8.0, G=0.01, rho_s=1.4),
                                         dict(cx=34.0, cy=32.0, R=8.0, G=0.02, rho_s=1.8)])).init()
    rho, _, _ = o2.macro()
    # a node deep inside both discs (lambda = 1 for each): rho_f plus the
    # average of the two excesses
    assert abs(rho[32, 29] - (1.0 + 0.5 * (0.4 + 0.8))) < 1e-15
    # deep inside one disc only: that disc's density
    assert abs(rho[32, 18] - 1.4) < 1e-15 and abs(rho[32, 38] - 1.8) < 1e-15


def _approach(eta, steps=400, U=0.03):
    # two discs whose blur zones already overlap, driven together by the flow
    n = 64
    cfg = workloads.make(nx=n, ny=n, tau=0.8, periodic_x=True, periodic_y=True, eta=eta,
                         solids=[dict(cx=20.0, cy=32.0, R=8.0, G=0.015, rho_s=1.0),
                                 dict(cx=37.0, cy=32.0, R=8.0, G=0.015, rho_s=1.0)])
    u0 = np.zeros((2, n, n))
    x = np.arange(n) + 0.5
    u0[0][:, x < 28.5] = U
    u0[0][:, x >= 28.5] = -U
    o = Oracle(**cfg).init(u0)
    dmin = np.inf
    for _ in range(steps // 20):
        o.step(20)
        dmin = min(dmin, o.diag_body(1)["centroid_x"] - o.diag_body(0)["centroid_x"])
    return dmin


def test_contact_keeps_colliding_solids_further_apart():
    d0, d1, d10 = _approach(0.0), _approach(1.0), _approach(10.0)
    assert d0 < d1 < d10
