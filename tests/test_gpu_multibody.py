"""Several solids (Sec. 3.6) on the HIP path against the FP64 CPU oracle.

Bars of the single-solid parity tests (FP64 1e-10, FP32 1e-5) on rho and u
(u against max |u|); every solid's reference map is compared on its own, its
node set must agree exactly, and its error is measured against the grid's
extent max(nx, ny) (a solid near the origin of its unwrapped frame has
|xi| near zero, so |xi| itself is no scale).  Cases: walled cavity (every
window the whole grid), a small periodic box (whole-axis windows, contact,
density contrast, gravity), a periodic box with sub-windows where one solid
sits on the periodic corner (windows wrapping both seams) and solids touch,
a lid-driven periodic channel (sub-windows along x, whole axis along y) in
FP64 and FP32, one solid through the several-solid path, graph replay
against eager launches, and the full-size suspension (4096^2, 400 solids,
FP32) on invariants.

FP32 stores xi as the displacement xi - x; when solids translate, its
rounding adds up to about (steps) x ulp(|xi - x|) / 2, so FP32 cases here run
lid-driven flows for 200 steps (a stream that carries the solids 5 nodes in
250 steps reaches 1e-4 absolute on xi and 3e-5 on u, on the single-solid path
as well).
"""
import numpy as np
import pytest

import workloads
from oracle import Oracle
from test_gpu_fp32 import TOL32
from test_gpu_parity import _np, rel

pytestmark = pytest.mark.gpu


def _sim(cfg, precision="f64", u0=None):
    from paper_2402_12696_amd import Sim
    return Sim(device="cuda:0", precision=precision, **cfg).init(u0)


def compare_mb(sim, ref, tol=1e-10, what=""):
    rho, ux, uy = _np(sim.macro())
    rr, ru, rv = ref.macro()
    umax = max(np.max(np.abs(ru)), np.max(np.abs(rv)))
    du = max(np.max(np.abs(ux - ru)), np.max(np.abs(uy - rv)))
    errs = {"rho": rel(rho, rr), "u": du / umax if umax > 0 else du}
    for b in range(ref.nsolid):
        X, Y, P = _np(sim.refmap(b))
        RX, RY, RP = ref.refmap(b)
        mg, mr = ~np.isnan(X), ~np.isnan(RX)
        mism = int(np.sum(mg != mr))
        assert mism == 0, f"{what}: solid {b} node sets differ at {mism} nodes"
        assert np.array_equal(P[mg] < 0, RP[mr] < 0), f"{what}: solid {b} solid sets differ"
        ext = max(ref.nx, ref.ny)
        errs[f"X{b}"] = max(np.max(np.abs(X[mr] - RX[mr])), np.max(np.abs(Y[mr] - RY[mr]))) / ext
    print(what, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{what}: {bad}"


def _run(cfg, steps, precision="f64", tol=1e-10, u0=None):
    sim = _sim(cfg, precision, u0)
    ref = Oracle(**cfg).init(u0)
    compare_mb(sim, ref, tol, f"{precision} step 0")
    done = 0
    for n in steps:
        sim.step(n - done)
        ref.step(n - done)
        done = n
        compare_mb(sim, ref, tol, f"{precision} step {n}")
    d = sim.diag()
    assert all(v == 0 for v in d["health"].values()), d["health"]
    dr = ref.diag()
    ext = max(ref.nx, ref.ny)
    assert abs(d["mass"] - dr["mass"]) < max(tol, 1e-12) * dr["mass"]
    for b in range(ref.nsolid):
        a, r = sim.diag_solid(b), ref.diag_body(b)
        assert abs(a["centroid_x"] - r["centroid_x"]) < tol * ext
        assert abs(a["centroid_y"] - r["centroid_y"]) < tol * ext
        assert a["n_band"] == r["n_band"] and a["n_solid"] == r["n_solid"]
    sim.close()


def _cavity3():
    return workloads.make(nx=96, ny=80, tau=0.8, lid_ux=0.08, gravity=(0.0, -1e-5),
                          solids=[dict(cx=30.0, cy=50.0, R=10.0, G=0.01, rho_s=1.2),
                                  dict(cx=52.5, cy=48.0, R=9.0, G=0.02, rho_s=1.5,
                                       shape="ellipse", b=6.0, theta=0.3),
                                  dict(cx=70.0, cy=26.0, R=8.0, G=0.01, rho_s=1.0)])


def test_three_solids_in_a_cavity_match_oracle():
    _run(_cavity3(), (1, 40, 400))


def _touching_periodic(n=72, **kw):
    # whole-axis windows (72 is not a multiple of 16); the zones stay clear of
    # the periodic seams, which such windows cannot cross
    return workloads.make(nx=n, ny=n, tau=0.8, periodic_x=True, periodic_y=True,
                          gravity=(0.0, -2e-5), **kw,
                          solids=[dict(cx=28.0, cy=36.0, R=8.0, G=0.015, rho_s=1.3),
                                  dict(cx=45.0, cy=37.0, R=8.0, G=0.015, rho_s=1.6)])


def test_touching_solids_in_a_periodic_box_match_oracle():
    n = 72
    u0 = np.zeros((2, n, n))
    x = np.arange(n) + 0.5
    u0[0][:, x < 36.5] = 0.03
    u0[0][:, x >= 36.5] = -0.03
    _run(_touching_periodic(n), (1, 30, 300), u0=u0)


def _windowed():
    # 192^2 periodic, 64-node windows: solid 0 sits on the periodic corner
    # (its window wraps both seams), solids 1 and 2 overlap in their blur zones
    return workloads.make(nx=192, ny=192, tau=0.75, periodic_x=True, periodic_y=True,
                          gravity=(0.0, -2e-5), body_window=64,
                          solids=[dict(cx=2.0, cy=189.0, R=10.0, G=0.01, rho_s=1.4),
                                  dict(cx=90.0, cy=100.0, R=12.0, G=0.02, rho_s=1.2,
                                       shape="ellipse", b=8.0, theta=1.0),
                                  dict(cx=110.5, cy=101.0, R=9.0, G=0.01, rho_s=1.8),
                                  dict(cx=150.0, cy=40.0, R=7.0, G=0.005, rho_s=1.3)])


def test_windowed_solids_across_the_periodic_seams_match_oracle():
    # a uniform stream (the solids drift across the seams) with noise on it
    n = 192
    rng = np.random.default_rng(11)
    u0 = workloads.uniform_velocity(n, n, 0.02, -0.01) + rng.normal(0.0, 5e-4, size=(2, n, n))
    _run(_windowed(), (1, 25, 250), "f64", 1e-10, u0=u0)


def _channel():
    # periodic along x (64-node sub-windows), walls and a lid along y
    return workloads.make(nx=192, ny=96, tau=0.75, periodic_x=True, lid_ux=0.06,
                          gravity=(0.0, -2e-5), body_window=64,
                          solids=[dict(cx=2.0, cy=40.0, R=10.0, G=0.01, rho_s=1.4),
                                  dict(cx=90.0, cy=50.0, R=12.0, G=0.02, rho_s=1.2,
                                       shape="ellipse", b=8.0, theta=1.0),
                                  dict(cx=110.5, cy=51.0, R=9.0, G=0.01, rho_s=1.8),
                                  dict(cx=150.0, cy=30.0, R=7.0, G=0.005, rho_s=1.3)])


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", TOL32)])
def test_lid_driven_periodic_channel_matches_oracle(precision, tol):
    _run(_channel(), (1, 25, 200), precision, tol)


def test_one_solid_through_the_several_solid_path():
    cfg = workloads.cavity_disc_64()
    cfg = dict(cfg, solid=None, solids=[cfg["solid"]])
    _run(cfg, (1, 100, 1000))


def test_graph_replay_equals_eager_with_several_solids():
    cfg = _windowed()
    a = _sim(cfg).step(40)
    b = _sim(cfg)
    b.set_option(3, 0)  # eager launches
    b.step(40)
    fa = _np(a.macro()) + sum((_np(a.refmap(k)) for k in range(4)), [])
    fb = _np(b.macro()) + sum((_np(b.refmap(k)) for k in range(4)), [])
    for x, y in zip(fa, fb):
        assert np.array_equal(np.nan_to_num(x, nan=-9.0), np.nan_to_num(y, nan=-9.0))


def test_suspension_4096_conserves_momentum_without_gravity():
    # the full-size suspension with g = 0 in a stream (FP64): the elastic and
    # contact stresses enter as divergences on a periodic grid, so the total
    # momentum (sum of c f + F/2) stays fixed up to rounding.  (FP32 storage
    # drifts by ~3e-6 of it in 200 steps: 16.8 M nodes x 200 steps of float
    # rounding.)
    cfg = dict(workloads.suspension(), gravity=(0.0, 0.0))
    n = cfg["nx"]
    sim = _sim(cfg, "f64", workloads.uniform_velocity(n, n, 0.01, -0.004))
    d0 = sim.diag()
    sim.step(200)
    d1 = sim.diag()
    assert all(v == 0 for v in d1["health"].values()), d1["health"]
    p0 = np.hypot(d0["mom_x"], d0["mom_y"])
    print("momentum change", d1["mom_x"] - d0["mom_x"], d1["mom_y"] - d0["mom_y"], "of", p0)
    assert abs(d1["mom_x"] - d0["mom_x"]) < 1e-9 * p0
    assert abs(d1["mom_y"] - d0["mom_y"]) < 1e-9 * p0
    sim.close()


def test_suspension_4096_invariants():
    # the full-size suspension: 400 solids on a 4096^2 periodic box, FP32
    cfg = workloads.suspension()
    sim = _sim(cfg, "f32")
    d0 = sim.diag()
    s0 = [sim.diag_solid(k)["n_solid"] for k in range(0, 400, 37)]
    sim.step(300)
    d1 = sim.diag()
    assert all(v == 0 for v in d1["health"].values()), d1["health"]
    assert abs(d1["mass"] - d0["mass"]) < 1e-6 * d0["mass"]
    s1 = [sim.diag_solid(k)["n_solid"] for k in range(0, 400, 37)]
    assert all(abs(a - b) <= 0.05 * a for a, b in zip(s0, s1))
    sim.close()


def test_suspension_recipe_at_reduced_size_matches_oracle():
    # the suspension's own recipe (seeded ellipses, density contrast, gravity,
    # periodic box, 128-node sub-windows) on a 384^2 box with 8 solids, 50
    # steps in FP64 against the oracle; a uniform stream sets the velocity
    # scale (from rest, gravity 1e-6 alone leaves max |u| ~ 1e-6 at step 1)
    cfg = workloads.suspension(n=384, nbody=8, seed=7)
    _run(cfg, (1, 10, 50), u0=workloads.uniform_velocity(384, 384, 0.01, 0.005))


@pytest.mark.parametrize("cfgf,u0f,steps", [
    (_cavity3, None, 60),
    (_touching_periodic, "shear", 40),
])
def test_stress_with_several_solids_matches_oracle(cfgf, u0f, steps):
    # the global half-edge stress of Eq. (3_6_global_stress) (blend of the
    # solids normalised by their summed fraction, plus the contact stress of
    # every pair) averaged over a node's four edges; the bar is the single-
    # solid one (a first difference of xi divided by small map gradients)
    cfg = cfgf()
    u0 = None
    if u0f == "shear":
        n = cfg["nx"]
        u0 = np.zeros((2, n, n))
        x = np.arange(n) + 0.5
        u0[0][:, x < n / 2 + 0.5] = 0.03
        u0[0][:, x >= n / 2 + 0.5] = -0.03
    sim, ref = _sim(cfg, u0=u0), Oracle(**cfg).init(u0)
    sim.step(steps)
    ref.step(steps)
    s, rs = _np(sim.stress()), ref.stress()
    for name, a, b in zip(("sxx", "sxy", "syy"), s, rs):
        assert np.max(np.abs(b)) > 0, name
        err = rel(a, b)
        print(name, f"{err:.2e}", flush=True)
        assert err < 1e-9, name
    # reading the stress changes neither the state nor the health counters
    sim.step(1)
    ref.step(1)
    compare_mb(sim, ref, 1e-10, f"step {steps + 1} after the read")
    assert all(v == 0 for v in sim.diag()["health"].values())
    sim.close()


def test_checkpoint_resume_is_bitwise_with_several_solids():
    cfg = _windowed()
    n = cfg["nx"]
    rng = np.random.default_rng(11)
    u0 = workloads.uniform_velocity(n, n, 0.02, -0.01) + rng.normal(0.0, 5e-4, size=(2, n, n))

    def fields(s):
        return _np(s.macro()) + sum((_np(s.refmap(k)) for k in range(4)), []) + _np(s.force())

    a = _sim(cfg, u0=u0).step(37)
    blob = a.save_state()
    a.step(50)
    ra = fields(a)
    # into a fresh context, and into one that has run on from other data
    b = _sim(cfg)
    b.load_state(blob)
    assert b.step_count == 37
    b.step(50)
    c = _sim(cfg, u0=u0).step(61)
    c.load_state(blob)
    assert c.step_count == 37
    c.step(50)
    for s in (b, c):
        for x, y in zip(ra, fields(s)):
            assert np.array_equal(np.nan_to_num(x, nan=-9.0), np.nan_to_num(y, nan=-9.0))
        assert all(v == 0 for v in s.diag()["health"].values())
    # a blob of another solid count is refused
    cfg3 = dict(cfg, solids=cfg["solids"][:3])
    d = _sim(cfg3)
    with pytest.raises(RuntimeError, match="does not match"):
        d.load_state(blob)
    for s in (a, b, c, d):
        s.close()


def _drifting():
    # periodic both ways with 64-node sub-windows; a stream carries the solids
    # 30 and 18 nodes in 600 steps, farther than their windows' margins, so
    # each window has to follow its solid (several moves per solid)
    return workloads.make(nx=128, ny=128, tau=0.8, periodic_x=True, periodic_y=True,
                          gravity=(0.0, -1e-5), body_window=64,
                          solids=[dict(cx=40.0, cy=50.0, R=8.0, G=0.01, rho_s=1.2),
                                  dict(cx=90.0, cy=80.0, R=9.0, G=0.015, rho_s=1.0,
                                       shape="ellipse", b=6.0, theta=0.4)])


def _drift_u0(n=128):
    rng = np.random.default_rng(3)
    return workloads.uniform_velocity(n, n, 0.05, 0.03) + rng.normal(0.0, 5e-4, size=(2, n, n))


def test_windows_follow_drifting_solids_and_match_oracle():
    # without the moves the zones would leave their windows (window_clip);
    # with them every node keeps its lattice position and value
    _run(_drifting(), (1, 150, 300, 600), "f64", 1e-10, u0=_drift_u0())


def test_moved_windows_survive_checkpoints_and_graph_replay():
    cfg, u0 = _drifting(), _drift_u0()

    def fields(s):
        return _np(s.macro()) + sum((_np(s.refmap(k)) for k in range(2)), [])

    a = _sim(cfg, u0=u0).step(400)
    blob = a.save_state()
    a.step(200)
    b = _sim(cfg)
    b.load_state(blob)
    b.step(200)
    e = _sim(cfg, u0=u0)
    e.set_option(3, 0)  # eager launches
    e.step(600)
    for s in (b, e):
        for x, y in zip(fields(a), fields(s)):
            assert np.array_equal(np.nan_to_num(x, nan=-9.0), np.nan_to_num(y, nan=-9.0))
        assert all(v == 0 for v in s.diag()["health"].values())
    for s in (a, b, e):
        s.close()
