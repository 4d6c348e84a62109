"""The one-launch extrapolation (all layers of Sec. 3.2 in one kernel, tiles
with recomputed margins, a one-block pass for tiles that need wider scan
windows) against the one-launch-per-layer path: the whole state after many
steps must be bitwise identical (populations, force, xi, phi, health), for
every block size, for the default choice, and with the margin check
tightened so that the one-block pass fits most of the zone.  The per-layer
path itself is held to the FP64 oracle by the parity tests."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

THIN = workloads.make(nx=128, ny=128, tau=0.8, lid_ux=0.08,
                      solid=dict(cx=64.0, cy=70.0, R=30.0, G=0.01, rho_s=1.0, shape="ellipse",
                                 b=3.0, theta=0.3))
HEAVY_WALLED = workloads.make(nx=96, ny=112, tau=0.7, lid_ux=0.05, gravity=(0.0, -1e-4),
                              solid=dict(cx=40.0, cy=60.0, R=14.0, G=0.02, rho_s=1.5,
                                         shape="ellipse", b=9.0, theta=-0.6))


def _state(sim):
    X, Y, P = [t.cpu().numpy() for t in sim.refmap()]
    fx, fy = [t.cpu().numpy() for t in sim.force()]
    return (sim.populations().cpu().numpy(), np.nan_to_num(X, nan=7.5), np.nan_to_num(Y, nan=7.5),
            np.nan_to_num(P, nan=7.5), fx, fy, sim.diag(raise_unstable=False)["health"])


def _run(cfg, prec, opt, steps, graph=True):
    from paper_2402_12696_amd import Sim
    from paper_2402_12696_amd import lbrmt as B
    sim = Sim(device="cuda:0", precision=prec, **cfg)
    sim.set_option(B.LBRMT_OPT_FUSED_FIT, opt)
    sim.set_option(B.LBRMT_OPT_GRAPH, 1 if graph else 0)
    sim.init()
    sim.step(steps)
    out = _state(sim)
    sim.close()
    return out


def _equal(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a[:6], b[:6])) and a[6] == b[6]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,cfg,steps", [("cavity64", workloads.cavity_disc_64(), 300),
                                            ("thin_ellipse", THIN, 200),
                                            ("heavy_ellipse", HEAVY_WALLED, 150)])
def test_one_launch_extrapolation_is_bitwise_the_per_layer_path(name, cfg, steps, prec):
    ref = _run(cfg, prec, 0, steps)
    assert not any(ref[6].values()), ref[6]
    for opt in (1024, 512, 256, 1, -1):
        assert _equal(ref, _run(cfg, prec, opt, steps)), (name, prec, opt)
    # eager launches too
    assert _equal(ref, _run(cfg, prec, 1024, steps, graph=False))


def test_one_launch_extrapolation_at_2048():
    cfg = workloads.cavity_disc_2048()
    ref = _run(cfg, "f64", 0, 24)
    for opt in (1024, 1):
        assert _equal(ref, _run(cfg, "f64", opt, 24)), opt


def test_fused_fit_option_values():
    from paper_2402_12696_amd import Sim
    from paper_2402_12696_amd import lbrmt as B
    sim = Sim(device="cuda:0", precision="f64", **workloads.cavity_disc_64())
    assert sim.get_option(B.LBRMT_OPT_FUSED_FIT) == -1
    for v in (0, 1, 256, 512, 1024, -1):
        sim.set_option(B.LBRMT_OPT_FUSED_FIT, v)
        assert sim.get_option(B.LBRMT_OPT_FUSED_FIT) == v
    for v in (2, 128, 2048, -2):
        with pytest.raises(Exception):
            sim.set_option(B.LBRMT_OPT_FUSED_FIT, v)
    sim.close()


def test_hold_option_refuses_a_held_and_capped_bulk_update():
    # a held bulk update with a cap on its workgroups is refused in either
    # order of the two calls; -1 (default) holds only an uncapped update
    from paper_2402_12696_amd import Sim
    from paper_2402_12696_amd import lbrmt as B
    sim = Sim(device="cuda:0", precision="f64", **workloads.cavity_disc_64())
    assert sim.get_option(B.LBRMT_OPT_HOLD_BULK) == -1
    sim.set_option(B.LBRMT_OPT_BULK_BLOCKS, 512)        # default hold: allowed
    with pytest.raises(B.LBRMTError, match="cannot be held"):
        sim.set_option(B.LBRMT_OPT_HOLD_BULK, 1)
    assert sim.get_option(B.LBRMT_OPT_HOLD_BULK) == -1
    sim.set_option(B.LBRMT_OPT_BULK_BLOCKS, 0)
    sim.set_option(B.LBRMT_OPT_HOLD_BULK, 1)
    with pytest.raises(B.LBRMTError, match="cannot be held"):
        sim.set_option(B.LBRMT_OPT_BULK_BLOCKS, 512)
    assert sim.get_option(B.LBRMT_OPT_BULK_BLOCKS) == 0
    for v in (0, -1):
        sim.set_option(B.LBRMT_OPT_HOLD_BULK, v)
        assert sim.get_option(B.LBRMT_OPT_HOLD_BULK) == v
    for v in (2, -2):
        with pytest.raises(B.LBRMTError):
            sim.set_option(B.LBRMT_OPT_HOLD_BULK, v)
    sim.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_early_bulk_tiles_are_bitwise_the_single_bulk_launch(prec):
    # part of the held bulk update launched when the previous step's chain
    # ends: the same state after graph replays (whole and partial six-step
    # runs) and eager steps, for several fractions, the whole grid included
    from paper_2402_12696_amd import Sim
    from paper_2402_12696_amd import lbrmt as B

    def run(early, graph=True):
        sim = Sim(device="cuda:0", precision=prec, **workloads.cavity_disc_256())
        sim.set_option(B.LBRMT_OPT_GRAPH, 1 if graph else 0)
        sim.set_option(B.LBRMT_OPT_BULK_EARLY, early)
        assert sim.get_option(B.LBRMT_OPT_BULK_EARLY) == early
        sim.init()
        for n in (7, 12, 5, 30, 1):
            sim.step(n)
        out = _state(sim)
        sim.close()
        return out

    ref = run(0)
    assert not any(ref[6].values()), ref[6]
    for early in (1, 150, 500, 1000, -1):
        assert _equal(ref, run(early)), early
    assert _equal(ref, run(300, graph=False))


def test_early_bulk_option_values():
    from paper_2402_12696_amd import Sim
    from paper_2402_12696_amd import lbrmt as B
    sim = Sim(device="cuda:0", precision="f64", **workloads.cavity_disc_64())
    assert sim.get_option(B.LBRMT_OPT_BULK_EARLY) == -1
    for v in (0, 1000, -1):
        sim.set_option(B.LBRMT_OPT_BULK_EARLY, v)
        assert sim.get_option(B.LBRMT_OPT_BULK_EARLY) == v
    for v in (-2, 1001):
        with pytest.raises(B.LBRMTError):
            sim.set_option(B.LBRMT_OPT_BULK_EARLY, v)
    sim.close()


def test_autotune_steps_chooses_a_mode_and_steps_like_lbrmt_step():
    from paper_2402_12696_amd import Sim
    from paper_2402_12696_amd import lbrmt as B
    cfg = workloads.cavity_disc_64()
    a = Sim(device="cuda:0", precision="f64", **cfg).init()
    a.step(5)
    mode, ms = a.autotune_steps(30)
    assert mode in (0, 1024) and ms > 0.0
    assert a.get_option(B.LBRMT_OPT_FUSED_FIT) == mode
    n = a.step_count
    assert n >= 5 + 2 * 30
    a.step(7)
    sa = _state(a)
    a.close()
    b = Sim(device="cuda:0", precision="f64", **cfg)
    b.set_option(B.LBRMT_OPT_FUSED_FIT, 0)
    b.init()
    b.step(n + 7)
    assert _equal(sa, _state(b))
    b.close()
    # several solids: no choice to make
    s = Sim(device="cuda:0", precision="f64", **workloads.make(
        nx=64, ny=64, tau=0.8, lid_ux=0.05,
        solids=[dict(cx=20.0, cy=32.0, R=6.0, G=0.01, rho_s=1.0),
                dict(cx=44.0, cy=32.0, R=6.0, G=0.01, rho_s=1.0)])).init()
    with pytest.raises(Exception):
        s.autotune_steps(12)
    s.close()


NEAR_WALL = workloads.make(nx=96, ny=80, tau=0.8, lid_ux=0.06,
                           solid=dict(cx=30.0, cy=14.5, R=11.0, G=0.01, rho_s=1.0))


@pytest.mark.parametrize("name,cfg,steps", [
    ("near_wall", NEAR_WALL, 120),
    ("layers3", dict(workloads.cavity_disc_64(), layers=3), 150),
    ("layers7", dict(workloads.cavity_disc_64(), layers=7), 150),
    ("rmax2_thin", dict(THIN, r_max=2), 120),
])
def test_one_launch_extrapolation_edge_cases(name, cfg, steps):
    # a window clipped by the walls; fewer layers (narrower margins); scan
    # windows capped at r = 2, so that fits fail and are counted
    for prec in ("f64", "f32"):
        ref = _run(cfg, prec, 0, steps)
        print(name, prec, ref[6])
        if name == "rmax2_thin":
            assert ref[6]["extrap_fail"] > 0  # the case exercises failed fits
        for opt in (1024, 1):
            assert _equal(ref, _run(cfg, prec, opt, steps)), (name, prec, opt, ref[6])


def test_one_launch_extrapolation_with_more_zone_tiles_than_blocks():
    # a disc of radius 1200 on 4096^2: some 600 zone tiles for 256 blocks
    cfg = workloads.make(nx=4096, ny=4096, tau=0.6, lid_ux=0.05,
                         solid=dict(cx=2048.0, cy=2200.0, R=1200.0, G=0.005, rho_s=1.0))
    ref = _run(cfg, "f32", 0, 12)
    assert _equal(ref, _run(cfg, "f32", 1024, 12))


def test_one_launch_extrapolation_over_a_long_deforming_run():
    # the 256^2 inverse-problem scene from a noisy initial velocity, 600 steps
    # (the solid deforms strongly; the run stays finite): bitwise equal
    from paper_2402_12696_amd import Sim
    from paper_2402_12696_amd import lbrmt as B
    cfg = workloads.make(nx=256, ny=256, tau=0.7, lid_ux=0.08,
                         solid=dict(cx=128.0, cy=153.6, R=40.0, G=0.01, rho_s=1.0))
    u0 = np.random.default_rng(5).normal(0.0, 1e-3, size=(2, 256, 256))
    out = []
    for prec in ("f64", "f32"):
        for opt in (0, 1024):
            sim = Sim(device="cuda:0", precision=prec, **cfg)
            sim.set_option(B.LBRMT_OPT_FUSED_FIT, opt)
            sim.init(u0)
            sim.step(600)
            out.append(_state(sim))
            sim.close()
    assert _equal(out[0], out[1]) and _equal(out[2], out[3])
    assert not out[0][6]["nonfinite"]
