"""The 2048 x 2048 cavity-disc workload at full size, in the launch
configuration the benchmark times: full-field parity with the oracle over the
first steps (eager, graph-replayed and eager again), and invariants over a
longer run that the oracle cannot afford."""
import numpy as np
import pytest

import workloads
from oracle import Oracle
from test_gpu_parity import compare

pytestmark = pytest.mark.gpu


def test_cavity_disc_2048_matches_oracle():
    cfg = workloads.cavity_disc_2048()
    from paper_2402_12696_amd import Sim
    sim = Sim(device="cuda:0", **cfg).init()
    ref = Oracle(**cfg).init()
    sim.step(13)
    ref.step(13)
    compare(sim, ref, what="cavity_disc_2048 step 13")


def test_cavity_disc_2048_conserves_mass():
    cfg = workloads.cavity_disc_2048()
    from paper_2402_12696_amd import Sim
    sim = Sim(device="cuda:0", **cfg).init()
    m0 = sim.diag()["mass"]
    sim.step(600)
    d = sim.diag()
    assert abs(d["mass"] - m0) / m0 < 1e-12
    assert d["max_u"] < 0.2 and d["n_solid"] > 2.9e5
    assert all(v == 0 for v in d["health"].values())
