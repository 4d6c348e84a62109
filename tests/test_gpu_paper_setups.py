"""The paper's benchmark setups on the GPU path: loose physical checks.

Soft disc in the lid-driven cavity at Re = 100 (Sec. 4.1) on a 160 x 160 grid
(80000 steps, the paper's grid study scaled as in ``paper_setups``): the solid
stays healthy and loses a few percent of its volume (the paper's grid study
spans 9.2 % at L = 80 down to 0.3 % at L = 640; this path gives 4.9 % at
L = 160, 1.2 % at L = 320 and 0.29 % at L = 640).  A heavier disc settles in a
closed box (Sec. 4.3) with its mass conserved.
"""
import pytest

import paper_setups

pytestmark = pytest.mark.gpu


def test_cavity_160_volume_change():
    r = paper_setups.run_cavity(160)
    assert r["health_ok"]
    assert -0.08 < r["volume_change"] < -0.02, r["volume_change"]
    # the disc is carried up towards the lid and back along the vortex
    assert 0.45 < r["cx"] < 0.65 and 0.55 < r["cy"] < 0.8


def test_heavy_disc_settles():
    d0, d1 = paper_setups.run_settling(steps=20000)
    assert all(v == 0 for v in d1["health"].values())
    assert d1["centroid_y"] < d0["centroid_y"] - 3.0
    assert abs(d1["mass"] / d0["mass"] - 1.0) < 1e-10
