"""lbrmt_diag_noalloc (scratch in the library's static device array) against
lbrmt_diag (scratch in the context's workspace), through the C ABI: the same
kernels in the same order, so the results must be identical bit for bit.
Two calls in a row on different contexts, the second smaller, so that the
second call runs on the array the first call left behind."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _diag(name, sim):
    from paper_2402_12696_amd import lbrmt as B
    out = B.lbrmt_diag_t()
    rc = getattr(B.lib(), name)(sim.ctx, ctypes.byref(out))
    vals = [getattr(out, k) for k, _ in B.lbrmt_diag_t._fields_ if k != "health"]
    return rc, np.array(vals, dtype=np.float64), list(out.health)


def _same(a, b):
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1], equal_nan=True), (a[1], b[1])
    assert a[2] == b[2]


def test_noalloc_diag_equals_diag_on_two_contexts_the_second_smaller():
    from paper_2402_12696_amd import Sim
    big = workloads.make(nx=160, ny=144, tau=0.7, lid_ux=0.06,
                         solid=dict(cx=80.0, cy=80.0, R=30.0, G=0.01, rho_s=1.2),
                         gravity=(0.0, -1e-5))
    small = workloads.cavity_disc_64()
    print("case: noalloc diag, 160x144 cavity FP64 then 64x64 cavity FP32", flush=True)
    a = Sim(device="cuda:0", **big).init()
    a.step(40)
    first = _diag("lbrmt_diag_noalloc", a)
    _same(first, _diag("lbrmt_diag", a))
    assert first[0] == 0 and first[1][1] > 160 * 144 * 0.99
    b = Sim(device="cuda:0", precision="f32", **small).init()
    b.step(25)
    second = _diag("lbrmt_diag_noalloc", b)
    _same(second, _diag("lbrmt_diag", b))
    assert second[1][1] < first[1][1]
    # the first context again, after the smaller one used the array
    _same(_diag("lbrmt_diag_noalloc", a), first)
    a.close()
    b.close()


def test_noalloc_diag_with_several_solids():
    from paper_2402_12696_amd import Sim
    cfg = workloads.make(nx=96, ny=80, tau=0.8, periodic_x=True, periodic_y=True,
                         gravity=(0.0, -2e-5),
                         solids=[dict(cx=30.0, cy=40.0, R=9.0, G=0.02, rho_s=1.4),
                                 dict(cx=64.0, cy=38.0, R=8.0, b=5.0, theta=0.4,
                                      shape="ellipse", G=0.015, rho_s=1.2)])
    print("case: noalloc diag, two solids on a 96x80 periodic box", flush=True)
    s = Sim(device="cuda:0", **cfg).init()
    s.step(30)
    _same(_diag("lbrmt_diag_noalloc", s), _diag("lbrmt_diag", s))
    s.close()
