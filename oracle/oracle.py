"""ctypes binding of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It loads ``liblbrmt_oracle.so`` (built
from ``lbrmt_oracle.c`` by ``__graft_entry__.build()``) and exposes the oracle's
step, reads and pointwise definitions as numpy arrays.  Parity unpinned
functions: none (every function is pinned by ``tests/test_oracle_*.py``).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbrmt_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32),
        ("tau", ctypes.c_double), ("lid_ux", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("fext_x", ctypes.c_double), ("fext_y", ctypes.c_double),
        ("rho_f", ctypes.c_double), ("eps", ctypes.c_double),
        ("layers", ctypes.c_int32), ("r_max", ctypes.c_int32),
        ("det_rel", ctypes.c_double), ("detJ_min", ctypes.c_double),
        ("reverse_order", ctypes.c_int32), ("lid_rho_mode", ctypes.c_int32),
        ("eta", ctypes.c_double),
    ]


class _Solid(ctypes.Structure):
    _fields_ = [("cx", ctypes.c_double), ("cy", ctypes.c_double), ("R", ctypes.c_double),
                ("G", ctypes.c_double), ("rho_s", ctypes.c_double),
                ("shape", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("b", ctypes.c_double), ("theta", ctypes.c_double)]


def _solid(d):
    """A solid description (``workloads`` keywords): a disc of radius R, or
    with ``shape="ellipse"`` an ellipse of semi-axes a = R and b whose a axis
    makes the angle theta with the x axis."""
    shape = d.get("shape", "disc")
    if shape not in ("disc", "ellipse"):
        raise ValueError(f"unknown solid shape {shape!r}")
    ell = shape == "ellipse"
    return _Solid(d["cx"], d["cy"], d["R"], d["G"], d["rho_s"], int(ell), 0,
                  float(d.get("b", d["R"])) if ell else d["R"],
                  float(d.get("theta", 0.0)) if ell else 0.0)


def phi0(solid, X, Y):
    """Reference level set of a solid description at reference point (X, Y)."""
    s = _solid(solid)
    return lib().orc_phi0(ctypes.byref(s), float(X), float(Y))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Solid), ctypes.c_int32]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_init.argtypes = [ctypes.c_void_p, _dp]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        for name in ("advect", "extrapolate", "relabel", "force", "collide_stream", "moments"):
            getattr(L, "orc_phase_" + name).argtypes = [ctypes.c_void_p]
        L.orc_step_count.restype = ctypes.c_int64
        L.orc_step_count.argtypes = [ctypes.c_void_p]
        L.orc_read_macro.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc_read_populations.argtypes = [ctypes.c_void_p, _dp]
        L.orc_read_force.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_read_refmap.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc_read_refmap_padded.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc_read_layers_padded.argtypes = [ctypes.c_void_p, _ip]
        L.orc_read_stress.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc_counters.argtypes = [ctypes.c_void_p, _lp]
        L.orc_diag.argtypes = [ctypes.c_void_p, _dp]
        L.orc_set_refmap_padded.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_set_populations.argtypes = [ctypes.c_void_p, _dp]
        L.orc_set_moments.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc_heaviside.restype = ctypes.c_double
        L.orc_heaviside.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_feq_sfc.argtypes = [ctypes.c_double] * 4 + [_dp]
        L.orc_guo.argtypes = [ctypes.c_double] * 4 + [_dp]
        L.orc_solid_stress.restype = ctypes.c_int
        L.orc_solid_stress.argtypes = [_dp, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_read_refmap_body.argtypes = [ctypes.c_void_p, ctypes.c_int32, _dp, _dp, _dp]
        L.orc_diag_body.argtypes = [ctypes.c_void_p, ctypes.c_int32, _dp]
        L.orc_nsolid.restype = ctypes.c_int32
        L.orc_nsolid.argtypes = [ctypes.c_void_p]
        L.orc_phi0.restype = ctypes.c_double
        L.orc_phi0.argtypes = [ctypes.POINTER(_Solid), ctypes.c_double, ctypes.c_double]
        L.orc_layers_mask.argtypes = [ctypes.c_int32, ctypes.c_int32, _u8p, ctypes.c_int32, _ip]
        L.orc_d2q9.argtypes = [_ip, _ip, _dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


# ---------------------------------------------------------------- pointwise

def heaviside(phi, eps):
    return lib().orc_heaviside(float(phi), float(eps))


def feq_sfc(rho, ux, uy, drho):
    out = np.zeros(9)
    lib().orc_feq_sfc(rho, ux, uy, drho, _d(out))
    return out


def guo(ux, uy, fx, fy):
    out = np.zeros(9)
    lib().orc_guo(ux, uy, fx, fy, _d(out))
    return out


def solid_stress(J, G, detJ_min=1e-12):
    J = np.ascontiguousarray(J, dtype=np.float64).reshape(4)
    out = np.zeros(3)
    ok = lib().orc_solid_stress(_d(J), G, detJ_min, _d(out))
    return bool(ok), out


def layers_mask(solid, L):
    solid = np.ascontiguousarray(solid, dtype=np.uint8)
    ny, nx = solid.shape
    out = np.zeros((ny, nx), dtype=np.int32)
    lib().orc_layers_mask(nx, ny, solid.ctypes.data_as(_u8p), L, out.ctypes.data_as(_ip))
    return out


def d2q9():
    cx = np.zeros(9, np.int32)
    cy = np.zeros(9, np.int32)
    w = np.zeros(9)
    lib().orc_d2q9(cx.ctypes.data_as(_ip), cy.ctypes.data_as(_ip), _d(w))
    return cx, cy, w


# ---------------------------------------------------------------- simulation

class Oracle:
    """One LBRMT simulation on the CPU oracle (keywords as in ``workloads``)."""

    def __init__(self, nx, ny, tau, lid_ux=0.0, periodic_x=False, periodic_y=False,
                 gravity=(0.0, 0.0), fext=(0.0, 0.0), rho_f=1.0, eps=1.5, layers=11,
                 r_max=8, det_rel=1e-8, detJ_min=1e-12, reverse_order=False, solid=None,
                 solids=None, eta=1.0, lid_rho_mode=0, **_ignored):
        p = _Params(nx, ny, int(periodic_x), int(periodic_y), tau, lid_ux,
                    gravity[0], gravity[1], fext[0], fext[1], rho_f, eps, layers, r_max,
                    det_rel, detJ_min, int(reverse_order), int(lid_rho_mode), eta)
        self.nx, self.ny = nx, ny
        if solid is not None and solids is not None:
            raise ValueError("give either solid or solids")
        bodies = [solid] if solid is not None else list(solids or [])
        self.nsolid = len(bodies)
        if bodies:
            arr = (_Solid * len(bodies))(*[_solid(b) for b in bodies])
            self._h = lib().orc_create(ctypes.byref(p), arr, len(bodies))
        else:
            self._h = lib().orc_create(ctypes.byref(p), None, 0)
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def init(self, u0=None):
        if u0 is None:
            lib().orc_init(self._h, None)
        else:
            u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(2, self.ny, self.nx)
            self._u0 = u0
            lib().orc_init(self._h, _d(u0))
        return self

    def step(self, n=1):
        lib().orc_step(self._h, int(n))
        return self

    def phase(self, name):
        getattr(lib(), "orc_phase_" + name)(self._h)

    @property
    def step_count(self):
        return lib().orc_step_count(self._h)

    def _plane(self):
        return np.zeros((self.ny, self.nx))

    def macro(self):
        r, u, v = self._plane(), self._plane(), self._plane()
        lib().orc_read_macro(self._h, _d(r), _d(u), _d(v))
        return r, u, v

    def populations(self):
        f = np.zeros((9, self.ny, self.nx))
        lib().orc_read_populations(self._h, _d(f))
        return f

    def force(self):
        fx, fy = self._plane(), self._plane()
        lib().orc_read_force(self._h, _d(fx), _d(fy))
        return fx, fy

    def refmap(self, body=0):
        """xi and phi of one solid on the interior nodes (NaN: no value)."""
        X, Y, phi = self._plane(), self._plane(), self._plane()
        lib().orc_read_refmap_body(self._h, int(body), _d(X), _d(Y), _d(phi))
        return X, Y, phi

    def refmap_padded(self):
        shp = (self.ny + 4, self.nx + 4)
        X, Y, phi = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        lib().orc_read_refmap_padded(self._h, _d(X), _d(Y), _d(phi))
        return X, Y, phi

    def layers_padded(self):
        out = np.zeros((self.ny + 4, self.nx + 4), np.int32)
        lib().orc_read_layers_padded(self._h, out.ctypes.data_as(_ip))
        return out

    def set_refmap_padded(self, X, Y):
        X = np.ascontiguousarray(X, dtype=np.float64)
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        lib().orc_set_refmap_padded(self._h, _d(X), _d(Y))

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        lib().orc_set_populations(self._h, _d(f))

    def set_moments(self, rho, ux, uy):
        a = [np.ascontiguousarray(x, dtype=np.float64) for x in (rho, ux, uy)]
        lib().orc_set_moments(self._h, *[_d(x) for x in a])

    def stress(self):
        a, b, c = self._plane(), self._plane(), self._plane()
        lib().orc_read_stress(self._h, _d(a), _d(b), _d(c))
        return a, b, c

    def counters(self):
        out = np.zeros(8, np.int64)
        lib().orc_counters(self._h, out.ctypes.data_as(_lp))
        return out

    def diag(self):
        out = np.zeros(10)
        lib().orc_diag(self._h, _d(out))
        keys = ["mass", "mom_x", "mom_y", "centroid_x", "centroid_y", "disp_x", "disp_y",
                "max_u", "n_solid", "n_band"]
        return dict(zip(keys, out.tolist()))

    def diag_body(self, body):
        out = np.zeros(6)
        lib().orc_diag_body(self._h, int(body), _d(out))
        keys = ["centroid_x", "centroid_y", "disp_x", "disp_y", "n_solid", "n_band"]
        return dict(zip(keys, out.tolist()))
