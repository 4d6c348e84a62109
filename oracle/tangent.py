"""ctypes binding of the tangent-linear oracle -- TEST INFRASTRUCTURE ONLY.

``liblbrmt_oracle_tangent.so`` is ``lbrmt_oracle.c`` compiled with every
floating-point number a dual number (value, tangent): the values are the
plain oracle's, bit for bit, and the tangents are the exact derivatives of the
discrete step along a seeded direction of the inputs (parameters, solid
properties, initial velocity).  Only the test-suite may import this module.

Every field and array that the plain oracle holds as a double comes back here
as a pair: ``value`` and ``tangent`` arrays of the same shape.
"""
import ctypes
import os

import numpy as np

from .oracle import _Params, _Solid, _solid

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbrmt_oracle_tangent.so")

_vp = ctypes.c_void_p


class _D(ctypes.Structure):
    _fields_ = [("v", ctypes.c_double), ("d", ctypes.c_double)]


def _dual_fields(fields):
    return [(n, _D if t is ctypes.c_double else t) for n, t in fields]


class _ParamsT(ctypes.Structure):
    _fields_ = _dual_fields(_Params._fields_)


class _SolidT(ctypes.Structure):
    _fields_ = _dual_fields(_Solid._fields_)


def _lift(src, cls, seed):
    """A dual-typed copy of a plain ctypes structure; ``seed`` maps field
    names to tangents (0 elsewhere)."""
    out = cls()
    unknown = set(seed) - {n for n, t in cls._fields_ if t is _D}
    if unknown:
        raise ValueError(f"no floating-point field {sorted(unknown)} to seed")
    for n, t in cls._fields_:
        x = getattr(src, n)
        setattr(out, n, _D(x, float(seed.get(n, 0.0))) if t is _D else x)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"tangent oracle library missing: {LIB_PATH} "
                               "(run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.orc_create.restype = _vp
        L.orc_create.argtypes = [ctypes.POINTER(_ParamsT), ctypes.POINTER(_SolidT), ctypes.c_int32]
        L.orc_destroy.argtypes = [_vp]
        L.orc_init.argtypes = [_vp, _vp]
        L.orc_step.argtypes = [_vp, ctypes.c_int64]
        for name in ("orc_read_macro", "orc_read_stress"):
            getattr(L, name).argtypes = [_vp, _vp, _vp, _vp]
        L.orc_read_populations.argtypes = [_vp, _vp]
        L.orc_read_force.argtypes = [_vp, _vp, _vp]
        L.orc_read_refmap_body.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp]
        L.orc_diag.argtypes = [_vp, _vp]
        L.orc_diag_body.argtypes = [_vp, ctypes.c_int32, _vp]
        L.orc_heaviside.restype = _D
        L.orc_heaviside.argtypes = [_D, _D]
        L.orc_phi0.restype = _D
        L.orc_phi0.argtypes = [ctypes.POINTER(_SolidT), _D, _D]
        L.orc_solid_stress.restype = ctypes.c_int
        L.orc_solid_stress.argtypes = [_vp, _D, _D, _vp]
        L.orc_feq_sfc.argtypes = [_D, _D, _D, _D, _vp]
        L.orc_guo.argtypes = [_D, _D, _D, _D, _vp]
        _lib = L
    return _lib


def _pairs(shape):
    return np.zeros(tuple(shape) + (2,))


def _ptr(a):
    return a.ctypes.data_as(_vp)


def _split(a):
    return a[..., 0].copy(), a[..., 1].copy()


def _dual(v, d=0.0):
    return _D(float(v), float(d))


# ---------------------------------------------------------------- pointwise

def heaviside(phi, dphi, eps, deps=0.0):
    r = lib().orc_heaviside(_dual(phi, dphi), _dual(eps, deps))
    return r.v, r.d


def phi0(solid, X, Y, dX=0.0, dY=0.0, dsolid=None):
    s = _lift(_solid(solid), _SolidT, dsolid or {})
    r = lib().orc_phi0(ctypes.byref(s), _dual(X, dX), _dual(Y, dY))
    return r.v, r.d


def solid_stress(J, dJ, G, dG=0.0, detJ_min=1e-12):
    Jd = np.stack([np.asarray(J, float).reshape(4), np.asarray(dJ, float).reshape(4)], axis=-1)
    Jd = np.ascontiguousarray(Jd)
    out = _pairs((3,))
    ok = lib().orc_solid_stress(_ptr(Jd), _dual(G, dG), _dual(detJ_min), _ptr(out))
    return bool(ok), out[:, 0].copy(), out[:, 1].copy()


def feq_sfc(rho, ux, uy, drho, tangents=(0.0, 0.0, 0.0, 0.0)):
    out = _pairs((9,))
    args = [_dual(v, d) for v, d in zip((rho, ux, uy, drho), tangents)]
    lib().orc_feq_sfc(*args, _ptr(out))
    return _split(out)


def guo(ux, uy, fx, fy, tangents=(0.0, 0.0, 0.0, 0.0)):
    out = _pairs((9,))
    args = [_dual(v, d) for v, d in zip((ux, uy, fx, fy), tangents)]
    lib().orc_guo(*args, _ptr(out))
    return _split(out)


# ---------------------------------------------------------------- simulation

class TangentOracle:
    """One LBRMT simulation on the tangent-linear oracle.  Keywords as in
    ``workloads`` and ``Oracle``; ``dparams`` seeds tangents of grid
    parameters (e.g. ``{"lid_ux": 1.0}``), ``dsolids`` those of the solids'
    fields (a list aligned with the solids, e.g. ``[{"G": 1.0}]``)."""

    _DIAG = ["mass", "mom_x", "mom_y", "centroid_x", "centroid_y", "disp_x", "disp_y",
             "max_u", "n_solid", "n_band"]

    def __init__(self, nx, ny, tau, lid_ux=0.0, periodic_x=False, periodic_y=False,
                 gravity=(0.0, 0.0), fext=(0.0, 0.0), rho_f=1.0, eps=1.5, layers=11,
                 r_max=8, det_rel=1e-8, detJ_min=1e-12, reverse_order=False, solid=None,
                 solids=None, eta=1.0, dparams=None, dsolids=None, **_ignored):
        p = _Params(nx, ny, int(periodic_x), int(periodic_y), tau, lid_ux,
                    gravity[0], gravity[1], fext[0], fext[1], rho_f, eps, layers, r_max,
                    det_rel, detJ_min, int(reverse_order), 0, eta)
        pt = _lift(p, _ParamsT, dparams or {})
        self.nx, self.ny = nx, ny
        if solid is not None and solids is not None:
            raise ValueError("give either solid or solids")
        bodies = [solid] if solid is not None else list(solids or [])
        dsolids = list(dsolids or [])
        if len(dsolids) > len(bodies):
            raise ValueError("more solid seeds than solids")
        dsolids += [{}] * (len(bodies) - len(dsolids))
        if bodies:
            arr = (_SolidT * len(bodies))(*[_lift(_solid(b), _SolidT, ds)
                                            for b, ds in zip(bodies, dsolids)])
            self._h = lib().orc_create(ctypes.byref(pt), arr, len(bodies))
        else:
            self._h = lib().orc_create(ctypes.byref(pt), None, 0)
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def init(self, u0=None, du0=None):
        """u0, du0: [2, ny, nx] initial velocity and its tangent (None: 0)."""
        if u0 is None and du0 is None:
            lib().orc_init(self._h, None)
            return self
        shp = (2, self.ny, self.nx)
        a = _pairs(shp)
        if u0 is not None:
            a[..., 0] = np.asarray(u0, float).reshape(shp)
        if du0 is not None:
            a[..., 1] = np.asarray(du0, float).reshape(shp)
        self._u0 = a
        lib().orc_init(self._h, _ptr(a))
        return self

    def step(self, n=1):
        lib().orc_step(self._h, int(n))
        return self

    def macro(self):
        """((rho, ux, uy), (d rho, d ux, d uy))"""
        a = [_pairs((self.ny, self.nx)) for _ in range(3)]
        lib().orc_read_macro(self._h, *[_ptr(x) for x in a])
        s = [_split(x) for x in a]
        return tuple(x[0] for x in s), tuple(x[1] for x in s)

    def populations(self):
        f = _pairs((9, self.ny, self.nx))
        lib().orc_read_populations(self._h, _ptr(f))
        return _split(f)

    def force(self):
        a = [_pairs((self.ny, self.nx)) for _ in range(2)]
        lib().orc_read_force(self._h, *[_ptr(x) for x in a])
        s = [_split(x) for x in a]
        return tuple(x[0] for x in s), tuple(x[1] for x in s)

    def refmap(self, body=0):
        a = [_pairs((self.ny, self.nx)) for _ in range(3)]
        lib().orc_read_refmap_body(self._h, int(body), *[_ptr(x) for x in a])
        s = [_split(x) for x in a]
        return tuple(x[0] for x in s), tuple(x[1] for x in s)

    def diag(self):
        """(values, tangents): two dicts with the keys of ``Oracle.diag``."""
        out = _pairs((10,))
        lib().orc_diag(self._h, _ptr(out))
        return (dict(zip(self._DIAG, out[:, 0].tolist())),
                dict(zip(self._DIAG, out[:, 1].tolist())))
