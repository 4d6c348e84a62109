"""Thin ctypes binding of ``liblbrmt.so`` (C ABI of ``include/lbrmt.h``).

Every ``lbrmt_*`` function here has the name, arguments and meaning of the C
call of the same name; it only marshals arguments (torch device tensors become
raw device pointers, the stream is torch's current HIP stream).  All the
arithmetic of the time step runs in the library's HIP kernels.  There is no
fallback: if the library is missing or no GPU is present, calls raise.

``Sim`` wraps one context with a workspace tensor for convenience.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbrmt.so")

LBRMT_OK, LBRMT_EINVAL, LBRMT_EWORKSPACE, LBRMT_EHIP, LBRMT_EUNSTABLE, LBRMT_ECAPACITY, \
    LBRMT_ESTATE = range(7)
LBRMT_FP64, LBRMT_FP32 = 0, 1
HEALTH_NAMES = ["advect_miss", "extrap_fail", "stress_miss", "detj", "detj_solid", "nonfinite",
                "window_clip", "list_overflow"]
KERNEL_NAMES = ["advect", "extrap", "relabel", "force", "lb_bulk", "lb_band"]
LBRMT_OPT_OVERLAP, LBRMT_OPT_LB_VARIANT, LBRMT_OPT_LB_VARIANT_COUNT, LBRMT_OPT_GRAPH = 0, 1, 2, 3
LBRMT_OPT_BULK_BLOCKS = 4
LBRMT_OPT_FUSED_FIT = 5
LBRMT_OPT_HOLD_BULK = 6
LBRMT_OPT_BULK_EARLY = 7


class lbrmt_grid_desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32),
        ("tau", ctypes.c_double), ("lid_ux", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("fext_x", ctypes.c_double), ("fext_y", ctypes.c_double),
        ("rho_f", ctypes.c_double), ("eps", ctypes.c_double),
        ("layers", ctypes.c_int32), ("r_max", ctypes.c_int32),
        ("det_rel", ctypes.c_double), ("detJ_min", ctypes.c_double),
        ("precision", ctypes.c_int32), ("body_window", ctypes.c_int32),
        ("eta", ctypes.c_double), ("kappa_J", ctypes.c_double),
        ("lid_rho_mode", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class lbrmt_solid_desc(ctypes.Structure):
    _fields_ = [
        ("shape", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("cx", ctypes.c_double), ("cy", ctypes.c_double),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("theta", ctypes.c_double),
        ("G", ctypes.c_double), ("rho_s", ctypes.c_double),
    ]


class lbrmt_diag_t(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("mass", ctypes.c_double),
        ("mom_x", ctypes.c_double), ("mom_y", ctypes.c_double),
        ("centroid_x", ctypes.c_double), ("centroid_y", ctypes.c_double),
        ("disp_x", ctypes.c_double), ("disp_y", ctypes.c_double),
        ("max_u", ctypes.c_double), ("n_solid", ctypes.c_double), ("n_band", ctypes.c_double),
        ("lambda_sum", ctypes.c_double),
        ("health", ctypes.c_uint32 * 8),
    ]


class lbrmt_validation_t(ctypes.Structure):
    _fields_ = [
        ("nu", ctypes.c_double), ("mach_lb", ctypes.c_double), ("reynolds", ctypes.c_double),
        ("tau_ok", ctypes.c_int32), ("mach_ok", ctypes.c_int32),
        ("solids_inside", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class LBRMTError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status}) {detail}".strip())


_lib = None
_vp = ctypes.c_void_p


def lib():
    """Load liblbrmt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "python -m paper_2402_12696_amd.build_lib")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "lbrmt_status_string": (ctypes.c_char_p, [ctypes.c_int]),
            "lbrmt_last_error": (ctypes.c_char_p, [_vp]),
            "lbrmt_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(lbrmt_grid_desc),
                                                     ctypes.c_int32,
                                                     ctypes.POINTER(ctypes.c_size_t)]),
            "lbrmt_create": (ctypes.c_int, [ctypes.POINTER(lbrmt_grid_desc), ctypes.c_int32, _vp,
                                            ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
            "lbrmt_destroy": (None, [_vp]),
            "lbrmt_add_solids": (ctypes.c_int, [_vp, ctypes.POINTER(lbrmt_solid_desc),
                                                ctypes.c_int32]),
            "lbrmt_init": (ctypes.c_int, [_vp, _vp]),
            "lbrmt_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
            "lbrmt_step_count": (ctypes.c_int64, [_vp]),
            "lbrmt_read_macro": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
            "lbrmt_read_populations": (ctypes.c_int, [_vp, _vp]),
            "lbrmt_read_force": (ctypes.c_int, [_vp, _vp, _vp]),
            "lbrmt_read_refmap": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp]),
            "lbrmt_read_stress": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
            "lbrmt_diag": (ctypes.c_int, [_vp, ctypes.POINTER(lbrmt_diag_t)]),
            "lbrmt_diag_noalloc": (ctypes.c_int, [_vp, ctypes.POINTER(lbrmt_diag_t)]),
            "lbrmt_diag_sums": (ctypes.c_int, [_vp, _vp]),
            "lbrmt_diag_solid": (ctypes.c_int, [_vp, ctypes.c_int32, _vp]),
            "lbrmt_snapshot_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
            "lbrmt_step_snapshot": (ctypes.c_int, [_vp, _vp]),
            "lbrmt_adjoint_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
            "lbrmt_adjoint_zero": (ctypes.c_int, [_vp, _vp]),
            "lbrmt_adjoint_loss": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, _vp]),
            "lbrmt_adjoint_step": (ctypes.c_int, [_vp, _vp, _vp]),
            "lbrmt_adjoint_init": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
            "lbrmt_state_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
            "lbrmt_save_state": (ctypes.c_int, [_vp, _vp]),
            "lbrmt_load_state": (ctypes.c_int, [_vp, _vp]),
            "lbrmt_debug_poke": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int64,
                                                ctypes.c_double]),
            "lbrmt_validate": (ctypes.c_int, [ctypes.POINTER(lbrmt_grid_desc),
                                              ctypes.POINTER(lbrmt_solid_desc), ctypes.c_int32,
                                              ctypes.POINTER(lbrmt_validation_t)]),
            "lbrmt_set_timing": (ctypes.c_int, [_vp, ctypes.c_int32]),
            "lbrmt_kernel_time": (ctypes.c_int, [_vp, ctypes.c_char_p,
                                                 ctypes.POINTER(ctypes.c_double),
                                                 ctypes.POINTER(ctypes.c_int64)]),
            "lbrmt_band_nodes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64),
                                                ctypes.POINTER(ctypes.c_int64)]),
            "lbrmt_set_option": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int64]),
            "lbrmt_get_option": (ctypes.c_int, [_vp, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_int64)]),
            "lbrmt_autotune": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_double)]),
            "lbrmt_autotune_steps": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_double)]),
            "lbrmt_batch_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(lbrmt_grid_desc),
                                                           ctypes.c_int32,
                                                           ctypes.POINTER(ctypes.c_size_t)]),
            "lbrmt_batch_create": (ctypes.c_int, [ctypes.POINTER(lbrmt_grid_desc),
                                                  ctypes.POINTER(lbrmt_solid_desc),
                                                  ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                                  _vp, ctypes.c_size_t, _vp,
                                                  ctypes.POINTER(_vp)]),
            "lbrmt_batch_destroy": (None, [_vp]),
            "lbrmt_batch_init": (ctypes.c_int, [_vp]),
            "lbrmt_batch_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
            "lbrmt_batch_size": (ctypes.c_int32, [_vp]),
            "lbrmt_batch_member": (_vp, [_vp, ctypes.c_int32]),
            "lbrmt_batch_set_option": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int64]),
            "lbrmt_batch_get_option": (ctypes.c_int, [_vp, ctypes.c_int32,
                                                      ctypes.POINTER(ctypes.c_int64)]),
            "lbrmt_batch_autotune": (ctypes.c_int, [_vp, ctypes.c_int32,
                                                    ctypes.POINTER(ctypes.c_int32),
                                                    ctypes.POINTER(ctypes.c_double)]),
            "lbrmt_batch_last_error": (ctypes.c_char_p, [_vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(status):
    return lib().lbrmt_status_string(int(status)).decode()


def _check(rc, where, ctx=None):
    if rc != LBRMT_OK:
        detail = ""
        if ctx:
            detail = lib().lbrmt_last_error(ctx).decode()
        raise LBRMTError(rc, where, detail)


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------ same-name calls

def make_grid_desc(nx, ny, tau, lid_ux=0.0, periodic_x=False, periodic_y=False,
                   gravity=(0.0, 0.0), fext=(0.0, 0.0), rho_f=1.0, eps=1.5, layers=11, r_max=8,
                   det_rel=1e-8, detJ_min=1e-12, precision="f64", body_window=0, eta=1.0,
                   kappa_J=0.25, lid_rho_mode=0, **_ignored):
    prec = {"f64": LBRMT_FP64, "f32": LBRMT_FP32}[precision]
    return lbrmt_grid_desc(nx, ny, int(periodic_x), int(periodic_y), tau, lid_ux,
                           gravity[0], gravity[1], fext[0], fext[1], rho_f, eps, layers, r_max,
                           det_rel, detJ_min, prec, int(body_window), float(eta),
                           float(kappa_J), int(lid_rho_mode), 0)


def _solid_list(cfg):
    if cfg.get("solid") is not None and cfg.get("solids") is not None:
        raise ValueError("give either solid or solids")
    if cfg.get("solids") is not None:
        return list(cfg["solids"])
    return [cfg["solid"]] if cfg.get("solid") else []


def make_solid_desc(cx, cy, R, G, rho_s, shape="disc", b=None, theta=0.0, **_ignored):
    """A disc of radius R, or (shape="ellipse") an ellipse of semi-axes R and
    b with its R axis at angle theta to the x axis."""
    if shape == "disc":
        return lbrmt_solid_desc(0, 0, cx, cy, R, 0.0, 0.0, G, rho_s)
    if shape == "ellipse":
        return lbrmt_solid_desc(1, 0, cx, cy, R, R if b is None else b, theta, G, rho_s)
    raise ValueError(f"unknown solid shape {shape!r}")


def lbrmt_workspace_bytes(desc, max_solids):
    out = ctypes.c_size_t(0)
    _check(lib().lbrmt_workspace_bytes(ctypes.byref(desc), max_solids, ctypes.byref(out)),
           "lbrmt_workspace_bytes")
    return out.value


def lbrmt_create(desc, max_solids, workspace, nbytes, stream=None):
    ctx = _vp()
    _check(lib().lbrmt_create(ctypes.byref(desc), max_solids, _ptr(workspace), nbytes,
                              stream if stream is not None else _stream(), ctypes.byref(ctx)),
           "lbrmt_create")
    return ctx


def lbrmt_destroy(ctx):
    lib().lbrmt_destroy(ctx)


def lbrmt_add_solids(ctx, solids):
    arr = (lbrmt_solid_desc * len(solids))(*solids)
    _check(lib().lbrmt_add_solids(ctx, arr, len(solids)), "lbrmt_add_solids", ctx)


def lbrmt_init(ctx, u0=None):
    _check(lib().lbrmt_init(ctx, _ptr(u0)), "lbrmt_init", ctx)


def lbrmt_step(ctx, n):
    _check(lib().lbrmt_step(ctx, int(n)), "lbrmt_step", ctx)


def lbrmt_step_count(ctx):
    return lib().lbrmt_step_count(ctx)


def lbrmt_read_macro(ctx, rho, ux, uy):
    _check(lib().lbrmt_read_macro(ctx, _ptr(rho), _ptr(ux), _ptr(uy)), "lbrmt_read_macro", ctx)


def lbrmt_read_populations(ctx, f9):
    _check(lib().lbrmt_read_populations(ctx, _ptr(f9)), "lbrmt_read_populations", ctx)


def lbrmt_read_force(ctx, fx, fy):
    _check(lib().lbrmt_read_force(ctx, _ptr(fx), _ptr(fy)), "lbrmt_read_force", ctx)


def lbrmt_read_refmap(ctx, solid, X, Y, phi):
    _check(lib().lbrmt_read_refmap(ctx, solid, _ptr(X), _ptr(Y), _ptr(phi)),
           "lbrmt_read_refmap", ctx)


def lbrmt_read_stress(ctx, sxx, sxy, syy):
    _check(lib().lbrmt_read_stress(ctx, _ptr(sxx), _ptr(sxy), _ptr(syy)), "lbrmt_read_stress",
           ctx)


def _diag_call(name, ctx, raise_unstable):
    out = lbrmt_diag_t()
    rc = getattr(lib(), name)(ctx, ctypes.byref(out))
    if rc != LBRMT_EUNSTABLE or raise_unstable:
        _check(rc, name, ctx)
    d = {k: getattr(out, k) for k, _ in lbrmt_diag_t._fields_ if k != "health"}
    d["health"] = dict(zip(HEALTH_NAMES, list(out.health)))
    d["status"] = rc
    return d


def lbrmt_diag(ctx, raise_unstable=True):
    return _diag_call("lbrmt_diag", ctx, raise_unstable)


def lbrmt_diag_noalloc(ctx, raise_unstable=True):
    return _diag_call("lbrmt_diag_noalloc", ctx, raise_unstable)


def lbrmt_diag_sums(ctx, out):
    """out: a device float64 tensor (view) of at least 11 elements."""
    _check(lib().lbrmt_diag_sums(ctx, _ptr(out)), "lbrmt_diag_sums", ctx)


def lbrmt_diag_solid(ctx, solid):
    out = (ctypes.c_double * 6)()
    _check(lib().lbrmt_diag_solid(ctx, int(solid), out), "lbrmt_diag_solid", ctx)
    keys = ["centroid_x", "centroid_y", "disp_x", "disp_y", "n_solid", "n_band"]
    return dict(zip(keys, list(out)))


def lbrmt_snapshot_bytes(ctx):
    out = ctypes.c_size_t(0)
    _check(lib().lbrmt_snapshot_bytes(ctx, ctypes.byref(out)), "lbrmt_snapshot_bytes", ctx)
    return out.value


def lbrmt_step_snapshot(ctx, snap):
    _check(lib().lbrmt_step_snapshot(ctx, _ptr(snap)), "lbrmt_step_snapshot", ctx)


def lbrmt_adjoint_bytes(ctx):
    out = ctypes.c_size_t(0)
    _check(lib().lbrmt_adjoint_bytes(ctx, ctypes.byref(out)), "lbrmt_adjoint_bytes", ctx)
    return out.value


def lbrmt_adjoint_zero(ctx, adj):
    _check(lib().lbrmt_adjoint_zero(ctx, _ptr(adj)), "lbrmt_adjoint_zero", ctx)


def lbrmt_adjoint_loss(ctx, adj, snap, which, coef):
    c = (ctypes.c_double * 8)(*[float(v) for v in coef])
    _check(lib().lbrmt_adjoint_loss(ctx, _ptr(adj), _ptr(snap), int(which), c),
           "lbrmt_adjoint_loss", ctx)


def lbrmt_adjoint_step(ctx, adj, snap):
    _check(lib().lbrmt_adjoint_step(ctx, _ptr(adj), _ptr(snap)), "lbrmt_adjoint_step", ctx)


def lbrmt_adjoint_init(ctx, adj, snap0, u0bar):
    gu = (ctypes.c_double * 2)()
    _check(lib().lbrmt_adjoint_init(ctx, _ptr(adj), _ptr(snap0), _ptr(u0bar), gu),
           "lbrmt_adjoint_init", ctx)
    return gu[0], gu[1]


def lbrmt_state_bytes(ctx):
    out = ctypes.c_size_t(0)
    _check(lib().lbrmt_state_bytes(ctx, ctypes.byref(out)), "lbrmt_state_bytes", ctx)
    return out.value


def lbrmt_save_state(ctx, buf):
    _check(lib().lbrmt_save_state(ctx, _ptr(buf)), "lbrmt_save_state", ctx)


def lbrmt_load_state(ctx, buf):
    _check(lib().lbrmt_load_state(ctx, _ptr(buf)), "lbrmt_load_state", ctx)


def lbrmt_debug_poke(ctx, field, index, value):
    _check(lib().lbrmt_debug_poke(ctx, field, int(index), float(value)), "lbrmt_debug_poke", ctx)


def lbrmt_validate(desc, solids=()):
    arr = (lbrmt_solid_desc * max(1, len(solids)))(*solids)
    out = lbrmt_validation_t()
    _check(lib().lbrmt_validate(ctypes.byref(desc), arr, len(solids), ctypes.byref(out)),
           "lbrmt_validate")
    return {k: getattr(out, k) for k, _ in lbrmt_validation_t._fields_ if k != "reserved"}


def lbrmt_set_timing(ctx, enable):
    _check(lib().lbrmt_set_timing(ctx, int(bool(enable))), "lbrmt_set_timing", ctx)


def lbrmt_kernel_time(ctx, name):
    ms = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    _check(lib().lbrmt_kernel_time(ctx, name.encode(), ctypes.byref(ms), ctypes.byref(n)),
           "lbrmt_kernel_time", ctx)
    return ms.value, n.value


def lbrmt_band_nodes(ctx):
    b = ctypes.c_int64(0)
    w = ctypes.c_int64(0)
    _check(lib().lbrmt_band_nodes(ctx, ctypes.byref(b), ctypes.byref(w)), "lbrmt_band_nodes", ctx)
    return b.value, w.value


def lbrmt_set_option(ctx, option, value):
    _check(lib().lbrmt_set_option(ctx, int(option), int(value)), "lbrmt_set_option", ctx)


def lbrmt_get_option(ctx, option):
    v = ctypes.c_int64(0)
    _check(lib().lbrmt_get_option(ctx, int(option), ctypes.byref(v)), "lbrmt_get_option", ctx)
    return v.value


def lbrmt_autotune(ctx, reps=5):
    v, ms = ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(lib().lbrmt_autotune(ctx, int(reps), ctypes.byref(v), ctypes.byref(ms)),
           "lbrmt_autotune", ctx)
    return v.value, ms.value


def lbrmt_autotune_steps(ctx, steps=60):
    v, ms = ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(lib().lbrmt_autotune_steps(ctx, int(steps), ctypes.byref(v), ctypes.byref(ms)),
           "lbrmt_autotune_steps", ctx)
    return v.value, ms.value


def _bcheck(rc, where, batch=None):
    if rc != LBRMT_OK:
        detail = lib().lbrmt_batch_last_error(batch).decode() if batch else ""
        raise LBRMTError(rc, where, detail)


def lbrmt_batch_workspace_bytes(descs):
    arr = (lbrmt_grid_desc * len(descs))(*descs)
    out = ctypes.c_size_t(0)
    _bcheck(lib().lbrmt_batch_workspace_bytes(arr, len(descs), ctypes.byref(out)),
            "lbrmt_batch_workspace_bytes")
    return out.value


def lbrmt_batch_create(descs, solids, has_solid, workspace, nbytes, stream=None):
    n = len(descs)
    d = (lbrmt_grid_desc * n)(*descs)
    s = (lbrmt_solid_desc * n)(*solids) if solids is not None else None
    h = (ctypes.c_int32 * n)(*[int(x) for x in has_solid]) if has_solid is not None else None
    b = _vp()
    _bcheck(lib().lbrmt_batch_create(d, s, h, n, _ptr(workspace), nbytes,
                                     stream if stream is not None else _stream(),
                                     ctypes.byref(b)), "lbrmt_batch_create")
    return b


def lbrmt_batch_destroy(batch):
    lib().lbrmt_batch_destroy(batch)


def lbrmt_batch_init(batch):
    _bcheck(lib().lbrmt_batch_init(batch), "lbrmt_batch_init", batch)


def lbrmt_batch_step(batch, n):
    _bcheck(lib().lbrmt_batch_step(batch, int(n)), "lbrmt_batch_step", batch)


def lbrmt_batch_size(batch):
    return lib().lbrmt_batch_size(batch)


def lbrmt_batch_member(batch, k):
    m = lib().lbrmt_batch_member(batch, int(k))
    if not m:
        raise LBRMTError(LBRMT_EINVAL, "lbrmt_batch_member", f"no member {k}")
    return _vp(m)


def lbrmt_batch_set_option(batch, option, value):
    _bcheck(lib().lbrmt_batch_set_option(batch, int(option), int(value)),
            "lbrmt_batch_set_option", batch)


def lbrmt_batch_get_option(batch, option):
    v = ctypes.c_int64(0)
    _bcheck(lib().lbrmt_batch_get_option(batch, int(option), ctypes.byref(v)),
            "lbrmt_batch_get_option", batch)
    return v.value


def lbrmt_batch_autotune(batch, reps=5):
    v, ms = ctypes.c_int32(0), ctypes.c_double(0.0)
    _bcheck(lib().lbrmt_batch_autotune(batch, int(reps), ctypes.byref(v), ctypes.byref(ms)),
            "lbrmt_batch_autotune", batch)
    return v.value, ms.value


# ------------------------------------------------------------ convenience

class Sim:
    """One LBRMT simulation on a GPU: workspace, context and typed reads.

    Keywords are those of ``workloads.make`` (nx, ny, tau, lid_ux, periodic_x,
    periodic_y, gravity, fext, rho_f, eps, layers, r_max, det_rel, detJ_min,
    solid={cx, cy, R, G, rho_s[, shape="ellipse", b, theta]}, or solids=[...]
    for several solids with eta and body_window) plus precision="f64"|"f32".
    """

    owner = True

    @classmethod
    def _view(cls, ctx, device, cfg):
        """Read-only view of a context owned elsewhere (a batch member)."""
        import torch
        self = cls.__new__(cls)
        self.torch = torch
        self.device = torch.device(device)
        self.cfg = dict(cfg)
        self.nx, self.ny = cfg["nx"], cfg["ny"]
        self.nsolid = len(_solid_list(cfg))
        self.ctx = ctx
        self.owner = False
        return self

    def __init__(self, device="cuda:0", **cfg):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("Sim needs a HIP GPU (torch.cuda) device")
        torch.cuda.set_device(self.device)
        self.cfg = dict(cfg)
        self.nx, self.ny = cfg["nx"], cfg["ny"]
        self.desc = make_grid_desc(**cfg)
        solids = _solid_list(cfg)
        self.nsolid = len(solids)
        # a list of solids takes the several-solid context, even for one
        cap = max(2, self.nsolid) if cfg.get("solids") is not None else self.nsolid
        nbytes = lbrmt_workspace_bytes(self.desc, cap)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        self.ctx = lbrmt_create(self.desc, cap, self._ws, nbytes)
        if solids:
            lbrmt_add_solids(self.ctx, [make_solid_desc(**b) for b in solids])

    def close(self):
        if getattr(self, "ctx", None):
            if self.owner:
                self.torch.cuda.synchronize(self.device)
                lbrmt_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _plane(self, *lead):
        return self.torch.empty(*lead, self.ny, self.nx, dtype=self.torch.float64,
                                device=self.device)

    def init(self, u0=None):
        if u0 is not None:
            u0 = self.torch.as_tensor(np.asarray(u0), dtype=self.torch.float64)
            u0 = u0.reshape(2, self.ny, self.nx).contiguous().to(self.device)
            self._u0 = u0
        lbrmt_init(self.ctx, u0)
        return self

    def step(self, n=1):
        lbrmt_step(self.ctx, n)
        return self

    @property
    def step_count(self):
        return lbrmt_step_count(self.ctx)

    def macro(self):
        r, u, v = self._plane(), self._plane(), self._plane()
        lbrmt_read_macro(self.ctx, r, u, v)
        return r, u, v

    def populations(self):
        f = self._plane(9)
        lbrmt_read_populations(self.ctx, f)
        return f

    def force(self):
        fx, fy = self._plane(), self._plane()
        lbrmt_read_force(self.ctx, fx, fy)
        return fx, fy

    def refmap(self, solid=0):
        X, Y, phi = self._plane(), self._plane(), self._plane()
        lbrmt_read_refmap(self.ctx, solid, X, Y, phi)
        return X, Y, phi

    def stress(self):
        a, b, c = self._plane(), self._plane(), self._plane()
        lbrmt_read_stress(self.ctx, a, b, c)
        return a, b, c

    def diag(self, raise_unstable=True):
        return lbrmt_diag(self.ctx, raise_unstable)

    def diag_solid(self, solid):
        """One solid's centroid, mean displacement and node counts."""
        return lbrmt_diag_solid(self.ctx, solid)

    def save_state(self):
        buf = self.torch.empty(lbrmt_state_bytes(self.ctx), dtype=self.torch.uint8,
                               device=self.device)
        lbrmt_save_state(self.ctx, buf)
        return buf

    def load_state(self, buf):
        lbrmt_load_state(self.ctx, buf)

    def poke(self, index, value):
        lbrmt_debug_poke(self.ctx, 0, index, value)

    def set_timing(self, enable):
        lbrmt_set_timing(self.ctx, enable)

    def kernel_time(self, name):
        return lbrmt_kernel_time(self.ctx, name)

    def band_nodes(self):
        return lbrmt_band_nodes(self.ctx)

    def set_option(self, option, value):
        lbrmt_set_option(self.ctx, option, value)

    def get_option(self, option):
        return lbrmt_get_option(self.ctx, option)

    def autotune(self, reps=5):
        return lbrmt_autotune(self.ctx, reps)

    def autotune_steps(self, steps=60):
        """Chooses the extrapolation launch mode by timing whole steps (the
        simulation advances by them); returns (LBRMT_OPT_FUSED_FIT, ms/step)."""
        return lbrmt_autotune_steps(self.ctx, steps)


class Batch:
    """Independent simulations stepped together (one launch per kernel for all
    members).  cfgs: a list of ``workloads.make`` configurations sharing the
    precision and layer count; members are read through ``member(k)``, a
    read-only ``Sim`` view."""

    def __init__(self, cfgs, device="cuda:0", precision=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("Batch needs a HIP GPU (torch.cuda) device")
        torch.cuda.set_device(self.device)
        self.cfgs = [dict(c, precision=precision) if precision else dict(c) for c in cfgs]
        descs = [make_grid_desc(**c) for c in self.cfgs]
        solids = [make_solid_desc(**c["solid"]) if c.get("solid") else
                  lbrmt_solid_desc(0, 0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0) for c in self.cfgs]
        has = [1 if c.get("solid") else 0 for c in self.cfgs]
        nbytes = lbrmt_batch_workspace_bytes(descs)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        self.batch = lbrmt_batch_create(descs, solids, has, self._ws, nbytes)
        self.members = [Sim._view(lbrmt_batch_member(self.batch, k), device, c)
                        for k, c in enumerate(self.cfgs)]

    def __len__(self):
        return len(self.members)

    def init(self):
        lbrmt_batch_init(self.batch)
        return self

    def step(self, n=1):
        lbrmt_batch_step(self.batch, n)
        return self

    def member(self, k):
        return self.members[k]

    def set_option(self, option, value):
        lbrmt_batch_set_option(self.batch, option, value)

    def get_option(self, option):
        return lbrmt_batch_get_option(self.batch, option)

    def autotune(self, reps=5):
        return lbrmt_batch_autotune(self.batch, reps)

    def close(self):
        if getattr(self, "batch", None):
            self.torch.cuda.synchronize(self.device)
            for m in self.members:
                m.ctx = None
            lbrmt_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
