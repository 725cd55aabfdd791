"""Thin ctypes binding of the C-ABI library ``libdg.so`` (include/dg.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Device memory and streams come from PyTorch tensors
(``tensor.data_ptr()``, ``torch.cuda.current_stream().cuda_stream``).  If the
library has not been built the calls raise; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdg.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EHIP, DG_EUNSUPPORTED, DG_ENONFINITE = 0, -1, -2, -3, -4, -5
CLOSURE_ISOTHERMAL, CLOSURE_LOCALLY_ISOTHERMAL, CLOSURE_ADIABATIC = 0, 1, 2
BC_PERIODIC, BC_FIXED_INITIAL, BC_GRADIENT_FREE = 0, 1, 2
PRECISION_FP64, PRECISION_MIXED = 0, 1
LIMITER_NONE, LIMITER_MODAL_DECAY, LIMITER_LEARNED = 0, 1, 2
RK_SSP33, RK_SSP22, RK_SSP54, RK_CASHKARP = 0, 1, 2, 3
FLUX_RUSANOV, FLUX_HLLC = 0, 1


class DGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dg error {code}: {msg}")
        self.code = code


class dg_config(C.Structure):
    _fields_ = [
        ("order", C.c_int), ("nvar", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
        ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
        ("closure", C.c_int), ("cs", C.c_double), ("h", C.c_double), ("gamma", C.c_double),
        ("bc", C.c_int), ("star", C.c_int), ("gm", C.c_double), ("r_core", C.c_double),
        ("q", C.c_double), ("eps", C.c_double), ("rp", C.c_double), ("phi0", C.c_double),
        ("damping", C.c_int), ("rd_in", C.c_double), ("rd_out", C.c_double),
        ("cfl", C.c_double), ("precision", C.c_int), ("sigma0", C.c_double), ("limiter", C.c_int),
        ("limiter_s0", C.c_double), ("mlp_theta", C.c_double), ("rk", C.c_int), ("positivity", C.c_int),
        ("pp_eps", C.c_double), ("flux", C.c_int),
    ]


@dataclasses.dataclass
class Config:
    """Problem statement; field meanings as in ``dg_config`` (include/dg.h)."""
    order: int = 3
    nvar: int = 3
    nx: int = 64
    ny: int = 64
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    closure: int = CLOSURE_ISOTHERMAL
    cs: float = 1.0
    h: float = 0.05
    gamma: float = 1.4
    bc: int = BC_PERIODIC
    star: int = 0
    gm: float = 1.0
    r_core: float = 0.4
    q: float = 0.0
    eps: float = 0.03
    rp: float = 1.0
    phi0: float = 0.0
    damping: int = 0
    rd_in: float = 0.4
    rd_out: float = 2.3
    cfl: float = 0.2
    precision: int = PRECISION_FP64
    sigma0: float = 1.0
    limiter: int = LIMITER_NONE
    limiter_s0: float = 0.0
    mlp_theta: float = 0.5
    rk: int = RK_SSP33
    positivity: int = 0
    pp_eps: float = 0.0
    flux: int = 0

    @property
    def n(self):
        return self.order

    @property
    def n_elem(self):
        return self.nx * self.ny

    @property
    def tile_width(self):
        """elements per tile of the state layout (64 / order)"""
        return 64 // self.order

    @property
    def tiles_x(self):
        return -(-self.nx // self.tile_width)

    @property
    def state_shape(self):
        """a state tensor in the element-tiled layout of dg.h:
        [j][tile][var][b][a][slot]"""
        return (self.ny, self.tiles_x, self.nvar, self.order, self.order, self.tile_width)

    def to_c(self) -> dg_config:
        c = dg_config()
        for f in dg_config._fields_:
            setattr(c, f[0], getattr(self, f[0]))
        return c

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


_lib = None


def lib():
    """Load libdg.so; raises if it was not built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, dp, cp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(dg_config)
        L.dg_get_nodes.argtypes = [cp, dp, dp]
        L.dg_state_size.argtypes = [cp]
        L.dg_state_size.restype = C.c_longlong
        L.dg_init.argtypes = [cp, dp, vp, vp, C.POINTER(vp)]
        L.dg_full_state.argtypes = [vp, vp, vp]
        L.dg_rhs.argtypes = [vp, C.c_double, vp, vp]
        L.dg_rk_step.argtypes = [vp, vp, vp, C.c_double, vp]
        L.dg_rk_step_torque.argtypes = [vp, vp, vp, C.c_double, vp, vp]
        L.dg_torque.argtypes = [vp, C.c_double, vp, vp, vp]
        L.dg_torque_noalloc.argtypes = [cp, C.c_double, vp, vp, vp, vp]
        L.dg_sync.argtypes = [vp]
        L.dg_free.argtypes = [vp]
        L.dg_profile_begin.argtypes = [vp]
        L.dg_profile_end.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.dg_troubled.argtypes = [vp, vp, C.c_int, vp, vp, vp]
        L.dg_positivity.argtypes = [vp, vp, vp, vp]
        L.dg_mlp_feature_scales.argtypes = [vp, dp]
        L.dg_mlp_features.argtypes = [vp, vp, vp]
        L.dg_mlp_params.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.dg_mlp_forward.argtypes = [vp, vp, C.c_long, vp]
        L.dg_mlp_train_step.argtypes = [vp, vp, vp, C.c_long, C.c_float, C.c_float, vp, vp]
        L.dg_capture.argtypes = [vp, vp, vp, vp, vp]
        L.dg_last_error.argtypes = [vp]
        L.dg_last_error.restype = C.c_char_p
        for name in ("dg_get_nodes", "dg_init", "dg_rhs", "dg_rk_step", "dg_rk_step_torque", "dg_torque",
                     "dg_sync", "dg_free",
                     "dg_profile_begin", "dg_profile_end", "dg_full_state", "dg_troubled", "dg_positivity",
                     "dg_mlp_feature_scales", "dg_mlp_features", "dg_mlp_params", "dg_mlp_forward",
                     "dg_mlp_train_step", "dg_capture", "dg_torque_noalloc"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


EXPORTS = ("dg_get_nodes", "dg_state_size", "dg_init", "dg_rhs", "dg_rk_step", "dg_rk_step_torque", "dg_torque",
           "dg_sync", "dg_free",
           "dg_last_error", "dg_profile_begin", "dg_profile_end", "dg_full_state", "dg_troubled", "dg_positivity",
           "dg_mlp_feature_scales", "dg_mlp_features", "dg_mlp_params", "dg_mlp_forward", "dg_mlp_train_step",
           "dg_capture", "dg_torque_noalloc")
MLP_NPARAM = 3169


def _check(rc, h=None):
    if rc != DG_OK:
        msg = lib().dg_last_error(h)
        raise DGError(rc, msg.decode() if msg else "")


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def dg_get_nodes(cfg: Config):
    E, nn = cfg.n_elem, cfg.order ** 2
    x = np.zeros(E * nn)
    y = np.zeros(E * nn)
    dp = C.POINTER(C.c_double)
    c = cfg.to_c()
    _check(lib().dg_get_nodes(C.byref(c), x.ctypes.data_as(dp), y.ctypes.data_as(dp)))
    return x.reshape(E, nn), y.reshape(E, nn)


class Handle:
    """Owns a dg_handle; frees it on close() or garbage collection."""

    def __init__(self, ptr: C.c_void_p, cfg: Config):
        self.ptr = ptr
        self.cfg = cfg

    def close(self):
        if self.ptr:
            lib().dg_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dg_state_size(cfg: Config) -> int:
    """doubles in one state array (padding included)"""
    c = cfg.to_c()
    n = lib().dg_state_size(C.byref(c))
    if n < 0:
        raise DGError(int(n), (lib().dg_last_error(None) or b"").decode())
    return int(n)


def to_planes(cfg: Config, u):
    """A state (tiled layout; torch tensor or numpy array) as [var][a*n + b][e]
    with e = j*nx + i, padding dropped (the layout the oracle uses)."""
    n, W, TX = cfg.order, cfg.tile_width, cfg.tiles_x
    x = u.reshape(cfg.state_shape)
    x = x.permute(2, 4, 3, 0, 1, 5) if hasattr(x, "permute") else x.transpose(2, 4, 3, 0, 1, 5)
    x = x.reshape(cfg.nvar, n * n, cfg.ny, TX * W)[..., :cfg.nx]
    return x.reshape(cfg.nvar, n * n, cfg.n_elem)


def from_planes(cfg: Config, planes, device="cuda"):
    """Inverse of to_planes: [var][a*n + b][e] (numpy) to a tensor in the
    tiled layout (padding zero)."""
    import torch
    n, W, TX = cfg.order, cfg.tile_width, cfg.tiles_x
    p = np.asarray(planes, dtype=np.float64).reshape(cfg.nvar, n, n, cfg.ny, cfg.nx)
    full = np.zeros((cfg.nvar, n, n, cfg.ny, TX * W))
    full[..., :cfg.nx] = p
    x = full.reshape(cfg.nvar, n, n, cfg.ny, TX, W).transpose(3, 4, 0, 2, 1, 5)  # [j][t][v][b][a][s]
    return torch.tensor(np.ascontiguousarray(x), device=device)


def dg_init(cfg: Config, prim, device="cuda"):
    """Project primitive node values ``prim`` ([var][E][n^2], host float64) and
    return (handle, u0) with u0 a device tensor in the state layout (the
    deviation from the equilibrium in the mixed-precision form)."""
    import torch
    prim = np.ascontiguousarray(prim, dtype=np.float64)
    if prim.shape != (cfg.nvar, cfg.n_elem, cfg.order ** 2):
        raise ValueError(f"prim has shape {prim.shape}, expected {(cfg.nvar, cfg.n_elem, cfg.order ** 2)}")
    u0 = torch.empty(cfg.state_shape, dtype=torch.float64, device=device)
    h = C.c_void_p()
    c = cfg.to_c()
    dp = C.POINTER(C.c_double)
    rc = lib().dg_init(C.byref(c), prim.ctypes.data_as(dp), _ptr(u0), _stream(), C.byref(h))
    _check(rc)
    return Handle(h, cfg), u0


def dg_rhs(h: Handle, t: float, u, rhs):
    _check(lib().dg_rhs(h.ptr, float(t), _ptr(u), _ptr(rhs)), h.ptr)


def dg_rk_step(h: Handle, u, t_dev, dt_fixed: float = 0.0, dt_used=None):
    _check(lib().dg_rk_step(h.ptr, _ptr(u), _ptr(t_dev), float(dt_fixed), _ptr(dt_used)), h.ptr)


def dg_rk_step_torque(h: Handle, u, t_dev, out, dt_fixed: float = 0.0, dt_used=None):
    """The torque of the state entering the step (u^n at t^n) into the device
    double out, then dg_rk_step (same bits as dg_torque before dg_rk_step)."""
    _check(lib().dg_rk_step_torque(h.ptr, _ptr(u), _ptr(t_dev), float(dt_fixed), _ptr(dt_used), _ptr(out)), h.ptr)


def dg_torque(h: Handle, u, out, t: float = 0.0, t_dev=None):
    _check(lib().dg_torque(h.ptr, float(t), _ptr(t_dev), _ptr(u), _ptr(out)), h.ptr)


def dg_torque_noalloc(cfg: Config, u, out, t: float = 0.0, t_dev=None, stream=None):
    """dg_torque without a handle and without allocating: partial sums in the
    library's static device scratch (FP64 states; calls on one GPU must not
    overlap).  stream: a hipStream_t value (default: torch's current stream)."""
    c = cfg.to_c()
    s = _stream() if stream is None else C.c_void_p(stream)
    _check(lib().dg_torque_noalloc(C.byref(c), float(t), _ptr(t_dev), _ptr(u), _ptr(out), s))


def dg_profile_begin(h: Handle):
    _check(lib().dg_profile_begin(h.ptr), h.ptr)


def dg_profile_end(h: Handle):
    """(summed stage-kernel ms, number of stage launches) since dg_profile_begin"""
    ms = C.c_double()
    n = C.c_int()
    _check(lib().dg_profile_end(h.ptr, C.byref(ms), C.byref(n)), h.ptr)
    return ms.value, n.value


def dg_full_state(h: Handle, dev, full):
    _check(lib().dg_full_state(h.ptr, _ptr(dev), _ptr(full)), h.ptr)


def dg_troubled(h: Handle, u, apply=False, flags=None, changed=None, sensor=None):
    _check(lib().dg_troubled(h.ptr, _ptr(u), int(bool(apply)), _ptr(flags), _ptr(changed), _ptr(sensor)), h.ptr)


def dg_positivity(h: Handle, u, changed=None, theta=None):
    """positivity limiter in place; changed: uint8 [E], theta: float64 [E, 2] (device)"""
    _check(lib().dg_positivity(h.ptr, _ptr(u), _ptr(changed), _ptr(theta)), h.ptr)


def dg_mlp_feature_scales(h: Handle):
    out = np.zeros(h.cfg.nvar)
    _check(lib().dg_mlp_feature_scales(h.ptr, out.ctypes.data_as(C.POINTER(C.c_double))), h.ptr)
    return out


def dg_mlp_features(h: Handle, u, feat):
    """feat: int16/uint16 device tensor [E, 64] receiving bf16 bit patterns"""
    _check(lib().dg_mlp_features(h.ptr, _ptr(u), _ptr(feat)), h.ptr)


def dg_mlp_params(h: Handle, set_params=None, get=False):
    fp = C.POINTER(C.c_float)
    src = None
    if set_params is not None:
        src = np.ascontiguousarray(set_params, dtype=np.float32)
        assert src.size == MLP_NPARAM
    out = np.zeros(MLP_NPARAM, dtype=np.float32) if get else None
    _check(lib().dg_mlp_params(h.ptr, src.ctypes.data_as(fp) if src is not None else None,
                               out.ctypes.data_as(fp) if out is not None else None), h.ptr)
    return out


def dg_mlp_forward(h: Handle, feat, n, logits):
    _check(lib().dg_mlp_forward(h.ptr, _ptr(feat), int(n), _ptr(logits)), h.ptr)


def dg_mlp_train_step(h: Handle, feat, labels, n, pos_weight=1.0, lr=1e-3, loss=None, grad=None):
    _check(lib().dg_mlp_train_step(h.ptr, _ptr(feat), _ptr(labels), int(n), float(pos_weight), float(lr),
                                   _ptr(loss), _ptr(grad)), h.ptr)


def dg_capture(h: Handle, feat=None, flags=None, labels=None, mlp_flags=None):
    _check(lib().dg_capture(h.ptr, _ptr(feat), _ptr(flags), _ptr(labels), _ptr(mlp_flags)), h.ptr)


def dg_sync(h: Handle):
    _check(lib().dg_sync(h.ptr), h.ptr)
