"""ctypes wrapper of the plain FP64 CPU oracle (``dg_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module; the product path never does.  It imports
nothing from the HIP package: configurations arrive as plain mappings of field
name to value (``dataclasses.asdict`` of any config object works).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "dg_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "dg_oracle_limiter.c")]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < max(
            [os.path.getmtime(f) for f in _SRCS] + [os.path.getmtime(os.path.join(_HERE, "dg_oracle.h"))]):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Cfg(C.Structure):
    _fields_ = [
        ("n", C.c_int), ("nvar", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
        ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
        ("closure", C.c_int), ("cs", C.c_double), ("h", C.c_double), ("gamma", C.c_double),
        ("bc", C.c_int), ("star", C.c_int), ("gm", C.c_double), ("r_core", C.c_double),
        ("q", C.c_double), ("eps", C.c_double), ("rp", C.c_double), ("phi0", C.c_double),
        ("damping", C.c_int), ("rd_in", C.c_double), ("rd_out", C.c_double),
        ("cfl", C.c_double), ("rk", C.c_int), ("positivity", C.c_int),
        ("pp_eps", C.c_double), ("flux", C.c_int),
    ]


_lib = None
_RHS_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double))


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.POINTER(C.c_double)
        cp = C.POINTER(_Cfg)
        _lib.or_gauss_legendre.argtypes = [C.c_int, P, P]
        _lib.or_phi.argtypes = [C.c_int, C.c_double]
        _lib.or_phi.restype = C.c_double
        _lib.or_dphi.argtypes = [C.c_int, C.c_double]
        _lib.or_dphi.restype = C.c_double
        _lib.or_nodes.argtypes = [cp, P, P]
        _lib.or_project.argtypes = [cp, P, P]
        _lib.or_eval_nodes.argtypes = [cp, P, P]
        _lib.or_rhs.argtypes = [cp, C.c_double, P, P, P]
        _lib.or_num_flux.argtypes = [cp, P, P, C.c_double, C.c_double, C.c_double, C.c_double, P]
        _lib.or_dt.argtypes = [cp, P]
        _lib.or_dt.restype = C.c_double
        _lib.or_rk_butcher.argtypes = [C.c_int, P, P, P, _RHS_FN, C.c_void_p, C.c_long, P,
                                       C.c_double, C.c_double]
        _lib.or_ssprk3_tableau.argtypes = [P, P, P]
        _lib.or_rk_tableau.argtypes = [C.c_int, P, P, P]
        _lib.or_rk_tableau.restype = C.c_int
        _lib.or_step.argtypes = [cp, P, C.c_double, C.c_double, P]
        _lib.or_step.restype = C.c_double
        _lib.or_damp.argtypes = [cp, P, P, C.c_double]
        _lib.or_torque.argtypes = [cp, C.c_double, P, P]
        _lib.or_torque.restype = C.c_double
        _lib.or_planet_pos.argtypes = [cp, C.c_double, P, P]
        U8 = C.POINTER(C.c_ubyte)
        _lib.or_indicator.argtypes = [cp, P, P]
        _lib.or_minmod.argtypes = [cp, P, P, U8, U8]
        _lib.or_gauss_lobatto.argtypes = [C.c_int, P, P]
        _lib.or_pp_lobatto_points.argtypes = [C.c_int]
        _lib.or_positivity.argtypes = [cp, P, U8, P]
        _lib.or_step_limited.argtypes = [cp, P, C.c_double, C.c_double, P, C.c_double]
        _lib.or_step_limited.restype = C.c_double
        _lib.or_mlp_features.argtypes = [cp, P, P, P]
        _lib.or_bf16.argtypes = [C.c_double]
        _lib.or_bf16.restype = C.c_double
        _lib.or_mlp_forward.argtypes = [P, P, C.c_long, C.c_int, P, P, P]
        _lib.or_mlp_loss_grad.argtypes = [P, P, P, C.c_long, C.c_double, C.c_int, P]
        _lib.or_mlp_loss_grad.restype = C.c_double
        _lib.or_adam.argtypes = [P, P, P, P, C.c_long, C.c_long, C.c_double, C.c_double, C.c_double,
                                 C.c_double]
    return _lib


_DEFAULTS = dict(n=3, nvar=3, nx=8, ny=8, x0=0.0, x1=1.0, y0=0.0, y1=1.0, closure=0, cs=1.0,
                 h=0.05, gamma=1.4, bc=0, star=0, gm=1.0, r_core=0.4, q=0.0, eps=0.03,
                 rp=1.0, phi0=0.0, damping=0, rd_in=0.4, rd_out=2.3, cfl=0.2, rk=0,
                 positivity=0, pp_eps=0.0, flux=0)


def cfg(fields=None, **kw):
    """Build the oracle configuration from a mapping and/or keywords.

    ``order`` is accepted as an alias of ``n``; unknown keys are ignored."""
    d = dict(_DEFAULTS)
    src = dict(fields or {})
    src.update(kw)
    if "order" in src:
        src["n"] = src["order"]
    for k in _DEFAULTS:
        if k in src:
            d[k] = src[k]
    c = _Cfg()
    for k, v in d.items():
        setattr(c, k, v)
    return c


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def n_elem(c):
    return c.nx * c.ny


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    if lib().or_gauss_legendre(n, _p(x), _p(w)) != 0:
        raise ValueError("n out of range")
    return x, w


def phi(a, x):
    return lib().or_phi(a, float(x))


def dphi(a, x):
    return lib().or_dphi(a, float(x))


def nodes(c):
    E, nn = n_elem(c), c.n * c.n
    x = np.zeros(E * nn)
    y = np.zeros(E * nn)
    lib().or_nodes(C.byref(c), _p(x), _p(y))
    return x.reshape(E, nn), y.reshape(E, nn)


def project(c, prim):
    """prim [var][E][n^2] -> modes u [var][n^2][E]"""
    prim = _f64(prim)
    u = np.zeros((c.nvar, c.n * c.n, n_elem(c)))
    lib().or_project(C.byref(c), _p(prim), _p(u))
    return u


def eval_nodes(c, u):
    u = _f64(u)
    out = np.zeros((c.nvar, n_elem(c), c.n * c.n))
    lib().or_eval_nodes(C.byref(c), _p(u), _p(out))
    return out


def rhs(c, t, u, u0=None):
    u = _f64(u)
    out = np.zeros_like(u)
    u0p = _p(_f64(u0)) if u0 is not None else None
    if c.bc == 1 and u0 is None:
        raise ValueError("bc == 1 needs the initial modes u0")
    keep = _f64(u0) if u0 is not None else None
    lib().or_rhs(C.byref(c), float(t), _p(u), _p(keep) if keep is not None else u0p, _p(out))
    return out


def num_flux(c, Ui, Uo, nx, ny, x=0.0, y=0.0):
    """the configured edge flux h(U_in, U_out) for outward normal (nx, ny)"""
    Ui, Uo = _f64(Ui), _f64(Uo)
    h = np.zeros(c.nvar)
    lib().or_num_flux(C.byref(c), _p(Ui), _p(Uo), float(nx), float(ny), float(x), float(y), _p(h))
    return h


def dt(c, u):
    return lib().or_dt(C.byref(c), _p(_f64(u)))


def ssprk3_tableau():
    A = np.zeros(9)
    b = np.zeros(3)
    cc = np.zeros(3)
    lib().or_ssprk3_tableau(_p(A), _p(b), _p(cc))
    return A.reshape(3, 3), b, cc


def rk_tableau(kind):
    """(A [s, s], b [s], c [s]) of an Appendix A table (0 SSP(3,3), 1 SSP(2,2),
    2 SSP(5,4), 3 Cash-Karp)."""
    A = np.zeros(36)
    b = np.zeros(6)
    cc = np.zeros(6)
    s = lib().or_rk_tableau(int(kind), _p(A), _p(b), _p(cc))
    if s < 0:
        raise ValueError(f"unknown RK table {kind}")
    return A.reshape(6, 6)[:s, :s].copy(), b[:s].copy(), cc[:s].copy()


def rk_butcher(A, b, cc, f, u, t, dt_):
    """Apply one Butcher-form RK step of the oracle to y' = f(t, y) (numpy f)."""
    A = _f64(A)
    b = _f64(b)
    cc = _f64(cc)
    u = _f64(u).copy()
    N = u.size

    def cb(_ctx, tt, yp, kp):
        y = np.ctypeslib.as_array(yp, shape=(N,))
        k = np.ctypeslib.as_array(kp, shape=(N,))
        k[:] = f(tt, y.copy())

    fn = _RHS_FN(cb)
    lib().or_rk_butcher(len(b), _p(A), _p(b), _p(cc), fn, None, N, _p(u), float(t), float(dt_))
    return u


def step(c, u, t, dt_fixed=0.0, u0=None):
    """One full step in place on a copy; returns (u_new, dt)."""
    u = _f64(u).copy()
    keep = _f64(u0) if u0 is not None else None
    if (c.bc == 1 or c.damping) and keep is None:
        raise ValueError("bc == 1 or damping needs the initial modes u0")
    d = lib().or_step(C.byref(c), _p(u), float(t), float(dt_fixed), _p(keep) if keep is not None else None)
    return u, d


def damp(c, u, u0, dt_):
    u = _f64(u).copy()
    lib().or_damp(C.byref(c), _p(u), _p(_f64(u0)), float(dt_))
    return u


def torque(c, t, u):
    s = C.c_double(0.0)
    g = lib().or_torque(C.byref(c), float(t), _p(_f64(u)), C.byref(s))
    return g, s.value


def planet_pos(c, t):
    x = C.c_double()
    y = C.c_double()
    lib().or_planet_pos(C.byref(c), float(t), C.byref(x), C.byref(y))
    return x.value, y.value


# ---------------------------------------------------------------- troubled cells
MLP_NPARAM = 3169


def _u8(a):
    return a.ctypes.data_as(C.POINTER(C.c_ubyte))


def indicator(c, u):
    s = np.zeros(n_elem(c))
    lib().or_indicator(C.byref(c), _p(_f64(u)), _p(s))
    return s


def minmod(c, u, u0, flags):
    """returns (limited u, changed mask)"""
    u = _f64(u).copy()
    fl = np.ascontiguousarray(flags, dtype=np.uint8)
    ch = np.zeros(n_elem(c), dtype=np.uint8)
    lib().or_minmod(C.byref(c), _p(u), _p(_f64(u0)), _u8(fl), _u8(ch))
    return u, ch.astype(bool)


def gauss_lobatto(L):
    x = np.zeros(L)
    w = np.zeros(L)
    if lib().or_gauss_lobatto(int(L), _p(x), _p(w)) != 0:
        raise ValueError("unsupported number of Gauss-Lobatto points")
    return x, w


def pp_lobatto_points(np_):
    return int(lib().or_pp_lobatto_points(int(np_)))


def positivity(c, u):
    """returns (limited u, changed mask, theta[E, 2])"""
    u = _f64(u).copy()
    ch = np.zeros(n_elem(c), dtype=np.uint8)
    th = np.zeros((n_elem(c), 2))
    lib().or_positivity(C.byref(c), _p(u), _u8(ch), _p(th))
    return u, ch.astype(bool), th


def step_limited(c, u, t, dt_fixed, u0, s0):
    """s0 = inf: no minmod flags (positivity alone if c.positivity)"""
    u = _f64(u).copy()
    d = lib().or_step_limited(C.byref(c), _p(u), float(t), float(dt_fixed), _p(_f64(u0)), float(s0))
    return u, d


def mlp_features(c, u, scale):
    f = np.zeros((n_elem(c), c.nvar * c.n * c.n))
    lib().or_mlp_features(C.byref(c), _p(_f64(u)), _p(_f64(scale)), _p(f))
    return f


def bf16(x):
    return lib().or_bf16(float(x))


def mlp_forward(par, x, bf16=True):
    x = _f64(x)
    nb = x.shape[0]
    z = np.zeros(nb)
    h1 = np.zeros((nb, 32))
    h2 = np.zeros((nb, 32))
    lib().or_mlp_forward(_p(_f64(par)), _p(x), nb, int(bf16), _p(z), _p(h1), _p(h2))
    return z, h1, h2


def mlp_loss_grad(par, x, y, pos_weight=1.0, bf16=True):
    x = _f64(x)
    g = np.zeros(MLP_NPARAM)
    loss = lib().or_mlp_loss_grad(_p(_f64(par)), _p(x), _p(_f64(y)), x.shape[0], float(pos_weight),
                                  int(bf16), _p(g))
    return loss, g


def adam(par, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    par = _f64(par).copy()
    m = _f64(m).copy()
    v = _f64(v).copy()
    lib().or_adam(_p(par), _p(_f64(grad)), _p(m), _p(v), par.size, int(t), lr, b1, b2, eps)
    return par, m, v
