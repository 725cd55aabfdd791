"""Host-side checks of the C-ABI library: it loads, exports every symbol the
header declares, validates configurations before touching a device, and its
node coordinates match the oracle's.  No kernel is launched here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1805_01443_amd import dg
from paper_1805_01443_amd import configs as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?(?:\w+\s+)*\w+\s*\**\s*(dg_\w+)\s*\(", txt, re.M))
    return names


def test_library_exports_every_declared_symbol():
    L = dg.lib()
    names = _declared_symbols()
    assert {"dg_init", "dg_rhs", "dg_rk_step", "dg_torque"} <= names
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(dg.EXPORTS) <= names


def test_nm_exports_are_c_symbols():
    out = os.popen("nm -D --defined-only " + dg.LIB_PATH).read()
    for n in _declared_symbols():
        assert re.search(r"\bT\s+" + n + r"\b", out), n


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_nodes_match_oracle(order):
    cfg = W.disc(nx=7, order=order).replace(ny=5)
    x, y = dg.dg_get_nodes(cfg)
    ox, oy = O.nodes(O.cfg(dataclass_fields(cfg)))
    assert np.max(np.abs(x - ox)) < 1e-15 and np.max(np.abs(y - oy)) < 1e-15


def dataclass_fields(cfg):
    import dataclasses
    return dataclasses.asdict(cfg)


@pytest.mark.parametrize("bad,code", [
    (dict(order=7), dg.DG_EUNSUPPORTED),
    (dict(order=1), dg.DG_EUNSUPPORTED),
    (dict(nx=0), dg.DG_EINVAL),
    (dict(nvar=4), dg.DG_EINVAL),
    (dict(x1=-1.0), dg.DG_EINVAL),
    (dict(cfl=0.0), dg.DG_EINVAL),
    (dict(closure=9), dg.DG_EINVAL),
    (dict(q=-1.0), dg.DG_EINVAL),
    (dict(rk=7), dg.DG_EINVAL),
    (dict(rk=dg.RK_CASHKARP, limiter=dg.LIMITER_MODAL_DECAY), dg.DG_EUNSUPPORTED),
    (dict(positivity=2), dg.DG_EINVAL),
    (dict(positivity=1, rk=dg.RK_SSP22), dg.DG_EUNSUPPORTED),
    (dict(pp_eps=-1.0), dg.DG_EINVAL),
    (dict(pp_eps=float("nan")), dg.DG_EINVAL),
    (dict(bc=3), dg.DG_EINVAL),
    (dict(flux=2), dg.DG_EINVAL),
    (dict(flux=dg.FLUX_HLLC), dg.DG_EUNSUPPORTED),  # isothermal closure
])
def test_init_rejects_bad_configs_without_a_device(bad, code):
    cfg = W.wave(nx=8).replace(**bad)
    prim = np.ones((3, 64, 9))
    h = C.c_void_p()
    c = cfg.to_c()
    dp = C.POINTER(C.c_double)
    rc = dg.lib().dg_init(C.byref(c), prim.ctypes.data_as(dp), C.c_void_p(8), None, C.byref(h))
    assert rc == code
    assert h.value is None
    assert dg.lib().dg_last_error(None)


def test_null_handle_calls_fail_cleanly():
    L = dg.lib()
    assert L.dg_rhs(None, 0.0, None, None) == dg.DG_EINVAL
    assert L.dg_rk_step(None, None, None, 0.0, None) == dg.DG_EINVAL
    assert L.dg_rk_step_torque(None, None, None, 0.0, None, None) == dg.DG_EINVAL
    assert L.dg_torque(None, 0.0, None, None, None) == dg.DG_EINVAL
    assert L.dg_sync(None) == dg.DG_EINVAL
    assert L.dg_free(None) == dg.DG_OK


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1805_01443_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"(import\s+oracle|from\s+oracle|liboracle|dg_oracle|or_rhs)", txt), fn


@pytest.mark.parametrize("cfg", [W.wave(nx=70, order=3).replace(ny=9), W.disc(nx=26, order=5),
                                 W.disc_ring(nx=40, order=4), W.wave(nx=5, order=2).replace(ny=3)])
def test_state_size_and_tiled_layout(cfg):
    """dg_state_size and the binding's layout conversion follow the formula of
    the state layout in dg.h: mode (a, b) of variable v of element (i, j) at
    ((t * nvar + v) * n + b) * n * W + a * W + s, t = j * TX + i / W, s = i % W."""
    n, Wd = cfg.order, 64 // cfg.order
    TX = -(-cfg.nx // Wd)
    size = dg.dg_state_size(cfg)
    assert size == cfg.nvar * n * n * TX * Wd * cfg.ny
    pl = np.random.default_rng(0).normal(size=(cfg.nvar, n * n, cfg.n_elem))
    u = np.zeros(size)
    for e in range(cfg.n_elem):
        i, j = e % cfg.nx, e // cfg.nx
        t, s = j * TX + i // Wd, i % Wd
        for v in range(cfg.nvar):
            for a in range(n):
                for b in range(n):
                    u[((t * cfg.nvar + v) * n + b) * n * Wd + a * Wd + s] = pl[v, a * n + b, e]
    assert np.array_equal(dg.to_planes(cfg, u), pl)
    assert np.array_equal(dg.from_planes(cfg, pl, device="cpu").numpy().ravel(), u)


def test_state_size_rejects_bad_config():
    with pytest.raises(dg.DGError):
        dg.dg_state_size(W.wave(nx=8).replace(order=9))


def test_state_size_limit_is_the_buffer_range():
    """State arrays are addressed through buffer resources of 2^31 - 1 bytes:
    the largest configuration below that is accepted, the next row is not
    (order 5, three variables: 600 bytes per padded element slot, 1896 slots
    per row)."""
    ok = W.disc(nx=1896, order=5).replace(ny=1887)
    assert dg.dg_state_size(ok) * 8 == 600 * 1896 * 1887 <= 2 ** 31 - 1
    with pytest.raises(dg.DGError):
        dg.dg_state_size(ok.replace(ny=1888))


def test_noalloc_torque_rejects_what_it_cannot_hold_without_a_device():
    """dg_torque_noalloc keeps its partial sums, one per tile, in a static
    array of 524288 doubles: a grid needing more is refused before any device
    call, and so is the deviation form (its states are not full states)."""
    # order 2: 32 elements per tile, 128 tiles per row: 537600 partial sums
    cfg = W.disc(nx=4096, order=2).replace(ny=4200)
    assert dg.dg_state_size(cfg) > 0
    with pytest.raises(dg.DGError) as ex:
        dg.dg_torque_noalloc(cfg, None, None, stream=0)
    assert ex.value.code == dg.DG_EUNSUPPORTED
    with pytest.raises(dg.DGError) as ex:
        dg.dg_torque_noalloc(W.disc_mixed(nx=16, order=3), None, None, stream=0)
    assert ex.value.code == dg.DG_EUNSUPPORTED
    with pytest.raises(dg.DGError) as ex:
        dg.dg_torque_noalloc(W.disc(nx=16, order=3), None, None, stream=0)
    assert ex.value.code == dg.DG_EINVAL
