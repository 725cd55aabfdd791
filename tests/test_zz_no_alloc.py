"""The allocation-free torque entry point (dg_torque_noalloc) against
dg_torque: same kernels and summation order, so the same bits, on two calls in
a row, the second on a smaller grid and order (the static scratch keeps the
first call's partial sums; the second call must not depend on them)."""
import numpy as np
import pytest

from paper_1805_01443_amd import configs as W
from paper_1805_01443_amd import dg

pytestmark = pytest.mark.gpu


def _torque_pair(T, cfg, t):
    prim = W.prim_for(cfg, "disc", seed=4)
    h, u = dg.dg_init(cfg, prim)
    t_dev = T.zeros(1, dtype=T.float64, device="cuda")
    for _ in range(2):
        dg.dg_rk_step(h, u, t_dev, 0.0, None)
    ref = T.zeros(1, dtype=T.float64, device="cuda")
    got = T.full((1,), float("nan"), dtype=T.float64, device="cuda")
    dg.dg_torque(h, u, ref, t_dev=t_dev)
    dg.dg_sync(h)
    dg.dg_torque_noalloc(cfg, u, got, t_dev=t_dev)
    T.cuda.synchronize()
    # host-side time argument instead of the device time
    got_t = T.full((1,), float("nan"), dtype=T.float64, device="cuda")
    dg.dg_torque_noalloc(cfg, u, got_t, t=float(t_dev.item()))
    ref_t = T.zeros(1, dtype=T.float64, device="cuda")
    dg.dg_torque(h, u, ref_t, t=float(t_dev.item()))
    T.cuda.synchronize()
    h.close()
    return ref.item(), got.item(), ref_t.item(), got_t.item()


def test_noalloc_torque_matches_dg_torque_bitwise_on_two_calls():
    import torch as T
    assert T.cuda.is_available()
    big = W.disc_sweep(nx=200, order=5)
    small = W.disc(nx=36, order=3, q=1e-3)
    for cfg in (big, small):
        print(f"[noalloc torque] {cfg.nx}x{cfg.ny} order {cfg.order}", flush=True)
        ref, got, ref_t, got_t = _torque_pair(T, cfg, 0.0)
        print(f"  dg_torque {ref!r}, dg_torque_noalloc {got!r}", flush=True)
        assert np.isfinite(ref) and ref != 0.0
        assert got == ref
        assert got_t == ref_t


def test_noalloc_torque_fills_the_scratch_exactly():
    """The largest grid the static scratch holds: order 2 on 4096 x 4096
    elements, 128 tiles of 32 elements per row, 524288 partial sums, every
    slot of the scratch; one more row is refused before any device work.
    Then a smaller call, which must not see the partials left behind."""
    import torch as T
    assert T.cuda.is_available()
    full = W.disc(nx=4096, order=2).replace(ny=4096)
    with pytest.raises(dg.DGError) as ex:
        dg.dg_torque_noalloc(full.replace(ny=4097), None, None, stream=0)
    assert ex.value.code == dg.DG_EUNSUPPORTED
    for cfg in (full, W.disc(nx=36, order=3, q=1e-3)):
        print(f"[noalloc torque] {cfg.nx}x{cfg.ny} order {cfg.order}", flush=True)
        ref, got, ref_t, got_t = _torque_pair(T, cfg, 0.0)
        print(f"  dg_torque {ref!r}, dg_torque_noalloc {got!r}", flush=True)
        assert np.isfinite(ref) and ref != 0.0
        assert got == ref
        assert got_t == ref_t
