"""The torque of eq. (5) formed inside a step (dg_rk_step_torque): the first
stage kernel forms the per-tile partials of the torque of the state entering
the step, u^n at t^n, from the node densities and planet offsets it
evaluates, and one more block of the last stage kernel adds them up in the
order of the final-sum kernel.  Against dg_torque before dg_rk_step on a
second handle from the same initial state: the same torque bits and the same
states at every step (SSP(3,3), SSP(2,2) and a Butcher table, where the sum
runs in stage 3, stage 2 and the last of six stages); and the torque of the
initial state against the oracle's (Sec. 5.2) to 1e-12 of the sum of |terms|.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_1805_01443_amd import configs as W
from paper_1805_01443_amd import dg

pytestmark = pytest.mark.gpu
TOL = 1e-12
STEPS = 4

CASES = [
    # locally isothermal with damping zones (the benchmark's kernels); rows
    # that end inside a tile (37 = 3 * 12 + 1 elements per row at order 5)
    ("disc_p4", W.disc(nx=37, order=5, q=1e-3).replace(ny=34), "disc", 3),
    # no damping, order 3
    ("disc_p2_undamped", W.disc(nx=30, order=3, q=1e-3).replace(damping=0), "disc", 4),
    # SSP(2,2)
    ("disc_p3_ssp22", W.disc(nx=33, order=4, q=1e-3).replace(ny=20, rk=dg.RK_SSP22), "disc", 5),
    # Cash-Karp in Butcher form: its first stage runs the same kernel
    ("disc_p3_cashkarp", W.disc(nx=20, order=4, q=1e-3).replace(ny=17, rk=dg.RK_CASHKARP), "disc", 6),
    # adiabatic ring, four variables, with the modal-decay limiter and the
    # positivity limiter (passes after every stage and after the damping)
    ("ring_p3_limited", W.disc_ring(nx=32, order=4).replace(ny=29, limiter=dg.LIMITER_MODAL_DECAY,
                                                             limiter_s0=-2.4, positivity=1), "disc_ring", 7),
    # the paper's disc: positivity scaling fused into the stage kernels
    ("paper_disc_pp", W.paper_disc(nx=24, order=5, q=1e-3).replace(ny=22), "paper_disc", None),
    # order 2, 32 elements per tile
    ("disc_p1", W.disc(nx=70, order=2, q=1e-3).replace(ny=9), "disc", 8),
    # the deviation form: the two calls one after the other
    ("disc_mixed_p2", W.disc_mixed(nx=24, order=3, seed=1, q=1e-3), "disc", 1),
]


def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU test needs a ROCm device"
    return T


@pytest.mark.parametrize("name,cfg,kind,seed", CASES, ids=[c[0] for c in CASES])
def test_torque_in_the_step_equals_torque_then_step(name, cfg, kind, seed):
    T = torch()
    oc = O.cfg(dataclasses.asdict(cfg))
    x, y = O.nodes(oc)
    prim = W.prim_for(cfg, kind, seed=seed, x=x, y=y)
    print(f"[torque in step] {name}", flush=True)
    ha, ua = dg.dg_init(cfg, prim)
    hb, ub = dg.dg_init(cfg, prim)
    ta = T.zeros(1, dtype=T.float64, device="cuda")
    tb = T.zeros(1, dtype=T.float64, device="cuda")
    qa = T.zeros(STEPS, dtype=T.float64, device="cuda")
    qb = T.zeros(STEPS, dtype=T.float64, device="cuda")
    full0 = T.empty_like(ua)
    dg.dg_full_state(ha, ua, full0)
    dg.dg_sync(ha)
    u0 = dg.to_planes(cfg, full0.detach().cpu().numpy())
    for k in range(STEPS):
        dg.dg_rk_step_torque(ha, ua, ta, qa[k:k + 1])
        dg.dg_torque(hb, ub, qb[k:k + 1], t_dev=tb)
        dg.dg_rk_step(hb, ub, tb, 0.0, None)
    dg.dg_sync(ha)
    dg.dg_sync(hb)
    print(f"  torques {qa.cpu().numpy()}, equal states {T.equal(ua, ub)}, equal torques {T.equal(qa, qb)}",
          flush=True)
    assert ta.item() == tb.item()
    assert T.equal(ua, ub)
    assert T.equal(qa, qb)
    assert np.isfinite(qa.cpu().numpy()).all()
    # the torque of the initial (full) state at t = 0 against the oracle's
    g, sabs = O.torque(oc, 0.0, u0)
    print(f"  t = 0: gpu {qa[0].item():.17e}, oracle {g:.17e}, sum|terms| {sabs:.3e}", flush=True)
    assert abs(qa[0].item() - g) <= TOL * sabs
    for h in (ha, hb):
        h.close()


def test_torque_sum_bits_with_many_tiles():
    """The benchmark's 512 x 512 order-5 disc: 22016 tile partials, so the
    in-stage sum runs the eight-load trips of the final-sum kernel's threads
    as well as their remainders; two steps, the torque bits and the states
    against dg_torque then dg_rk_step on a second handle."""
    T = torch()
    cfg = W.disc(nx=512, order=5)
    oc = O.cfg(dataclasses.asdict(cfg))
    x, y = O.nodes(oc)
    prim = W.prim_for(cfg, "disc", seed=0, x=x, y=y)
    print("[torque in step] disc 512x512 order 5, 22016 partials", flush=True)
    ha, ua = dg.dg_init(cfg, prim)
    hb, ub = dg.dg_init(cfg, prim)
    ta = T.zeros(1, dtype=T.float64, device="cuda")
    tb = T.zeros(1, dtype=T.float64, device="cuda")
    qa = T.zeros(2, dtype=T.float64, device="cuda")
    qb = T.zeros(2, dtype=T.float64, device="cuda")
    for k in range(2):
        dg.dg_rk_step_torque(ha, ua, ta, qa[k:k + 1])
        dg.dg_torque(hb, ub, qb[k:k + 1], t_dev=tb)
        dg.dg_rk_step(hb, ub, tb, 0.0, None)
    dg.dg_sync(ha)
    dg.dg_sync(hb)
    print(f"  torques {qa.cpu().numpy()} / {qb.cpu().numpy()}", flush=True)
    assert T.equal(qa, qb)
    assert T.equal(ua, ub)
    assert ta.item() == tb.item()
    for h in (ha, hb):
        h.close()
