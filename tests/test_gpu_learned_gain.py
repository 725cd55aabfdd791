"""What the trained troubled-cell network gains, on the GPU.

The committed network (paper_1805_01443_amd/mlp_ring_p3.json, trained by
``python -m paper_1805_01443_amd.learned`` on seeds 0-5 of the ring workload at
256^2, order 4, threshold chosen on seed 6) runs the held-out seed 7 for 24000
steps (t = 3.25, past the steepening of the ring into shocks), next to the same
run without a troubled-cell limiter (positivity limiter only) and with minmod
on every element.  The plain modal-decay indicator is the referee: at the end it
flags the elements that still carry oscillations.

Gains measured here: (1) against no troubled-cell limiter, the residual
oscillation left at the end drops from ~0.3 % of the elements to the plain
pipeline's level; (2) against limiting every element, the density stays within
a few per cent of the plain pipeline's instead of ~20 %, and the step is ~1.8x
cheaper; (3) the network's flags on its own run miss at most 1 % of the plain
indicator's."""
import numpy as np
import pytest

from paper_1805_01443_amd import configs as W
from paper_1805_01443_amd import dg
from paper_1805_01443_amd import learned

pytestmark = pytest.mark.gpu

NX, STEPS, SEED, EVERY = 256, 24000, 7, 400


def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


def run(limiter, s0, theta, params, capture=False):
    """final state, end-of-run sensor share, ms/step, closed-loop (tp, fn, fp)"""
    import time
    T = torch()
    cfg = learned.ring_config(NX, limiter=limiter, theta=theta, s0=s0)
    prim = W.prim_for(cfg, "disc_ring", seed=SEED)
    h, u = dg.dg_init(cfg, prim)
    if limiter == dg.LIMITER_LEARNED:
        dg.dg_mlp_params(h, set_params=params)
    E = cfg.n_elem
    lab = T.zeros(E, dtype=T.uint8, device="cuda")
    mf = T.zeros(E, dtype=T.uint8, device="cuda")
    t_dev = T.zeros(1, dtype=T.float64, device="cuda")
    tp = fn = fp = 0
    T.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(STEPS):
        cap = capture and (k + 1) % EVERY == 0
        if cap:
            dg.dg_capture(h, flags=lab, mlp_flags=mf)
        dg.dg_rk_step(h, u, t_dev, 0.0, None)
        if cap:
            y, m = lab.bool(), mf.bool()
            tp += int((y & m).sum())
            fn += int((y & ~m).sum())
            fp += int((~y & m).sum())
    dg.dg_sync(h)
    ms = (time.perf_counter() - t0) * 1e3 / STEPS
    h.close()
    # the referee: the plain sensor on the final state
    hq, _ = dg.dg_init(learned.ring_config(NX, s0=s0), prim)
    dg.dg_troubled(hq, u, apply=False, flags=lab)
    dg.dg_sync(hq)
    hq.close()
    return u, float(lab.float().mean().item()), ms, (tp, fn, fp)


def test_trained_network_gains_over_no_indicator_and_over_limiting_everywhere():
    lp = learned.load_params()
    assert lp is not None, "the trained network file is missing"
    s0, theta = lp["s0"], lp["theta"]
    u_p, osc_p, ms_p, _ = run(dg.LIMITER_MODAL_DECAY, s0, theta, None)
    u_l, osc_l, ms_l, (tp, fn, fp) = run(dg.LIMITER_LEARNED, s0, theta, lp["params"], capture=True)
    u_n, osc_n, ms_n, _ = run(dg.LIMITER_NONE, s0, theta, None)
    u_a, osc_a, ms_a, _ = run(dg.LIMITER_MODAL_DECAY, -1e300, theta, None)
    cfg = learned.ring_config(NX)
    rho = {k: dg.to_planes(cfg, v)[0] for k, v in (("plain", u_p), ("learned", u_l), ("none", u_n), ("all", u_a))}
    dif = {k: float(((rho[k] - rho["plain"]) ** 2).sum().sqrt() / (rho["plain"] ** 2).sum().sqrt())
           for k in ("learned", "none", "all")}
    miss = fn / max(tp + fn, 1)
    print(f"[gain] residual oscillation (sensor share at the end): plain {osc_p:.5%}, learned {osc_l:.5%}, "
          f"none {osc_n:.5%}, all {osc_a:.5%}", flush=True)
    print(f"[gain] density rel L2 vs plain: {dif}; ms/step plain {ms_p:.3f} learned {ms_l:.3f} "
          f"none {ms_n:.3f} all {ms_a:.3f}; closed-loop miss {miss:.4f} ({tp + fn} positives, {fp} false alarms)",
          flush=True)
    for v in (u_p, u_l, u_n, u_a):
        assert bool(torch().isfinite(v).all())
    # (1) oscillation control: no worse than the plain pipeline's, far below none
    assert osc_n > 0.0
    assert osc_l <= osc_p + 0.1 * osc_n
    # (2) accuracy and cost against limiting every element
    assert dif["learned"] < 0.25 * dif["all"]
    assert ms_l < ms_a
    # (3) the referee's miss rate on the network's own run
    assert miss <= 0.01
