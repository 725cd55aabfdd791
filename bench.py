"""Throughput of the DG hot path on one MI355X.

Workload (default): the planet-disc problem at order 5 (P4, 5x5 Gauss points),
512 x 512 elements on [-2.5, 2.5]^2, locally isothermal h = 0.05, FP64, planet
q = 1e-5 on a fixed orbit, damping zones r < 0.4 and r > 2.3; each step is one
SSP-RK3 step (device CFL reduction, three fused stage kernels, damping) plus
the planet torque.  Inputs are synthetic (seeded formulas), resident in HBM
before timing starts.

Prints one JSON line: DOF-stage updates/s (DOF = nx ny m^2, three stages per
step), the roofline position of the fused stage kernel (HIP events around each
stage launch on the library's stream) and the oracle's throughput on the host
cores for a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector, published


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--order", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison run")
    ap.add_argument("--no-limited", action="store_true", help="skip the modal vs learned limiter comparison")
    ap.add_argument("--no-shard", action="store_true", help="skip the one-GPU-share (1024 x 128 strip) run")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 1024^2 order sweep")
    ap.add_argument("--ring-nx", type=int, default=1024)
    ap.add_argument("--ring-steps", type=int, default=200)
    ap.add_argument("--mixed-nx", type=int, default=1024)
    ap.add_argument("--mixed-steps", type=int, default=2000)
    ap.add_argument("--sweep-steps", type=int, default=20)
    ap.add_argument("--cpu-child", nargs=3, metavar=("NX", "ORDER", "STEPS"), default=None,
                    help=argparse.SUPPRESS)
    ap.add_argument("--seed", type=int, default=None,
                    help="seeded disc: Sigma0 and 1e-4 density noise from the seed, q = 3e-5")
    ap.add_argument("--sweep", action="store_true",
                    help="orders 2..5 at --nx (FP64): per-order throughput and roofline fraction")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device copy of known size (HBM counter calibration)")
    return ap.parse_args()


def calibrate_copy():
    """A plain streaming kernel over 2 GiB, five times: b = a * 1 reads 2 GiB and
    writes 2 GiB with ordinary vector loads and stores (torch's elementwise
    kernel; the runtime's blit copy uses another load path).  Its PMC byte
    counters, divided by 2 GiB, give the counter-to-HBM-bytes factors."""
    import torch
    n = 1 << 28  # doubles: 2 GiB
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    print(json.dumps({"copy_bytes_read_per_launch": n * 8, "copy_bytes_written_per_launch": n * 8,
                      "launches": 5, "GBps_read_plus_write": 2 * 5 * n * 8 / el / 1e9}), flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for fn in ("dg_kernels.hip", "dg_internal.h", "dg_pp.h", "dg_mlp.h"):
        with open(os.path.join(ROOT, "paper_1805_01443_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per stage launch from committed rocprofv3 PMC counters, if they
    were taken on the current kernel source (else None)."""
    fn = os.path.join(ROOT, "profiles", "k_stage_traffic.json")
    if not os.path.exists(fn):
        return None
    with open(fn) as f:
        d = json.load(f)
    rec = d.get(workload)
    if not rec or rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def flop_per_element_stage(n, nvar):
    """Count model of one fused stage per element (sum-factorised contractions,
    1 MAC = 2 FLOP, divide and sqrt as 1 FLOP): volume interpolation 2n^3,
    traces 8n^2, projection 5n^3 and lift 8n^2 MAC per variable, minus n^3 for
    the source-free density equation; about 45 pointwise FLOP per volume node
    and per edge point pair; 4 FLOP per DOF for the stage combination."""
    mac = nvar * (7 * n ** 3 + 16 * n ** 2) - n ** 3
    return 2 * mac + 45 * n * n + 90 * n + 4 * nvar * n * n


def fp64_model(cfg, avg_launch_s):
    f = flop_per_element_stage(cfg.order, cfg.nvar) * cfg.n_elem
    ach = f / avg_launch_s / 1e12
    return {"flop_per_launch": f, "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / FP64_PEAK_TFLOPS, "note": "FLOP from the count model, not from counters"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(nx, order, steps):
    """The oracle as it stands on the disc at nx^2 and this order: `steps`
    full steps (CFL dt, three SSP-RK3 stages, damping) plus the torque after
    each, plain C FP64 with OpenMP over the elements; DOF-stage updates per
    second and the seconds taken."""
    import oracle as O
    from paper_1805_01443_amd import configs as W
    O.build()
    cfg = W.disc(nx=nx, order=order)
    oc = O.cfg(dataclasses.asdict(cfg))
    # the oracle's own node coordinates: this leg loads no HIP library
    x, y = O.nodes(oc)
    prim = W.prim_for(cfg, "disc", x=x, y=y)
    u0 = O.project(oc, prim)
    t0 = time.perf_counter()
    u, t = u0, 0.0
    for _ in range(steps):
        u, dt = O.step(oc, u, t, 0.0, u0=u0)
        t += dt
        O.torque(oc, t, u)
    el = time.perf_counter() - t0
    return cfg.nx * cfg.ny * order ** 2 * 3 * steps / el, el


def cpu_baseline(nx, order):
    """The oracle on the host cores, before the GPU is touched: all threads on
    six steps of the benchmark disc (about 10 s on 16 threads), and one thread
    (a child process with OMP_NUM_THREADS=1) on two steps of the same disc at
    128^2 (same work per element; the rate is per DOF-stage)."""
    import subprocess
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    steps = 6
    v, el = oracle_rate(nx, order, steps)
    out = {"value": v, "unit": "DOF-stage/s", "cores": threads, "kind": "oracle",
           "sample": f"{steps} full steps (CFL dt, 3 SSP-RK3 stages, damping) + torque each, of the same "
                     f"{nx}x{nx} order-{order} disc, plain C FP64, OpenMP over elements ({threads} threads), "
                     f"{el:.1f} s",
           "cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-child", "128", str(order), "2"],
                       env=env, capture_output=True, text=True, timeout=600)
    if r.returncode == 0 and r.stdout.strip():
        one = json.loads(r.stdout.strip().splitlines()[-1])
        out["one_thread"] = {"value": one["value"], "unit": "DOF-stage/s", "cores": 1,
                             "sample": f"2 full steps + torque of the same disc at 128x128, order {order}, "
                                       f"OMP_NUM_THREADS=1, {one['seconds']:.1f} s"}
        out["threads_speedup"] = v / one["value"]
    else:
        out["one_thread"] = {"error": (r.stderr or "")[-400:]}
    return out


def run_disc(cfg, prim, steps, warmup, profile):
    """Warm up, then time `steps` SSP-RK3 steps, each with the torque of the
    state entering it (dg_rk_step_torque); returns timings, the torque series
    of the timed steps and the final full state (device)."""
    import torch

    from paper_1805_01443_amd import dg
    h, u = dg.dg_init(cfg, prim)
    t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    torques = torch.zeros(steps + warmup, dtype=torch.float64, device="cuda")
    for k in range(warmup):
        dg.dg_rk_step_torque(h, u, t_dev, torques[k:k + 1])
    dg.dg_sync(h)
    if profile:
        dg.dg_profile_begin(h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        dg.dg_rk_step_torque(h, u, t_dev, torques[warmup + k:warmup + k + 1])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage_ms, launches = dg.dg_profile_end(h) if profile else (0.0, 0)
    dg.dg_sync(h)
    full = torch.empty_like(u)
    dg.dg_full_state(h, u, full)
    torch.cuda.synchronize()
    res = {"elapsed": t1 - t0, "stage_ms": stage_ms, "launches": launches, "torques": torques[warmup:].clone(),
           "full": full, "t_end": float(t_dev.item())}
    h.close()
    return res


NCAP = 10  # captured steps before the timed ones (limited forms)


def run_limited(a):
    """The ring workload (order 4, adiabatic, 1024^2 by default) with the plain
    modal-decay indicator and with the learned indicator, both followed by
    minmod and the positivity limiter: step rate of each and the density
    difference after the timed steps, on two states.
      smooth: the ring from t = 0.  At 1024^2 the plain sensor flags no element
              for t < 1 (31 500 steps): this times the indicators' cost alone.
      jump:   the same ring with density and pressure doubled inside r = 1.6,
              an edge through the middle of elements that both pipelines must
              limit from the first step.
    Each run first takes NCAP untimed steps that capture the plain indicator's
    flags and labels and the network's flags on the run's own last-stage states
    (the learned run's miss and false-alarm rates against the labels), then the
    timed steps."""
    import numpy as np
    import torch

    from paper_1805_01443_amd import configs as W
    from paper_1805_01443_amd import dg, learned
    lp = learned.load_params()
    if lp is None:
        params, theta, s0, src = learned.init_params(0), 0.5, learned.default_s0(4), "untrained (He init)"
    else:
        params, theta, s0, src = lp["params"], lp["theta"], lp["s0"], "trained, " + learned.PARAMS_FILE.split(os.sep)[-1]
    res = {"workload": f"ring{a.ring_nx}_p3_adiabatic_fp64_seed0", "network": src, "theta": theta, "s0": s0}
    for state in ("smooth", "jump"):
        steps = a.ring_steps if state == "smooth" else max(a.ring_steps // 2, 1)
        out, rho = {}, {}
        for name, lim in (("modal", dg.LIMITER_MODAL_DECAY), ("learned", dg.LIMITER_LEARNED)):
            cfg = learned.ring_config(a.ring_nx, limiter=lim, theta=theta, s0=s0)
            prim = W.prim_for(cfg, "disc_ring", seed=0)
            if state == "jump":
                x, y = dg.dg_get_nodes(cfg)
                inside = np.sqrt(x ** 2 + y ** 2) < 1.6
                prim[0] = np.where(inside, 2.0 * prim[0], prim[0])
                prim[3] = np.where(inside, 2.0 * prim[3], prim[3])
            h, u = dg.dg_init(cfg, prim)
            if lim == dg.LIMITER_LEARNED:
                dg.dg_mlp_params(h, set_params=params)
            t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
            # the first NCAP steps (untimed): the plain indicator's flags and
            # labels (flagged and altered by minmod) on each step's last-stage
            # state before limiting, and with the learned limiter the
            # network's flags on the same states
            E = cfg.n_elem
            fl = torch.zeros(E, dtype=torch.uint8, device="cuda")
            lab = torch.zeros(E, dtype=torch.uint8, device="cuda")
            mf = torch.zeros(E, dtype=torch.uint8, device="cuda")
            conf = {"labels": 0, "flagged": 0, "mlp_flags": 0, "miss": 0, "false_alarm": 0, "elements": 0}
            for _ in range(NCAP):
                dg.dg_capture(h, flags=fl, labels=lab, mlp_flags=mf if lim == dg.LIMITER_LEARNED else None)
                dg.dg_rk_step(h, u, t_dev, 0.0, None)
                torch.cuda.synchronize()
                conf["labels"] += int(lab.sum().item())
                conf["flagged"] += int(fl.sum().item())
                conf["elements"] += E
                if lim == dg.LIMITER_LEARNED:
                    conf["mlp_flags"] += int(mf.sum().item())
                    conf["miss"] += int(((lab == 1) & (mf == 0)).sum().item())
                    conf["false_alarm"] += int(((lab == 0) & (mf == 1)).sum().item())
            dg.dg_sync(h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                dg.dg_rk_step(h, u, t_dev, 0.0, None)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            dg.dg_sync(h)
            dofs = cfg.n_elem * cfg.order ** 2
            rec = {"value": dofs * 3 * steps / el, "unit": "DOF-stage/s", "ms_per_step": el * 1e3 / steps,
                   "plain_flagged_per_step": conf["flagged"] / NCAP, "plain_labels_per_step": conf["labels"] / NCAP}
            if lim == dg.LIMITER_LEARNED:
                rec["mlp_flagged_per_step"] = conf["mlp_flags"] / NCAP
                rec["miss_rate"] = conf["miss"] / conf["labels"] if conf["labels"] else None
                neg = conf["elements"] - conf["labels"]
                rec["false_alarm_rate"] = conf["false_alarm"] / neg if neg else None
            rho[name] = dg.to_planes(cfg, u)[0].clone()
            out[name] = rec
            h.close()
        out["learned_speedup_vs_modal"] = out["modal"]["ms_per_step"] / out["learned"]["ms_per_step"]
        out["density_rel_L2_diff"] = float(((rho["learned"] - rho["modal"]) ** 2).sum().sqrt()
                                           / (rho["modal"] ** 2).sum().sqrt())
        out["timed_steps"] = steps
        out["captured_steps_before_timing"] = NCAP
        res[state] = out
    return res


def run_shard(a, order):
    """One GPU's share of the 1024^2 disc split into eight strips of 1024 x 128
    elements: the strip y in [0, 0.625] (the planet's orbit crosses it), run
    alone with fixed-initial edges standing in for the neighbours' halo.  Same
    kernels, same element size as the 1024^2 disc."""
    from paper_1805_01443_amd import configs as W
    base = W.disc(nx=1024, order=order)
    cfg = base.replace(ny=128, y0=0.0, y1=(base.y1 - base.y0) / 8)
    r = run_disc(cfg, W.prim_for(cfg, "disc"), a.steps, a.warmup, profile=True)
    state_bytes = cfg.nvar * order ** 2 * cfg.n_elem * 8
    avg = r["stage_ms"] / 1e3 / max(r["launches"], 1)
    ach = state_bytes * 8.0 / 3.0 / avg / 1e9
    dofs = cfg.n_elem * order ** 2
    return {"workload": f"disc1024_strip128_p{order - 1}_fp64", "nx": cfg.nx, "ny": cfg.ny,
            "y_range": [cfg.y0, cfg.y1], "dofs": dofs,
            "value": dofs * 3 * a.steps / r["elapsed"], "unit": "DOF-stage/s",
            "ms_per_step": r["elapsed"] * 1e3 / a.steps, "stage_kernel_us": avg * 1e6,
            "hbm_GBps_alg": ach, "hbm_frac": ach / HBM_PEAK_GBPS,
            "note": "one of eight 1024x128 strips of the 1024^2 disc on one GPU; no halo exchange "
                    "(fixed-initial strip edges)"}


def disc_workload(a, order):
    from paper_1805_01443_amd import configs as W
    if a.seed is None:
        cfg = W.disc(nx=a.nx, order=order)
        return cfg, W.prim_for(cfg, "disc"), 1.0
    cfg = W.disc_sweep(nx=a.nx, order=order)
    return cfg, W.prim_for(cfg, "disc", seed=a.seed), W.sigma0_of(a.seed)


def sweep(a, nx, steps, seed):
    """FP64 throughput per order on the seeded disc at nx^2 (orders 2..5)."""
    from paper_1805_01443_amd import configs as W
    rows = []
    for order in (2, 3, 4, 5):
        cfg = W.disc_sweep(nx=nx, order=order)
        r = run_disc(cfg, W.prim_for(cfg, "disc", seed=seed), steps, a.warmup, profile=True)
        state_bytes = cfg.nvar * order ** 2 * cfg.n_elem * 8
        avg = r["stage_ms"] / 1e3 / max(r["launches"], 1)
        ach = state_bytes * 8.0 / 3.0 / avg / 1e9
        rows.append({"order": order, "p": order - 1, "dofs": cfg.n_elem * order ** 2,
                     "dof_stage_per_s": cfg.n_elem * order ** 2 * 3 * steps / r["elapsed"],
                     "ms_per_step": r["elapsed"] * 1e3 / steps, "stage_kernel_us": avg * 1e6,
                     "hbm_GBps_alg": ach, "hbm_frac": ach / HBM_PEAK_GBPS,
                     "fp64_model": fp64_model(cfg, avg)})
        del r
    return {"workload": f"disc{nx}_seed{seed}_orders2to5_fp64", "steps": steps, "rows": rows}


def run_mixed(a):
    """The mixed-precision deviation form against the FP64 path on the seeded
    1024^2 order-5 disc (q = 3e-5), --mixed-steps steps each with the torque
    every step: speeds, the torque series' largest difference relative to its
    largest value, and the relative L2 difference of the final density modes
    (Parseval: the orthonormal modes' L2 norm is the density's L2 norm over
    |K|).  The deviation's own error: the final difference relative to the
    largest deviation of the FP64 state from the equilibrium."""
    from paper_1805_01443_amd import configs as W
    from paper_1805_01443_amd import dg
    cfg = W.disc_sweep(nx=a.mixed_nx, order=5)
    prim = W.prim_for(cfg, "disc", seed=0)
    r64 = run_disc(cfg, prim, a.mixed_steps, a.warmup, profile=True)
    cm = W.disc_mixed(nx=a.mixed_nx, order=5, seed=0)
    rm = run_disc(cm, prim, a.mixed_steps, a.warmup, profile=True)
    g64, gm = r64["torques"], rm["torques"]
    rho64 = dg.to_planes(cfg, r64["full"])[0]
    rhom = dg.to_planes(cm, rm["full"])[0]
    dens_l2 = float(((rhom - rho64) ** 2).sum().sqrt() / (rho64 ** 2).sum().sqrt())
    tq_err = float((gm - g64).abs().max() / g64.abs().max())
    dofs = W.dofs(cfg)
    return {"workload": f"disc{a.mixed_nx}_p4_seed0_mixed_vs_fp64", "steps": a.mixed_steps,
            "fp64": {"value": dofs * 3 * a.mixed_steps / r64["elapsed"], "unit": "DOF-stage/s",
                     "ms_per_step": r64["elapsed"] * 1e3 / a.mixed_steps,
                     "stage_kernel_us": r64["stage_ms"] * 1e3 / max(r64["launches"], 1)},
            "mixed": {"value": dofs * 3 * a.mixed_steps / rm["elapsed"], "unit": "DOF-stage/s",
                      "ms_per_step": rm["elapsed"] * 1e3 / a.mixed_steps,
                      "stage_kernel_us": rm["stage_ms"] * 1e3 / max(rm["launches"], 1)},
            "speedup_vs_fp64": r64["elapsed"] / rm["elapsed"],
            "torque_series_rel_err_vs_fp64": tq_err, "density_rel_L2_err_vs_fp64": dens_l2,
            "t_end": rm["t_end"],
            "note": "FP32 deviation terms linearised about the projected equilibrium (its volume-node "
                    "values and tabulated edge traces); FP64 L(u_eq), state, stage combination, "
                    "damping, dt and torque"}


def progress(msg):
    """One line per finished leg on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    a = parse()
    if a.calibrate_copy:
        calibrate_copy()
        return
    if a.cpu_child:
        nx, order, steps = (int(v) for v in a.cpu_child)
        v, el = oracle_rate(nx, order, steps)
        print(json.dumps({"value": v, "seconds": el}), flush=True)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU only; sharding over several GPUs is a "
                                   "design, not an implemented path", "n_gpus": a.gpus}))
        sys.exit(2)
    # torch first (its HIP runtime is the one the library then binds to), then
    # the oracle's timings, before the GPU is initialised
    import torch

    cpu = None if a.no_cpu_baseline else cpu_baseline(a.nx, a.order)
    if cpu is not None:
        progress("oracle baseline done")

    from paper_1805_01443_amd import configs as W

    torch.cuda.set_device(0)
    if a.sweep:
        print(json.dumps(sweep(a, a.nx, a.steps, 0 if a.seed is None else a.seed)), flush=True)
        return
    cfg, prim, sigma0 = disc_workload(a, a.order)
    r64 = run_disc(cfg, prim, a.steps, a.warmup, profile=True)
    progress(f"timed steps done: {cfg.nx}^2 order {cfg.order}")
    el = r64["elapsed"]
    dofs = W.dofs(cfg)
    value = dofs * 3 * a.steps / el
    state_bytes = cfg.nvar * cfg.order ** 2 * cfg.n_elem * 8
    # algorithmic bytes of the three stage launches of a step: read u^(i),
    # read u^n (stages 2 and 3), write u^(i+1): 2 + 3 + 3 state passes
    alg_bytes_per_launch = state_bytes * 8.0 / 3.0
    avg_launch_s = r64["stage_ms"] / 1e3 / max(r64["launches"], 1)
    achieved = alg_bytes_per_launch / avg_launch_s / 1e9
    workload = f"disc{cfg.nx}_p{cfg.order - 1}_fp64" + ("" if a.seed is None else f"_seed{a.seed}")
    traffic = measured_traffic(workload)
    out = {
        "metric": "DOF-stage updates/s (p=4, FP64) at parity 1e-12 vs FP64 oracle",
        "value": value,
        "unit": "DOF-stage/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": el * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "nx": cfg.nx, "ny": cfg.ny, "order": cfg.order,
                   "closure": "locally_isothermal", "h": cfg.h, "q": cfg.q, "eps": cfg.eps,
                   "dofs": dofs, "stages_per_step": 3, "torque_every_step": True,
                   "torque_entering_last_step": float(r64["torques"][-1].item()), "t_end": r64["t_end"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": "k_stage_c (fused RK stage, N lanes per element)", "avg_launch_us": avg_launch_s * 1e6,
                     "alg_bytes_per_launch": alg_bytes_per_launch},
        "fp64_model": fp64_model(cfg, avg_launch_s),
    }
    del r64
    forms = {}
    if not a.no_sweep:
        forms["sweep1024"] = sweep(a, 1024, a.sweep_steps, 0)
        progress("order sweep done")
    if not a.no_mixed:
        forms["mixed"] = run_mixed(a)
        progress("mixed form done")
    if not a.no_shard:
        forms["shard"] = run_shard(a, cfg.order)
        progress("strip done")
    if not a.no_limited:
        forms["limited"] = run_limited(a)
        progress("limited forms done")
    if forms:
        out["forms"] = forms
    if cpu is not None:
        out["cpu_baseline"] = cpu
        out["cpu_baseline"]["gpu_over_cpu"] = value / cpu["value"]
        if "value" in cpu.get("one_thread", {}):
            out["cpu_baseline"]["gpu_over_one_thread"] = value / cpu["one_thread"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
