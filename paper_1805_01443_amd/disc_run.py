"""Long run of a planet-disc set-up with the torque on the planet recorded
every step (eq. (5)), normalised as in Sec. 5.2: gamma Gamma / Gamma_0 with
Gamma_0 = Sigma(r_p) Omega_p^2 r_p^4 q / h^2 (gamma = 1 for the locally
isothermal disc).  Workloads: the paper's adiabatic disc (Sec. 5.1) or the
locally isothermal benchmark disc; any Runge-Kutta table of Appendix A.

    python -m paper_1805_01443_amd.disc_run --nx 320 --order 5 --orbits 10 --out torque.json
    python -m paper_1805_01443_amd.disc_run --workload disc --nx 512 --rk 3 --orbits 1

Every step runs in the library's kernels; this module only drives them and
copies the torque series back in chunks.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import configs as W
from . import dg


def gamma0(cfg, sigma_p):
    """Gamma_0 = Sigma(r_p) Omega_p^2 r_p^4 q / h^2 with Omega_p^2 = GM / r_p^3."""
    om2 = cfg.gm / cfg.rp ** 3
    return sigma_p * om2 * cfg.rp ** 4 * cfg.q / cfg.h ** 2


def run(nx, order, orbits, rk=dg.RK_SSP33, chunk=2000, every=50, log=print, workload="paper_disc"):
    import torch
    if workload == "paper_disc":
        cfg = W.paper_disc(nx=nx, order=order)
        # the positivity limiter is built for SSP(3,3) only
        cfg = cfg.replace(rk=rk, positivity=1 if rk == dg.RK_SSP33 else 0)
    else:
        cfg = W.disc(nx=nx, order=order).replace(rk=rk)
    prim = W.prim_for(cfg, workload)
    h, u = dg.dg_init(cfg, prim)
    t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    tq = torch.zeros(chunk, dtype=torch.float64, device="cuda")
    if workload == "paper_disc":
        g0 = gamma0(cfg, 1.0 / (1.0 + math.exp((cfg.rp - 1.75) / (cfg.rp * cfg.h))))
        gam = cfg.gamma
    else:
        g0 = gamma0(cfg, cfg.sigma0 / math.sqrt(cfg.rp))
        gam = 1.0
    t_end = 2.0 * math.pi * orbits
    times, torques = [], []
    steps, el = 0, 0.0
    while True:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(chunk):
            dg.dg_rk_step_torque(h, u, t_dev, tq[k:k + 1], 0.0, dt_dev)
        torch.cuda.synchronize()
        el += time.perf_counter() - t0
        dg.dg_sync(h)
        steps += chunk
        t = t_dev.item()
        # sample every `every` steps; times are reconstructed from the
        # end-of-chunk time and the last dt (dt changes slowly)
        vals = tq.cpu().numpy()
        dt = dt_dev.item()
        for k in range(every - 1, chunk, every):
            times.append(t - (chunk - 1 - k) * dt)
            torques.append(float(gam * vals[k] / g0))
        log(f"[disc] {steps} steps, t = {t:.3f} ({t / (2 * math.pi):.2f} orbits), "
            f"gamma Gamma/Gamma0 = {torques[-1]:+.4f}, {el * 1e3 / steps:.3f} ms/step")
        if t >= t_end:
            break
    h.close()
    return {"workload": f"{workload}{nx}_p{order - 1}", "nx": nx, "order": order, "rk": rk, "steps": steps,
            "t_end": t, "orbits": t / (2 * math.pi), "ms_per_step": el * 1e3 / steps, "gamma0": g0,
            "dofs": nx * nx * order * order, "time": times, "gamma_torque_over_gamma0": torques}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=("paper_disc", "disc"), default="paper_disc")
    ap.add_argument("--nx", type=int, default=320)
    ap.add_argument("--order", type=int, default=5)
    ap.add_argument("--orbits", type=float, default=10.0)
    ap.add_argument("--rk", type=int, default=dg.RK_SSP33)
    ap.add_argument("--chunk", type=int, default=2000)
    ap.add_argument("--every", type=int, default=50)
    ap.add_argument("--out", default="paper_disc_torque.json")
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    res = run(a.nx, a.order, a.orbits, a.rk, a.chunk, a.every, log=lambda m: print(m, flush=True),
              workload=a.workload)
    with open(a.out, "w") as f:
        json.dump(res, f)
    tq = np.array(res["gamma_torque_over_gamma0"])
    n = len(tq)
    print(json.dumps({k: res[k] for k in ("workload", "steps", "t_end", "orbits", "ms_per_step", "gamma0")}
                     | {"torque_last_orbit_mean": float(tq[-max(n // max(int(res["orbits"]), 1), 1):].mean())}),
          flush=True)


if __name__ == "__main__":
    main()
