"""Learned troubled-cell indicator: data, training and evaluation on the GPU.

Workload: the adiabatic disc at order 4 (P3) with an over-pressure ring that
steepens into shocks (``configs.disc_ring``).  The plain pipeline (modal-decay
sensor + minmod) is run with seeded initial data; every ``every`` steps the
state of the last stage before limiting is captured (``dg_capture``): its bf16
features and the plain indicator's flags, which are the labels.  All positives
and as many random negatives are kept.  The MLP is trained with the
library's own forward/backward/Adam kernels (``dg_mlp_train_step``), the flag
threshold is chosen on a validation seed for a miss rate <= 1 %, and on a test
seed the learned limiter runs the same workload while its flags are compared
with the plain labels on the same states (miss and false-alarm rates); the
torque and density of the two runs and their step times are compared too.

Index selection and batching use PyTorch tensor indexing (data plumbing); all
method arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import configs as W
from . import dg


def default_s0(order: int) -> float:
    """Threshold of the modal-decay sensor: -4 log10(p + 1)."""
    return -4.0 * math.log10(order)


def ring_config(nx, order=4, limiter=dg.LIMITER_MODAL_DECAY, theta=0.5, s0=None):
    return W.disc_ring(nx=nx, order=order).replace(
        limiter=limiter, limiter_s0=default_s0(order) if s0 is None else s0, mlp_theta=theta)


PARAMS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mlp_ring_p3.json")


def load_params(path=PARAMS_FILE):
    """Trained parameters, flag threshold and sensor threshold from a JSON file
    written by ``main`` (``--params-out``); None if there is none."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    p = np.asarray(d["params"], dtype=np.float32)
    if p.size != dg.MLP_NPARAM:
        raise ValueError(f"{path}: {p.size} parameters, expected {dg.MLP_NPARAM}")
    return {"params": p, "theta": float(d["theta"]), "s0": float(d["s0"]), "meta": d.get("meta", {})}


def save_params(path, params, theta, s0, meta):
    with open(path, "w") as f:
        json.dump({"params": [float(v) for v in params], "theta": theta, "s0": s0, "meta": meta}, f)


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    p = np.zeros(dg.MLP_NPARAM, dtype=np.float32)
    p[:2048] = rng.normal(0, math.sqrt(2.0 / 64), 2048)
    p[2080:3104] = rng.normal(0, math.sqrt(2.0 / 32), 1024)
    p[3136:3168] = rng.normal(0, math.sqrt(1.0 / 32), 32)
    return p


def collect(seed, nx, steps, every, cap, torch, s0=None, log=print):
    """Run the plain pipeline; returns (features int16 [N, 64], labels float [N],
    per-capture positive counts, steps run).  A run whose state turns
    non-finite (the plain limiter does not preserve positivity) stops there and
    keeps the samples captured before."""
    cfg = ring_config(nx, s0=s0)
    prim = W.prim_for(cfg, "disc_ring", seed=seed)
    h, u = dg.dg_init(cfg, prim)
    E = cfg.n_elem
    feat = torch.zeros((E, 64), dtype=torch.int16, device="cuda")
    lab = torch.zeros(E, dtype=torch.uint8, device="cuda")
    t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(1000 + seed)
    xs, ys, npos = [], [], []
    done = 0
    for k in range(steps):
        cap_now = (k + 1) % every == 0
        if cap_now:
            dg.dg_capture(h, feat=feat, flags=lab)
        dg.dg_rk_step(h, u, t_dev, 0.0, None)
        if cap_now:
            try:
                dg.dg_sync(h)
            except dg.DGError as err:
                log(f"[collect] seed {seed}: stopped at step {k + 1} ({err})")
                break
            pos = torch.nonzero(lab).flatten()
            neg = torch.nonzero(lab == 0).flatten()
            npos.append(int(pos.numel()))
            if pos.numel() > cap:
                pos = pos[torch.randperm(pos.numel(), device="cuda", generator=g)[:cap]]
            nneg = min(max(int(pos.numel()), 64), neg.numel())
            neg = neg[torch.randperm(neg.numel(), device="cuda", generator=g)[:nneg]]
            idx = torch.cat([pos, neg])
            xs.append(feat[idx].clone())
            ys.append(torch.cat([torch.ones(pos.numel(), device="cuda"), torch.zeros(neg.numel(), device="cuda")]))
        done = k + 1
    try:
        dg.dg_sync(h)
    except dg.DGError:
        pass
    log(f"[collect] seed {seed}: {done} steps, t_end {t_dev.item():.4f}, positives per capture "
        f"{npos[:3]}...{npos[-3:]} (total {sum(npos)})")
    h.close()
    return torch.cat(xs), torch.cat(ys), npos, done


def train(h, X, Y, epochs, batch, lr, seed, torch, log=print):
    n = X.shape[0]
    npos = float(Y.sum().item())
    pos_weight = (n - npos) / max(npos, 1.0)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=g)
        tot, nb = 0.0, 0
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            xb = X[idx].contiguous()
            yb = Y[idx].contiguous()
            dg.dg_mlp_train_step(h, xb, yb, xb.shape[0], pos_weight=pos_weight, lr=lr, loss=loss)
            tot += loss.item()
            nb += 1
        hist.append(tot / max(nb, 1))
        log(f"[train] epoch {ep}: mean loss {hist[-1]:.5f}")
    return hist, pos_weight


def rates(prob, y, theta):
    f = prob > theta
    pos = y > 0.5
    miss = float((~f & pos).sum()) / max(int(pos.sum()), 1)
    fa = float((f & ~pos).sum()) / max(int((~pos).sum()), 1)
    return miss, fa


def evaluate_run(seed, nx, steps, every, params, theta, torch, s0=None, log=print):
    """Plain and learned limiter on the same seeded workload: step times,
    torque series and final density difference, and the learned flags vs the
    plain labels on the learned run's captured states.  Runs stop at the first
    non-finite state; the comparison covers the steps both completed."""
    out = {}
    res = {}
    for name, lim in (("plain", dg.LIMITER_MODAL_DECAY), ("learned", dg.LIMITER_LEARNED)):
        cfg = ring_config(nx, limiter=lim, theta=theta, s0=s0)
        prim = W.prim_for(cfg, "disc_ring", seed=seed)
        h, u = dg.dg_init(cfg, prim)
        if lim == dg.LIMITER_LEARNED:
            dg.dg_mlp_params(h, set_params=params)
        E = cfg.n_elem
        lab = torch.zeros(E, dtype=torch.uint8, device="cuda")
        mf = torch.zeros(E, dtype=torch.uint8, device="cuda")
        t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
        tq = torch.zeros(steps, dtype=torch.float64, device="cuda")
        tp = fp = fn = tn = 0
        # timed run in chunks (no captures; a finiteness check between chunks)
        chunk = max(every, 1)
        done, el = 0, 0.0
        while done < steps:
            n = min(chunk, steps - done)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(done, done + n):
                dg.dg_rk_step(h, u, t_dev, 0.0, None)
                dg.dg_torque(h, u, tq[k:k + 1], t_dev=t_dev)
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
            try:
                dg.dg_sync(h)
            except dg.DGError:
                log(f"[eval] {name}: non-finite state after step {done + n}")
                break
            done += n
        res[name] = {"u": u.clone(), "tq": tq.clone(), "elapsed": el, "steps": done}
        if lim == dg.LIMITER_LEARNED:
            h2, u2 = dg.dg_init(cfg, prim)
            dg.dg_mlp_params(h2, set_params=params)
            t2 = torch.zeros(1, dtype=torch.float64, device="cuda")
            ncap = 0
            for k in range(done):
                cap = (k + 1) % every == 0
                if cap:
                    dg.dg_capture(h2, flags=lab, mlp_flags=mf)
                dg.dg_rk_step(h2, u2, t2, 0.0, None)
                if cap:
                    y = lab.bool()
                    m = mf.bool()
                    tp += int((y & m).sum())
                    fn += int((y & ~m).sum())
                    fp += int((~y & m).sum())
                    tn += int((~y & ~m).sum())
                    ncap += 1
            h2.close()
            out["captured_states"] = ncap
            out["miss_rate"] = fn / max(tp + fn, 1)
            out["false_alarm_rate"] = fp / max(fp + tn, 1)
            out["label_positives"] = tp + fn
            out["mlp_flags"] = tp + fp
        h.close()
    a, b = res["plain"], res["learned"]
    n = min(a["steps"], b["steps"])
    out["steps_completed"] = {"plain": a["steps"], "learned": b["steps"]}
    if a["steps"] == b["steps"]:
        rho_p, rho_l = dg.to_planes(cfg, a["u"])[0], dg.to_planes(cfg, b["u"])[0]
        out["density_rel_L2_diff"] = float(((rho_l - rho_p) ** 2).sum().sqrt() / (rho_p ** 2).sum().sqrt())
    if n > 0:
        out["torque_series_rel_diff"] = float((b["tq"][:n] - a["tq"][:n]).abs().max() / a["tq"][:n].abs().max())
    out["ms_per_step_plain"] = a["elapsed"] * 1e3 / max(a["steps"], 1)
    out["ms_per_step_learned"] = b["elapsed"] * 1e3 / max(b["steps"], 1)
    out["speedup_learned_vs_plain"] = out["ms_per_step_plain"] / out["ms_per_step_learned"]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--every", type=int, default=25)
    ap.add_argument("--cap", type=int, default=4096)
    ap.add_argument("--train-seeds", type=int, nargs="*", default=[0, 1, 2, 3, 4, 5])
    ap.add_argument("--val-seed", type=int, default=6)
    ap.add_argument("--test-seed", type=int, default=7)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default="learned_result.json")
    ap.add_argument("--params-out", default=None)
    ap.add_argument("--s0", type=float, default=None, help="modal-decay threshold (default -4 log10(order))")
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)

    def log(msg):
        print(msg, flush=True)

    t_start = time.time()
    Xs, Ys = [], []
    for s in a.train_seeds:
        X, Y, _, _ = collect(s, a.nx, a.steps, a.every, a.cap, torch, a.s0, log)
        Xs.append(X)
        Ys.append(Y)
    X = torch.cat(Xs)
    Y = torch.cat(Ys)
    Xv, Yv, _, _ = collect(a.val_seed, a.nx, a.steps, a.every, a.cap, torch, a.s0, log)
    log(f"[data] train {X.shape[0]} samples ({int(Y.sum().item())} positive), val {Xv.shape[0]}")
    # a handle is needed to own the network; any configuration with the limiter works
    cfg = ring_config(64)
    h, _ = dg.dg_init(cfg, W.prim_for(cfg, "disc_ring", seed=0))
    dg.dg_mlp_params(h, set_params=init_params(0))
    t_tr = time.time()
    hist, pw = train(h, X, Y, a.epochs, a.batch, a.lr, 0, torch, log)
    t_tr = time.time() - t_tr
    params = dg.dg_mlp_params(h, get=True)
    zv = torch.zeros(Xv.shape[0], dtype=torch.float32, device="cuda")
    dg.dg_mlp_forward(h, Xv, Xv.shape[0], zv)
    pv = torch.sigmoid(zv).cpu().numpy()
    yv = Yv.cpu().numpy()
    theta = 0.5
    for th in np.linspace(0.95, 0.01, 95):
        miss, _ = rates(pv, yv, th)
        if miss <= 0.01:
            theta = float(th)
            break
    vmiss, vfa = rates(pv, yv, theta)
    log(f"[val] theta {theta:.3f}: miss {vmiss:.4f}, false alarm (balanced sample) {vfa:.4f}")
    h.close()
    s0 = default_s0(4) if a.s0 is None else a.s0
    ev = evaluate_run(a.test_seed, a.nx, a.steps, a.every, params, theta, torch, s0, log)
    res = {"nx": a.nx, "order": 4, "steps": a.steps, "s0": s0, "every": a.every, "train_seeds": a.train_seeds,
           "val_seed": a.val_seed, "test_seed": a.test_seed, "train_samples": int(X.shape[0]),
           "train_positives": int(Y.sum().item()), "pos_weight": pw, "epochs": a.epochs, "batch": a.batch,
           "lr": a.lr, "loss_history": hist, "train_seconds": t_tr, "theta": theta,
           "val_miss": vmiss, "val_false_alarm_balanced": vfa, "test": ev,
           "wall_seconds": time.time() - t_start}
    log(json.dumps(res))
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1)
    if a.params_out:
        save_params(a.params_out, params, theta, s0,
                    {k: res[k] for k in ("nx", "steps", "every", "train_seeds", "val_seed", "test_seed",
                                         "train_samples", "train_positives", "epochs", "val_miss")})


if __name__ == "__main__":
    main()
