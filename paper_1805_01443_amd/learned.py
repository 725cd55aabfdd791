"""Learned troubled-cell indicator: data, training and evaluation on the GPU.

Workload: the adiabatic disc at order 4 (P3) with an over-pressure ring that
steepens into shocks (``configs.disc_ring``).  The plain pipeline (modal-decay
sensor + minmod) is run with seeded initial data; every ``every`` steps the
state of the last stage before limiting is captured (``dg_capture``): its bf16
features and the plain indicator's flags, which are the labels.  All positives
and as many random negatives are kept.  The MLP is trained with the
library's own forward/backward/Adam kernels (``dg_mlp_train_step``).  Then, in
DAgger iterations, the learned limiter itself runs the training seeds and the
states it visits (where its misses let oscillations grow) are labelled by the
plain indicator and added to the data before retraining.  The flag threshold
is chosen on a validation seed for a miss rate <= 1 %.  Besides the ring runs,
every seed contributes a short run from its jump state (density and pressure
multiplied inside a seeded radius: a discontinuity the smooth ring does not
produce at these times), whose first steps are all captured.  On a test seed the
learned limiter runs the same workload while its flags are compared with the
plain labels on the same states (miss and false-alarm rates); torque, density,
residual oscillation and step time are compared with the plain indicator, with
no troubled-cell limiter and with minmod on every element.

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
from . import synth


def default_s0(order: int) -> float:
    """Threshold of the modal-decay sensor: -4 log10(p + 1)."""
    return -4.0 * math.log10(order)


def ring_config(nx, order=4, limiter=dg.LIMITER_MODAL_DECAY, theta=0.5, s0=None, positivity=1):
    """The ring workload with a troubled-cell limiter and (by default) the
    positivity-preserving limiter behind it: component-wise minmod alone can
    leave negative point pressures behind the ring's shocks."""
    return W.disc_ring(nx=nx, order=order).replace(
        limiter=limiter, limiter_s0=default_s0(order) if s0 is None else s0, mlp_theta=theta,
        positivity=positivity)


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


def ring_prim(cfg, seed, jump=None):
    """Initial data of the ring workload; jump: None, or (r_j, f) to multiply
    density and pressure by f inside r < r_j."""
    prim = W.prim_for(cfg, "disc_ring", seed=seed)
    if jump is None:
        return prim
    x, y = dg.dg_get_nodes(cfg)
    return synth.apply_jump(prim, x, y, *jump)


def collect(seed, nx, steps, every, cap, torch, s0=None, log=print, positivity=1, params=None, theta=0.5,
            jump=False, cap_first=0):
    """Run the plain pipeline (or, with ``params``, the learned limiter with
    that network: the states it visits, labelled by the plain indicator);
    returns (features int16 [N, 64], labels float [N], per-capture positive
    counts, steps run).  With ``jump`` the ring starts with the seed's density
    and pressure jump (synth.ring_jump); the first ``cap_first`` steps are
    captured, then every ``every``-th.  A run whose state turns non-finite
    stops there and keeps the samples captured before."""
    lim = dg.LIMITER_MODAL_DECAY if params is None else dg.LIMITER_LEARNED
    cfg = ring_config(nx, limiter=lim, theta=theta, s0=s0, positivity=positivity)
    prim = ring_prim(cfg, seed, synth.ring_jump(seed) if jump else None)
    h, u = dg.dg_init(cfg, prim)
    if params is not None:
        dg.dg_mlp_params(h, set_params=params)
    E = cfg.n_elem
    feat = torch.zeros((E, 64), dtype=torch.int16, device="cuda")
    lab = torch.zeros(E, dtype=torch.uint8, device="cuda")
    t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(1000 + seed)
    xs, ys, npos = [], [], []
    done = 0
    for k in range(steps):
        cap_now = k < cap_first or (k + 1) % every == 0
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
    log(f"[collect] seed {seed}{' jump' if jump else ''} ({'learned' if params is not None else 'plain'}): "
        f"{done} steps, "
        f"t_end {t_dev.item():.4f}, positives per capture "
        f"{npos[:3]}...{npos[-3:]} (total {sum(npos)})")
    h.close()
    return torch.cat(xs), torch.cat(ys), npos, done


def symmetry_maps(order=4, nvar=4):
    """Column maps of the eight mirror/transpose images of a feature row
    f[v*n*n + a*n + b]: image[:, j] = f[:, src[j]] with the sign flipped where
    flip[j].  x mirror: mode (a, b) of a scalar changes sign with (-1)^a and
    m_x with -(-1)^a; y mirror likewise with b and m_y; transpose swaps a <-> b
    and m_x <-> m_y.  The modal-decay sensor (and so the label) is invariant
    under all eight."""
    n = order
    maps = []
    for tr in (0, 1):
        for rx in (0, 1):
            for ry in (0, 1):
                src = np.zeros(nvar * n * n, dtype=np.int64)
                flip = np.zeros(nvar * n * n, dtype=bool)
                for v in range(nvar):
                    for a in range(n):
                        for b in range(n):
                            vs, as_, bs = v, a, b
                            if tr:
                                vs = {1: 2, 2: 1}.get(v, v)
                                as_, bs = b, a
                            neg = False
                            if rx:
                                neg ^= (a % 2 == 1) ^ (v == 1)
                            if ry:
                                neg ^= (b % 2 == 1) ^ (v == 2)
                            j = v * n * n + a * n + b
                            src[j] = vs * n * n + as_ * n + bs
                            flip[j] = neg
                maps.append((src, flip))
    return maps


def augment_positives(X, Y, torch):
    """Append the seven other mirror/transpose images of every positive sample
    (bf16 bit patterns: a sign flip is the top bit)."""
    pos = torch.nonzero(Y > 0.5).flatten()
    Xp = X[pos]
    extra = []
    for src, flip in symmetry_maps()[1:]:
        img = Xp[:, torch.as_tensor(src, device=X.device)]
        mask = torch.as_tensor(np.where(flip, -32768, 0).astype(np.int16), device=X.device)
        extra.append(img ^ mask)
    Xa = torch.cat([X] + extra)
    Ya = torch.cat([Y, torch.ones(Xp.shape[0] * len(extra), device=Y.device)])
    return Xa, Ya


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


def pick_theta(h, Xv, Yv, torch):
    """The largest threshold on a 0.01 grid with a validation miss rate <= 1 %."""
    zv = torch.zeros(Xv.shape[0], dtype=torch.float32, device="cuda")
    dg.dg_mlp_forward(h, Xv, Xv.shape[0], zv)
    pv = torch.sigmoid(zv).cpu().numpy()
    yv = Yv.cpu().numpy()
    for th in np.linspace(0.95, 0.01, 95):
        miss, _ = rates(pv, yv, th)
        if miss <= 0.01:
            return float(th)
    return 0.01


def rates(prob, y, theta):
    f = prob > theta
    pos = y > 0.5
    miss = float((~f & pos).sum()) / max(int(pos.sum()), 1)
    fa = float((f & ~pos).sum()) / max(int((~pos).sum()), 1)
    return miss, fa


# troubled-cell treatments compared on the test seed: the plain indicator (the
# reference), the learned one, none (positivity limiter only) and minmod on
# every element (a sensor threshold below any value)
TREATMENTS = (("plain", dg.LIMITER_MODAL_DECAY, None), ("learned", dg.LIMITER_LEARNED, None),
              ("none", dg.LIMITER_NONE, None), ("all", dg.LIMITER_MODAL_DECAY, -1e300))


def evaluate_run(seed, nx, steps, every, params, theta, torch, s0=None, log=print, positivity=1,
                 treatments=TREATMENTS):
    """Each treatment on the same seeded workload: step times, torque series,
    final density, and the share of elements the plain sensor flags at the end
    (residual oscillation); the learned flags against the plain labels on the
    learned run's own states (miss and false-alarm rates).  A run stops at its
    first non-finite state; comparisons with the plain run cover the steps both
    completed."""
    out = {}
    res = {}
    for name, lim, s0_over in treatments:
        cfg = ring_config(nx, limiter=lim, theta=theta, s0=s0 if s0_over is None else s0_over,
                          positivity=positivity)
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
        # residual oscillation: elements the plain sensor (threshold s0) flags
        cs = ring_config(nx, s0=s0, positivity=positivity)
        hq, _ = dg.dg_init(cs, prim)
        dg.dg_troubled(hq, u, apply=False, flags=lab)
        dg.dg_sync(hq)
        hq.close()
        flagged = float(lab.float().mean().item())
        res[name] = {"u": u.clone(), "tq": tq.clone(), "elapsed": el, "steps": done, "t": t_dev.item(),
                     "flagged": flagged}
        log(f"[eval] {name}: {done} steps to t = {t_dev.item():.4f}, {el * 1e3 / max(done, 1):.3f} ms/step, "
            f"sensor flags {flagged:.4%} of the elements at the end")
        if name == "plain":
            # open loop: the network on the plain run's own states
            h2, u2 = dg.dg_init(cfg, prim)
            hn, _ = dg.dg_init(ring_config(64), W.prim_for(ring_config(64), "disc_ring", seed=0))
            dg.dg_mlp_params(hn, set_params=params)
            feat = torch.zeros((E, 64), dtype=torch.int16, device="cuda")
            z = torch.zeros(E, dtype=torch.float32, device="cuda")
            thf = np.float32(theta)
            zthr = float(np.log(thf / (np.float32(1.0) - thf)))
            t2 = torch.zeros(1, dtype=torch.float64, device="cuda")
            otp = ofn = ofp = otn = 0
            for k in range(done):
                cap = (k + 1) % every == 0
                if cap:
                    dg.dg_capture(h2, feat=feat, flags=lab)
                dg.dg_rk_step(h2, u2, t2, 0.0, None)
                if cap:
                    dg.dg_mlp_forward(hn, feat, E, z)
                    y = lab.bool()
                    m = z > zthr
                    otp += int((y & m).sum())
                    ofn += int((y & ~m).sum())
                    ofp += int((~y & m).sum())
                    otn += int((~y & ~m).sum())
            h2.close()
            hn.close()
            out["open_loop"] = {"states": "the plain run's", "miss_rate": ofn / max(otp + ofn, 1),
                                "false_alarm_rate": ofp / max(ofp + otn, 1), "label_positives": otp + ofn,
                                "mlp_flags": otp + ofp}
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
            out["closed_loop"] = {"states": "the learned run's own", "captured": ncap,
                                  "miss_rate": fn / max(tp + fn, 1), "false_alarm_rate": fp / max(fp + tn, 1),
                                  "label_positives": tp + fn, "mlp_flags": tp + fp}
        h.close()
    a = res["plain"]
    out["runs"] = {}
    for name, r in res.items():
        d = {"steps": r["steps"], "t_end": r["t"], "ms_per_step": r["elapsed"] * 1e3 / max(r["steps"], 1),
             "sensor_flagged_fraction_at_end": r["flagged"]}
        n = min(a["steps"], r["steps"])
        if name != "plain" and r["steps"] == a["steps"]:
            rho_p, rho_x = dg.to_planes(cfg, a["u"])[0], dg.to_planes(cfg, r["u"])[0]
            d["density_rel_L2_diff_vs_plain"] = float(((rho_x - rho_p) ** 2).sum().sqrt() / (rho_p ** 2).sum().sqrt())
        if name != "plain" and n > 0:
            d["torque_series_rel_diff_vs_plain"] = float(
                (r["tq"][:n] - a["tq"][:n]).abs().max() / a["tq"][:n].abs().max())
        out["runs"][name] = d
    if "learned" in res:
        out["speedup_learned_vs_plain"] = out["runs"]["plain"]["ms_per_step"] / out["runs"]["learned"]["ms_per_step"]
    return out


def evaluate_jump(seed, nx, steps, params, theta, torch, s0=None, log=print, positivity=1):
    """The seed's jump state (synth.ring_jump): the network's flags against
    the plain labels on every step's last-stage state, on the plain run's
    states (open loop) and on the learned limiter's own (closed loop)."""
    out = {"jump": list(synth.ring_jump(seed)), "steps": steps}
    for name, lim in (("open_loop", dg.LIMITER_MODAL_DECAY), ("closed_loop", dg.LIMITER_LEARNED)):
        cfg = ring_config(nx, limiter=lim, theta=theta, s0=s0, positivity=positivity)
        prim = ring_prim(cfg, seed, synth.ring_jump(seed))
        h, u = dg.dg_init(cfg, prim)
        dg.dg_mlp_params(h, set_params=params)
        E = cfg.n_elem
        feat = torch.zeros((E, 64), dtype=torch.int16, device="cuda")
        lab = torch.zeros(E, dtype=torch.uint8, device="cuda")
        z = torch.zeros(E, dtype=torch.float32, device="cuda")
        thf = np.float32(theta)
        zthr = float(np.log(thf / (np.float32(1.0) - thf)))
        t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
        tp = fn = fp = tn = 0
        for _ in range(steps):
            dg.dg_capture(h, feat=feat, flags=lab)
            dg.dg_rk_step(h, u, t_dev, 0.0, None)
            dg.dg_mlp_forward(h, feat, E, z)
            y = lab.bool()
            m = z > zthr
            tp += int((y & m).sum())
            fn += int((y & ~m).sum())
            fp += int((~y & m).sum())
            tn += int((~y & ~m).sum())
        dg.dg_sync(h)
        h.close()
        out[name] = {"miss_rate": fn / max(tp + fn, 1), "false_alarm_rate": fp / max(fp + tn, 1),
                     "label_positives": tp + fn, "mlp_flags": tp + fp}
        log(f"[eval jump] {name}: miss {out[name]['miss_rate']:.4f}, false alarm {out[name]['false_alarm_rate']:.5f}, "
            f"{tp + fn} positives over {steps} steps")
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
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default="learned_result.json")
    ap.add_argument("--params-out", default=None)
    ap.add_argument("--s0", type=float, default=None, help="modal-decay threshold (default -4 log10(order))")
    ap.add_argument("--no-positivity", action="store_true", help="without the positivity-preserving limiter")
    ap.add_argument("--dagger", type=int, default=2,
                    help="iterations of data from the learned limiter's own runs, labelled by the plain indicator")
    ap.add_argument("--jump-steps", type=int, default=0,
                    help="steps of a run from each seed's jump state (0: none), its first 20 captured")
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)

    def log(msg):
        print(msg, flush=True)

    t_start = time.time()
    pos = 0 if a.no_positivity else 1
    Xs, Ys = [], []

    def runs(seed, params=None, theta=0.5):
        """the seed's ring run and, with --jump-steps, its jump run"""
        X, Y, _, _ = collect(seed, a.nx, a.steps, a.every, a.cap, torch, a.s0, log, pos, params=params, theta=theta)
        xs, ys = [X], [Y]
        if a.jump_steps > 0:
            X, Y, _, _ = collect(seed, a.nx, a.jump_steps, a.every, a.cap, torch, a.s0, log, pos, params=params,
                                 theta=theta, jump=True, cap_first=min(20, a.jump_steps))
            xs.append(X)
            ys.append(Y)
        return torch.cat(xs), torch.cat(ys)

    for s in a.train_seeds:
        X, Y = runs(s)
        Xs.append(X)
        Ys.append(Y)
    Xv, Yv = runs(a.val_seed)
    Xvs, Yvs = [Xv], [Yv]
    # a handle is needed to own the network; any configuration with the limiter works
    cfg = ring_config(64)
    h, _ = dg.dg_init(cfg, W.prim_for(cfg, "disc_ring", seed=0))
    dg.dg_mlp_params(h, set_params=init_params(0))
    t_tr = time.time()
    X, Y = augment_positives(torch.cat(Xs), torch.cat(Ys), torch)
    log(f"[data] iteration 0: train {X.shape[0]} samples ({int(Y.sum().item())} positive, mirror images included)")
    hist, pw = train(h, X, Y, a.epochs, a.batch, a.lr, 0, torch, log)
    theta = pick_theta(h, torch.cat(Xvs), torch.cat(Yvs), torch)
    # DAgger: the learned limiter's own runs (states it visits when it misses),
    # labelled by the plain indicator, added to the data; retrain
    for rnd in range(1, a.dagger + 1):
        params = dg.dg_mlp_params(h, get=True)
        for s in a.train_seeds:
            X, Y = runs(s, params, theta)
            Xs.append(X)
            Ys.append(Y)
        Xv, Yv = runs(a.val_seed, params, theta)
        Xvs.append(Xv)
        Yvs.append(Yv)
        X, Y = augment_positives(torch.cat(Xs), torch.cat(Ys), torch)
        log(f"[data] iteration {rnd}: train {X.shape[0]} samples ({int(Y.sum().item())} positive, mirror images "
            f"included), data collected with theta {theta:.3f}")
        h2, p2 = train(h, X, Y, a.epochs, a.batch, a.lr, rnd, torch, log)
        hist += h2
        pw = p2
        theta = pick_theta(h, torch.cat(Xvs), torch.cat(Yvs), torch)
    t_tr = time.time() - t_tr
    Xv, Yv = torch.cat(Xvs), torch.cat(Yvs)
    log(f"[data] val {Xv.shape[0]} samples ({int(Yv.sum().item())} positive)")
    params = dg.dg_mlp_params(h, get=True)
    theta = pick_theta(h, Xv, Yv, torch)
    zv = torch.zeros(Xv.shape[0], dtype=torch.float32, device="cuda")
    dg.dg_mlp_forward(h, Xv, Xv.shape[0], zv)
    vmiss, vfa = rates(torch.sigmoid(zv).cpu().numpy(), Yv.cpu().numpy(), theta)
    log(f"[val] theta {theta:.3f}: miss {vmiss:.4f}, false alarm (balanced sample) {vfa:.4f}")
    h.close()
    s0 = default_s0(4) if a.s0 is None else a.s0
    ev = evaluate_run(a.test_seed, a.nx, a.steps, a.every, params, theta, torch, s0, log, pos)
    if a.jump_steps > 0:
        ev["jump"] = evaluate_jump(a.test_seed, a.nx, min(20, a.jump_steps), params, theta, torch, s0, log, pos)
    res = {"nx": a.nx, "jump_steps": a.jump_steps, "order": 4, "steps": a.steps, "s0": s0, "positivity": pos, "every": a.every,
           "dagger_iterations": a.dagger, "train_seeds": a.train_seeds, "val_samples": int(Xv.shape[0]),
           "val_positives": int(Yv.sum().item()),
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
                    {k: res[k] for k in ("nx", "steps", "jump_steps", "positivity", "every", "train_seeds", "val_seed",
                                         "test_seed", "train_samples", "train_positives", "epochs", "val_miss")})


if __name__ == "__main__":
    main()
