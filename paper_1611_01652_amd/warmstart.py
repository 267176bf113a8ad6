"""Learned warm start of contact impulses, end to end on the GPU.

1. label: the plain solver iterated to the residual tolerance on the chain
   distribution writes (features, converged impulse) records (rollout_solve);
2. train: the per-contact network is fitted to the records by mean-squared
   error with Adam, with the library's matrix-core forward/backward kernels;
3. evaluate: on held-out envs, the same tolerance-mode rollout with the plain
   and with the learned warm start: sweeps per env-step to the tolerance
   (sweeps a rejected learned start cost included), fallbacks, env-steps/s.

Every step runs in the library; torch provides device memory, the stream and
the sampling of minibatches.

    python -m paper_1611_01652_amd.warmstart --label-envs 4096 --eval-envs 2048
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import workloads as W
from .sim import Simulator, WarmStartNet


def _dev(w):
    import torch
    x0 = torch.tensor(np.ascontiguousarray(w.x0.T), dtype=torch.float32, device="cuda")
    u = torch.tensor(np.ascontiguousarray(w.u), dtype=torch.float32, device="cuda")
    return x0, u


def label(n_envs, T, seed_salt=100, rec_every=2, cap=10_000_000, tol=1e-5):
    """Training records [n, 16] (CUDA float32) from the plain solver, ordered
    by (env, step, contact code) so that training is reproducible."""
    import torch
    w = W.warm_start_chains(n_envs=n_envs, T=T, seed_salt=seed_salt, tol=tol)
    s = Simulator(w)
    x0, u = _dev(w)
    r = s.rollout_solve(x0, u, rec_cap=cap, rec_every=rec_every, want_final=False)
    torch.cuda.synchronize()
    n = min(int(r["n_records"].item()), cap)
    rec = r["records"][:n]
    ints = rec[:, 12:15].contiguous().view(torch.int32).to(torch.int64)
    key = (ints[:, 0] * (1 << 12) + ints[:, 1]) * (1 << 27) + ints[:, 2]
    order = torch.argsort(key)
    s.close()
    return rec.index_select(0, order).contiguous(), int(r["iters"].sum().item()) / float(w.T_env.sum())


def train(rec, steps=3000, batch=4096, lr=1e-3, seed=0, w0=None, log_every=500, huber=0.05):
    """Fit the network to the corrections of the carried impulses (Huber loss:
    the bulk of contacts need small corrections, a few impacts very large
    ones); starts from a zero output layer, i.e. from the plain warm start.
    Returns (net, [(step, loss on a fixed evaluation batch)])."""
    import torch
    net = WarmStartNet(W.wsn_init(seed_salt=seed, zero_output=True) if w0 is None else w0)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    n = rec.shape[0]
    probe = rec[torch.randint(0, n, (min(n, 65536),), device="cuda", generator=gen)].contiguous()
    log = []
    for it in range(steps):
        idx = torch.randint(0, n, (batch,), device="cuda", generator=gen)
        net.loss_grad(rec.index_select(0, idx), huber=huber, relative=True)
        # learning rate: constant, then linearly to a tenth over the last half
        f = 1.0 if it < steps // 2 else 1.0 - 0.9 * (it - steps // 2) / max(1, steps - steps // 2)
        net.adam(lr * f)
        if log_every and (it % log_every == 0 or it == steps - 1):
            log.append((it, float(net.loss_grad(probe, huber=huber, relative=True)[0].item())))
    return net, log


def evaluate(ws_w, n_envs, T, seed_salt=200, tol=1e-5, reps=2, fb_iters=5, fb_tol=1e-3):
    """Tolerance-mode rollout on held-out envs with the plain (ws_w None) or
    the learned warm start."""
    import torch
    w = W.warm_start_chains(n_envs=n_envs, T=T, seed_salt=seed_salt, tol=tol, ws_w=ws_w, fb_iters=fb_iters,
                            fb_tol=fb_tol)
    s = Simulator(w)
    x0, u = _dev(w)
    r = s.rollout_solve(x0, u)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        r = s.rollout_solve(x0, u)
        b.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    es = float(w.T_env.sum())
    out = dict(sweeps_per_env_step=float(r["iters"].sum().item()) / es,
               fallback_frac=float(r["fallbacks"].sum().item()) / es,
               env_steps_per_s=es / (min(ms) * 1e-3), ms=min(ms),
               nonfinite_envs=int((r["flags"] & 1).ne(0).sum().item()))
    s.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--label-envs", type=int, default=4096)
    ap.add_argument("--eval-envs", type=int, default=2048)
    ap.add_argument("--T", type=int, default=500)
    ap.add_argument("--rec-every", type=int, default=2)
    ap.add_argument("--cap", type=int, default=10_000_000)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--huber", type=float, default=0.05)
    ap.add_argument("--eval-tols", type=str, default="1e-5,1e-4")
    ap.add_argument("--fb-tols", type=str, default="1e-3",
                    help="fallback thresholds to evaluate (contact-row residual after 5 sweeps)")
    a = ap.parse_args(argv)
    t0 = time.time()
    rec, label_sweeps = label(a.label_envs, a.T, rec_every=a.rec_every, cap=a.cap, tol=a.tol)
    t1 = time.time()
    print(json.dumps(dict(stage="label", records=int(rec.shape[0]), seconds=round(t1 - t0, 2),
                          plain_sweeps_per_env_step=round(label_sweeps, 2))), flush=True)
    net, log = train(rec, steps=a.steps, batch=a.batch, lr=a.lr, huber=a.huber)
    t2 = time.time()
    print(json.dumps(dict(stage="train", seconds=round(t2 - t1, 2), loss=log)), flush=True)
    wl = net.w.cpu().numpy().astype(np.float64)
    out = []
    for tol in [float(v) for v in a.eval_tols.split(",")]:
        plain = evaluate(None, a.eval_envs, a.T, tol=tol)
        for fbt in [float(v) for v in a.fb_tols.split(",")]:
            learned = evaluate(wl, a.eval_envs, a.T, tol=tol, fb_tol=fbt)
            res = dict(stage="evaluate", tol=tol, fb_tol=fbt, held_out_envs=a.eval_envs, T=a.T, plain=plain,
                       learned=learned, sweep_ratio=learned["sweeps_per_env_step"] / plain["sweeps_per_env_step"],
                       speedup=learned["env_steps_per_s"] / plain["env_steps_per_s"])
            print(json.dumps(res), flush=True)
            out.append(res)
    return out, wl


if __name__ == "__main__":
    main()
