"""Policy search for the quadruped's controller (section 2.2): gradient of the
mean forward speed with respect to the controller's weights through the
hand-written adjoint, Adam with the gradient norm clipped to 1 (section 3.2).

The episodes are cut to a fixed horizon: over the full 500..2000 steps the
gradient of this chaotic system overflows FP32 (the remedies of section 3.2,
shorter horizons or a decaying gradient, are left for later).  An env whose
adjoint still overflows is left out of the weight gradient by the library
(flagged SIM_FLAG_GRAD_NONFINITE).

    python -m paper_1611_01652_amd.train_controller --envs 1024 --T 200 --iters 50
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import workloads as W
from .sim import Adam, Simulator


def train(n_envs=1024, T=200, iters=50, lr=1e-3, max_norm=1.0, seed_salt=0, log=None):
    import torch
    w = W.quadruped(n_envs=n_envs, T_min=T, T_max=T, seed_salt=seed_salt)
    s = Simulator(w)
    x0 = torch.tensor(np.ascontiguousarray(w.x0.T), dtype=torch.float32, device="cuda")
    wt = torch.tensor(w.extra["mlp"]["w"], dtype=torch.float32, device="cuda")
    opt = Adam(wt, lr=lr, max_norm=max_norm)
    dl = torch.full((n_envs,), 1.0 / n_envs, device="cuda")   # the mean loss over envs
    ws = s.workspace()
    hist = []
    for it in range(iters + 1):
        r = s.rollout(x0, wt)
        loss = float(r["loss"].mean().item())
        if it == iters:
            hist.append(dict(iter=it, loss=loss))
            break
        g = s.rollout_grad(x0, wt, r["ckpt"], dl, workspace=ws)
        opt.step(g["g_u"])
        hist.append(dict(iter=it, loss=loss, grad_norm=float(opt.grad_norm.item()),
                         nonfinite_envs=int((r["flags"] & 1).ne(0).sum().item()),
                         overflowed_gradients=int((g["flags"] & 4).ne(0).sum().item())))
        if log and (it % log == 0):
            print(json.dumps(hist[-1]), flush=True)
    s.close()
    return hist, wt


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--envs", type=int, default=1024)
    ap.add_argument("--T", type=int, default=200)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--lr", type=float, default=3e-4)
    a = ap.parse_args(argv)
    t0 = time.time()
    hist, _ = train(a.envs, a.T, a.iters, a.lr, log=10)
    best = min(hist, key=lambda h: h["loss"])
    print(json.dumps(dict(zero_policy_loss=hist[0]["loss"], final_loss=hist[-1]["loss"], best_loss=best["loss"],
                          best_iter=best["iter"], seconds=round(time.time() - t0, 2))))


if __name__ == "__main__":
    main()
