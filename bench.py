"""Benchmark: forward + adjoint env-steps/s of the batched rigid-body step.

One "step" of this benchmark is one pass of the whole hot path over the
workload: `rollout` (T time steps of every env, with checkpoints) followed by
`rollout_grad` (recompute from the checkpoints + hand-written reverse sweep),
i.e. E * T env-steps forward and backward.  Inputs are resident in HBM before
the timed region.  The workload is the 4096 planar 3-link arms x 1000 steps
one (synthetic, seeded); `--workload chains` runs the 16384 uneven 3D chains
x 500, `--workload quadruped` the 1024 legged robots with an MLP controller.

Printed: one JSON line with the throughput, a roofline object for the
dominant kernel (the reverse sweep, timed by events the library records
around it), a gradient check of sampled envs against the FP64 oracle, and
the oracle's own CPU throughput on a bounded sample (rank 0, N = 1).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+adjoint env-steps/s at grad rel-err<=1e-3 vs FP64 oracle; % HBM roofline"
HBM_PEAK_GBS = 8000.0
CHECK_HORIZON = 40   # steps of the gradient check of the chaotic workloads
FP32_VECTOR_PEAK_TFLOPS = 157.3


def algorithmic_bytes_per_env_step(w):
    """Bytes a step must move if it were its own kernel with the state in HBM
    (struct-of-arrays): state in/out, warm-start impulses in/out, torques in,
    checkpoint writes / K_ck; the adjoint adds the recompute (a forward plus
    the segment buffer write), and the reverse sweep (segment buffer read,
    state and impulse adjoints in/out, torques in, torque adjoints out)."""
    E = w.n_envs
    nb = w.n_bodies / E
    nj = w.n_joints / E
    lam = 5 * nj  # hinge rows; contact candidates are added for contact models
    ng = (w.sphere_flags & 1).sum() / E if w.ground else 0
    lam += 4 * ng
    state = 72 * nb
    fwd = 2 * state + 2 * 4 * lam + 4 * nj + (state + 4 * lam) / w.ckpt_every
    seg = state + 4 * lam
    rev = seg + 2 * state + 2 * 4 * lam + 4 * nj + 4 * nj
    grad_kernel = fwd + seg + rev
    return dict(fwd=fwd, grad_kernel=grad_kernel, total=fwd + grad_kernel)


def flops_per_env_step(w, n_sample=8):
    """Operation counts from the oracle's counting scalar (forward) and the
    edges of its reverse-mode tape (2 flops each) on sampled envs/steps."""
    from oracle import Oracle
    E = w.n_envs
    envs = sorted(set(np.linspace(0, E - 1, min(n_sample, E)).astype(int).tolist()))
    ws = w.subset(envs).with_steps(min(w.T_max, 120))
    o = Oracle(ws)
    tr = o.rollout(traj=True)["traj"]
    f, r = 0.0, 0.0
    n = 0
    for t in (0, ws.T_max // 2, ws.T_max - 1):
        x = tr[t]
        for e in range(ws.n_envs):
            f += o.count_flops(e, x=x, u=ws.u[t] if ws.u is not None and ws.u.size else None, t=t)
            r += 2 * o.count_tape_edges(e, x=x, u=ws.u[t] if ws.u is not None and ws.u.size else None, t=t)
            n += 1
    return f / n, r / n


def make_workload(name):
    from paper_1611_01652_amd import workloads as W
    if name == "arms":
        return W.planar_arms(n_envs=4096, T=1000)
    if name == "chains":
        return W.uneven_chains(n_envs=16384, T=500)
    if name == "quadruped":
        # the controller as initialised for training: zero output layer
        return W.quadruped(n_envs=1024)
    raise SystemExit(f"unknown workload {name}")


def controls(w):
    """The control input of rollout: the torque tape, or the controller weights."""
    mlp = (getattr(w, "extra", None) or {}).get("mlp")
    return np.asarray(mlp["w"] if mlp is not None else w.u, dtype=np.float32)


def grad_check(w, got_gu, got_gx0, n=4):
    """Max relative gradient error of sampled envs of the benchmark's own
    result against the oracle."""
    from oracle import Oracle
    envs = sorted(set(np.linspace(0, w.n_envs - 1, n).astype(int).tolist()))
    ws = w.subset(envs)
    ref = Oracle(ws).rollout_grad()
    return _worst(w, envs, ws, ref, got_gu, got_gx0), len(envs)


def grad_check_short(w, T, n=4):
    """Chaotic workloads: sampled envs over their first T steps, run by the
    library on their own, against the oracle (the full horizon's gradients
    differ by FP32 rounding amplified along the trajectory)."""
    import torch
    from oracle import Oracle
    from paper_1611_01652_amd.sim import Simulator
    envs = sorted(set(np.linspace(0, w.n_envs - 1, n).astype(int).tolist()))
    ws = w.subset(envs).with_steps(T)
    s = Simulator(ws)
    x0 = torch.tensor(np.ascontiguousarray(ws.x0.T), dtype=torch.float32, device="cuda")
    u = torch.tensor(np.ascontiguousarray(controls(ws)), dtype=torch.float32, device="cuda")
    r = s.rollout(x0, u)
    g = s.rollout_grad(x0, u, r["ckpt"], torch.ones(ws.n_envs, device="cuda"))
    torch.cuda.synchronize()
    ref = Oracle(ws).rollout_grad()
    gu = g["g_u"].cpu().numpy().astype(np.float64)
    gx0 = g["g_x0"].cpu().numpy().T.astype(np.float64)
    s.close()
    if "g_w" in ref:
        # the controller's weight gradient (what training uses); the legged
        # robot's dL/dx0 hinges on stick-slip decisions of its feet
        return float(np.linalg.norm(gu - ref["g_w"]) / max(np.linalg.norm(ref["g_w"]), 1e-30)), len(envs)
    return _worst(ws, list(range(len(envs))), ws, ref, gu, gx0), len(envs)


def _worst(w, envs, ws, ref, got_gu, got_gx0):
    worst = 0.0
    for i, e in enumerate(envs):
        j0, j1 = w.env_joint_off[e], w.env_joint_off[e + 1]
        b0, b1 = w.env_body_off[e], w.env_body_off[e + 1]
        rj0, rj1 = ws.env_joint_off[i], ws.env_joint_off[i + 1]
        rb0, rb1 = ws.env_body_off[i], ws.env_body_off[i + 1]
        for got, r in ((got_gu[:, j0:j1], ref["g_u"][:, rj0:rj1]), (got_gx0[b0:b1], ref["g_x0"][rb0:rb1])):
            nr = np.linalg.norm(r)
            if nr > 1e-8:
                worst = max(worst, float(np.linalg.norm(got - r) / nr))
    return worst


def cpu_baseline(w, seconds=15.0):
    """The oracle (FP64, tape reverse mode) on the host cores, fwd + gradient,
    on a bounded sample of envs of the same workload."""
    from oracle import Oracle
    threads = min(os.cpu_count() or 1, 16)
    n = 2 * threads
    ws = w.subset(list(range(n)))
    # shorten the horizon if a full pass would exceed the time budget
    t0 = time.time()
    Oracle(ws.with_steps(min(w.T_max, 50))).rollout_grad(threads=threads)
    per_step = (time.time() - t0) / (n * min(w.T_max, 50))
    T = int(max(20, min(w.T_max, seconds / max(per_step * n, 1e-9))))
    wt = ws.with_steps(T)
    o = Oracle(wt)
    t0 = time.time()
    o.rollout(threads=threads)
    o.rollout_grad(threads=threads)
    el = time.time() - t0
    return {"value": n * T / el, "unit": "env-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} envs x {T} steps of the same workload, forward + tape gradient, FP64, "
                      f"{threads} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="arms", choices=["arms", "chains", "quadruped"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not implemented)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1611_01652_amd.sim import Simulator

    w = make_workload(args.workload)
    sim = Simulator(w)
    x0 = torch.tensor(np.ascontiguousarray(w.x0.T), dtype=torch.float32, device="cuda")
    u = torch.tensor(np.ascontiguousarray(controls(w)), dtype=torch.float32, device="cuda")
    dl = torch.ones(w.n_envs, dtype=torch.float32, device="cuda")
    ws_buf = sim.workspace()
    env_steps = float(np.sum(w.T_env))

    def one_step(ev=None):
        r = sim.rollout(x0, u, want_ckpt=True, want_final=False)
        if ev is not None:
            ev[0].record()
        g = sim.rollout_grad(x0, u, r["ckpt"], dl, workspace=ws_buf)
        if ev is not None:
            ev[1].record()
        return r, g

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    mk = lambda: torch.cuda.Event(enable_timing=True)   # noqa: E731
    evs = [(mk(), mk()) for _ in range(args.steps)]
    fwd_evs = [(mk(), mk()) for _ in range(args.steps)]
    # rollout_grad's phases (recompute, reverse sweep), recorded by the library
    # on the launch stream
    phase_evs = [[mk() for _ in range(4)] for _ in range(args.steps)]
    for e in [e for p in phase_evs for e in p]:
        e.record()   # creates the event
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        fwd_evs[k][0].record()
        r = sim.rollout(x0, u, want_ckpt=True, want_final=False)
        fwd_evs[k][1].record()
        sim.time_grad(phase_evs[k])
        evs[k][0].record()
        g = sim.rollout_grad(x0, u, r["ckpt"], dl, workspace=ws_buf)
        evs[k][1].record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.time_grad(None)
    ms_per_step = el * 1e3 / args.steps
    grad_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    fwd_ms = float(np.mean([a.elapsed_time(b) for a, b in fwd_evs]))
    rec_ms = float(np.mean([p[0].elapsed_time(p[1]) for p in phase_evs]))
    rev_ms = float(np.mean([p[2].elapsed_time(p[3]) for p in phase_evs]))
    mode = {1: "replay", 2: "segment", 3: "trajectory"}[sim.info.grad_store]
    value = env_steps / (el / args.steps)
    flags = r["flags"].cpu().numpy()[: w.n_envs]

    check, n_checked, horizon = None, None, None
    if not args.no_check:
        if args.workload == "arms":
            check, n_checked = grad_check(w, g["g_u"].cpu().numpy().astype(np.float64),
                                          g["g_x0"].cpu().numpy().T.astype(np.float64))
            horizon = int(w.T_max)
        else:
            # contact-rich chains and the legged robot are chaotic over the full
            # horizon; the controller's weight gradient is a sum over all envs
            horizon = CHECK_HORIZON
            check, n_checked = grad_check_short(w, horizon)
    fl_fwd, fl_rev = flops_per_env_step(w)
    by = algorithmic_bytes_per_env_step(w)
    # algorithmic flops of the reverse sweep kernel per env-step: the reverse,
    # plus the forward it recomputes (segment mode) and replays (replay mode)
    rev_kernel_flops = fl_rev + {"trajectory": 0, "segment": 1, "replay": 2}[mode] * fl_fwd
    achieved_tflops = rev_kernel_flops * env_steps / (rev_ms * 1e-3) / 1e12
    rec_tflops = fl_fwd * env_steps / (rec_ms * 1e-3) / 1e12 if mode == "trajectory" else None
    hbm_gbs = by["total"] * env_steps / (el / args.steps) / 1e9
    from paper_1611_01652_amd import traffic as TR
    traffic = TR.load(args.workload)   # None unless measured on the current kernel sources
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": {"arms": "planar-arms", "chains": "uneven-chains",
                                "quadruped": "quadruped-mlp-controller"}[args.workload],
                   "envs": w.n_envs, "T": int(w.T_max), "bodies": w.n_bodies, "joints": w.n_joints,
                   "pgs_iters": w.n_iters, "dt": w.dt, "ckpt_every": w.ckpt_every,
                   "parallelism": "single GPU, envs over one-wave workgroups"},
        "fwd_env_steps_per_s": env_steps / (fwd_ms * 1e-3),
        "fwd_ms": fwd_ms,
        "grad_ms": grad_ms,
        "grad_store": mode,
        "grad_phases_ms": {"recompute": rec_ms, "reverse": rev_ms},
        "grad_check": {"max_rel_err": check, "envs": None if check is None else n_checked, "horizon": horizon,
                       "tolerance": 1e-3, "ok": None if check is None else bool(check <= 1e-3)},
        "env_flags_nonzero": int((flags != 0).sum()),
        "roofline": {"bound": "alu", "kernel": "k_rollout_grad", "achieved": achieved_tflops,
                     "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "flops_per_env_step": {"forward": fl_fwd, "reverse": fl_rev, "kernel": rev_kernel_flops},
                     "kernel_ms": rev_ms},
        "recompute_roofline": None if rec_tflops is None else {
            "bound": "alu", "kernel": "k_recompute", "achieved": rec_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": rec_tflops / FP32_VECTOR_PEAK_TFLOPS, "kernel_ms": rec_ms},
        "hbm_roofline": {"achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm_gbs / HBM_PEAK_GBS,
                         "bytes_per_env_step": by["total"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
