"""Benchmark: forward + adjoint env-steps/s of the batched rigid-body step.

One "step" of this benchmark is one pass of the whole hot path over the
workload: `rollout` (T time steps of every env, with checkpoints) followed by
`rollout_grad` (recompute from the checkpoints + hand-written reverse sweep),
i.e. E * T env-steps forward and backward.  Inputs are resident in HBM before
the timed region.  The default workload is the largest single-GPU one: 16384
uneven 3D hinge chains of 2..32 spheres with ground and self contact, 500
steps (synthetic, seeded).  `--workload arms` runs the 4096 planar 3-link arms
x 1000 steps, `--workload quadruped` the 1024 legged robots with an MLP
controller.  `--workload camera` measures the differentiable camera instead
(section 3.4): one step is an image of every env at the paper's frame size
and the gradient of a weighted sum of it with respect to the bodies' poses.

Printed: one JSON line with the throughput, a roofline object for the
reverse sweep kernel of one call (one launch per size bucket, all running at
once; timed by events the library records around them, and each bucket's
launch on its own stream), a gradient check of the timed launch's own
gradients against the FP64 oracle, and the oracle's own CPU throughput on a
bounded sample.  The
oracle runs only in the CPU-baseline leg: its timed full-horizon run over the
sampled envs is also the reference of the gradient check.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# The size buckets of an uneven workload run at once, one stream each.  HIP
# maps streams onto GPU_MAX_HW_QUEUES hardware queues (4 unless set, and
# machines may export 4), and the kernels of streams that share a queue run
# one after another: 16 buckets on 4 queues run as 4 serial chains (measured:
# 1988 ms per chains step against 1896 ms with a queue per bucket).  Give
# every bucket a queue of its own: at least 32 (read once, when HIP starts).
if int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0) < 32:
    os.environ["GPU_MAX_HW_QUEUES"] = "32"

METRIC = "fwd+adjoint env-steps/s at grad rel-err<=1e-3 vs FP64 oracle; % HBM roofline"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
GRAD_TOL = 1e-3
NOISE = 2.0 ** -24            # FP32-sized relative noise of the oracle's conditioning runs
WORKLOAD_NAMES = {"arms": "planar-arms", "chains": "uneven-chains", "quadruped": "quadruped-mlp-controller"}


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


def stratified(w, n):
    """n envs at evenly spaced quantiles of the body count (ties by index)."""
    nb = np.diff(w.env_body_off)
    order = np.argsort(nb, kind="stable")
    n = min(n, w.n_envs)
    return sorted(set(order[((np.arange(n) + 0.5) / n * len(order)).astype(int)].tolist()))


def cpu_threads():
    """Worker threads for the oracle: the CPUs this process may run on, at
    most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except Exception:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def physical_cores():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        cps = int(re.search(r"Core\(s\) per socket:\s+(\d+)", out).group(1))
        soc = int(re.search(r"Socket\(s\):\s+(\d+)", out).group(1))
        return cps * soc
    except Exception:
        return None


# ---------------------------------------------------------------- algorithmic counts
def stored_counts(name):
    """Operations per env-step by body count, {bodies: (forward, reverse)}, as
    the oracle's counters gave them (tests/golden/flop_counts.py writes them)."""
    with open(os.path.join(ROOT, "tests", "golden", "flop_counts.json")) as fh:
        d = json.load(fh)[name]
    return {int(k): tuple(v) for k, v in d.items()}


def algorithmic_bytes_per_env_step(w):
    """Bytes a step must move if it were its own kernel with the state in HBM
    (struct-of-arrays), per env of the workload on average: state in/out,
    warm-start impulses in/out, torques in, checkpoint writes / K_ck; the
    adjoint adds the recompute (a forward plus the segment buffer write) and
    the reverse sweep (segment buffer read, state and impulse adjoints in/out,
    torques in, torque adjoints out)."""
    E = w.n_envs
    nb = w.n_bodies / E
    nj = w.n_joints / E
    lam = 5 * nj
    if w.ground:
        lam += 4 * (w.sphere_flags & 1).sum() / E
    state = 72 * nb
    fwd = 2 * state + 2 * 4 * lam + 4 * nj + (state + 4 * lam) / w.ckpt_every
    seg = state + 4 * lam
    rev = seg + 2 * state + 2 * 4 * lam + 4 * nj + 4 * nj
    return dict(fwd=fwd, grad_kernel=fwd + seg + rev, total=fwd + fwd + seg + rev)


# ---------------------------------------------------------------- gradient check
GRAD_KEYS = ("g_x0", "g_u", "g_inv_mass", "g_inv_inertia", "g_mu", "g_damping", "g_anchor_p", "g_anchor_c")


def _rel(a, b, floor=0.0):
    """|a - b| / max(|b|, floor), absolute below 1e-8."""
    n = max(float(np.linalg.norm(b)), floor)
    d = np.linalg.norm(np.asarray(a) - np.asarray(b))
    return d / n if n >= 1e-8 else d


# An array far below the env's state gradient |dL/dx0| (e.g. dL/du of a servo
# at its limit on all but a few steps) is compared against 1e-5 of that scale:
# FP32 forms every array from adjoints of that size.
GRAD_SCALE_FLOOR = 1e-5


def _env_grads(g, w, e, local_b, local_j, local_e):
    """Gradient arrays of one env: g holds the arrays of the workload w, the
    env's bodies / joints / index in it are local_b / local_j / local_e."""
    out = {}
    for k in GRAD_KEYS:
        if k not in g:
            continue
        if k == "g_u":
            out[k] = g[k][:, local_j]
        elif k == "g_mu":
            out[k] = g[k][local_e:local_e + 1]
        elif k in ("g_damping", "g_anchor_p", "g_anchor_c"):
            out[k] = g[k][local_j]
        else:
            out[k] = g[k][local_b]
    return out


def grad_check(w, envs, got, ref, noisy):
    """The timed launch's gradients (got, arrays of the whole workload) against
    the oracle's (ref, of the sampled envs `envs` as their own workload), on
    the sampled envs whose oracle gradient is stable under FP32-sized noise
    (each of `noisy` within half the tolerance): over the full horizon the
    others are chaotic, FP32 and FP64 trajectories part and so do their
    gradients.  Every array the call returns is compared."""
    ws = w.subset(envs)
    nb = np.diff(w.env_body_off)
    stable, errs = [], []
    for i, e in enumerate(envs):
        lb = np.arange(ws.env_body_off[i], ws.env_body_off[i + 1])
        lj = np.arange(ws.env_joint_off[i], ws.env_joint_off[i + 1])
        r = _env_grads(ref, ws, i, lb, lj, i)
        fl = GRAD_SCALE_FLOOR * float(np.linalg.norm(r["g_x0"]))
        if any(max((_rel(_env_grads(g, ws, i, lb, lj, i)[k], r[k], fl) for k in r if r[k].size), default=0.0)
               >= 0.5 * GRAD_TOL for g in noisy):
            continue
        gb = np.arange(w.env_body_off[e], w.env_body_off[e + 1])
        gj = np.arange(w.env_joint_off[e], w.env_joint_off[e + 1])
        a = _env_grads(got, w, e, gb, gj, e)
        stable.append(e)
        errs.append(max((_rel(a[k], r[k], fl) for k in r if r[k].size), default=0.0))
    worst = max(errs) if errs else None
    errs = np.array(errs)
    beyond = [(int(stable[i]), int(nb[stable[i]]), float(errs[i])) for i in np.argsort(-errs) if errs[i] > GRAD_TOL]
    return {"max_rel_err": worst, "tolerance": GRAD_TOL, "ok": None if worst is None else bool(worst <= GRAD_TOL),
            "horizon": int(w.T_max), "sampled_envs": len(envs), "envs_checked": len(stable),
            "envs_within_tolerance": int((errs <= GRAD_TOL).sum()),
            "median_rel_err": float(np.median(errs)) if len(errs) else None,
            "beyond_tolerance": beyond[:8],
            "bodies_of_checked": sorted(set(nb[stable].tolist())) if stable else [],
            "arrays": [k for k in GRAD_KEYS if k in got],
            "criterion": f"sampled envs whose oracle gradient moves by less than half the tolerance under "
                         f"FP32-sized noise ({len(noisy)} draws); the rest are beyond their non-chaotic horizon"}


# ---------------------------------------------------------------- CPU baseline
def cpu_baseline(w, n_envs=256, per_core_seconds=5.0, noisy_draws=8):
    """The oracle (FP64, tape reverse mode) on the host cores, forward +
    gradient of the full horizon, on n_envs envs of the workload at evenly
    spaced quantiles of the body count; the per-core figure comes from one
    thread on a quarter of the sample.  The run's gradients, and those of
    `noisy_draws` runs with FP32-sized noise (untimed), are returned as the
    reference of the gradient check."""
    from oracle import Oracle
    threads = cpu_threads()
    envs = stratified(w, n_envs)
    ws = w.subset(envs)
    o = Oracle(ws)
    t0 = time.time()
    o.rollout(threads=threads)
    ref = o.rollout_grad(threads=threads)
    el = time.time() - t0
    value = float(np.sum(ws.T_env)) / el
    sub = [envs[i] for i in range(0, len(envs), 4)]
    wp = w.subset(sub)
    cal = 5
    t1 = time.time()
    op = Oracle(wp.with_steps(cal))
    op.rollout(threads=1)
    op.rollout_grad(threads=1)
    pstep = (time.time() - t1) / cal
    Tp = int(max(cal, min(w.T_max, per_core_seconds / max(pstep, 1e-9))))
    op = Oracle(wp.with_steps(Tp))
    t1 = time.time()
    op.rollout(threads=1)
    op.rollout_grad(threads=1)
    elp = time.time() - t1
    per_core = float(np.minimum(np.asarray(wp.T_env), Tp).sum()) / elp
    noisy = [Oracle(ws, noise=NOISE, noise_seed=k).rollout_grad(threads=threads) for k in range(noisy_draws)]
    base = {"value": value, "unit": "env-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(envs)} envs at evenly spaced quantiles of the body count, full horizon "
                      f"({int(np.sum(ws.T_env))} env-steps), forward + tape gradient, FP64, {threads} threads; "
                      f"per core: {len(sub)} of them x {Tp} steps on one thread",
            "seconds": el, "per_core": per_core, "all_core": value, "threads": threads,
            "nproc": os.cpu_count(), "physical_cores": physical_cores()}
    return base, envs, ref, noisy


# ---------------------------------------------------------------- camera
# Operations of a pixel's ray as the renderer defines it, counted from its
# arithmetic: the ray through the pixel centre and |d|^2 (26), then per
# sphere of the env the centre p + R o (18), the ray's closest approach to it
# and the discriminant (24), the root (3); the ground's hit parameter (1).
# Shading the hit (<= 55, the gradient's adjoint <= 139) is not counted, so
# the achieved rate is a lower bound.
CAM_RAY_FLOPS, CAM_SPHERE_FLOPS = 27, 45


def camera_scene(n_envs=1024, seed_salt=12):
    """Envs of the chain distribution with 2..16 spheres at their initial
    poses, seen from the side and above at the paper's 288 x 96 frame, with
    seeded smooth textures."""
    from paper_1611_01652_amd import workloads as W
    rng = np.random.default_rng(seed_salt)
    w = W.uneven_chains(n_envs=n_envs, T=4, seed_salt=seed_salt, sizes=rng.integers(2, 17, n_envs))
    cam = W.pinhole_camera((0.3, -3.5, 1.6), (0.0, 0.0, 0.3), focal=1.0, pitch=1.6 / 288, width=288, height=96)
    return w, cam, W.synthetic_texture(64, 32, 5), W.synthetic_texture(64, 64, 6), 0.25


def camera_cpu_baseline(w, cam, ts, tg, cell, n_envs=16):
    """The oracle's image and gradient (FP64, tape reverse mode) on n_envs
    envs at evenly spaced quantiles of the sphere count, one thread."""
    from oracle import Camera, Oracle
    envs = stratified(w, n_envs)
    ws = w.subset(envs)
    o = Oracle(ws)
    c = Camera()
    c.pos[:] = [float(v) for v in cam["pos"]]
    c.axes[:] = [float(v) for v in np.asarray(cam["axes"]).reshape(9)]
    c.focal, c.pitch, c.width, c.height = cam["focal"], cam["pitch"], cam["width"], cam["height"]
    t0 = time.time()
    img = o.render(c, ts, tg, cell)
    o.render_grad(c, ts, tg, cell, np.ones_like(img))
    el = time.time() - t0
    return {"value": img.size / el, "unit": "pixels/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(envs)} envs at evenly spaced quantiles of the sphere count, image and gradient of "
                      f"the sum of the image, {cam['width']} x {cam['height']}, FP64, one thread",
            "seconds": el, "nproc": os.cpu_count(), "physical_cores": physical_cores()}


def bench_camera(args):
    import torch
    from paper_1611_01652_amd.sim import Simulator
    w, cam, ts, tg, cell = camera_scene()
    sim = Simulator(w)
    xd = torch.tensor(np.ascontiguousarray(w.x0.T), dtype=torch.float32, device="cuda")
    tsd = torch.tensor(ts, dtype=torch.float32, device="cuda")
    tgd = torch.tensor(tg, dtype=torch.float32, device="cuda")
    print(f"bench: camera {w.n_envs} envs x {cam['width']} x {cam['height']}", file=sys.stderr, flush=True)
    img = sim.render(xd, cam, tsd, tgd, cell)
    wd = torch.ones_like(img)
    g = sim.render_grad(xd, cam, tsd, tgd, cell, wd)
    for _ in range(args.warmup):
        sim.render(xd, cam, tsd, tgd, cell, out=img)
        sim.render_grad(xd, cam, tsd, tgd, cell, wd, out=g)
    torch.cuda.synchronize()
    mk = lambda: torch.cuda.Event(enable_timing=True)   # noqa: E731
    evs = [[mk() for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        # both calls launch on torch's current stream, where the events sit
        evs[k][0].record()
        sim.render(xd, cam, tsd, tgd, cell, out=img)
        evs[k][1].record()
        g = sim.render_grad(xd, cam, tsd, tgd, cell, wd, out=g)
        evs[k][2].record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    print("bench: timed region done", file=sys.stderr, flush=True)
    render_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    grad_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    n_pix = img.numel()
    ns = np.diff(w.env_sphere_off)
    flops = float(cam["width"] * cam["height"] * (CAM_RAY_FLOPS + CAM_SPHERE_FLOPS * ns).sum())
    from paper_1611_01652_amd import traffic as TR
    # HBM bytes per launch from the counters (None unless measured on the
    # current kernel sources)
    traffic = {"k_render_grad": TR.load("camera"), "k_render": TR.load_other("camera", "k_render", 1)}
    roof = lambda ms, name: {   # noqa: E731
        "bound": "alu", "kernel": name, "achieved": flops / (ms * 1e-3) / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s", "frac": flops / (ms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic[name],
        "flops_per_launch": flops, "kernel_ms": ms}
    line = {
        "metric": "camera image + gradient pixels/s", "value": n_pix / (el / args.steps), "unit": "pixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "camera", "envs": w.n_envs, "width": cam["width"], "height": cam["height"],
                   "spheres": int(ns.sum()), "pixels": n_pix},
        "render_ms": render_ms, "render_grad_ms": grad_ms,
        "image_pixels_per_s": n_pix / (render_ms * 1e-3), "gradient_pixels_per_s": n_pix / (grad_ms * 1e-3),
        "roofline": roof(grad_ms, "k_render_grad") if grad_ms >= render_ms else roof(render_ms, "k_render"),
        "render_roofline": roof(render_ms, "k_render"),
        "render_grad_roofline": roof(grad_ms, "k_render_grad"),
        "finite": bool(torch.isfinite(img).all().item() and torch.isfinite(g).all().item()),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = camera_cpu_baseline(w, cam, ts, tg, cell)
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chains", choices=["arms", "chains", "quadruped", "camera"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-keep", action="store_true",
                    help="in trajectory mode, recompute the working sets from the checkpoints instead of keeping "
                         "them in the rollout")
    ap.add_argument("--fuse", action="store_true",
                    help="with kept working sets, call rollout_and_grad (each bucket's reverse right after its own "
                         "forward) instead of rollout_keep and rollout_grad_kept one after the other")
    ap.add_argument("--tune", metavar="CACHE", default=None,
                    help="team widths from the tune cache at CACHE (JSON); when the model is not in it yet, tuned "
                         "on the whole forward + gradient call (one bucket's width at a time) and stored there")
    ap.add_argument("--tune-steps", type=int, default=None,
                    help="time the tuning trials on a copy of the workload cut to this many steps (default: the "
                         "full horizon; shorter copies measured to mislead for the chains)")
    ap.add_argument("--grad-mem-gib", type=float, default=None,
                    help="memory for the reverse sweep's saved working sets (default: what the device has free "
                         "less a 12 GiB margin)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                                   "(sharding over GPUs is a design note, not implemented)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "camera":
        bench_camera(args)
        return

    import torch
    from paper_1611_01652_amd.sim import Simulator

    w = make_workload(args.workload)
    # the reverse sweep keeps every step's working set when the device's memory
    # allows (recomputed in one parallel pass), else one segment's at a time
    free, _ = torch.cuda.mem_get_info()
    gib = args.grad_mem_gib if args.grad_mem_gib is not None else max(1.0, free / 2**30 - 12.0)
    w.extra = dict(w.extra or {})
    w.extra["grad_mem_limit"] = int(gib * 2**30)
    sim = Simulator(w)
    teams_from = "default"
    if args.tune:
        from paper_1611_01652_amd import tune_cache as TC
        dev_u = lambda ws: torch.tensor(np.ascontiguousarray(controls(ws)), dtype=torch.float32,  # noqa: E731
                                        device="cuda")
        _, teams_from = TC.tuned_teams(
            sim, dev_u, args.tune, short_T=args.tune_steps,
            log=lambda t, ms: print(f"bench: tune trial {t}: {ms:.1f} ms", file=sys.stderr, flush=True))
    print(f"bench: {args.workload} {w.n_envs} envs x {w.T_max} steps, {len(sim.teams())} buckets, teams "
          f"{sim.teams().tolist()} ({teams_from})", file=sys.stderr, flush=True)
    x0 = torch.tensor(np.ascontiguousarray(w.x0.T), dtype=torch.float32, device="cuda")
    u = torch.tensor(np.ascontiguousarray(controls(w)), dtype=torch.float32, device="cuda")
    dl = torch.ones(w.n_envs, dtype=torch.float32, device="cuda")
    ws_buf = sim.workspace()
    env_steps = float(np.sum(w.T_env))
    # trajectory mode: the rollout keeps every step's working set in the
    # workspace and the reverse reads them without recomputing them
    keep = ws_buf if sim.info.grad_store == 3 and not args.no_keep else None
    fused = keep is not None and args.fuse

    def one_step():
        if fused:
            return sim.rollout_and_grad(x0, u, dl, keep)
        r = sim.rollout(x0, u, want_ckpt=True, want_final=False, keep=keep)
        return r, sim.rollout_grad(x0, u, r["ckpt"], dl, workspace=ws_buf, kept=keep)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    mk = lambda: torch.cuda.Event(enable_timing=True)   # noqa: E731
    n_b = len(sim.teams())
    evs = [(mk(), mk()) for _ in range(args.steps)]
    fwd_evs = [(mk(), mk()) for _ in range(args.steps)]
    # rollout_grad's phases and each bucket's reverse kernel, recorded by the
    # library on the streams the kernels run on
    phase_evs = [[mk() for _ in range(4)] for _ in range(args.steps)]
    bucket_evs = [[mk() for _ in range(2 * n_b)] for _ in range(args.steps)]
    for e in [e for p in phase_evs + bucket_evs for e in p]:
        e.record()   # creates the event
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        sim.time_grad(phase_evs[k])
        sim.time_buckets(bucket_evs[k])
        if fused:
            # one call: the "reverse" phase events span it
            fwd_evs[k][0].record()
            r, g = sim.rollout_and_grad(x0, u, dl, keep)
            fwd_evs[k][1].record()
            evs[k][0].record()
            evs[k][1].record()
        else:
            fwd_evs[k][0].record()
            r = sim.rollout(x0, u, want_ckpt=True, want_final=False, keep=keep)
            fwd_evs[k][1].record()
            evs[k][0].record()
            g = sim.rollout_grad(x0, u, r["ckpt"], dl, workspace=ws_buf, kept=keep)
            evs[k][1].record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.time_grad(None)
    sim.time_buckets(None)
    print("bench: timed region done", file=sys.stderr, flush=True)
    ms_per_step = el * 1e3 / args.steps
    grad_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    fwd_ms = float(np.mean([a.elapsed_time(b) for a, b in fwd_evs]))
    call_ms = fwd_ms if fused else None
    if fused:
        # the forward's own rate: the keeping rollout alone, after the timed
        # region (the fused call cannot separate it)
        fe = [(mk(), mk()) for _ in range(args.steps)]
        for a_, b_ in fe:
            a_.record()
            sim.rollout(x0, u, want_ckpt=False, want_final=False, keep=keep)
            b_.record()
        torch.cuda.synchronize()
        fwd_ms, grad_ms = float(np.mean([a.elapsed_time(b) for a, b in fe])), None
    rec_ms = float(np.mean([p[0].elapsed_time(p[1]) for p in phase_evs]))
    rev_ms = float(np.mean([p[2].elapsed_time(p[3]) for p in phase_evs]))
    bucket_ms = np.array([[p[2 * i].elapsed_time(p[2 * i + 1]) for i in range(n_b)] for p in bucket_evs]).mean(0)
    mode = {1: "replay", 2: "segment", 3: "trajectory"}[sim.info.grad_store]
    value = env_steps / (el / args.steps)
    flags = r["flags"].cpu().numpy()[: w.n_envs]

    # algorithmic flops: per body count, the oracle's counts (stored)
    counts = stored_counts(args.workload)
    nb = np.diff(w.env_body_off)
    T_env = np.asarray(w.T_env, dtype=np.float64)
    f_fwd = np.array([counts[b][0] for b in nb])
    f_rev = np.array([counts[b][1] for b in nb])
    # the reverse sweep kernel recomputes (segment mode) or replays (replay
    # mode) the forward besides reversing it
    k_fwd = {"trajectory": 0, "segment": 1, "replay": 2}[mode]
    kern_flops_env = (f_rev + k_fwd * f_fwd) * T_env
    # the fused call's span holds the forward kernels too
    call_flops_env = kern_flops_env + (f_fwd * T_env if fused else 0.0)
    of_env = sim.env_buckets()
    bucket_flops = np.array([kern_flops_env[of_env == i].sum() for i in range(n_b)])
    dom = int(np.argmax(bucket_ms))
    teams = sim.teams()
    achieved = bucket_flops[dom] / (bucket_ms[dom] * 1e-3) / 1e12
    phase_tflops = call_flops_env.sum() / (rev_ms * 1e-3) / 1e12
    # (a forward that keeps the working sets leaves the reverse no recompute)
    rec_tflops = float((f_fwd * T_env).sum() / (rec_ms * 1e-3) / 1e12) if mode == "trajectory" and keep is None \
        else None
    by = algorithmic_bytes_per_env_step(w)
    hbm_gbs = by["total"] * env_steps / (el / args.steps) / 1e9
    from paper_1611_01652_amd import traffic as TR
    # (None unless measured on the current kernel sources)
    traffic = TR.load(args.workload, all_buckets=True)
    traffic_dom = TR.load(args.workload, bucket=dom)
    if fused and traffic is not None:
        # the fused call's span holds the forward kernels' launches too
        fwd_traffic = TR.load_other(args.workload, "k_rollout_keep", n_b)
        traffic = None if fwd_traffic is None else traffic + fwd_traffic

    got = None
    if not args.no_check and args.workload != "quadruped":
        got = {k: g[k].cpu().numpy().astype(np.float64) for k in GRAD_KEYS if k != "g_x0"}
        got["g_x0"] = g["g_x0"].cpu().numpy().T.astype(np.float64)
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
        "config": {"workload": WORKLOAD_NAMES[args.workload],
                   "envs": w.n_envs, "T": int(w.T_max), "bodies": w.n_bodies, "joints": w.n_joints,
                   "pgs_iters": w.n_iters, "dt": w.dt, "ckpt_every": w.ckpt_every,
                   "parallelism": "single GPU, envs over one-wave workgroups, size buckets on concurrent streams",
                   "teams": teams_from},
        "fwd_env_steps_per_s": env_steps / (fwd_ms * 1e-3),
        "fwd_ms": fwd_ms,
        "grad_ms": grad_ms,
        "grad_store": mode,
        "forward_keeps_working_sets": keep is not None,
        "fused_call": fused,
        "fused_call_ms": call_ms,
        "grad_phases_ms": {"recompute": rec_ms, "reverse": rev_ms},
        "grad_check": None,
        "env_flags_nonzero": int((flags != 0).sum()),
        # the reverse kernel of one call: one launch per size bucket, all
        # running at once on forked streams and sharing the CUs, timed from
        # the first launch's start to the last one's end
        "roofline": {"bound": "alu", "kernel": (f"k_rollout_keep + k_rollout_grad ({n_b} concurrent bucket "
                                                "pipelines, one rollout_and_grad call)") if fused else
                     f"k_rollout_grad ({n_b} concurrent bucket launches)"
                     if n_b > 1 else f"k_rollout_grad<{int(teams[0])}, {0 if mode == 'replay' else 1}>",
                     "achieved": phase_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": phase_tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "flops_per_launch": float(call_flops_env.sum()), "kernel_ms": rev_ms},
        # the longest of those launches, timed on its own stream (its share
        # of the CUs varies as the other buckets start and finish)
        "dominant_launch": {"kernel": f"k_rollout_grad<{int(teams[dom])}, {0 if mode == 'replay' else 1}>",
                            "bucket": dom, "bucket_envs": int((of_env == dom).sum()), "achieved": achieved,
                            "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic_dom,
                            "flops_per_launch": float(bucket_flops[dom]), "kernel_ms": float(bucket_ms[dom])},
        "buckets": [{"team": int(teams[i]), "envs": int((of_env == i).sum()), "reverse_ms": float(bucket_ms[i]),
                     "tflops": float(bucket_flops[i] / (bucket_ms[i] * 1e-3) / 1e12)} for i in range(n_b)],
        "flops_per_env_step": {"forward": float((f_fwd * T_env).sum() / env_steps),
                               "reverse": float((f_rev * T_env).sum() / env_steps)},
        "recompute_roofline": None if rec_tflops is None else {
            "bound": "alu", "kernel": "k_recompute", "achieved": rec_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": rec_tflops / FP32_VECTOR_PEAK_TFLOPS, "kernel_ms": rec_ms},
        "hbm_roofline": {"achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm_gbs / HBM_PEAK_GBS,
                         "bytes_per_env_step": by["total"]},
    }
    if not args.no_cpu_baseline:
        base, envs, ref, noisy = cpu_baseline(w)
        line["cpu_baseline"] = base
        if got is not None:
            line["grad_check"] = grad_check(w, envs, got, ref, noisy)
        print("bench: cpu baseline and gradient check done", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
