"""A persisted cache of the tile autotuner's choices.

`sim_tune` times each size bucket of a model at the team widths its LDS
admits and keeps the fastest (results do not depend on the width).  Tuning
costs a rollout and a gradient per candidate, so the widths are stored in a
JSON file under a key of what they depend on: the model's bucket structure
(each env's bucket and the default widths), the envs' body counts, the solver
sweeps, the reverse sweep's memory mode, the device and the library's ABI
version.  A model seen before gets its widths back without timing anything.

Two objectives.  "bucket": sim_tune, each bucket timed alone.  "call": the
buckets of a model run at once on their own streams and share the CUs, so a
bucket's time alone is not what the call takes; this objective times the
whole forward + gradient call and changes one bucket's width at a time
(coordinate descent over the buckets in bucket order), keeping a change
only when the call gets faster by more than `gain` (5 %: calls of the
16384-chain model vary by about 3 % from run to run).

A bucket's work grows linearly with the horizon while its tiles do not
depend on it, so a model is tuned on a copy of itself cut to a short horizon
whose buckets are the same (checked: same default widths, same bucket for
every env); the widths then apply to the full horizon.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np


def cache_key(sim) -> str:
    """The key of a model's tuning: what the fastest widths depend on."""
    import torch
    from . import sim as S
    w = sim.w
    h = hashlib.sha256()
    for a in (sim.teams(), sim.env_buckets(), np.diff(np.asarray(w.env_body_off))):
        h.update(np.ascontiguousarray(a, dtype=np.int64).tobytes())
    dev = torch.cuda.get_device_name(torch.cuda.current_device()) if torch.cuda.is_available() else "none"
    h.update(json.dumps([int(w.n_iters), int(sim.info.grad_store), S.ABI_VERSION, dev]).encode())
    return h.hexdigest()[:24]


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def call_ms(sim, x0, u, reps=2):
    """Milliseconds of one forward + gradient call of the whole model (the
    rollout keeping the working sets in trajectory mode), the best of reps."""
    import torch
    dl = torch.ones(sim.info.n_envs, device="cuda")
    ws = sim.workspace()
    keep = ws if sim.info.grad_store == 3 else None
    best = None
    for k in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        r = sim.rollout(x0, u, want_final=False, keep=keep)
        sim.rollout_grad(x0, u, r["ckpt"], dl, workspace=ws, kept=keep)
        b.record()
        torch.cuda.synchronize()
        if k:   # (the first call warms up)
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
    del ws
    return best


def tune_call(sim, x0, u, gain=0.05, reps=2, log=None):
    """Coordinate descent over the buckets' team widths on the whole call's
    time; returns the widths it keeps (and leaves them set).  log, if given,
    is called with (widths, ms) after every timed trial."""
    from .sim import SimError
    teams = sim.teams().copy()
    best = call_ms(sim, x0, u, reps)
    if log is not None:
        log(teams.tolist(), best)
    for i in range(len(teams)):
        t = int(teams[i]) * 2
        while t <= 64:
            trial = teams.copy()
            trial[i] = t
            try:
                sim.set_teams(trial)
            except SimError:
                break
            ms = call_ms(sim, x0, u, reps)
            if log is not None:
                log(trial.tolist(), ms)
            if ms < best * (1.0 - gain):
                best, teams = ms, trial
            t *= 2
        sim.set_teams(teams)
    return teams


def tuned_teams(sim, make_controls, path, short_T=50, with_grad=True, max_candidates=3, objective="call",
                log=None):
    """Team widths for `sim` from the cache at `path`, tuning and storing them
    when the model is not there yet, and applies them (sim_set_teams).
    make_controls(w) gives the control input of a workload w on the device
    (the tape or the controller's weights).  objective: "call" (the whole
    call timed, with the gradient) or "bucket" (sim_tune).  short_T: the
    horizon of the copy that is timed (None: the model itself).  log: as
    tune_call's.  Returns (widths, "cache" or "tuned")."""
    import torch
    from .sim import Simulator
    if objective not in ("call", "bucket"):
        raise ValueError("objective must be 'call' or 'bucket'")
    key = cache_key(sim) + ":" + objective
    cache = _load(path)
    if key in cache:
        teams = np.asarray(cache[key]["teams"], np.int32)
        sim.set_teams(teams)
        return teams, "cache"
    w = sim.w
    ws = w.with_steps(min(int(short_T), int(w.T_max))) if short_T else w
    tuner = Simulator(ws) if short_T else sim
    try:
        same = (np.array_equal(tuner.teams(), sim.teams()) and np.array_equal(tuner.env_buckets(), sim.env_buckets()))
        if not same:
            # the short copy tiles differently: tune the model itself
            tuner.close()
            tuner, ws = sim, w
        x0 = torch.tensor(np.ascontiguousarray(ws.x0.T), dtype=torch.float32, device="cuda")
        if objective == "bucket":
            teams = tuner.tune(x0, make_controls(ws), with_grad=with_grad, max_candidates=max_candidates)
        else:
            teams = tune_call(tuner, x0, make_controls(ws), log=log)
        torch.cuda.synchronize()
    finally:
        if tuner is not sim:
            tuner.close()
    sim.set_teams(teams)
    cache = _load(path)
    cache[key] = {"teams": [int(t) for t in teams], "tuned_on_steps": int(ws.T_max), "envs": int(w.n_envs),
                  "objective": objective}
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1)
    os.replace(tmp, path)
    return teams, "tuned"
