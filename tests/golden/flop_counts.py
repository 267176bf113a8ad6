"""Writes flop_counts.json: algorithmic operations per env-step of the
benchmark workloads, counted by the FP64 oracle (its counting scalar for the
forward step, twice the edges of its reverse-mode tape for the reverse), for
one env of each body count, averaged over a few steps of that env's own
trajectory.  Calls only the oracle; the benchmark reads the stored counts.

    python tests/golden/flop_counts.py
"""
from __future__ import annotations

import functools
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "flop_counts.json")
TIMES = (0, 100, 250, 400)


NAMES = ("arms", "chains", "quadruped")


@functools.lru_cache(maxsize=None)
def workload(name):
    """The benchmark's workload of that name (the same seeded generator)."""
    from paper_1611_01652_amd import workloads as W
    if name == "arms":
        return W.planar_arms(n_envs=4096, T=1000)
    if name == "chains":
        return W.uneven_chains(n_envs=16384, T=500)
    return W.quadruped(n_envs=1024)


def count(w, B, times=TIMES):
    """(forward, reverse) operations per env-step for the first env with B bodies."""
    from oracle import Oracle
    nb = np.diff(w.env_body_off)
    e = int(np.where(nb == B)[0][0])
    Tm = int(w.T_env[e])
    ts = sorted(set(min(t, max(Tm - 1, 0)) for t in times))
    ws = w.subset([e]).with_steps(max(ts) + 1)
    o = Oracle(ws)
    tr = o.rollout(traj=True)["traj"]
    f = r = 0.0
    for t in ts:
        u = ws.u[t] if ws.u is not None and ws.u.size else None
        f += o.count_flops(0, x=tr[t], u=u, t=t)
        r += 2 * o.count_tape_edges(0, x=tr[t], u=u, t=t)
    return f / len(ts), r / len(ts)


def main():
    out = {"note": "operations per env-step by body count: [forward, reverse]", "times": list(TIMES)}
    for name in NAMES:
        w = workload(name)
        sizes = sorted(set(np.diff(w.env_body_off).tolist()))
        out[name] = {str(B): list(count(w, B)) for B in sizes}
        print(name, len(sizes), "body counts", flush=True)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
