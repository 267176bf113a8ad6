"""TEST INFRASTRUCTURE ONLY: runs the multi-lane host build of the kernel
source (kernel_lanes.cpp) on named cases, each under three lane schedules
(ascending, descending, seeded random), and prints one JSON line per case:
whether the schedules gave the same bits, and the largest relative
difference to the FP64 oracle.  Started by tests/test_kernel_host_lanes.py in
a process of its own (the library may be built with AddressSanitizer)."""
import ctypes as C
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Oracle                                  # noqa: E402
from paper_1611_01652_amd import workloads as W           # noqa: E402
from test_kernel_host_fp64 import _desc64, _rel           # noqa: E402

KEYS = ("loss", "x_final", "g_x0", "g_u", "g_inv_mass", "g_inv_inertia", "g_mu", "g_damping", "g_anchor_p",
        "g_anchor_c")


def _bouncy(w, e, seed):
    w.restitution = np.random.default_rng(seed).uniform(0.0, e, size=w.n_envs).astype(np.float32)
    return w


def _pile(n, T):
    rng = np.random.default_rng(1)
    pos = np.c_[rng.uniform(-0.1, 0.1, (n, 2)), rng.uniform(0.05, 0.2, n)]
    return W.free_spheres(pos, [0.1] * n, [1.0] * n, T=T)


def _store(w, mode):
    w.extra = dict(w.extra or {})
    w.extra["grad_store"] = mode
    return w


CASES = {
    "arms": lambda: W.planar_arms(n_envs=3, T=40),
    "chains": lambda: W.uneven_chains(n_envs=4, T=25, seed_salt=2),
    "chains-replay": lambda: _store(W.uneven_chains(n_envs=3, T=20, seed_salt=4), "replay"),
    "chains-segment": lambda: _store(W.uneven_chains(n_envs=3, T=20, seed_salt=5), "segment"),
    "quadruped": lambda: W.quadruped(n_envs=3, T_min=8, T_max=12,
                                     mlp_w=W.mlp_init(zero_output=False, out_scale=0.3)),
    "quadruped-rec": lambda: W.quadruped(n_envs=3, T_min=8, T_max=12, rec=3,
                                         mlp_w=W.mlp_init(W.rec_sizes(W.MLP_SIZES, 3), zero_output=False,
                                                          out_scale=0.3)),
    "quadruped-wave": lambda: W.quadruped(n_envs=9, T_min=6, T_max=9,
                                          mlp_w=W.mlp_init(zero_output=False, out_scale=0.3)),
    "servo-chains": lambda: W.servo_chains(3, 20),
    "bouncy-chains": lambda: _bouncy(W.uneven_chains(n_envs=2, T=70, seed_salt=6), 0.8, 3),
    "balls": lambda: W.paper_ball_throws(n_envs=3, T=80),
    # 12 overlapping spheres: more active contacts than the env's capacity
    "overflow": lambda: _pile(12, 5),
}
SOLVE_CASES = {
    "solve-learned": lambda: W.warm_start_chains(n_envs=4, T=25, seed_salt=3, ws_w=W.wsn_init(seed_salt=2),
                                                 fb_tol=1e-3),
}


def _lib(path):
    lib = C.CDLL(path)
    lib.kl_rollout_grad.restype = C.c_longlong
    lib.kl_rollout_solve.restype = C.c_longlong
    lib.kl_set_ring.argtypes = [C.c_int]
    return lib


def run_grad(lib, w, sched, seed, min_team, tpw):
    d, keep = _desc64(w)
    E, B, J = w.n_envs, w.n_bodies, w.n_joints
    p = lambda a: a.ctypes.data_as(C.c_void_p)   # noqa: E731
    x0 = np.ascontiguousarray(w.x0.T)
    mlp = w.extra.get("mlp") if getattr(w, "extra", None) else None
    if mlp is not None:
        u = np.ascontiguousarray(np.asarray(mlp["w"], np.float64))
        gu0 = np.zeros(len(u))
    else:
        u = np.ascontiguousarray(w.u if w.u is not None and w.u.size else np.zeros((max(w.T_max, 1), 1)))
        gu0 = np.zeros((max(w.T_max, 1), max(J, 1)))
    out = dict(loss=np.zeros(E), x_final=np.zeros((18, B)), g_x0=np.zeros((18, B)), g_u=gu0,
               g_inv_mass=np.zeros(B), g_inv_inertia=np.zeros((B, 3)), g_mu=np.zeros(E),
               g_damping=np.zeros(max(J, 1)), g_anchor_p=np.zeros((max(J, 1), 3)), g_anchor_c=np.zeros((max(J, 1), 3)))
    err = C.create_string_buffer(512)
    n = lib.kl_rollout_grad(C.byref(d), p(x0), p(u), p(np.ones(E)), p(out["loss"]), p(out["x_final"]),
                            p(out["g_x0"]), p(out["g_u"]), p(out["g_inv_mass"]), p(out["g_inv_inertia"]),
                            p(out["g_mu"]), p(out["g_damping"]), p(out["g_anchor_p"]), p(out["g_anchor_c"]),
                            int(sched), int(seed), int(min_team), int(tpw), err, 512)
    if n < 0:
        raise RuntimeError(err.value.decode())
    out["x_final"] = out["x_final"].T
    out["g_x0"] = out["g_x0"].T
    if mlp is not None:
        out["g_w"] = out.pop("g_u")
    else:
        out["g_u"] = out["g_u"][:, :J]
    for k in ("g_damping", "g_anchor_p", "g_anchor_c"):
        out[k] = out[k][:J]
    return out, n


def run_solve(lib, w, sched, seed, min_team, tpw):
    d, keep = _desc64(w)
    E, B = w.n_envs, w.n_bodies
    p = lambda a: a.ctypes.data_as(C.c_void_p)   # noqa: E731
    x0 = np.ascontiguousarray(w.x0.T)
    u = np.ascontiguousarray(w.u if w.u is not None and w.u.size else np.zeros((max(w.T_max, 1), 1)))
    loss, xf = np.zeros(E), np.zeros((18, B))
    it, fb = np.zeros(E, np.int32), np.zeros(E, np.int32)
    cap = 20000
    rec = np.zeros((cap, 16))
    nrec = C.c_longlong(0)
    err = C.create_string_buffer(512)
    n = lib.kl_rollout_solve(C.byref(d), p(x0), p(u), p(loss), p(xf), p(it), p(fb), p(rec), C.c_longlong(cap),
                             C.c_int(3), int(sched), int(seed), int(min_team), int(tpw), C.byref(nrec), err, 512)
    if n < 0:
        raise RuntimeError(err.value.decode())
    rec = rec[: min(nrec.value, cap)].copy()
    rec[:, 12:15] = rec[:, 12:15].copy().view(np.int64)
    rec = rec[np.lexsort((rec[:, 14], rec[:, 13], rec[:, 12]))]
    return dict(loss=loss, x_final=xf.T, iters=it, fallbacks=fb, records=rec), n


def main():
    lib = _lib(sys.argv[1])
    min_team = int(sys.argv[2])
    tpw = int(sys.argv[3])
    names = sys.argv[4:]
    if names and names[0] == "--ring":   # every env keeps a ring of the impulse history
        lib.kl_set_ring(1)
        names = names[1:]
    for name in names:
        solve = name in SOLVE_CASES
        w = (SOLVE_CASES if solve else CASES)[name]()
        runs = []
        phases = 0
        try:
            for sched, seed in ((0, 1), (1, 1), (2, 7)):
                r, n = (run_solve if solve else run_grad)(lib, w, sched, seed, min_team, tpw)
                runs.append(r)
                phases += n
        except RuntimeError as e:
            print(json.dumps({"case": name, "error": str(e)}), flush=True)
            continue
        same = all(np.array_equal(runs[0][k], r[k]) for r in runs[1:] for k in runs[0])
        o = Oracle(w)
        if solve:
            ref = o.rollout_ex(rec_every=3, rec_cap=20000)
            diff = max(_rel(runs[0]["x_final"], ref["x_final"]), _rel(runs[0]["loss"], ref["loss"]))
            counts = bool(np.array_equal(runs[0]["iters"], ref["iters"]) and
                          np.array_equal(runs[0]["fallbacks"], ref["fallbacks"]))
        else:
            ref = dict(o.rollout_grad())
            roll = o.rollout()
            ref["x_final"] = roll["x_final"]
            ref["loss"] = roll["loss"]
            diff = max(_rel(runs[0][k], ref[k]) for k in list(KEYS) + ["g_w"]
                       if k in ref and k in runs[0] and np.asarray(ref[k]).size)
            counts = True
        print(json.dumps({"case": name, "schedules_agree": bool(same), "max_rel_diff": float(diff),
                          "counts_agree": counts, "phases": int(phases)}), flush=True)


if __name__ == "__main__":
    main()
