"""Replayable step graphs and the tile autotuner (GPU).

A captured step sequence must reproduce the eager sim_step loop bit for bit
on every replay (the graph holds only kernels: queue resets are fill
kernels, not memsets), with the program's own eager work and
synchronisations between replays, and the eager loop matches the FP64
oracle's steps.  rollout and rollout_grad (several buckets on forked
streams) captured together in one graph by stream capture replay bit for bit
too.  Re-tiling by the autotuner must not change any result bit, since the
sweep order does not depend on the team width.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from gpu_helpers import STATE_TOL, state_errors, to_dev
from oracle import Oracle
from paper_1611_01652_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _eager_steps(s, x0, u_rows, lam0, t0, n):
    x, lam = x0.clone(), lam0.clone()
    for k in range(n):
        uk = u_rows if s.info.n_params else u_rows[k]
        x, lam, flags = s.step(x, uk, lam, t0 + k)
    return x, lam, flags


def _check_graph_replays(s, x0, u_rows, t0, n, reps=3):
    import torch
    lam0 = torch.zeros(max(s.info.lam_size, 1), device="cuda")
    xe, le, fe = _eager_steps(s, x0, u_rows, lam0, t0, n)
    torch.cuda.synchronize()
    xbuf = torch.zeros((2,) + tuple(x0.shape), device="cuda")
    lam = torch.zeros_like(lam0)
    flags = torch.zeros(max(s.info.n_envs, 1), dtype=torch.int32, device="cuda")
    g = s.step_graph(n, xbuf, u_rows, lam, t0=t0, flags=flags)
    try:
        for r in range(reps):
            xbuf[0].copy_(x0)
            xbuf[1].zero_()
            lam.zero_()
            flags.fill_(7)
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(xbuf[n % 2], xe), ("replay", r, (xbuf[n % 2] - xe).abs().max().item())
            assert torch.equal(lam, le), ("replay lambda", r)
            assert torch.equal(flags[: s.info.n_envs], fe[: s.info.n_envs]), ("replay flags", r)
            # the program's own eager work between replays
            xe2, _, _ = _eager_steps(s, x0, u_rows, lam0, t0, 1)
            torch.cuda.synchronize()
            assert torch.isfinite(xe2).all()
    finally:
        g.close()


def test_step_graph_matches_eager_steps_on_several_buckets():
    import torch
    from paper_1611_01652_amd.sim import Simulator
    w = W.uneven_chains(n_envs=160, T=40, seed_salt=21)
    s = Simulator(w)
    assert len(s.teams()) > 1, "want several buckets (fork/join inside the graph)"
    x0, u = to_dev(w)
    _say("case step graph, chains 160 envs x 12 steps, buckets", s.teams().tolist())
    _check_graph_replays(s, x0, u[:12].contiguous(), 0, 12)
    # the eager steps (the graph's bits) against the oracle's
    xe, _, _ = _eager_steps(s, x0, u[:12].contiguous(), torch.zeros(max(s.info.lam_size, 1), device="cuda"), 0, 12)
    o = Oracle(w)
    x, lam = np.asarray(w.x0, np.float64), np.zeros(o.lam_size)
    for t in range(12):
        x, lam = o.step(x, lam, w.u[t], t)
    se = state_errors(w, xe.cpu().numpy().T.astype(np.float64), x)
    assert (se <= STATE_TOL).all(), se.max()
    _say("case step graph, odd step count 5 from row 3")
    _check_graph_replays(s, x0, u[3:8].contiguous(), 3, 5)
    s.close()


def test_step_graph_with_controller_and_clock_offset():
    import torch
    from paper_1611_01652_amd.sim import Simulator
    w = W.quadruped(n_envs=24, T_min=40, T_max=40, mlp_w=W.mlp_init(zero_output=False, out_scale=0.1))
    s = Simulator(w)
    x0, _ = to_dev(w)
    wt = torch.tensor(w.extra["mlp"]["w"], dtype=torch.float32, device="cuda")
    _say("case step graph with controller, t0 = 7, 9 steps")
    _check_graph_replays(s, x0, wt, 7, 9)
    from paper_1611_01652_amd.sim import SimError
    xbuf = torch.zeros((2,) + tuple(x0.shape), device="cuda")
    lam = torch.zeros(max(s.info.lam_size, 1), device="cuda")
    with pytest.raises(SimError):
        s.step_graph(5, xbuf, wt, lam, t0=38)     # t0 + n_steps > T_max
    s.close()


@pytest.mark.parametrize("keep", [False, True])
def test_rollout_and_gradient_captured_in_one_graph(keep):
    # one call of rollout (or rollout with kept working sets) and rollout_grad
    # captured by torch's stream capture: every replay equals the eager calls
    # bit for bit, with eager calls and synchronisations between replays
    import torch
    from paper_1611_01652_amd.sim import Simulator
    w = W.uneven_chains(n_envs=96, T=40, seed_salt=24)
    s = Simulator(w)
    assert len(s.teams()) > 1, "want several buckets (forked streams inside the capture)"
    assert s.info.grad_store == 3
    x0, u = to_dev(w)
    dl = torch.ones(w.n_envs, device="cuda")
    ws = s.workspace()

    def calls():
        r = s.rollout(x0, u, keep=ws if keep else None)
        g = s.rollout_grad(x0, u, r["ckpt"], dl, workspace=None if keep else ws, kept=ws if keep else None)
        return [r["loss"], r["x_final"], r["ckpt"]] + [g[k] for k in sorted(g)]

    ref = [t.clone() for t in calls()]
    torch.cuda.synchronize()
    _say("case captured rollout + rollout_grad, chains 96 envs x 40 steps, keep", keep)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        calls()   # warm-up on the capture's stream, as torch asks
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        outs = calls()
    try:
        for rep_ in range(3):
            for t in outs:
                t.fill_(float("nan") if t.is_floating_point() else -1)
            graph.replay()
            torch.cuda.synchronize()
            for k, (a, b) in enumerate(zip(outs, ref)):
                assert torch.equal(a, b), ("replay", rep_, k)
            eager = calls()
            torch.cuda.synchronize()
            for a, b in zip(eager, ref):
                assert torch.equal(a, b)
    finally:
        del graph
    s.close()


def test_tune_keeps_every_result_bit():
    import torch
    from paper_1611_01652_amd.sim import SimError, Simulator
    w = W.uneven_chains(n_envs=256, T=60, seed_salt=22)
    s = Simulator(w)
    x0, u = to_dev(w)
    dl = torch.ones(w.n_envs, device="cuda")

    def run():
        r = s.rollout(x0, u)
        g = s.rollout_grad(x0, u, r["ckpt"], dl)
        torch.cuda.synchronize()
        return [r["loss"], r["x_final"], r["ckpt"]] + [g[k] for k in sorted(g)]

    before_teams = s.teams()
    ref = run()
    _say("case tune, chains 256 envs x 60 steps, teams", before_teams.tolist())
    chosen = s.tune(x0, u, with_grad=True, max_candidates=3)
    _say("  chosen", chosen.tolist())
    assert len(chosen) == len(before_teams)
    assert (chosen >= before_teams).all() and all(int(t) & (int(t) - 1) == 0 for t in chosen)
    assert np.array_equal(s.teams(), chosen)
    for a, b in zip(run(), ref):
        assert torch.equal(a, b)
    wide = np.minimum(before_teams * 2, 64)
    s.set_teams(wide)
    for a, b in zip(run(), ref):
        assert torch.equal(a, b)
    bad = before_teams.copy()
    if bad[0] > 1:
        bad[0] //= 2
        with pytest.raises(SimError):
            s.set_teams(bad)
    with pytest.raises(SimError):
        s.set_teams(before_teams[:-1])
    # a live graph holds the tile lists: re-tiling is refused until it is gone
    xbuf = torch.zeros((2,) + tuple(x0.shape), device="cuda")
    lam = torch.zeros(max(s.info.lam_size, 1), device="cuda")
    g = s.step_graph(2, xbuf, u[:2].contiguous(), lam)
    with pytest.raises(SimError):
        s.set_teams(before_teams)
    g.close()
    s.set_teams(before_teams)
    for a, b in zip(run(), ref):
        assert torch.equal(a, b)
    s.close()


def test_reverse_sweep_memory_modes_give_the_same_gradient_bits():
    # the reverse sweep replays each step, or reloads the working set saved by
    # the recompute of its segment, or by the recompute of all segments at
    # once in a separate launch; the arithmetic is the same, so every bit must
    # agree (chains: several buckets and a ragged last segment; quadruped:
    # controller, episode lengths that differ per env)
    import torch
    from paper_1611_01652_amd.sim import Simulator
    quad = W.quadruped(n_envs=16, T_min=30, T_max=45, mlp_w=W.mlp_init(zero_output=False, out_scale=0.1))
    quad.ckpt_every = 8
    cases = (W.uneven_chains(n_envs=64, T=60, seed_salt=23), quad)
    for w in cases:
        outs = []
        for mode in ("trajectory", "segment", "replay"):
            w.extra = dict(w.extra or {})
            w.extra["grad_store"] = mode
            s = Simulator(w)
            assert s.info.grad_store == {"replay": 1, "segment": 2, "trajectory": 3}[mode]
            x0, u = to_dev(w)
            if "mlp" in w.extra:
                u = torch.tensor(w.extra["mlp"]["w"], dtype=torch.float32, device="cuda")
            r = s.rollout(x0, u)
            g = s.rollout_grad(x0, u, r["ckpt"], torch.ones(w.n_envs, device="cuda"))
            torch.cuda.synchronize()
            outs.append({k: v.clone() for k, v in g.items()})
            _say("case reverse sweep", w.name, "mode", mode, "workspace MB", s.info.workspace_bytes / 1e6)
            s.close()
        for o in outs[1:]:
            for k in outs[0]:
                assert torch.equal(outs[0][k], o[k]), k


def test_tune_cache_tunes_once_then_reuses(tmp_path):
    # the first model is tuned on a short copy of itself and stored; a second
    # handle of the same model gets the stored widths without timing; results
    # keep every bit
    import torch
    from paper_1611_01652_amd import tune_cache as TC
    from paper_1611_01652_amd.sim import Simulator
    w = W.uneven_chains(n_envs=256, T=120, seed_salt=23)
    x0, u = to_dev(w)
    dl = torch.ones(w.n_envs, device="cuda")
    path = str(tmp_path / "tune.json")
    make_u = lambda ws: to_dev(ws)[1]   # noqa: E731

    def run(s):
        r = s.rollout(x0, u)
        g = s.rollout_grad(x0, u, r["ckpt"], dl)
        torch.cuda.synchronize()
        return [r["loss"], r["x_final"]] + [g[k] for k in sorted(g)]

    s = Simulator(w)
    default = s.teams()
    ref = run(s)
    teams, how = TC.tuned_teams(s, make_u, path, short_T=30, objective="bucket")
    _say("case tune cache, chains 256 envs x 120 steps: default", default.tolist(), "tuned", teams.tolist(), how)
    assert how == "tuned" and np.array_equal(s.teams(), teams)
    assert (teams >= default).all()
    for a, b in zip(run(s), ref):
        assert torch.equal(a, b)
    s.close()
    s2 = Simulator(w)
    teams2, how2 = TC.tuned_teams(s2, make_u, path, short_T=30, objective="bucket")
    assert how2 == "cache" and np.array_equal(teams2, teams) and np.array_equal(s2.teams(), teams)
    for a, b in zip(run(s2), ref):
        assert torch.equal(a, b)
    # the whole-call objective: its own cache entry, widths never below the
    # default, every result bit kept
    s2.set_teams(default)
    teams3, how3 = TC.tuned_teams(s2, make_u, path, short_T=30, objective="call")
    _say("   whole-call objective:", teams3.tolist(), how3)
    assert how3 == "tuned" and (teams3 >= default).all() and np.array_equal(s2.teams(), teams3)
    for a, b in zip(run(s2), ref):
        assert torch.equal(a, b)
    s2.close()
