"""What any warm start can save on the chain distribution solved to 1e-5,
measured with the FP64 oracle (tolerance mode, plain warm start at factor 1,
cap 1000 sweeps).

At sampled steps of seeded chain trajectories, the same step is solved again
from four starts: the carried impulses (the plain warm start); the carried
joint impulses with the step's converged contact impulses (a perfect
per-contact predictor, the most a learned contact warm start can reach); the
converged joint impulses with the carried contact impulses; and the converged
impulses of both.  "Converged" is the step's own solve, so:

* restarted at its own converged impulses, a step that reached the tolerance
  stops after exactly one sweep (the sweep that measures the residual);
* a sizable share of the steps reach the 1000-sweep cap from the plain start,
  and most of them reach it again from their own final iterate: a chain
  resting on the ground with friction is statically indeterminate, and the
  iteration creeps along the internal force (hinge and friction impulses
  together) that the dynamics leaves free, so no start near the capped
  iterate ends the solve sooner;
* on the steps that converge, the perfect per-contact start saves little of
  the sweeps, the exact joint impulses save more, and both together save
  everything: the sweep count is set by the chains' joint modes.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import Oracle
from paper_1611_01652_amd import workloads as W

CAP = 1000


@pytest.fixture(scope="module")
def samples():
    base = W.warm_start_chains(n_envs=256, T=300, seed_salt=200, tol=1e-5, max_iters=CAP)
    nb = np.diff(base.env_body_off)
    # 24 envs at evenly spaced quantiles of the body count
    order = np.argsort(nb, kind="stable")
    envs = sorted(set(order[((np.arange(24) + 0.5) / 24 * len(order)).astype(int)].tolist()))
    out = {k: [] for k in ("plain", "contacts", "joints", "both")}
    for e in envs:
        w = base.subset([e])
        o = Oracle(w)
        nj5 = 5 * w.n_joints
        x, lam = np.asarray(w.x0, np.float64), np.zeros(o.lam_size)
        for t in range(w.T_max):
            xn, ln = o.step(x, lam, w.u[t], t)
            if t >= 20 and t % 20 == 0:
                w1 = w.with_steps(1)
                w1.u = w.u[t:t + 1].copy()

                def sweeps(l0):
                    return int(Oracle(w1, lam0=l0).rollout_ex(x0=x)["iters"][0])
                out["plain"].append(sweeps(lam))
                out["contacts"].append(sweeps(np.concatenate([lam[:nj5], ln[nj5:]])))
                out["joints"].append(sweeps(np.concatenate([ln[:nj5], lam[nj5:]])))
                out["both"].append(sweeps(ln))
            x, lam = xn, ln
    return {k: np.array(v) for k, v in out.items()}


def test_a_converged_step_restarted_at_its_solution_takes_one_sweep(samples):
    conv = samples["plain"] < CAP
    assert conv.sum() >= 100
    assert (samples["both"][conv] == 1).all()


def test_indeterminate_resting_steps_reach_the_cap_from_any_nearby_start(samples):
    capped = samples["plain"] >= CAP
    print("steps at the cap from the plain start:", capped.mean())
    assert capped.mean() >= 0.2
    # from the capped solve's own final iterate most reach the cap again
    assert (samples["both"][capped] >= CAP).mean() >= 0.5


def test_a_perfect_contact_predictor_saves_little(samples):
    conv = samples["plain"] < CAP
    p = samples["plain"][conv].sum()
    ratio = {k: samples[k][conv].sum() / p for k in ("contacts", "joints", "both")}
    print("sweeps relative to the plain start on converging steps:", ratio)
    assert ratio["contacts"] >= 0.85
    assert ratio["joints"] < ratio["contacts"]
    assert ratio["both"] <= 0.05


def test_a_resting_chain_creeps_along_its_indeterminate_internal_force():
    # a 3-body chain resting on the ground (seeded env, step 192): its solve
    # reaches the tolerance only after ~2e4 sweeps; meanwhile a hinge impulse
    # and the friction impulses at the contacts keep growing together, the
    # internal force that friction and the hinges can trade
    base = W.warm_start_chains(n_envs=256, T=200, seed_salt=200, tol=1e-5)
    w = base.subset([26])
    assert w.n_bodies == 3
    o = Oracle(w)
    x, lam = np.asarray(w.x0, np.float64), np.zeros(o.lam_size)
    for t in range(192):
        x, lam = o.step(x, lam, w.u[t], t)
    assert np.allclose(x[:, 2], w.sphere_radius, atol=1e-3)   # every sphere on the ground
    res = {}
    for cap in (1000, 4000, 16000, 64000):
        w1 = w.with_steps(1)
        w1.u = w.u[192:193].copy()
        w1.extra = dict(w1.extra, solve=dict(mode=1, tol=1e-5, max_iters=cap))
        r = Oracle(w1, lam0=lam).rollout_ex(x0=x)
        res[cap] = (int(r["iters"][0]), r["lam_final"].copy())
    assert [res[c][0] for c in (1000, 4000, 16000)] == [1000, 4000, 16000]
    assert 16000 < res[64000][0] < 64000
    nj5 = 5 * w.n_joints
    grow = np.abs(res[16000][1]) - np.abs(res[1000][1])
    assert grow[:nj5].max() > 5e-3 and grow[nj5:].max() > 5e-3
