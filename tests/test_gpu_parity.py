"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances: states within 1e-4 and gradients within 1e-3 relative (per env,
per group / array), on each env's non-chaotic horizon (gpu_helpers: states at
every checkpoint before the env's horizon, gradients of every env whose oracle
gradient is stable under 4-ulp noise; no env may miss).  The coverage floors
of each case sit just below what the criterion yields on it.  Sizes span
several tiles and a ragged tail; the full-size launches are compared on
sampled envs computed one by one by the oracle.
"""
import numpy as np
import pytest

from gpu_helpers import (GRAD_TOL, STATE_TOL, compare_with_oracle, gpu_run, grad_errors, grad_stable, rel,
                         state_errors, to_dev)
from oracle import Oracle
from paper_1611_01652_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _compare(w, got, check_grad=True, state_frac=0.0, grad_frac=1.0, checkpoints=0):
    rep = compare_with_oracle(w, got, check_grad=check_grad, min_state_frac=state_frac, min_grad_frac=grad_frac,
                              min_checkpoints=checkpoints)
    _say("  ", rep)
    return rep


def test_ball_throw_full():
    w = W.ball_throw()
    _say("case ball-throw T=300")
    got = gpu_run(w)
    _compare(w, got)


def test_planar_arms_subset_all_steps():
    w = W.planar_arms(n_envs=96, T=1000)      # 3 tiles of 32 at the narrowest team
    _say("case planar-arms 96 x 1000")
    got = gpu_run(w)
    # no arm stays non-chaotic over all 1000 steps; the criterion yields 413
    # (env, checkpoint) state comparisons and 61.5 % gradient-stable arms
    _compare(w, got, grad_frac=0.55, checkpoints=380)


def test_planar_arms_quarter_horizon_every_env():
    w = W.planar_arms(n_envs=96, T=250)
    _say("case planar-arms 96 x 250")
    # the criterion yields 19.8 % of the arms non-chaotic over the 250 steps,
    # 386 checkpoint comparisons and 77 % gradient-stable arms
    _compare(w, gpu_run(w), state_frac=0.18, grad_frac=0.7, checkpoints=360)


def test_planar_arms_full_size_sampled():
    # the arm benchmark's launch (trajectory mode, the rollout keeping the
    # working sets); 16 evenly spaced envs by the per-env protocol (12 of
    # them gradient-stable over the 1000 steps)
    import bench
    w = W.planar_arms(n_envs=4096, T=1000)
    _say("case planar-arms 4096 x 1000 (the arm benchmark's launch), sampled")
    got = gpu_run(w, keep=True)
    sample = bench.stratified(w, 16)
    ws = w.subset(sample)
    _compare(ws, _sampled(got, w, sample), grad_frac=7 / 16, checkpoints=50)


def test_uneven_chains_subset():
    w = W.uneven_chains(n_envs=40, T=100, seed_salt=1)
    _say("case uneven-chains 40 x 100")
    got = gpu_run(w)
    assert (got["flags"] == 0).all()
    # yields 22.5 % non-chaotic, 78 checkpoint comparisons, 55 % gradient-stable
    _compare(w, got, state_frac=0.2, grad_frac=0.5, checkpoints=70)


def _sampled(got, w, sample):
    """The arrays of the sampled envs, as their own workload lays them out."""
    b = np.concatenate([np.arange(w.env_body_off[e], w.env_body_off[e + 1]) for e in sample])
    j = np.concatenate([np.arange(w.env_joint_off[e], w.env_joint_off[e + 1]) for e in sample])
    out = dict(loss=got["loss"][sample], x_final=got["x_final"][b], flags=got["flags"][sample],
               ckpt_states=got["ckpt_states"][:, b])
    for k in ("g_x0", "g_inv_mass", "g_inv_inertia"):
        if k in got:
            out[k] = got[k][b]
    for k in ("g_damping", "g_anchor_p", "g_anchor_c"):
        if k in got:
            out[k] = got[k][j]
    if "g_u" in got:
        out["g_u"] = got["g_u"][:, j]
    if "g_mu" in got:
        out["g_mu"] = got["g_mu"][sample]
    return out


def test_uneven_chains_full_size_sampled():
    # the benchmark's launch: 16384 chains x 500 steps with the benchmark's
    # memory limit (the free device memory less 12 GiB), which gives
    # trajectory mode, the rollout keeping every step's working set and the
    # reverse reading them, all size buckets; 64 envs at evenly spaced
    # quantiles of the body count are compared by the per-env protocol.  Over
    # 500 steps the criterion yields 142 checkpoint comparisons and 4
    # gradient-stable envs of the 64.
    import torch
    import bench
    w = W.uneven_chains(n_envs=16384, T=500)
    free, _ = torch.cuda.mem_get_info()
    w.extra = dict(w.extra or {}, grad_mem_limit=int(max(1.0, free / 2**30 - 12.0) * 2**30))
    _say("case uneven-chains 16384 x 500 (full size, the benchmark's launch), sampled")
    from paper_1611_01652_amd.sim import Simulator
    s = Simulator(w)
    try:
        assert s.info.grad_store == 3
        got = gpu_run(w, sim=s, keep=True)
    finally:
        s.close()
        torch.cuda.empty_cache()
    assert (got["flags"] == 0).mean() > 0.99
    sample = bench.stratified(w, 64)
    ws = w.subset(sample)
    _compare(ws, _sampled(got, w, sample), grad_frac=3 / 64, checkpoints=130)


def test_sim_step_from_contact_state():
    w = W.uneven_chains(n_envs=12, T=80, seed_salt=2)
    o = Oracle(w)
    x, lam = w.x0.copy(), np.zeros(o.lam_size)
    for t in range(60):
        x, lam = o.step(x, lam, w.u[t], t)
    assert (lam != 0).sum() > 50
    xn, ln = o.step(x, lam, w.u[60], 60)
    import torch
    from paper_1611_01652_amd.sim import Simulator
    _say("case sim_step from a contact state")
    s = Simulator(w)
    xd = torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float32, device="cuda")
    ud = torch.tensor(w.u[60], dtype=torch.float32, device="cuda")
    ld = torch.tensor(lam, dtype=torch.float32, device="cuda")
    xo, lo, flags = s.step(xd, ud, ld)
    torch.cuda.synchronize()
    assert (flags.cpu().numpy()[: w.n_envs] == 0).all()
    se = state_errors(w, xo.cpu().numpy().T.astype(np.float64), xn)
    assert (se <= STATE_TOL).all(), se.max()
    assert rel(lo.cpu().numpy()[: o.lam_size], ln) <= 1e-4


def test_ragged_lengths_and_degenerate_envs():
    # episode lengths 0..T, a body without joints or spheres, and the other envs
    a = W.uneven_chains(n_envs=6, T=90, sizes=[2, 5, 3, 9, 2, 4], seed_salt=3)
    a.T_env = np.array([90, 0, 37, 1, 64, 90], np.int32)
    _say("case ragged episode lengths")
    got = gpu_run(a)
    _compare(a, got, grad_frac=0.5)   # 3 of the 6 envs have stable gradients
    assert np.all(got["g_u"][37:, a.env_joint_off[2]:a.env_joint_off[3]] == 0)
    assert np.all(got["g_x0"][a.env_body_off[1]:a.env_body_off[2]] == 0)
    b = W.single_sphere(p=(0, 0, 1.0), v=(0.3, 0, 0), ground=False, T=40)
    b.sphere_flags[:] = 0
    _say("case lone body")
    _compare(b, gpu_run(b))


def test_zero_iterations_and_empty_model():
    w = W.uneven_chains(n_envs=5, T=30, seed_salt=4)
    w.n_iters = 0
    _say("case zero sweeps")
    _compare(w, gpu_run(w))
    e = W.uneven_chains(n_envs=1, T=3).subset([])
    from paper_1611_01652_amd.sim import Simulator
    s = Simulator(e)
    assert s.info.n_envs == 0


def test_nonfinite_env_is_flagged_and_isolated():
    w = W.uneven_chains(n_envs=6, T=50, seed_salt=6)
    _say("case NaN in one env")
    clean = gpu_run(w, grad=False)
    bad = w.with_steps(w.T_max)
    bad.x0 = w.x0.copy()
    bad.x0[w.env_body_off[2], 12] = np.nan
    got = gpu_run(bad, grad=False)
    assert got["flags"][2] & 1
    others = [e for e in range(w.n_envs) if e != 2]
    assert (got["flags"][others] == 0).all()
    assert np.array_equal(got["loss"][others], clean["loss"][others])


def test_contact_overflow_is_flagged():
    rng = np.random.default_rng(1)
    pos = np.c_[rng.uniform(-0.1, 0.1, (12, 2)), rng.uniform(0.05, 0.2, 12)]
    w = W.free_spheres(pos, [0.1] * 12, [1.0] * 12, T=5)
    _say("case contact overflow")
    got = gpu_run(w, grad=False)
    assert got["flags"][0] & 2


@pytest.mark.parametrize("make", [lambda: W.uneven_chains(n_envs=20, T=60, seed_salt=7),
                                  lambda: W.planar_arms(n_envs=40, T=120),
                                  lambda: W.servo_chains(20, 60, seed_salt=7)])
def test_bitwise_determinism_and_team_invariance(make):
    # chains (free floating) and arms (world-attached base joints: the paired
    # hinge forms with the world slot as side a), and chains on servos (the
    # motor row's pair exchange), at their default team widths and at 64
    # lanes per env give the same bits
    w = make()
    _say("case determinism", w.name)
    a = gpu_run(w)
    b = gpu_run(w)
    w2 = w.with_steps(w.T_max)
    w2.min_team = 64
    c = gpu_run(w2)
    for k in ("loss", "x_final", "g_x0", "g_u", "g_mu", "g_inv_mass", "g_inv_inertia", "g_damping", "g_anchor_p",
              "g_anchor_c"):
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k


def test_gradient_matches_fp32_finite_differences():
    import torch
    from paper_1611_01652_amd.sim import Simulator
    w = W.planar_arms(n_envs=4, T=200)
    _say("case FP32 central differences")
    s = Simulator(w)
    x0, u = to_dev(w)
    r = s.rollout(x0, u)
    g = s.rollout_grad(x0, u, r["ckpt"], torch.ones(4, device="cuda"))["g_u"].cpu().numpy()
    h = 1e-2
    for (t, j) in [(0, 0), (50, 4), (120, 7), (199, 11)]:
        up = u.clone()
        um = u.clone()
        up[t, j] += h
        um[t, j] -= h
        e = j // 3
        fd = (s.rollout(x0, up)["loss"][e].item() - s.rollout(x0, um)["loss"][e].item()) / (2 * h)
        assert abs(g[t, j] - fd) <= 1e-2 * abs(fd) + 2e-5, (t, j, g[t, j], fd)


def test_autograd_function_matches_rollout_grad():
    import torch
    from paper_1611_01652_amd.autograd import rollout_loss
    from paper_1611_01652_amd.sim import Simulator
    w = W.planar_arms(n_envs=8, T=150)
    _say("case autograd.Function")
    s = Simulator(w)
    x0, u = to_dev(w)
    x0.requires_grad_(True)
    u.requires_grad_(True)
    loss = rollout_loss(s, x0, u)
    wts = torch.linspace(0.5, 1.5, 8, device="cuda")
    (loss * wts).sum().backward()
    o = Oracle(w).rollout_grad(dloss=np.linspace(0.5, 1.5, 8))
    assert rel(u.grad.cpu().numpy().astype(np.float64), o["g_u"]) <= GRAD_TOL
    assert rel(x0.grad.cpu().numpy().T.astype(np.float64), o["g_x0"]) <= GRAD_TOL


def _quadruped_run(w, grad=True):
    import torch
    from paper_1611_01652_amd.sim import Simulator
    s = Simulator(w)
    x0, _ = to_dev(w)
    wt = torch.tensor(w.extra["mlp"]["w"], dtype=torch.float32, device="cuda")
    r = s.rollout(x0, wt)
    out = dict(loss=r["loss"].cpu().numpy().astype(np.float64), x_final=r["x_final"].cpu().numpy().T.astype(np.float64),
               flags=r["flags"].cpu().numpy()[: w.n_envs])
    if grad:
        g = s.rollout_grad(x0, wt, r["ckpt"], torch.ones(w.n_envs, device="cuda"))
        out["g_w"] = g["g_u"].cpu().numpy().astype(np.float64)
        out["g_x0"] = g["g_x0"].cpu().numpy().T.astype(np.float64)
        out["g_mu"] = g["g_mu"].cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    return s, out


def _weight_gradient_blocks(w, got_w, ref_w):
    sizes = w.extra["mlp"]["sizes"]
    off = 0
    for a_, b_ in zip(sizes[:-1], sizes[1:]):
        for n in (a_ * b_, b_):
            blk = slice(off, off + n)
            assert rel(got_w[blk], ref_w[blk]) <= GRAD_TOL, (off, rel(got_w[blk], ref_w[blk]))
            off += n
    assert off == len(ref_w)


def test_quadruped_controller_forward_and_weight_gradient():
    # ragged episode lengths; controller output layer small but non-zero so
    # that every layer's gradient is exercised.  States, losses and per-env
    # gradients by the per-env protocol (the criterion yields 95 % of the
    # robots non-chaotic over their episodes and 64 % gradient-stable); the
    # weight gradient, a sum over envs, over the gradient-stable robots as a
    # launch of their own
    w = W.quadruped(n_envs=64, T_min=30, T_max=60, mlp_w=W.mlp_init(zero_output=False, out_scale=0.1))
    _say("case quadruped + MLP controller 64 envs, T 30..60")
    from paper_1611_01652_amd.sim import Simulator
    s = Simulator(w)
    assert s.info.n_params == 19976
    got = gpu_run(w, sim=s)
    _compare(w, got, state_frac=0.9, grad_frac=0.55)
    stable = np.where(grad_stable(w, Oracle(w).rollout_grad()))[0].tolist()
    ws = w.subset(stable)
    _say("   weight gradient over", len(stable), "gradient-stable robots")
    sub = gpu_run(ws)
    _weight_gradient_blocks(ws, sub["g_w"], Oracle(ws).rollout_grad()["g_w"])


def test_quadruped_zero_policy_gradient_reaches_output_layer_only():
    # the zero-initialised output layer (section 3.2) passes no gradient to the
    # hidden layers at the first update; only W3 and b3 move
    w = W.quadruped(n_envs=16, T_min=40, T_max=40)
    _say("case quadruped zero policy")
    s, got = _quadruped_run(w)
    ref = Oracle(w).rollout_grad()
    n_hidden = 128 * 18 + 128 + 128 * 128 + 128
    assert np.abs(got["g_w"][:n_hidden]).max() == 0.0
    assert rel(got["g_w"][n_hidden:], ref["g_w"][n_hidden:]) <= GRAD_TOL


@pytest.mark.parametrize("rec", [0, 4])
def test_quadruped_sim_step_with_controller(rec):
    # with a recurrent controller the carried block holds h^t after the
    # impulses; one step from a state reached by the oracle
    import torch
    w = W.quadruped(n_envs=8, T_min=40, T_max=40, rec=rec,
                    mlp_w=W.mlp_init(W.rec_sizes(W.MLP_SIZES, rec), zero_output=False, out_scale=0.1))
    o = Oracle(w)
    x, lam = w.x0.copy(), np.zeros(o.lam_size)
    for t in range(25):
        x, lam = o.step(x, lam, None, t)
    xn, ln = o.step(x, lam, None, 25)
    from paper_1611_01652_amd.sim import Simulator
    _say("case quadruped sim_step t=25, recurrent units", rec)
    s = Simulator(w)
    xd = torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float32, device="cuda")
    wt = torch.tensor(w.extra["mlp"]["w"], dtype=torch.float32, device="cuda")
    ld = torch.tensor(lam, dtype=torch.float32, device="cuda")
    xo, lo, flags = s.step(xd, wt, ld, t_index=25)
    torch.cuda.synchronize()
    se = state_errors(w, xo.cpu().numpy().T.astype(np.float64), xn)
    assert (se <= STATE_TOL).all(), se.max()
    if rec:
        assert np.abs(lam[-rec:]).max() > 0.01
        assert rel(lo.cpu().numpy()[: o.lam_size], ln) <= 1e-4


@pytest.mark.parametrize("make,alpha,frac", [(lambda: W.planar_arms(n_envs=48, T=300), 0.95, 0.9),
                                             (lambda: W.uneven_chains(n_envs=24, T=120, seed_salt=5), 0.8, 0.2)])
def test_gradient_decay_matches_oracle(make, alpha, frac):
    # section 3.2's gradient decay: the carried adjoints shrink by alpha per
    # reversed step; the per-env protocol against the oracle with the same
    # alpha (yields 96 % gradient-stable arms, 25 % of the chains)
    w = make()
    w.grad_decay = alpha
    _say("case gradient decay", w.name, alpha)
    got = gpu_run(w)
    _compare(w, got, grad_frac=frac)
    exact = w.with_steps(w.T_max)
    exact.grad_decay = 1.0
    g1 = gpu_run(exact)
    assert np.abs(got["g_x0"]).sum() < np.abs(g1["g_x0"]).sum()   # the decay shrinks the far-past terms


def test_recurrent_controller_matches_oracle():
    # eq. (g) with memory: 8 recurrent units carried after the impulses.
    # States and losses by the per-env protocol (96 % of the robots
    # non-chaotic over their episodes); the per-env dL/dx0 of these robots
    # moves by up to 4e-3 under 4-ulp noise (stick-slip of the feet), so the
    # gradient compared is dL/dW over the batch, whose noisy oracle runs stay
    # within 3e-5 of the clean one
    import gpu_helpers as H
    rec = 8
    sizes = W.rec_sizes(W.MLP_SIZES, rec)
    w = W.quadruped(n_envs=48, T_min=20, T_max=45, rec=rec, mlp_w=W.mlp_init(sizes, zero_output=False, out_scale=0.1))
    _say("case recurrent controller, quadruped 48 envs, 8 units")
    got = gpu_run(w)
    _compare(w, got, state_frac=0.9, grad_frac=0.0)
    ref = Oracle(w).rollout_grad()["g_w"]
    for k in range(4):
        noisy = Oracle(w, noise=H.GRAD_NOISE, noise_seed=k).rollout_grad()["g_w"]
        assert rel(noisy, ref) < 0.5 * GRAD_TOL
    _weight_gradient_blocks(w, got["g_w"], ref)


@pytest.mark.parametrize("make", [lambda: W.planar_arms(n_envs=40, T=130),
                                  lambda: W.uneven_chains(n_envs=24, T=110, seed_salt=3),
                                  lambda: W.servo_chains(12, 80)])
def test_rollout_keep_and_grad_kept_equal_rollout_and_grad(make):
    # trajectory mode: the rollout that keeps every step's working set and the
    # reverse without a recompute give the bits of rollout + rollout_grad
    import torch
    from paper_1611_01652_amd.sim import Simulator
    w = make()
    w.extra = dict(w.extra or {}, grad_store="trajectory")
    _say("case rollout_keep", w.name, w.n_envs)
    s = Simulator(w)
    x0, u = to_dev(w)
    dl = torch.ones(w.n_envs, device="cuda")
    r = s.rollout(x0, u)
    g = s.rollout_grad(x0, u, r["ckpt"], dl)
    ws = s.workspace()
    rk = s.rollout(x0, u, keep=ws)
    gk = s.rollout_grad(x0, u, None, dl, kept=ws)
    torch.cuda.synchronize()
    for k in ("loss", "x_final", "ckpt"):
        assert torch.equal(r[k], rk[k]), k
    for k in ("g_x0", "g_u", "g_inv_mass", "g_inv_inertia", "g_mu", "g_damping", "g_anchor_p", "g_anchor_c"):
        assert torch.equal(g[k], gk[k]), k


@pytest.mark.parametrize("make", [lambda: W.planar_arms(n_envs=40, T=130),
                                  lambda: W.uneven_chains(n_envs=48, T=110, seed_salt=5),
                                  lambda: W.quadruped(n_envs=24, T_min=20, T_max=45,
                                                      mlp_w=W.mlp_init(zero_output=False, out_scale=0.1))])
def test_rollout_and_grad_equals_rollout_keep_and_grad_kept(make):
    # the fused call (each bucket's reverse right after its own forward, one
    # join) gives the bits of rollout_keep + rollout_grad_kept, including the
    # controller's weight gradient; run twice to see that nothing depends on
    # what an earlier call left in the workspace
    import torch
    from paper_1611_01652_amd.sim import Simulator
    w = make()
    w.extra = dict(w.extra or {}, grad_store="trajectory")
    s = Simulator(w)
    _say("case rollout_and_grad", w.name, w.n_envs, "buckets", len(s.teams()))
    x0, u = to_dev(w)
    mlp = (w.extra or {}).get("mlp")
    if mlp is not None:
        u = torch.tensor(np.asarray(mlp["w"], np.float32), device="cuda")
    dl = torch.linspace(0.5, 1.5, w.n_envs, device="cuda")
    ws = s.workspace()
    rk = s.rollout(x0, u, keep=ws)
    gk = s.rollout_grad(x0, u, None, dl, kept=ws)
    ws2 = s.workspace()
    for _ in range(2):
        rf, gf = s.rollout_and_grad(x0, u, dl, ws2, want_ckpt=True, want_final=True)
        torch.cuda.synchronize()
        for k in ("loss", "x_final", "lam_final", "ckpt", "flags"):
            assert torch.equal(rk[k][: rf[k].numel()].reshape(rf[k].shape), rf[k]), k
        for k in ("g_x0", "g_u", "g_inv_mass", "g_inv_inertia", "g_mu", "g_damping", "g_anchor_p", "g_anchor_c",
                  "flags"):
            assert torch.equal(gk[k], gf[k]), k


def test_rollout_keep_is_refused_outside_trajectory_mode():
    import torch
    from paper_1611_01652_amd.sim import SimError, Simulator
    w = W.uneven_chains(n_envs=4, T=60, seed_salt=4)
    w.extra = dict(w.extra or {}, grad_store="segment")
    s = Simulator(w)
    x0, u = to_dev(w)
    ws = s.workspace()
    with pytest.raises(SimError, match="trajectory"):
        s.rollout(x0, u, keep=ws)
    with pytest.raises(SimError, match="trajectory"):
        s.rollout_grad(x0, u, None, torch.ones(w.n_envs, device="cuda"), kept=ws)
    with pytest.raises(SimError, match="trajectory"):
        s.rollout_and_grad(x0, u, torch.ones(w.n_envs, device="cuda"), ws)
