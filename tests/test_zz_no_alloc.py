"""The allocation-free reverse mode (rollout_grad_noalloc) against rollout_grad.

Both entry points run the same kernels on the same inputs, so the results
must be bit for bit the same; the second call in a row uses a smaller model,
with the scratch still holding the first call's contents.  A model whose
workspace exceeds the scratch is refused before any launch.
"""
import numpy as np
import pytest

from gpu_helpers import to_dev
from paper_1611_01652_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("g_x0", "g_u", "g_inv_mass", "g_inv_inertia", "g_mu", "g_damping", "g_anchor_p", "g_anchor_c", "flags")


def _say(*a):
    print(*a, flush=True)


def _both(w, controls=None):
    import torch
    from paper_1611_01652_amd.sim import NOALLOC_SCRATCH_BYTES, Simulator
    s = Simulator(w)
    assert 0 < s.info.workspace_bytes <= NOALLOC_SCRATCH_BYTES, s.info.workspace_bytes
    x0, u = to_dev(w)
    if controls is not None:
        u = torch.tensor(controls, dtype=torch.float32, device="cuda")
    r = s.rollout(x0, u)
    dl = torch.linspace(0.5, 1.5, w.n_envs, device="cuda")
    ref = s.rollout_grad(x0, u, r["ckpt"], dl)
    got = s.rollout_grad(x0, u, r["ckpt"], dl, no_alloc=True)
    torch.cuda.synchronize()
    for k in KEYS:
        a, b = got[k].cpu().numpy(), ref[k].cpu().numpy()
        assert a.shape == b.shape, k
        assert np.array_equal(a, b), (k, np.abs(a - b).max())
    nz = float(np.abs(ref["g_x0"].cpu().numpy()).max())
    assert nz > 0
    s.close()
    return s.info


def test_noalloc_equals_rollout_grad_two_calls_second_smaller():
    # first call: contact chains with a controller-free tape in the mode the
    # memory limit picks; second call, smaller: arms (its scratch content is
    # the first call's)
    a = W.uneven_chains(n_envs=24, T=80, seed_salt=3)
    a.extra["grad_mem_limit"] = 64 << 20
    _say("case no-alloc: uneven-chains 24 x 80")
    ia = _both(a)
    b = W.planar_arms(n_envs=8, T=60)
    _say("case no-alloc: planar-arms 8 x 60 (smaller, after the first)")
    ib = _both(b)
    assert ib.workspace_bytes < ia.workspace_bytes


def test_noalloc_with_a_controller_then_a_smaller_model():
    # the controller's tape rows and weight-gradient partials live in the
    # scratch too
    q = W.quadruped(n_envs=6, T_min=20, T_max=35, mlp_w=W.mlp_init(zero_output=False, out_scale=0.1))
    _say("case no-alloc: quadruped 6 x 20..35 with the controller")
    iq = _both(q, controls=np.asarray(q.extra["mlp"]["w"], np.float32))
    c = W.uneven_chains(n_envs=3, T=30, seed_salt=8)
    _say("case no-alloc: uneven-chains 3 x 30 (smaller)")
    ic = _both(c)
    assert ic.workspace_bytes < iq.workspace_bytes


def test_noalloc_refuses_a_workspace_beyond_the_scratch():
    import torch
    from paper_1611_01652_amd.sim import NOALLOC_SCRATCH_BYTES, SimError, Simulator
    w = W.uneven_chains(n_envs=64, T=400, seed_salt=2)
    _say("case no-alloc: refusal of a large workspace")
    s = Simulator(w)
    assert s.info.workspace_bytes > NOALLOC_SCRATCH_BYTES
    x0, u = to_dev(w)
    ck = torch.zeros(max(int(s.info.ckpt_floats), 1), device="cuda")
    with pytest.raises(SimError, match="exceeds the allocation-free scratch"):
        s.rollout_grad(x0, u, ck, torch.ones(w.n_envs, device="cuda"), no_alloc=True)
    s.close()
