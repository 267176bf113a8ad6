"""GPU parity of the differentiable camera (section 3.4) against the FP64
oracle: images and the gradient of sum(w * image) with respect to every
body's position and rotation.

Which object a ray hits is a discrete decision that FP32 and FP64 can take
differently for a ray that grazes a silhouette, so the comparison covers the
pixels whose hit object the oracle keeps when every body moves by 1e-4 (at
least 85 % of them): there the images agree to 1e-4 (colours in [0, 1]) and
the gradients, with the weights on those pixels only, to 1e-3 relative per
env and array (positions, rotations), the tolerance of the state gradients.
The reduction is in a fixed order, so the gradient is bitwise reproducible.
"""
from __future__ import annotations

import time

import numpy as np
import pytest

from gpu_helpers import GRAD_TOL, rel
from oracle import Camera, Oracle
from paper_1611_01652_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _ocam(c):
    o = Camera()
    o.pos[:] = [float(v) for v in c["pos"]]
    o.axes[:] = [float(v) for v in np.asarray(c["axes"]).reshape(9)]
    o.focal, o.pitch, o.width, o.height = c["focal"], c["pitch"], c["width"], c["height"]
    return o


def _scene(n_envs=6, steps=40, seed_salt=31, sizes=None):
    # chains of 3..12 spheres after some steps of falling and tumbling (turned
    # bodies), seen from the side and above
    if sizes is None:
        sizes = np.random.default_rng(seed_salt).integers(3, 13, n_envs)
    n_envs = len(sizes)
    w = W.uneven_chains(n_envs=n_envs, T=steps, seed_salt=seed_salt, sizes=sizes)
    o = Oracle(w)
    x, lam = np.asarray(w.x0, np.float64), np.zeros(o.lam_size)
    for t in range(steps):
        x, lam = o.step(x, lam, w.u[t], t)
    x = W.f32(x)
    return w, x


def _stable_mask(o, cam, ts, tg, cell, x, eps=1e-4):
    base = o.render(cam, ts, tg, cell, x=x)
    stable = np.ones(base.shape, bool)
    for k in (0, 1, 2):
        for s in (-eps, eps):
            xp = x.copy()
            xp[:, k] += s
            stable &= np.abs(o.render(cam, ts, tg, cell, x=xp) - base) < 1e-2
    return base, stable


# (50 x 31 = 1550 pixels: six full workgroups of 256 and a ragged tail of 14;
# the last case puts envs at the gradient's limit of 16 spheres)
@pytest.mark.parametrize("width,height,sizes", [(96, 48, None), (288, 96, None), (50, 31, None),
                                                (96, 48, (16, 2, 16, 9))])
def test_images_and_gradients_match_oracle(width, height, sizes):
    import torch
    from paper_1611_01652_amd.sim import Simulator
    w, x = _scene(sizes=None if sizes is None else np.array(sizes))
    cam = W.pinhole_camera((0.3, -3.5, 1.6), (0.0, 0.0, 0.3), focal=1.0, pitch=1.6 / width, width=width,
                           height=height)
    ts, tg, cell = W.synthetic_texture(32, 16, 3), W.synthetic_texture(24, 24, 4), 0.25
    o = Oracle(w)
    oc = _ocam(cam)
    ref, stable = _stable_mask(o, oc, ts, tg, cell, x)
    _say(f"case camera {width}x{height}, {w.n_envs} envs, stable pixels {stable.mean():.3f}, "
         f"pixels that hit an object {(ref > 0).mean():.3f}")
    assert stable.mean() >= 0.85
    s = Simulator(w)
    xd = torch.tensor(np.ascontiguousarray(x.T), dtype=torch.float32, device="cuda")
    tsd = torch.tensor(ts, dtype=torch.float32, device="cuda")
    tgd = torch.tensor(tg, dtype=torch.float32, device="cuda")
    img = s.render(xd, cam, tsd, tgd, cell).cpu().numpy().astype(np.float64)
    err = np.abs(img - ref)[stable]
    _say("   image: max error on stable pixels", err.max(), "pixels that differ elsewhere",
         int((np.abs(img - ref)[~stable] > 1e-4).sum()))
    assert err.max() <= 1e-4
    # gradient of sum(w * image), weights on the stable pixels
    wts = np.random.default_rng(7).normal(size=ref.shape) * stable
    g_ref = o.render_grad(oc, ts, tg, cell, wts, x=x)
    wd = torch.tensor(wts, dtype=torch.float32, device="cuda")
    g1 = s.render_grad(xd, cam, tsd, tgd, cell, wd)
    g2 = s.render_grad(xd, cam, tsd, tgd, cell, wd)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    g = g1.cpu().numpy().T.astype(np.float64)
    worst = 0.0
    for e in range(w.n_envs):
        b = slice(w.env_body_off[e], w.env_body_off[e + 1])
        for cols in (slice(0, 3), slice(3, 12)):
            worst = max(worst, rel(g[b, cols], g_ref[b, cols]))
    _say("   gradient: worst relative error per env and array", worst)
    assert worst <= GRAD_TOL
    assert np.abs(g[:, 12:]).max() == 0.0


def test_image_of_an_env_with_more_spheres_than_one_staging_chunk():
    # 70 unjointed spheres in one env (no pair contacts, so the model fits the
    # step's LDS): the image kernel stages an env's spheres 64 at a time, and
    # the nearest hit must be found across the chunks; a ragged frame
    import torch
    from paper_1611_01652_amd.sim import Simulator
    rng = np.random.default_rng(41)
    n = 70
    pos = np.column_stack([rng.uniform(-1.0, 1.0, n), rng.uniform(-1.0, 1.0, n), rng.uniform(0.1, 0.9, n)])
    w = W.free_spheres(pos, rng.uniform(0.05, 0.15, n), rng.uniform(0.5, 2.0, n), T=1)
    w.sphere_flags = (np.asarray(w.sphere_flags) & ~2).astype(np.int32)
    cam = W.pinhole_camera((0.2, -3.0, 1.2), (0.0, 0.0, 0.4), focal=1.0, pitch=1.6 / 40, width=40, height=27)
    ts, tg, cell = W.synthetic_texture(32, 16, 8), W.synthetic_texture(24, 24, 9), 0.25
    o = Oracle(w)
    ref, stable = _stable_mask(o, _ocam(cam), ts, tg, cell, W.f32(np.asarray(w.x0, np.float64)))
    _say(f"case camera {n} spheres in one env, 40x27, stable pixels {stable.mean():.3f}, "
         f"pixels that show a sphere or the ground {(ref > 0).mean():.3f}")
    assert stable.mean() >= 0.85
    s = Simulator(w)
    xd = torch.tensor(np.ascontiguousarray(w.x0.T), dtype=torch.float32, device="cuda")
    tsd = torch.tensor(ts, dtype=torch.float32, device="cuda")
    tgd = torch.tensor(tg, dtype=torch.float32, device="cuda")
    img = s.render(xd, cam, tsd, tgd, cell)
    err = np.abs(img.cpu().numpy().astype(np.float64) - ref)[stable]
    _say("   image: max error on stable pixels", err.max())
    assert err.max() <= 1e-4


def test_too_many_spheres_for_the_gradient_is_refused():
    import torch
    from paper_1611_01652_amd.sim import SimError, Simulator
    w = W.uneven_chains(n_envs=2, T=4, seed_salt=1, sizes=np.array([17, 3]))
    s = Simulator(w)
    cam = W.pinhole_camera((0.0, -3.0, 1.0), (0.0, 0.0, 0.3), width=16, height=8)
    xd = torch.tensor(np.ascontiguousarray(w.x0.T), dtype=torch.float32, device="cuda")
    t = torch.full((4, 4), 0.5, device="cuda")
    img = s.render(xd, cam, t, t, 0.5)
    torch.cuda.synchronize()
    assert img.shape == (2, 8, 16)
    with pytest.raises(SimError):
        s.render_grad(xd, cam, t, t, 0.5, torch.ones_like(img))


def test_camera_throughput():
    # the paper's frame size on 1024 envs of the chain distribution (up to
    # 16 spheres): pixels per second of the image and of its gradient
    import torch
    from paper_1611_01652_amd.sim import Simulator
    rng = np.random.default_rng(11)
    w = W.uneven_chains(n_envs=1024, T=4, seed_salt=12, sizes=rng.integers(2, 17, 1024))
    s = Simulator(w)
    cam = W.pinhole_camera((0.3, -3.5, 1.6), (0.0, 0.0, 0.3), focal=1.0, pitch=1.6 / 288, width=288, height=96)
    xd = torch.tensor(np.ascontiguousarray(w.x0.T), dtype=torch.float32, device="cuda")
    tsd = torch.tensor(W.synthetic_texture(64, 32, 5), dtype=torch.float32, device="cuda")
    tgd = torch.tensor(W.synthetic_texture(64, 64, 6), dtype=torch.float32, device="cuda")
    img = s.render(xd, cam, tsd, tgd, 0.25)
    wd = torch.ones_like(img)
    s.render_grad(xd, cam, tsd, tgd, 0.25, wd)
    torch.cuda.synchronize()
    n_pix = img.numel()
    out = {}
    for name, fn in (("render", lambda: s.render(xd, cam, tsd, tgd, 0.25)),
                     ("render_grad", lambda: s.render_grad(xd, cam, tsd, tgd, 0.25, wd))):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            fn()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 5
        out[name] = (ms, n_pix / (ms * 1e-3))
    _say("   camera 1024 envs x 288 x 96:", {k: f"{v[0]:.2f} ms, {v[1]:.3g} pixels/s" for k, v in out.items()})
    assert torch.isfinite(img).all()
