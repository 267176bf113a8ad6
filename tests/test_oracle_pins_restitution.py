"""Pins of the FP64 oracle's restitution and final-state loss (the ball of
section 2.1.1: diameter 1 m, friction 1, restitution 0.5, asked to lie still
at (10, 0) after 5 s, its six initial velocities optimised by gradient
descent through time).

Each expected value comes from mechanics or a construction, never from the
oracle itself:

* a sphere touching the ground and falling at v takes, in one step, the
  vertical velocity -e (v - g dt): restitution reverses e times the approach
  speed at the predicted velocity, for e = 1/4, 1/2, 1; a sphere a little
  above the ground that would reach it within the step bounces the same way;
  one that would not reach it falls freely; one approaching slower than the
  threshold stops dead (the plain contact); a deep penetration leaves at the
  Baumgarte push-out speed when that is the faster
* a dropped ball: every bounce obeys the same law, the bounces end once the
  approach is slower than the threshold, and the ball then lies still
* two equal spheres meeting head-on with no gravity: momentum is conserved
  and the relative velocity is reversed and scaled by e
* e = 0 everywhere leaves every result bit for bit as without restitution,
  and a resting ball with e > 0 does not move
* the final-state loss of a body in free flight is the closed form
  |p_xy(T) - target|^2 + |v|^2 + |omega|^2 with its gradient; through
  bounces, sliding and rolling the reverse-mode gradient with respect to the
  six initial velocities equals central differences
* gradient descent on the six parameters, started from a throw with
  backspin, meets the paper's criterion (0.01 m from the target, speeds below
  0.01) at 5 s
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_1611_01652_amd import workloads as W

F32 = lambda v: float(np.float32(v))   # noqa: E731
G_DT = F32(9.81) * F32(0.01)


def _ball(p, v, w=(0, 0, 0), e=0.5, T=1, mu=1.0, gravity=(0.0, 0.0, -9.81)):
    wl = W.single_sphere(p=p, v=v, w=w, r=0.5, mu=mu, T=T, dt=0.01, gravity=gravity)
    wl.restitution = np.array([e], np.float32)
    return wl


@pytest.mark.parametrize("e", [0.25, 0.5, 1.0])
def test_touching_ball_rebounds_at_e_times_its_approach(e):
    vz = -3.0
    w = _ball((0, 0, 0.5), (0, 0, vz), e=e)
    x1 = Oracle(w).rollout()["x_final"][0]
    e32 = F32(e)
    assert x1[14] == pytest.approx(-e32 * (vz - G_DT), rel=1e-12, abs=1e-12)
    assert np.abs(x1[[12, 13, 15, 16, 17]]).max() < 1e-12


def test_ball_that_reaches_the_ground_within_the_step_bounces():
    vz = -3.0
    # gap 0.01 m: the predicted approach (3.0981 m/s over 10 ms) closes it
    x1 = Oracle(_ball((0, 0, 0.51), (0, 0, vz))).rollout()["x_final"][0]
    assert x1[14] == pytest.approx(-0.5 * (vz - G_DT), rel=1e-12)
    # gap 0.04 m (a contact candidate, margin 0.05): not reached, free fall
    x1 = Oracle(_ball((0, 0, 0.54), (0, 0, vz))).rollout()["x_final"][0]
    assert x1[14] == pytest.approx(vz - G_DT, rel=1e-12)


def test_deep_penetration_keeps_the_faster_push_out():
    # 0.2 m deep: Baumgarte asks for beta 0.2 m / dt = 4 m/s, faster than
    # e times the 1.1 m/s approach, so the push-out decides
    x1 = Oracle(_ball((0, 0, 0.3), (0, 0, -1.0))).rollout()["x_final"][0]
    gap = F32(0.3) - F32(0.5)
    assert x1[14] == pytest.approx(-F32(0.2) * gap / F32(0.01), rel=1e-12)
    # 0.01 m deep, fast approach: e times the approach is the faster
    x1 = Oracle(_ball((0, 0, 0.49), (0, 0, -3.0))).rollout()["x_final"][0]
    assert x1[14] == pytest.approx(-0.5 * (-3.0 - G_DT), rel=1e-12)


def test_slow_approach_does_not_bounce():
    # 0.3 m/s is below the 0.5 m/s threshold: the plain contact stops it
    x1 = Oracle(_ball((0, 0, 0.5), (0, 0, -0.3))).rollout()["x_final"][0]
    assert abs(x1[14]) < 1e-12
    assert x1[2] == pytest.approx(0.5, abs=1e-12)


def test_dropped_ball_bounces_by_the_law_then_rests():
    T = 400
    w = _ball((0, 0, 1.5), (0, 0, 0), T=T)
    tr = Oracle(w).rollout(traj=True)["traj"][:, 0, :]
    vz = tr[:, 14]
    ups = [t for t in range(T) if vz[t] < 0 and vz[t + 1] > 0]
    assert len(ups) >= 3
    for t in ups:
        assert vz[t + 1] == pytest.approx(-0.5 * (vz[t] - G_DT), rel=1e-12)
        assert vz[t] - G_DT < -0.5   # bounced: approach above the threshold
    # the last bounce came down faster than the threshold; after it the ball rests
    last = ups[-1]
    assert np.abs(tr[-1, 12:18]).max() < 1e-9
    assert tr[-1, 2] == pytest.approx(0.5, abs=1e-6)
    # an approach slower than the threshold after the last bounce
    down = [t for t in range(last + 1, T) if vz[t] < 0 and vz[t + 1] >= -1e-12 and tr[t + 1, 2] < 0.5 + 1e-6]
    assert down and vz[down[0]] - G_DT > -0.5


@pytest.mark.parametrize("e", [0.0, 0.5, 1.0])
def test_equal_spheres_head_on(e):
    w = W.free_spheres([(0, 0, 2), (1.0, 0, 2)], [0.5, 0.5], [1.0, 1.0],
                       velocities=np.array([[1.0, 0, 0], [-1.0, 0, 0]]), ground=False, gravity=(0, 0, 0))
    w.restitution = np.array([e], np.float32)
    x1 = Oracle(w).rollout()["x_final"]
    e32 = F32(e)
    assert x1[0, 12] == pytest.approx(-e32, abs=1e-12)
    assert x1[1, 12] == pytest.approx(e32, abs=1e-12)
    assert abs(x1[0, 12] + x1[1, 12]) < 1e-12
    assert np.abs(x1[:, [13, 14, 15, 16, 17]]).max() < 1e-12


def test_zero_restitution_is_bitwise_no_restitution():
    w = W.uneven_chains(n_envs=6, T=60, seed_salt=3)
    a = Oracle(w).rollout_grad()
    w.restitution = np.zeros(w.n_envs, np.float32)
    b = Oracle(w).rollout_grad()
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def test_resting_ball_with_restitution_does_not_move():
    w = W.paper_ball(T=200)
    o = Oracle(w)
    r = o.rollout()
    np.testing.assert_array_equal(r["x_final"], np.asarray(w.x0, np.float64))
    # the loss is the squared distance to the target, nothing else
    assert r["loss"][0] == pytest.approx(100.0, abs=1e-12)


def test_final_state_loss_in_free_flight_closed_form():
    v, om, T = np.array([1.5, -0.5, 0.25]), np.array([0.3, -0.2, 0.7]), 37
    w = W.paper_ball(v0=v, w0=om, T=T)
    w.ground, w.gravity = 0, (0.0, 0.0, 0.0)
    v32, w32 = np.float32(v).astype(np.float64), np.float32(om).astype(np.float64)
    x0 = np.asarray(w.x0[0], np.float64)
    pT = x0[:3] + T * F32(0.01) * v32
    d = pT[:2] - np.array([10.0, 0.0])
    o = Oracle(w)
    L = o.rollout()["loss"][0]
    assert L == pytest.approx(d @ d + v32 @ v32 + w32 @ w32, rel=1e-12)
    g = o.rollout_grad()["g_x0"][0]
    gv = 2 * np.append(d, 0.0) * T * F32(0.01) + 2 * v32
    np.testing.assert_allclose(g[12:15], gv, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(g[15:18], 2 * w32, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(g[0:2], 2 * d, rtol=1e-10)


@pytest.mark.parametrize("v0,w0,T", [((3, 1, 4), (2, -5, 1), 150), ((2, -1, 3), (1, 2, -3), 200),
                                     ((5, 0, 5), (0, -15, 0), 300)])
def test_gradient_through_bounces_equals_central_differences(v0, w0, T):
    w = W.paper_ball(v0=v0, w0=w0, T=T)
    o = Oracle(w)
    g = o.rollout_grad()["g_x0"][0, 12:18]
    x0 = np.asarray(w.x0, np.float64)
    h = 1e-6
    fd = np.zeros(6)
    for i, k in enumerate(range(12, 18)):
        xp, xm = x0.copy(), x0.copy()
        xp[0, k] += h
        xm[0, k] -= h
        fd[i] = (o.rollout(x0=xp)["loss"][0] - o.rollout(x0=xm)["loss"][0]) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-6 * np.abs(fd).max()


def test_gradient_descent_reaches_the_target():
    """Gradient descent with momentum from a throw with backspin; from rest
    the descent settles in a rolling optimum instead (a rolling ball keeps its
    speed in this model), so the start is a throw."""
    th = np.array([5.0, 0.0, 5.0, 0.0, -15.0, 0.0])
    vel = np.zeros(6)
    done = False
    for it in range(600):
        w = W.paper_ball(v0=th[:3], w0=th[3:])
        o = Oracle(w)
        xf = o.rollout()["x_final"][0]
        if (np.hypot(xf[0] - 10.0, xf[1]) < 0.01 and np.linalg.norm(xf[12:15]) < 0.01
                and np.linalg.norm(xf[15:18]) < 0.01):
            done = True
            break
        g = o.rollout_grad()["g_x0"][0, 12:18]
        vel = 0.9 * vel - 0.02 * g
        th = th + vel
    assert done, (it, xf)
