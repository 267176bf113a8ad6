"""Pins of the FP64 oracle's servo motors (section 2.1: gain, maximal torque
and maximal velocity; the arm of section 3.2 has 30 1/s, 30 N m, 45 deg/s).

Each expected value comes from the motor law or mechanics, never from the
oracle itself.  A sphere centred on a world hinge (the motor row is then
decoupled from the hinge's other rows) is driven by a servo:

* below both limits the hinge rate after one step is exactly
  gain (theta* - theta), with the hinge angle read from a constructed pose
* a large error gives exactly +-vmax
* a weak motor saturates: the rate is the torque limit times dt over the
  inertia about the axis
* over many steps the angle converges monotonically to the target
* between free bodies the motor's impulses are internal: the change of total
  angular momentum over a step is still the moment of the hinge's point
  impulses at anchor points err apart (the motor adds none)
* with servos the tape entries are target angles, not torques: a zero tape
  on a hanging arm holds it near zero angle instead of letting it fall
* the reverse-mode gradient with respect to the target angles and the
  initial state equals central differences, with the motor below its limits,
  at them on some steps, and at them on nearly all
"""
import math

import numpy as np
import pytest

from oracle import Oracle
from paper_1611_01652_amd import workloads as W

F32 = lambda v: float(np.float32(v))   # noqa: E731


def _hinged(theta0, gain, torque, vmax, T=1, r=0.05):
    """Sphere centred on a world hinge along y, rotated -theta0 (hinge angle
    -theta0), no gravity."""
    w = W.pendulum(L=0.0, r=r, theta0=theta0, T=T, dt=0.001)
    w.gravity = (0.0, 0.0, 0.0)
    return W.with_servos(w, gain=gain, torque=torque, vmax=vmax)


def _hinge_angle(x):
    R = x[3:12].reshape(3, 3)
    ub = R @ np.array([1.0, 0.0, 0.0])
    return math.atan2(np.cross([1.0, 0.0, 0.0], ub) @ np.array([0.0, 1.0, 0.0]), ub[0])


def test_rate_below_the_limits_is_gain_times_error():
    w = _hinged(0.1, gain=5.0, torque=30.0, vmax=math.radians(45.0))
    x0 = np.asarray(w.x0, np.float64)
    th = _hinge_angle(x0[0])
    assert th == pytest.approx(-0.1, abs=1e-7)
    for target in (0.0, -0.05, -0.2):
        x1, _ = Oracle(w).step(x0, None, np.array([target]), 0)
        assert x1[0, 16] == pytest.approx(F32(5.0) * (target - th), rel=1e-11)
        assert abs(x1[0, 15]) < 1e-12 and abs(x1[0, 17]) < 1e-12


@pytest.mark.parametrize("target", [1.0, -1.2])
def test_large_error_runs_at_the_velocity_limit(target):
    vmax = math.radians(45.0)
    w = _hinged(0.1, gain=30.0, torque=30.0, vmax=vmax)
    x1, _ = Oracle(w).step(np.asarray(w.x0, np.float64), None, np.array([target]), 0)
    assert x1[0, 16] == pytest.approx(math.copysign(F32(vmax), target), rel=1e-11)


@pytest.mark.parametrize("target", [0.0, 0.5, -0.6])
def test_weak_motor_saturates_at_its_torque(target):
    # 0.5 rad/s asked of a 1e-3 kg m^2 sphere in 1 ms needs 0.5 N m; 0.05
    # allowed (the target angle is not also applied as a torque)
    w = _hinged(0.1, gain=5.0, torque=0.05, vmax=math.radians(45.0))
    x1, lam = Oracle(w).step(np.asarray(w.x0, np.float64), None, np.array([target]), 0)
    inv_i = float(w.inv_inertia[0, 1])
    sgn = 1.0 if target > -0.1 else -1.0
    assert x1[0, 16] == pytest.approx(sgn * inv_i * F32(0.05) * F32(0.001), rel=1e-11)
    assert lam[5] == pytest.approx(sgn * F32(0.05) * F32(0.001), rel=1e-12)


def test_motor_acts_about_the_parent_axis():
    # the child tilted 0.2 rad off the hinge axis: the hinge's angular rows
    # pull it back, and the motor sets the rate about the parent's axis (y)
    w = _hinged(0.1, gain=5.0, torque=30.0, vmax=math.radians(45.0))
    Rt = np.asarray(w.x0[0, 3:12], np.float64).reshape(3, 3) @ W._rot((1, 0, 0), 0.2)
    x0 = np.asarray(w.x0, np.float64).copy()
    x0[0, 3:12] = Rt.reshape(9)
    ub = Rt @ np.array([1.0, 0.0, 0.0])
    th = math.atan2(np.cross([1.0, 0.0, 0.0], ub)[1], ub[0])
    x1, _ = Oracle(w).step(x0, None, np.array([0.0]), 0)
    assert x1[0, 16] == pytest.approx(F32(5.0) * (0.0 - th), rel=1e-9)
    assert abs(x1[0, 15]) > 1.0   # the realignment about x is under way


def test_angle_converges_to_the_target():
    w = _hinged(0.3, gain=5.0, torque=30.0, vmax=math.radians(45.0), T=2000)
    w.u = np.full((2000, 1), 0.2, np.float32)
    tr = Oracle(w).rollout(traj=True)["traj"][:, 0, :]
    err = np.array([abs(F32(0.2) - _hinge_angle(x)) for x in tr])
    assert err[0] == pytest.approx(0.5, abs=1e-6)
    assert (np.diff(err) <= 1e-12).all()
    assert err[-1] < 1e-3


def test_free_chain_with_servos_keeps_the_angular_momentum_balance():
    base = W.free_chain(n=5, T=40, torque_sigma=0.0)
    w = W.with_servos(base, gain=30.0, torque=2.0, vmax=2.0,
                      targets=W.servo_targets(40, base.n_joints, amp=0.8, hold=10))
    o = Oracle(w)
    m, I = 1.0 / w.inv_mass, 1.0 / w.inv_inertia
    x, lam = w.x0.astype(np.float64), np.zeros(o.lam_size)
    worst, motor = 0.0, 0.0
    for t in range(40):
        xn, ln = o.step(x, lam, w.u[t], t)
        if t >= 2:   # after the first renormalisations R is orthonormal to ~1e-9
            dL = _ang_mom(xn, m, I, R_at=x) - _ang_mom(x, m, I)
            mom, scale = np.zeros(3), 0.0
            for j in range(w.n_joints):
                a, b = w.joint_parent[j], w.joint_child[j]
                Ra, Rb = x[a, 3:12].reshape(3, 3), x[b, 3:12].reshape(3, 3)
                err = (x[b, :3] + Rb @ w.anchor_c[j]) - (x[a, :3] + Ra @ w.anchor_p[j])
                Lam = ln[6 * j:6 * j + 3]
                mom += np.cross(err, Lam)
                scale += np.linalg.norm(Lam)
                motor = max(motor, abs(ln[6 * j + 5]))
            worst = max(worst, np.linalg.norm(dL - mom) / max(scale, 1e-12))
        x, lam = xn, ln
    assert motor > 1e-3   # the motors acted
    assert worst < 1e-7, worst


def _ang_mom(x, m, I, R_at=None):
    L = np.zeros(3)
    for b in range(x.shape[0]):
        R = (x if R_at is None else R_at)[b, 3:12].reshape(3, 3)
        L += np.cross(x[b, :3], m[b] * x[b, 12:15]) + R @ np.diag(I[b]) @ R.T @ x[b, 15:18]
    return L


def test_zero_tape_holds_a_hanging_arm():
    # a pendulum released 0.3 rad from the bottom: without servos a zero
    # torque tape lets it swing through the bottom; with a servo the zero
    # tape is a target angle of 0 and the arm settles there
    free = W.pendulum(L=0.5, r=0.05, theta0=0.3, T=3000, dt=0.001)
    held = W.with_servos(free, gain=10.0, torque=30.0, vmax=2.0)
    th_free = [_hinge_angle(x) for x in Oracle(free).rollout(traj=True)["traj"][:, 0, :]]
    th_held = [_hinge_angle(x) for x in Oracle(held).rollout(traj=True)["traj"][:, 0, :]]
    assert min(th_free) < -0.25 and max(th_free) > 0.25   # swings to the other side
    assert max(abs(v) for v in th_held[-500:]) < 1e-3
    assert all(v <= 1e-9 for v in th_held)   # approaches 0 from below, never overshooting


def _fd_check(w, keys, h=1e-6, tol=1e-6):
    o = Oracle(w)
    g = o.rollout_grad()
    base_u = np.asarray(w.u, np.float64)
    for key, idx in keys:
        if key == "g_u":
            up, um = base_u.copy(), base_u.copy()
            up[idx] += h
            um[idx] -= h
            wp, wm = W.with_servos(w, w.servo_gain, w.servo_torque, w.servo_vmax), \
                W.with_servos(w, w.servo_gain, w.servo_torque, w.servo_vmax)
            wp.u, wm.u = up, um
            fd = (Oracle(wp).rollout()["loss"].sum() - Oracle(wm).rollout()["loss"].sum()) / (2 * h)
        else:
            x0 = np.asarray(w.x0, np.float64)
            xp, xm = x0.copy(), x0.copy()
            xp[idx] += h
            xm[idx] -= h
            fd = (o.rollout(x0=xp)["loss"].sum() - o.rollout(x0=xm)["loss"].sum()) / (2 * h)
        got = g[key][idx]
        assert abs(got - fd) <= tol * max(abs(fd), 1e-3), (key, idx, got, fd)


@pytest.mark.parametrize("gain,torque,vmax,sat_lo,sat_hi", [(5.0, 200.0, 10.0, 0, 0), (10.0, 50.0, 3.0, 20, 200),
                                                           (30.0, 0.4, 0.6, 300, 360)])
def test_gradient_through_servos_equals_central_differences(gain, torque, vmax, sat_lo, sat_hi):
    # a 3-link arm, gravity in its plane, following held targets: limits never
    # reached, reached on some steps, and reached on nearly all
    base = W.planar_arms(n_envs=1, T=120, seed_salt=3)
    base.gravity = (0.0, -9.81, 0.0)
    w = W.with_servos(base, gain=gain, torque=torque, vmax=vmax,
                      targets=W.servo_targets(120, base.n_joints, amp=0.8, hold=30))
    keys = [("g_u", (t, j)) for t, j in ((0, 0), (15, 1), (29, 2), (45, 0), (90, 2))]
    keys += [("g_x0", (1, 16)), ("g_x0", (2, 0)), ("g_x0", (0, 12))]
    _fd_check(w, keys)
    # the regime asked for: motor impulses at the torque limit
    o = Oracle(w)
    x, lam = np.asarray(w.x0, np.float64), np.zeros(o.lam_size)
    sat = 0
    for t in range(120):
        x, lam = o.step(x, lam, w.u[t], t)
        sat += sum(abs(abs(lam[6 * j + 5]) - F32(torque) * F32(w.dt)) < 1e-12 for j in range(w.n_joints))
    assert sat_lo <= sat <= sat_hi, sat
