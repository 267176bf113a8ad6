"""Pins of the oracle's tolerance-mode solve, learned warm start, fallback and
training records, against closed forms, brute force and library routines.

* bfloat16 rounding equals torch's float32 -> bfloat16 conversion (nearest,
  ties to even) on float32 values, ties included.
* the network's index layout: weights that route input k to hidden unit k and
  back out reproduce the (rounded) input exactly; its outputs correct the
  carried impulses (a zero network is the plain warm start).
* a ball at rest: one sweep per step once warm (two on the first step), and
  2 T with a carried impulse scaled by 0.85; its records are the closed forms
  v_n = -g dt, target lambda_n / m_n = g dt, m_n = m, m_t = 2 m / 7.
* to a tight tolerance the frictionless sphere pile reaches the LCP solution
  found by enumerating active sets.
* a learned warm start rejected before any sweep reproduces the plain solve
  bit for bit; rejected after 5 sweeps it costs exactly 5 sweeps per fallback.
* the network reference's Huber loss and gradient against finite differences.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import REC, WSN_PARAMS, Oracle, _load
from paper_1611_01652_amd import workloads as W


def test_parameter_count_of_the_warm_start_network():
    assert WSN_PARAMS == W.WSN_PARAMS == 4867
    assert W.wsn_init().size == 4867


def test_bf16_rounding_equals_torch_conversion():
    import torch
    lib = _load()
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e-3, 1000), rng.normal(0, 300, 1000)])
    x = x.astype(np.float32)
    # exact ties: the 17th bit set and nothing below it
    bits = rng.integers(0, 2 ** 31, size=500, dtype=np.int64).astype(np.uint32)
    ties = ((bits & np.uint32(0xFFFF0000)) | np.uint32(0x8000)).view(np.float32)
    ties = ties[np.isfinite(ties) & (np.abs(ties) > 1e-30) & (np.abs(ties) < 1e30)]
    x = np.concatenate([x, ties])
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([lib.oracle_bf16(float(v)) for v in x])
    np.testing.assert_array_equal(got, ref)


def _routing_net():
    """W1 routes input k to hidden unit k (k < 7) and -x_k to unit 7 + k,
    W2 copies hidden units, W3 takes outputs o = h[4 + o] - h[11 + o]: the net
    returns the rounded inputs 4..6 (the plain warm start over its masses)."""
    I, H, O = 7, 64, 3
    W1 = np.zeros((H, I)); W2 = np.eye(H); W3 = np.zeros((O, H))
    for k in range(I):
        W1[k, k] = 1.0
        W1[I + k, k] = -1.0
    for o in range(O):
        W3[o, 4 + o] = 1.0
        W3[o, I + 4 + o] = -1.0
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3.ravel(), np.zeros(O)])


def _rest(T, warm):
    w = W.single_sphere(p=(0.2, -0.1, 0.1), T=T)
    w.warm = warm
    w.extra = dict(solve=dict(mode=1, tol=1e-5, max_iters=1000))
    return w


@pytest.mark.parametrize("warm,expected", [(1.0, lambda T: T + 1), (0.85, lambda T: 2 * T)])
def test_ball_at_rest_sweep_count(warm, expected):
    T = 50
    r = Oracle(_rest(T, warm)).rollout_ex()
    assert r["iters"][0] == expected(T)
    assert r["fallbacks"][0] == 0


def test_ball_at_rest_records_are_closed_form():
    T = 6
    w = _rest(T, 1.0)
    r = Oracle(w).rollout_ex(rec_every=1, rec_cap=100)
    rec = r["records"]
    assert r["n_records"] == T and rec.shape == (T, REC)
    m = 1.0 / w.inv_mass[0]
    gdt = float(np.float32(9.81)) * float(np.float32(w.dt))
    np.testing.assert_allclose(rec[:, 0], 0.0, atol=1e-15)            # gap / dt
    np.testing.assert_allclose(rec[:, 1], -gdt, rtol=1e-12)            # J_n v at the predicted velocity
    np.testing.assert_allclose(rec[:, 2:4], 0.0, atol=1e-15)           # tangential velocities
    np.testing.assert_allclose(rec[0, 4], 0.0, atol=1e-15)             # no carried impulse at t = 0
    np.testing.assert_allclose(rec[1:, 4], gdt, rtol=1e-12)            # carried m g dt over m_n
    np.testing.assert_allclose(rec[:, 7], gdt, rtol=1e-12)             # converged m g dt over m_n
    np.testing.assert_allclose(rec[:, 8:10], 0.0, atol=1e-15)
    np.testing.assert_allclose(rec[:, 10], m, rtol=1e-12)              # m_n = m
    # m_t = 2/(K11 + K22) with lever arm (0, 0, -r): K11 = 1/m + r^2/I_y, K22 = 1/m + r^2/I_x
    # (= 2 m / 7 for a solid sphere, up to the FP32 rounding of the inputs)
    r2, ii = float(w.sphere_radius[0]) ** 2, w.inv_inertia[0]
    mt = 2.0 / (2.0 * w.inv_mass[0] + r2 * (ii[0] + ii[1]))
    np.testing.assert_allclose(rec[:, 11], mt, rtol=1e-12)
    assert abs(mt - 2.0 * m / 7.0) < 1e-6
    np.testing.assert_array_equal(rec[:, 12], 0)
    np.testing.assert_array_equal(rec[:, 13], np.arange(T))
    np.testing.assert_array_equal(rec[:, 14], (1 << 24) | 0)


def test_zero_network_is_the_plain_warm_start():
    # the network corrects the carried impulses: zero outputs leave them as
    # they are, so the resting ball needs one sweep per step once warm
    T = 30
    w = _rest(T, 1.0)
    w.extra["ws"] = dict(w=np.zeros(W.WSN_PARAMS), fb_iters=5, fb_tol=1e-3)
    r = Oracle(w).rollout_ex()
    assert r["fallbacks"][0] == 0
    assert r["iters"][0] == T + 1
    xp = Oracle(_rest(T, 1.0)).rollout_ex()["x_final"]
    np.testing.assert_allclose(r["x_final"], xp, rtol=0, atol=1e-12)


def test_routing_network_doubles_the_carried_impulse():
    # the routing net returns the rounded carried impulse over its mass, so the
    # learned start is twice the carried one (up to bfloat16 rounding): on the
    # resting ball the first sweep removes the excess, the second confirms
    T = 30
    w = _rest(T, 1.0)
    w.extra["ws"] = dict(w=_routing_net(), fb_iters=5, fb_tol=1e-3)
    r = Oracle(w).rollout_ex()
    assert r["fallbacks"][0] == 0
    assert r["iters"][0] == 2 * T
    xp = Oracle(_rest(T, 1.0)).rollout_ex()["x_final"]
    np.testing.assert_allclose(r["x_final"], xp, rtol=0, atol=1e-9)


def test_frictionless_pile_tolerance_mode_reaches_lcp_solution():
    from test_oracle_pins import _lcp_brute_force
    r = 0.1
    pos = np.array([[0.0, 0.0, r], [0.19, 0.0, r], [0.095, 0.0, r + 0.17]])
    rng = np.random.default_rng(3)
    vel = rng.normal(0, 0.5, size=(3, 3))
    w = W.free_spheres(pos, [r, r, r], [1.0, 2.0, 0.7], velocities=vel, mu=0.0, n_iters=1, T=1)
    w.extra = dict(solve=dict(mode=1, tol=1e-13, max_iters=100000))
    out = Oracle(w).rollout_ex()
    assert 10 < out["iters"][0] < 100000
    # the same LCP as the fixed-sweep pin, solved by enumeration
    P, rad, invm = w.x0[:, :3], w.sphere_radius, w.inv_mass
    dt, beta = float(np.float32(w.dt)), float(np.float32(w.beta))   # the FP32 inputs
    vstar = w.x0[:, 12:15] + dt * np.array([0, 0, -float(np.float32(9.81))])
    rows = []
    for i in range(3):
        C = P[i, 2] - rad[i]
        if C < w.spec_margin:
            J = np.zeros(9); J[3 * i + 2] = 1.0
            rows.append((J, C))
    for i in range(3):
        for j in range(i + 1, 3):
            d = P[j] - P[i]
            L = np.linalg.norm(d)
            C = L - rad[i] - rad[j]
            if C < w.spec_margin:
                n = d / L
                J = np.zeros(9); J[3 * i:3 * i + 3] = -n; J[3 * j:3 * j + 3] = n
                rows.append((J, C))
    Jm = np.array([q[0] for q in rows])
    b = np.array([(max(C, 0) + beta * min(C, 0)) / dt for _, C in rows])
    Minv = np.repeat(invm, 3)
    K = Jm @ (Minv[:, None] * Jm.T)
    lam = _lcp_brute_force(K, Jm @ vstar.reshape(9) + b)
    v_exp = vstar.reshape(9) + Minv * (Jm.T @ lam)
    np.testing.assert_allclose(out["x_final"][:, 12:15].reshape(9), v_exp, rtol=0, atol=1e-9)


def _chains(ws_w=None, fb_iters=5, fb_tol=1e-3):
    return W.warm_start_chains(n_envs=6, T=120, seed_salt=7, ws_w=ws_w, fb_iters=fb_iters, fb_tol=fb_tol)


def test_rejection_before_any_sweep_reproduces_the_plain_solve():
    plain = Oracle(_chains()).rollout_ex()
    rej = Oracle(_chains(ws_w=W.wsn_init(seed_salt=1), fb_iters=0, fb_tol=-1.0)).rollout_ex()
    np.testing.assert_array_equal(rej["x_final"], plain["x_final"])
    np.testing.assert_array_equal(rej["lam_final"], plain["lam_final"])
    np.testing.assert_array_equal(rej["iters"], plain["iters"])
    # every step with at least one row (all steps: the chains have joints)
    np.testing.assert_array_equal(rej["fallbacks"], 120)


def test_rejection_after_five_sweeps_costs_five_sweeps_each():
    plain = Oracle(_chains()).rollout_ex()
    # a network whose normal output is -1000 m/s starts every contact from
    # zero impulses (the projection then zeroes the tangential ones)
    wz = np.zeros(W.WSN_PARAMS)
    wz[4864] = -1000.0
    rej = Oracle(_chains(ws_w=wz, fb_iters=5, fb_tol=-1.0)).rollout_ex()
    off = _chains().env_body_off
    same = np.array([np.array_equal(rej["x_final"][a:b], plain["x_final"][a:b]) for a, b in zip(off[:-1], off[1:])])
    assert same.sum() >= 4, same
    d = rej["iters"] - plain["iters"]
    np.testing.assert_array_equal(d[same], 5 * rej["fallbacks"][same])
    assert (rej["fallbacks"][same] > 0).all()


def test_gradient_is_refused_in_tolerance_mode():
    o = Oracle(_chains())
    lib = o.lib
    import ctypes as C
    z = np.zeros(10 ** 6)
    dp = z.ctypes.data_as(C.POINTER(C.c_double))
    x0 = np.ascontiguousarray(o.w.x0, dtype=np.float64)
    rc = lib.oracle_rollout_grad(C.byref(o._m), x0.ctypes.data_as(C.POINTER(C.c_double)), dp, dp, dp, dp, dp,
                                 dp, dp, dp, None, None, None, 1)
    assert rc == -1


def test_network_reference_gradient_matches_finite_differences():
    from oracle import wsnet
    rng = np.random.default_rng(5)
    w = W.wsn_init(seed_salt=3).astype(np.float64) + rng.normal(0, 0.05, W.WSN_PARAMS)
    X = rng.normal(0, 1, (9, 7))
    T = rng.normal(0, 1, (9, 3))
    L, g = wsnet.loss_grad(w, X, T)
    assert abs(L - ((wsnet.forward(w, X) - T) ** 2).sum() / 9) < 1e-12
    idx = rng.choice(W.WSN_PARAMS, 300, replace=False)
    idx = np.concatenate([idx, np.arange(4864, 4867), np.arange(448, 452)])   # output and first biases
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (wsnet.loss_grad(wp, X, T)[0] - wsnet.loss_grad(wm, X, T)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_network_reference_layout_with_routing_weights():
    from oracle import wsnet
    rng = np.random.default_rng(6)
    X = np.abs(rng.normal(0, 1, (5, 7)))
    # the routing net returns x[:, 4:7] (ReLU of x minus ReLU of -x)
    np.testing.assert_allclose(wsnet.forward(_routing_net(), X), X[:, 4:7], rtol=0, atol=1e-15)
    np.testing.assert_allclose(wsnet.forward(_routing_net(), -X), -X[:, 4:7], rtol=0, atol=1e-15)


def test_adam_first_step_moves_each_weight_by_lr():
    from oracle import wsnet
    g = np.array([3.0, -0.5, 1e-3])
    w, m, v = wsnet.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01, eps=0.0)
    np.testing.assert_allclose(w, -0.01 * np.sign(g), rtol=1e-12)


def test_network_reference_huber_gradient_matches_finite_differences():
    from oracle import wsnet
    rng = np.random.default_rng(8)
    w = W.wsn_init(seed_salt=4).astype(np.float64)
    X = rng.normal(0, 1, (11, 7))
    T = rng.normal(0, 2, (11, 3))
    L, g = wsnet.loss_grad(w, X, T, huber=0.5)
    L2, _ = wsnet.loss_grad(w, X, T)
    assert L < L2                                  # the errors beyond 0.5 are damped
    idx = np.concatenate([rng.choice(W.WSN_PARAMS, 200, replace=False), np.arange(4864, 4867)])
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (wsnet.loss_grad(wp, X, T, huber=0.5)[0] - wsnet.loss_grad(wm, X, T, huber=0.5)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
