"""Seeded synthetic workloads shaped like the paper's robot models.

This module only *builds inputs*: body masses and inertias, sphere geometry,
hinge frames, initial poses, control tapes and loss targets.  It contains no
part of the time step itself (no forces, no constraint rows, no solver, no
integration), so that both the FP64 oracle and the GPU path can consume the
identical inputs without sharing any of the method's arithmetic.

Every floating-point value is drawn in float64 and rounded to float32, then
stored as float64 again: both sides therefore see exactly the same
FP32-representable numbers, and input rounding is never part of a parity
error.

Model format (flat arrays over all environments, CSR offsets per env):

=================  =========  ====================================================
key                shape      meaning
=================  =========  ====================================================
env_body_off       [E+1]      first body of each env (global body index)
env_joint_off      [E+1]      first joint of each env
env_sphere_off     [E+1]      first collision sphere of each env
inv_mass           [B]        1/m
inv_inertia        [B,3]      inverse of the diagonal body-frame inertia
sphere_body        [S]        global body index carrying the sphere
sphere_offset      [S,3]      sphere centre in the body frame
sphere_radius      [S]
sphere_flags       [S]        bit 0: touches the ground, bit 1: touches spheres
joint_parent       [J]        global body index, or -1 for the world
joint_child        [J]        global body index
anchor_p/anchor_c  [J,3]      hinge point in parent (or world) / child frame
axis_p/axis_c      [J,3]      unit hinge axis in parent (or world) / child frame
perp_p/perp_c      [J,3]      unit vector perpendicular to the axis, per frame
damping            [J]        viscous joint damping [N m s / rad]
mu                 [E]        Coulomb friction coefficient of the env
loss_body          [E]        global body index whose centre enters the loss
target             [E,3]      loss target
T_env              [E]        steps simulated for the env (<= T_max)
x0                 [B,18]     p(3), R(9, row-major), v(3), omega(3) per body
u                  [T_max,J]  joint torque tape (None for a controller)
=================  =========  ====================================================

Scalars: dt, gravity (3), beta, gamma, spec_margin, n_iters, warm (factor on
carried impulses), ground (0/1), loss_kind, loss_mask, T_max.  Bodies connected by a joint never collide.
Each body carries at most one sphere with bit 1 set.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, Optional

import numpy as np

SEED_BASE = 1611016520

# loss kinds (the per-env task cost l(x, p) of the paper's eq. (L))
LOSS_FINAL_SQDIST = 0   # sum_k mask_k (p_k(T) - target_k)^2
LOSS_MEAN_DIST = 1      # (1/T) sum_{t=1..T} |mask*(p(t) - target)|
LOSS_NEG_MEAN_VELX = 2  # -(p_x(T) - p_x(0)) / (T dt)
LOSS_FINAL_STATE = 3    # sum_k mask_k (p_k(T) - target_k)^2 + |v(T)|^2 + |omega(T)|^2

SPHERE_GROUND = 1
SPHERE_PAIR = 2


def f32(a):
    """Round to float32 and widen back, so both sides see identical values."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def rng_for(cfg: int, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + cfg + 1000 * salt))


def _rot(axis, ang):
    """Rotation matrix about a unit axis (Rodrigues), for building poses."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    k = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * k + (1 - math.cos(ang)) * (k @ k)


@dataclass
class Workload:
    name: str
    n_envs: int
    env_body_off: np.ndarray
    env_joint_off: np.ndarray
    env_sphere_off: np.ndarray
    inv_mass: np.ndarray
    inv_inertia: np.ndarray
    sphere_body: np.ndarray
    sphere_offset: np.ndarray
    sphere_radius: np.ndarray
    sphere_flags: np.ndarray
    joint_parent: np.ndarray
    joint_child: np.ndarray
    anchor_p: np.ndarray
    anchor_c: np.ndarray
    axis_p: np.ndarray
    axis_c: np.ndarray
    perp_p: np.ndarray
    perp_c: np.ndarray
    damping: np.ndarray
    mu: np.ndarray
    loss_body: np.ndarray
    target: np.ndarray
    T_env: np.ndarray
    x0: np.ndarray
    u: Optional[np.ndarray]
    dt: float = 0.01
    gravity: tuple = (0.0, 0.0, -9.81)
    beta: float = 0.2
    gamma: float = 0.0
    spec_margin: float = 0.05
    n_iters: int = 20
    warm: float = 0.85
    ground: int = 1
    loss_kind: int = LOSS_FINAL_SQDIST
    loss_mask: int = 7
    T_max: int = 0
    ckpt_every: int = 50
    min_team: int = 0
    grad_decay: float = 1.0   # alpha: carried adjoints shrink by this per step (1: exact gradient)
    restitution: Optional[np.ndarray] = None   # [E] coefficient e per env (None: 0)
    rest_threshold: float = 0.5                # approach speed (m/s) below which no bounce
    # servo motors: with servo_gain set, every hinge is a velocity motor and u
    # holds target angles; gain (1/s), maximal torque (N m), maximal rate (rad/s) [J]
    servo_gain: Optional[np.ndarray] = None
    servo_torque: Optional[np.ndarray] = None
    servo_vmax: Optional[np.ndarray] = None
    extra: Dict = field(default_factory=dict)

    @property
    def n_bodies(self):
        return int(self.env_body_off[-1])

    @property
    def n_joints(self):
        return int(self.env_joint_off[-1])

    @property
    def n_spheres(self):
        return int(self.env_sphere_off[-1])

    def subset(self, envs) -> "Workload":
        """A new workload holding only the listed envs (order kept)."""
        envs = [int(e) for e in envs]
        bo, jo, so = self.env_body_off, self.env_joint_off, self.env_sphere_off
        bidx = np.concatenate([np.arange(bo[e], bo[e + 1]) for e in envs]) if envs else np.zeros(0, int)
        jidx = np.concatenate([np.arange(jo[e], jo[e + 1]) for e in envs]) if envs else np.zeros(0, int)
        sidx = np.concatenate([np.arange(so[e], so[e + 1]) for e in envs]) if envs else np.zeros(0, int)
        bmap = -np.ones(self.n_bodies + 1, dtype=np.int64)
        bmap[bidx] = np.arange(len(bidx))

        def remap(a):
            a = np.asarray(a, dtype=np.int64)
            return np.where(a < 0, -1, bmap[np.maximum(a, 0)]).astype(np.int32)

        def offs(o):
            return np.concatenate([[0], np.cumsum([o[e + 1] - o[e] for e in envs])]).astype(np.int32)

        return Workload(
            name=self.name + "-subset", n_envs=len(envs),
            env_body_off=offs(bo), env_joint_off=offs(jo), env_sphere_off=offs(so),
            inv_mass=self.inv_mass[bidx], inv_inertia=self.inv_inertia[bidx],
            sphere_body=remap(self.sphere_body[sidx]), sphere_offset=self.sphere_offset[sidx],
            sphere_radius=self.sphere_radius[sidx], sphere_flags=self.sphere_flags[sidx],
            joint_parent=remap(self.joint_parent[jidx]), joint_child=remap(self.joint_child[jidx]),
            anchor_p=self.anchor_p[jidx], anchor_c=self.anchor_c[jidx],
            axis_p=self.axis_p[jidx], axis_c=self.axis_c[jidx],
            perp_p=self.perp_p[jidx], perp_c=self.perp_c[jidx], damping=self.damping[jidx],
            mu=self.mu[envs], loss_body=remap(self.loss_body[envs]), target=self.target[envs],
            T_env=self.T_env[envs], x0=self.x0[bidx],
            u=None if self.u is None else self.u[:, jidx],
            dt=self.dt, gravity=self.gravity, beta=self.beta, gamma=self.gamma,
            spec_margin=self.spec_margin, n_iters=self.n_iters, warm=self.warm, ground=self.ground,
            loss_kind=self.loss_kind, loss_mask=self.loss_mask, T_max=self.T_max,
            ckpt_every=self.ckpt_every, min_team=self.min_team, grad_decay=self.grad_decay,
            restitution=None if self.restitution is None else self.restitution[envs],
            rest_threshold=self.rest_threshold,
            servo_gain=None if self.servo_gain is None else self.servo_gain[jidx],
            servo_torque=None if self.servo_torque is None else self.servo_torque[jidx],
            servo_vmax=None if self.servo_vmax is None else self.servo_vmax[jidx], extra=dict(self.extra))

    def with_steps(self, T: int) -> "Workload":
        """Same model, horizon cut to T steps (tape truncated)."""
        import copy
        w = copy.copy(self)
        w.T_max = int(T)
        w.T_env = np.minimum(self.T_env, T).astype(np.int32)
        w.u = None if self.u is None else self.u[:T].copy()
        return w


class _Builder:
    """Accumulates bodies/joints/spheres env by env."""

    def __init__(self):
        self.bodies = []   # (inv_mass, inv_inertia[3], x0[18])
        self.joints = []   # dict
        self.spheres = []  # (body, offset, radius, flags)
        self.env_b = [0]
        self.env_j = [0]
        self.env_s = [0]

    def body(self, mass, inertia_diag, p, R, v=(0, 0, 0), w=(0, 0, 0)):
        x = np.zeros(18)
        x[0:3] = p
        x[3:12] = np.asarray(R).reshape(9)
        x[12:15] = v
        x[15:18] = w
        self.bodies.append((1.0 / mass, 1.0 / np.asarray(inertia_diag, dtype=np.float64), x))
        return len(self.bodies) - 1

    def sphere(self, body, offset, radius, flags):
        self.spheres.append((body, np.asarray(offset, dtype=np.float64), radius, flags))

    def joint(self, parent, child, anchor_p, anchor_c, axis_p, axis_c, perp_p, perp_c, damping):
        self.joints.append(dict(parent=parent, child=child, anchor_p=anchor_p, anchor_c=anchor_c,
                                axis_p=axis_p, axis_c=axis_c, perp_p=perp_p, perp_c=perp_c,
                                damping=damping))

    def end_env(self):
        self.env_b.append(len(self.bodies))
        self.env_j.append(len(self.joints))
        self.env_s.append(len(self.spheres))

    def arrays(self):
        B, J, S = len(self.bodies), len(self.joints), len(self.spheres)
        out = dict(
            env_body_off=np.array(self.env_b, np.int32), env_joint_off=np.array(self.env_j, np.int32),
            env_sphere_off=np.array(self.env_s, np.int32),
            inv_mass=f32([b[0] for b in self.bodies]),
            inv_inertia=f32(np.array([b[1] for b in self.bodies]).reshape(B, 3)),
            x0=f32(np.array([b[2] for b in self.bodies]).reshape(B, 18)),
            sphere_body=np.array([s[0] for s in self.spheres], np.int32).reshape(S),
            sphere_offset=f32(np.array([s[1] for s in self.spheres]).reshape(S, 3)),
            sphere_radius=f32(np.array([s[2] for s in self.spheres]).reshape(S)),
            sphere_flags=np.array([s[3] for s in self.spheres], np.int32).reshape(S),
        )
        jk = ["anchor_p", "anchor_c", "axis_p", "axis_c", "perp_p", "perp_c"]
        out["joint_parent"] = np.array([j["parent"] for j in self.joints], np.int32).reshape(J)
        out["joint_child"] = np.array([j["child"] for j in self.joints], np.int32).reshape(J)
        for k in jk:
            out[k] = f32(np.array([j[k] for j in self.joints], dtype=np.float64).reshape(J, 3))
        out["damping"] = f32(np.array([j["damping"] for j in self.joints]).reshape(J))
        return out


def sphere_inertia(m, r):
    return [0.4 * m * r * r] * 3


def box_inertia(m, a, b, c):
    return [m / 12 * (b * b + c * c), m / 12 * (a * a + c * c), m / 12 * (a * a + b * b)]


def rod_inertia(m, L, eps=0.01):
    return [m / 12 * eps * eps, m / 12 * L * L, m / 12 * L * L]


# --------------------------------------------------------------------------
# cfg1: ball throw (paper section 2.1.1, batch 1)
# --------------------------------------------------------------------------
def ball_throw(seed_salt: int = 0, T: int = 300) -> Workload:
    rng = rng_for(1, seed_salt)
    v0 = rng.uniform(-2.0, 6.0, size=3)
    tgt = np.array([rng.uniform(1.0, 5.0), rng.uniform(-1.0, 1.0), 0.0])
    r, m = 0.1, 1.0
    b = _Builder()
    b.body(m, sphere_inertia(m, r), p=(0, 0, r), R=np.eye(3), v=v0)
    b.sphere(0, (0, 0, 0), r, SPHERE_GROUND)
    b.end_env()
    a = b.arrays()
    return Workload(name="ball-throw", n_envs=1, **a, mu=f32([1.0]), loss_body=np.array([0], np.int32),
                    target=f32(tgt[None]), T_env=np.array([T], np.int32), u=np.zeros((T, 0)),
                    dt=0.01, ground=1, loss_kind=LOSS_FINAL_SQDIST, loss_mask=3, T_max=T,
                    ckpt_every=50)


def shell_inertia(m, r):
    return [2.0 / 3.0 * m * r * r] * 3


def paper_ball(v0=(0.0, 0.0, 0.0), w0=(0.0, 0.0, 0.0), n_envs: int = 1, T: int = 500, dt: float = 0.01,
               e: float = 0.5, mu: float = 1.0, target=(10.0, 0.0)) -> Workload:
    """The ball of section 2.1.1: 1 m diameter, friction 1, restitution 0.5,
    starting at rest on the ground at (0, 0) and asked to lie still at (10, 0)
    after 5 s (T = 500 steps of 10 ms).  The six parameters are the initial
    velocity and angular velocity.  Mass 1 kg with a thin-shell inertia
    (2/3 m r^2), as a soccer ball.  The loss is the squared xy distance to
    the target plus |v|^2 + |omega|^2 at T.  v0 and w0 are [3] or [n_envs, 3]."""
    r, m = 0.5, 1.0
    v0 = np.broadcast_to(np.asarray(v0, np.float64), (n_envs, 3))
    w0 = np.broadcast_to(np.asarray(w0, np.float64), (n_envs, 3))
    b = _Builder()
    for k in range(n_envs):
        b.body(m, shell_inertia(m, r), p=(0, 0, r), R=np.eye(3), v=v0[k], w=w0[k])
        b.sphere(k, (0, 0, 0), r, SPHERE_GROUND)
        b.end_env()
    a = b.arrays()
    tg = np.array([target[0], target[1], 0.0])
    return Workload(name="paper-ball", n_envs=n_envs, **a, mu=f32(np.full(n_envs, mu)),
                    loss_body=np.arange(n_envs, dtype=np.int32), target=f32(np.tile(tg, (n_envs, 1))),
                    T_env=np.full(n_envs, T, np.int32), u=np.zeros((T, 0)), dt=dt, ground=1,
                    loss_kind=LOSS_FINAL_STATE, loss_mask=3, T_max=T, ckpt_every=50,
                    restitution=f32(np.full(n_envs, e)))


def paper_ball_throws(n_envs: int = 256, T: int = 500, seed_salt: int = 0) -> Workload:
    """A batch of the section 2.1.1 ball with seeded throws: initial velocity
    (U(2, 10), U(-2, 2), U(0, 6)) m/s and angular velocity (U(-5, 5),
    U(-25, 5), U(-5, 5)) rad/s (mostly backspin), each asked to lie still at
    (10, 0) after T steps."""
    rng = rng_for(11, seed_salt)
    v0 = np.stack([rng.uniform(2, 10, n_envs), rng.uniform(-2, 2, n_envs), rng.uniform(0, 6, n_envs)], 1)
    w0 = np.stack([rng.uniform(-5, 5, n_envs), rng.uniform(-25, 5, n_envs), rng.uniform(-5, 5, n_envs)], 1)
    w = paper_ball(v0=v0, w0=w0, n_envs=n_envs, T=T)
    w.name = "paper-ball-throws"
    return w


# --------------------------------------------------------------------------
# cfg2: planar 3-link arms, open-loop torque tape
# --------------------------------------------------------------------------
def planar_arms(n_envs: int = 4096, T: int = 1000, seed_salt: int = 0, n_links: int = 3) -> Workload:
    rng = rng_for(2, seed_salt)
    b = _Builder()
    r_pt = 0.05
    base = np.array([0.0, 0.0, 1.0])
    targets = []
    for e in range(n_envs):
        L = rng.uniform(0.3, 0.6, size=n_links)
        m = rng.uniform(0.5, 2.0, size=n_links)
        th = rng.uniform(-0.5, 0.5, size=n_links)
        phi = 0.0
        pos = base.copy()
        ids = []
        for i in range(n_links):
            phi += th[i]
            Rz = _rot((0, 0, 1), phi)
            pos = pos + L[i] * np.array([math.cos(phi), math.sin(phi), 0.0])
            ids.append(b.body(m[i], sphere_inertia(m[i], r_pt), p=pos, R=Rz))
        for i in range(n_links):
            parent = ids[i - 1] if i > 0 else -1
            anchor_p = (0, 0, 0) if i > 0 else tuple(base)
            b.joint(parent, ids[i], anchor_p, (-L[i], 0, 0), (0, 0, 1), (0, 0, 1), (1, 0, 0), (1, 0, 0), 0.1)
        rad = rng.uniform(0.2, 0.9 * L.sum())
        ang = rng.uniform(-math.pi, math.pi)
        targets.append([rad * math.cos(ang), rad * math.sin(ang), base[2]])
        b.end_env()
    a = b.arrays()
    J = n_links * n_envs
    u = f32(rng.normal(0.0, 0.5, size=(T, J)))
    ee = a["env_body_off"][1:] - 1
    return Workload(name="planar-arms", n_envs=n_envs, **a, mu=f32(np.zeros(n_envs)),
                    loss_body=ee.astype(np.int32), target=f32(np.array(targets)),
                    T_env=np.full(n_envs, T, np.int32), u=u, dt=0.005, ground=0, gravity=(0.0, 0.0, 0.0),
                    loss_kind=LOSS_MEAN_DIST, loss_mask=7, T_max=T, ckpt_every=50)


# --------------------------------------------------------------------------
# cfg4: uneven 3D hinge chains of spheres with ground and self contact
# --------------------------------------------------------------------------
def chain_sizes(n_envs, rng, lo=2, hi=32):
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi + 1), size=n_envs))).astype(int).clip(lo, hi)


def uneven_chains(n_envs: int = 16384, T: int = 500, seed_salt: int = 0, sizes=None) -> Workload:
    rng = rng_for(4, seed_salt)
    if sizes is None:
        sizes = chain_sizes(n_envs, rng)
    b = _Builder()
    targets, mus = [], []
    for e in range(n_envs):
        nb = int(sizes[e])
        r = rng.uniform(0.05, 0.15, size=nb)
        m = rng.uniform(0.5, 2.0, size=nb)
        axes = [np.array([0.0, 1.0, 0.0]) if i % 2 == 0 else np.array([0.0, 0.0, 1.0]) for i in range(nb - 1)]
        ang = rng.uniform(-0.5, 0.5, size=max(nb - 1, 0))
        yaw0 = rng.uniform(-math.pi, math.pi)
        clear = rng.uniform(0.2, 0.7)
        Rs = [_rot((0, 0, 1), yaw0)]
        ps = [np.zeros(3)]
        d = [r[i] + r[i + 1] + 0.05 for i in range(nb - 1)]
        for i in range(nb - 1):
            Rn = Rs[i] @ _rot(axes[i], ang[i])
            pn = ps[i] + Rs[i] @ np.array([d[i] / 2, 0, 0]) + Rn @ np.array([d[i] / 2, 0, 0])
            Rs.append(Rn)
            ps.append(pn)
        lowest = min(ps[i][2] - r[i] for i in range(nb))
        lift = clear - lowest
        ids = []
        for i in range(nb):
            p = ps[i] + np.array([0, 0, lift])
            ids.append(b.body(m[i], sphere_inertia(m[i], r[i]), p=p, R=Rs[i]))
            b.sphere(ids[-1], (0, 0, 0), r[i], SPHERE_GROUND | SPHERE_PAIR)
        for i in range(nb - 1):
            b.joint(ids[i], ids[i + 1], (d[i] / 2, 0, 0), (-d[i] / 2, 0, 0), axes[i], axes[i],
                    (1, 0, 0), (1, 0, 0), 0.05)
        targets.append([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.0, 0.5)])
        mus.append(rng.uniform(0.3, 1.0))
        b.end_env()
    a = b.arrays()
    J = int(a["env_joint_off"][-1])
    u = f32(rng.normal(0.0, 0.2, size=(T, J)))
    tip = a["env_body_off"][1:] - 1
    return Workload(name="uneven-chains", n_envs=n_envs, **a, mu=f32(mus), loss_body=tip.astype(np.int32),
                    target=f32(np.array(targets)), T_env=np.full(n_envs, T, np.int32), u=u,
                    dt=0.005, ground=1, loss_kind=LOSS_FINAL_SQDIST, loss_mask=7, T_max=T,
                    ckpt_every=50)


WSN_SIZES = (7, 64, 64, 3)     # per-contact warm-start network
WSN_PARAMS = 7 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3


def warm_start_chains(n_envs: int = 16384, T: int = 500, seed_salt: int = 0, tol: float = 1e-5,
                      max_iters: int = 1000, ws_w=None, fb_iters: int = 5, fb_tol: float = 1e-3) -> Workload:
    """The uneven-chain distribution solved to a residual tolerance instead of
    a fixed sweep count, with the plain warm start at factor 1 (the carried
    impulses themselves) or, with ws_w, the learned warm start of contacts."""
    w = uneven_chains(n_envs=n_envs, T=T, seed_salt=seed_salt)
    w.name = "warm-start-chains"
    w.warm = 1.0
    w.extra = dict(w.extra or {})
    w.extra["solve"] = dict(mode=1, tol=float(tol), max_iters=int(max_iters))
    if ws_w is not None:
        w.extra["ws"] = dict(w=np.asarray(ws_w, np.float64), fb_iters=int(fb_iters), fb_tol=float(fb_tol))
    return w


def wsn_init(seed_salt: int = 0, scale: float = 1.0, zero_output: bool = False) -> np.ndarray:
    """Seeded He-uniform initial weights of the warm-start network, FP32
    values: W1[64][7] b1[64] W2[64][64] b2[64] W3[3][64] b3[3].  With
    zero_output the output layer is zero: the network then leaves the carried
    impulses unchanged (the plain warm start)."""
    rng = rng_for(5, seed_salt)
    parts = []
    for fan_in, fan_out in ((7, 64), (64, 64), (64, 3)):
        lim = scale * math.sqrt(6.0 / fan_in)
        wl = rng.uniform(-lim, lim, size=fan_out * fan_in)
        parts.append(np.zeros_like(wl) if (zero_output and fan_out == 3) else wl)
        parts.append(np.zeros(fan_out))
    return f32(np.concatenate(parts))


# --------------------------------------------------------------------------
# small hand-made models for closed-form checks
# --------------------------------------------------------------------------
def single_sphere(p, v=(0, 0, 0), w=(0, 0, 0), r=0.1, m=1.0, mu=1.0, ground=True, T=100, dt=0.01,
                  gravity=(0.0, 0.0, -9.81), n_iters=20, R=None) -> Workload:
    b = _Builder()
    b.body(m, sphere_inertia(m, r), p=p, R=np.eye(3) if R is None else R, v=v, w=w)
    b.sphere(0, (0, 0, 0), r, SPHERE_GROUND if ground else 0)
    b.end_env()
    a = b.arrays()
    return Workload(name="sphere", n_envs=1, **a, mu=f32([mu]), loss_body=np.array([0], np.int32),
                    target=f32(np.zeros((1, 3))), T_env=np.array([T], np.int32), u=np.zeros((T, 0)),
                    dt=dt, gravity=tuple(gravity), ground=int(ground), loss_kind=LOSS_FINAL_SQDIST,
                    loss_mask=7, T_max=T, n_iters=n_iters)


def pendulum(L=1.0, m=1.0, r=0.05, theta0=0.1, T=200, dt=0.001, damping=0.0, n_iters=20,
             beta=0.2) -> Workload:
    """A sphere hanging from a world hinge whose axis is y; swings in the x-z plane."""
    b = _Builder()
    pivot = np.array([0.0, 0.0, 2.0])
    # body hangs at angle theta0 from -z toward +x; the rotation of the
    # body frame follows the rod so that the anchor stays at (0, 0, L) local.
    Ry = _rot((0, 1, 0), -theta0)
    p = pivot + Ry @ np.array([0.0, 0.0, -L])
    bi = b.body(m, sphere_inertia(m, r), p=p, R=Ry)
    b.joint(-1, bi, tuple(pivot), (0, 0, L), (0, 1, 0), (0, 1, 0), (1, 0, 0), (1, 0, 0), damping)
    b.end_env()
    a = b.arrays()
    return Workload(name="pendulum", n_envs=1, **a, mu=f32([0.0]), loss_body=np.array([0], np.int32),
                    target=f32(np.zeros((1, 3))), T_env=np.array([T], np.int32), u=np.zeros((T, 1)),
                    dt=dt, ground=0, loss_kind=LOSS_FINAL_SQDIST, loss_mask=7, T_max=T,
                    n_iters=n_iters, beta=beta)


def free_chain(n=4, T=200, dt=0.005, seed_salt=0, gravity=(0.0, 0.0, 0.0), ground=False,
               torque_sigma=0.3) -> Workload:
    """A free-floating 3D chain (the uneven-chain recipe at a fixed size)."""
    w = uneven_chains(n_envs=1, T=T, seed_salt=seed_salt, sizes=[n])
    w.gravity = tuple(gravity)
    w.ground = int(ground)
    rng = rng_for(9, seed_salt)
    w.u = f32(rng.normal(0.0, torque_sigma, size=(T, w.n_joints)))
    w.dt = dt
    w.x0 = w.x0.copy()
    # random initial body velocities so that momentum is non-trivial
    w.x0[:, 12:18] = f32(rng.normal(0.0, 0.5, size=(w.n_bodies, 6)))
    return w


def free_spheres(positions, radii, masses, velocities=None, mu=0.0, ground=True, T=1, dt=0.01,
                 n_iters=20, gravity=(0.0, 0.0, -9.81)) -> Workload:
    """Unjointed spheres in one env, each touching the ground and each other."""
    b = _Builder()
    n = len(positions)
    velocities = np.zeros((n, 3)) if velocities is None else velocities
    for i in range(n):
        bi = b.body(masses[i], sphere_inertia(masses[i], radii[i]), p=positions[i], R=np.eye(3), v=velocities[i])
        b.sphere(bi, (0, 0, 0), radii[i], SPHERE_GROUND | SPHERE_PAIR)
    b.end_env()
    a = b.arrays()
    return Workload(name="spheres", n_envs=1, **a, mu=f32([mu]), loss_body=np.array([0], np.int32),
                    target=f32(np.zeros((1, 3))), T_env=np.array([T], np.int32), u=np.zeros((T, 0)),
                    dt=dt, gravity=tuple(gravity), ground=int(ground), loss_kind=LOSS_FINAL_SQDIST,
                    loss_mask=7, T_max=T, n_iters=n_iters)


def with_servos(w: Workload, gain=30.0, torque=30.0, vmax=math.radians(45.0), targets=None) -> Workload:
    """A copy of a workload whose hinges are all servo motors (section 2.1;
    the arm of section 3.2 has gain 30 1/s, 30 N m and 45 deg/s): the control
    tape then holds target angles (rad), `targets` [T, J] or the given
    workload's tape as it stands."""
    import copy
    s = copy.copy(w)
    J = w.n_joints
    s.servo_gain = f32(np.broadcast_to(np.asarray(gain, np.float64), (J,)))
    s.servo_torque = f32(np.broadcast_to(np.asarray(torque, np.float64), (J,)))
    s.servo_vmax = f32(np.broadcast_to(np.asarray(vmax, np.float64), (J,)))
    if targets is not None:
        s.u = f32(targets)
    s.name = w.name + "-servo"
    return s


def servo_targets(T: int, J: int, seed_salt: int = 0, amp: float = 0.6, hold: int = 40) -> np.ndarray:
    """Seeded target-angle tape [T, J]: uniform targets in [-amp, amp] rad,
    each held for `hold` steps."""
    rng = rng_for(12, seed_salt)
    n = (T + hold - 1) // hold
    return f32(np.repeat(rng.uniform(-amp, amp, size=(n, J)), hold, axis=0)[:T])


def servo_arms(n_envs: int = 96, T: int = 300, gain: float = 10.0, torque: float = 50.0, vmax: float = 3.0,
               seed_salt: int = 3) -> Workload:
    """3-link arms with gravity in their plane, every hinge a servo following
    seeded targets held for 30 steps."""
    base = planar_arms(n_envs=n_envs, T=T, seed_salt=seed_salt)
    base.gravity = (0.0, -9.81, 0.0)
    return with_servos(base, gain=gain, torque=torque, vmax=vmax,
                       targets=servo_targets(T, base.n_joints, seed_salt=seed_salt, amp=0.8, hold=30))


def servo_chains(n_envs: int = 40, T: int = 100, gain: float = 20.0, torque: float = 5.0, vmax: float = 3.0,
                 seed_salt: int = 2) -> Workload:
    """The uneven chains with every hinge a servo following seeded targets
    held for 25 steps."""
    base = uneven_chains(n_envs=n_envs, T=T, seed_salt=seed_salt)
    return with_servos(base, gain=gain, torque=torque, vmax=vmax,
                       targets=servo_targets(T, base.n_joints, seed_salt=seed_salt, amp=0.5, hold=25))


def mlp_param_count(sizes, skip_input_to_output=False):
    """Parameters of a dense net with biases (optionally the output layer also
    reads the input layer, as the gait controller of section 3.3 does)."""
    n = 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        n += a * b + b
    if skip_input_to_output:
        n += sizes[0] * sizes[-1]
    return n


# --------------------------------------------------------------------------
# quadruped with a neural controller (sections 3.1, 3.3)
# --------------------------------------------------------------------------
MLP_SIZES = (18, 128, 128, 8)


def cylinder_z_inertia(m, L, r):
    """Solid cylinder of length L and radius r along the body z axis."""
    return [m * (3 * r * r + L * L) / 12, m * (3 * r * r + L * L) / 12, m * r * r / 2]


def mlp_init(sizes=MLP_SIZES, seed_salt=0, zero_output=True, scale=1.0, out_scale=1.0):
    """Dense net parameters in the order W1[h1][in] b1 W2[h2][h1] b2 W3[out][h2] b3;
    hidden weights N(0, scale^2/fan_in), biases zero, output layer zero
    (the controller starts as the zero policy, section 3.2) or, for tests,
    N(0, out_scale^2/fan_in)."""
    rng = rng_for(3, 100 + seed_salt)
    parts = []
    n = len(sizes) - 1
    for li, (a, b) in enumerate(zip(sizes[:-1], sizes[1:])):
        if li == n - 1 and zero_output:
            W = np.zeros((b, a))
        elif li == n - 1:
            W = rng.normal(0.0, out_scale / math.sqrt(a), size=(b, a))
        else:
            W = rng.normal(0.0, scale / math.sqrt(a), size=(b, a))
        parts += [W.reshape(-1), np.zeros(b)]
    return f32(np.concatenate(parts))


def quadruped(n_envs: int = 1024, T_min: int = 500, T_max: int = 2000, seed_salt: int = 0,
              mlp_w=None, rec: int = 0) -> Workload:
    """Box torso (1 kg, 0.30 x 0.15 x 0.06 m) and four legs of two 0.10 m
    cylinders (r 0.025, 0.125 kg each), hips and knees hinged about the body y
    axis with damping 0.01, sphere feet r = 0.05 touching the ground; legs
    straight and feet on the ground at t = 0.  Four spheres (r = 0.03) inside
    the torso touch the ground too.  (With 75 % of the mass in the torso the
    42 g legs make the explicit damping term unstable at dt = 0.01,
    dt c / I > 2, and the 20-sweep solve diverge under any active policy.)"""
    rng = rng_for(3, seed_salt)
    b = _Builder()
    L, mleg, r_leg, r_foot = 0.10, 0.125, 0.025, 0.05
    hips = [(0.12, 0.09), (0.12, -0.09), (-0.12, 0.09), (-0.12, -0.09)]
    h = 2 * L + r_foot
    mus = []
    for e in range(n_envs):
        yaw = 0.0
        R0 = np.eye(3)
        torso = b.body(1.0, box_inertia(1.0, 0.30, 0.15, 0.06), p=(0, 0, h), R=R0)
        # four spheres inside the cuboid let the spine touch the ground (section 3.1)
        for (sx, sy) in ((0.12, 0.045), (0.12, -0.045), (-0.12, 0.045), (-0.12, -0.045)):
            b.sphere(torso, (sx, sy, 0.0), 0.03, SPHERE_GROUND)
        for (hx, hy) in hips:
            up = b.body(mleg, cylinder_z_inertia(mleg, L, r_leg), p=(hx, hy, h - L / 2), R=R0)
            lo = b.body(mleg, cylinder_z_inertia(mleg, L, r_leg), p=(hx, hy, h - 1.5 * L), R=R0)
            b.sphere(lo, (0, 0, -L / 2), r_foot, SPHERE_GROUND)
            b.joint(torso, up, (hx, hy, 0.0), (0, 0, L / 2), (0, 1, 0), (0, 1, 0), (1, 0, 0), (1, 0, 0), 0.01)
            b.joint(up, lo, (0, 0, -L / 2), (0, 0, L / 2), (0, 1, 0), (0, 1, 0), (1, 0, 0), (1, 0, 0), 0.01)
        mus.append(rng.uniform(0.5, 1.0))
        b.end_env()
        del yaw
    a = b.arrays()
    T_env = rng.integers(T_min, T_max + 1, size=n_envs).astype(np.int32)
    w = Workload(name="quadruped", n_envs=n_envs, **a, mu=f32(mus),
                 loss_body=a["env_body_off"][:-1].astype(np.int32), target=f32(np.zeros((n_envs, 3))),
                 T_env=T_env, u=None, dt=0.01, ground=1, loss_kind=LOSS_NEG_MEAN_VELX, loss_mask=1,
                 T_max=int(T_env.max()), ckpt_every=50)
    sizes = rec_sizes(MLP_SIZES, rec)
    w.extra["mlp"] = dict(sizes=sizes, w=mlp_init(sizes) if mlp_w is None else np.asarray(mlp_w, np.float64),
                          clock_hz=1.5, rec=int(rec))
    return w


def rec_sizes(sizes, rec):
    """Layer sizes of the controller with `rec` recurrent units (eq. (g)): the
    input gains h^t, the output gains the pre-activation of h^{t+1}."""
    return (sizes[0] + rec, sizes[1], sizes[2], sizes[3] + rec)


# --------------------------------------------------------------------------
# the differentiable camera (section 3.4): camera poses and textures
# --------------------------------------------------------------------------
def pinhole_camera(pos, look_at, up=(0.0, 0.0, 1.0), focal=1.0, pitch=1.0 / 144, width=288, height=96) -> dict:
    """A camera at `pos` whose optical axis points at `look_at`: axes rows
    (right, up, optical axis), the projection plane at `focal`, pixels of
    `pitch` on it (the paper's frames are 288 x 96).  Values rounded to
    float32 so both sides see the same camera."""
    pos = np.asarray(pos, np.float64)
    ez = np.asarray(look_at, np.float64) - pos
    ez /= np.linalg.norm(ez)
    ex = np.cross(ez, np.asarray(up, np.float64))
    ex /= np.linalg.norm(ex)
    ey = np.cross(ex, ez)
    return dict(pos=f32(pos), axes=f32(np.stack([ex, ey, ez])), focal=float(f32(focal)), pitch=float(f32(pitch)),
                width=int(width), height=int(height))


def synthetic_texture(nx: int, ny: int, seed_salt: int = 0, n_waves: int = 6) -> np.ndarray:
    """A seeded smooth grayscale texture [ny, nx] in [0, 1]: a sum of plane
    waves that tile the texture (stand-in for the paper's photographs,
    which are not available)."""
    rng = rng_for(13, seed_salt)
    a, b = np.meshgrid(np.arange(nx), np.arange(ny))
    t = np.full((ny, nx), 0.5)
    for _ in range(n_waves):
        kx, ky = rng.integers(-4, 5), rng.integers(-4, 5)
        t += rng.uniform(0.02, 0.08) * np.sin(2 * np.pi * (kx * a / nx + ky * b / ny) + rng.uniform(0, 2 * np.pi))
    return f32(np.clip(t, 0.0, 1.0))
