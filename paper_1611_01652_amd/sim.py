"""ctypes binding of the C ABI in include/sim.h (argument marshalling only).

Every step of the simulation runs in the HIP library ``libsim_hip.so``; this
module only converts a workload description into ``sim_model_desc``, owns the
handle, and passes device pointers of torch tensors.  There is no CPU path:
loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsim_hip.so")

SIM_OK = 0
FLAG_NONFINITE = 1
FLAG_CONTACT_OVERFLOW = 2

# layout of the descriptor and info structs below (SIM_ABI_VERSION)
ABI_VERSION = 10

# reverse sweep memory modes (sim_model_desc.grad_store)
GRAD_STORE = {"auto": 0, "replay": 1, "segment": 2, "trajectory": 3}

_I32P = C.POINTER(C.c_int32)
_F32P = C.POINTER(C.c_float)


class SimDesc(C.Structure):
    _fields_ = [
        ("n_envs", C.c_int32),
        ("env_body_off", _I32P), ("env_joint_off", _I32P), ("env_sphere_off", _I32P),
        ("inv_mass", _F32P), ("inv_inertia", _F32P),
        ("sphere_body", _I32P), ("sphere_offset", _F32P), ("sphere_radius", _F32P), ("sphere_flags", _I32P),
        ("joint_parent", _I32P), ("joint_child", _I32P),
        ("anchor_p", _F32P), ("anchor_c", _F32P), ("axis_p", _F32P), ("axis_c", _F32P),
        ("perp_p", _F32P), ("perp_c", _F32P), ("damping", _F32P),
        ("mu", _F32P), ("loss_body", _I32P), ("target", _F32P), ("T_env", _I32P),
        ("T_max", C.c_int32), ("dt", C.c_float), ("gravity", C.c_float * 3),
        ("beta", C.c_float), ("gamma", C.c_float), ("spec_margin", C.c_float), ("warm", C.c_float),
        ("n_iters", C.c_int32), ("ground", C.c_int32), ("loss_kind", C.c_int32), ("loss_mask", C.c_int32),
        ("ckpt_every", C.c_int32), ("min_team", C.c_int32),
        ("ctrl_kind", C.c_int32), ("mlp_sizes", C.c_int32 * 4), ("clock_hz", C.c_float),
        ("solve_mode", C.c_int32), ("tol", C.c_float), ("max_iters", C.c_int32),
        ("ws_kind", C.c_int32), ("ws_net", _F32P), ("fb_iters", C.c_int32), ("fb_tol", C.c_float),
        ("grad_store", C.c_int32), ("grad_mem_limit", C.c_int64),
        ("use_grad_decay", C.c_int32), ("grad_decay", C.c_float), ("mlp_rec", C.c_int32),
        ("restitution", _F32P), ("rest_threshold", C.c_float),
        ("servo", C.c_int32), ("servo_gain", _F32P), ("servo_torque", _F32P), ("servo_vmax", _F32P),
    ]


class SimInfo(C.Structure):
    _fields_ = [
        ("n_envs", C.c_int32), ("n_bodies", C.c_int32), ("n_joints", C.c_int32),
        ("lam_size", C.c_int32), ("n_ckpt", C.c_int32),
        ("ckpt_floats", C.c_int64), ("workspace_bytes", C.c_int64),
        ("max_lds_bytes", C.c_int32), ("n_tiles", C.c_int32), ("n_params", C.c_int32),
        ("grad_store", C.c_int32),
    ]


def make_desc(w):
    """Build a SimDesc for a workload; returns (desc, keepalive list)."""
    keep = []

    def f(a):
        arr = np.ascontiguousarray(np.asarray(a, dtype=np.float32)).reshape(-1)
        if arr.size == 0:
            arr = np.zeros(1, np.float32)
        keep.append(arr)
        return arr.ctypes.data_as(_F32P)

    def i(a):
        arr = np.ascontiguousarray(np.asarray(a, dtype=np.int32)).reshape(-1)
        if arr.size == 0:
            arr = np.zeros(1, np.int32)
        keep.append(arr)
        return arr.ctypes.data_as(_I32P)

    d = SimDesc()
    d.n_envs = w.n_envs
    d.env_body_off = i(w.env_body_off)
    d.env_joint_off = i(w.env_joint_off)
    d.env_sphere_off = i(w.env_sphere_off)
    d.inv_mass = f(w.inv_mass)
    d.inv_inertia = f(w.inv_inertia)
    d.sphere_body = i(w.sphere_body)
    d.sphere_offset = f(w.sphere_offset)
    d.sphere_radius = f(w.sphere_radius)
    d.sphere_flags = i(w.sphere_flags)
    d.joint_parent = i(w.joint_parent)
    d.joint_child = i(w.joint_child)
    for k in ("anchor_p", "anchor_c", "axis_p", "axis_c", "perp_p", "perp_c", "damping"):
        setattr(d, k, f(getattr(w, k)))
    d.mu = f(w.mu)
    d.loss_body = i(w.loss_body)
    d.target = f(w.target)
    d.T_env = i(w.T_env)
    d.T_max = w.T_max
    d.dt = w.dt
    d.gravity = (C.c_float * 3)(*w.gravity)
    d.beta, d.gamma, d.spec_margin, d.warm = w.beta, w.gamma, w.spec_margin, w.warm
    d.n_iters, d.ground, d.loss_kind, d.loss_mask = w.n_iters, w.ground, w.loss_kind, w.loss_mask
    d.ckpt_every = w.ckpt_every
    d.min_team = int(getattr(w, 'min_team', 0) or 0)
    mlp = w.extra.get("mlp") if getattr(w, "extra", None) else None
    if mlp is not None:
        d.ctrl_kind = 1
        d.mlp_sizes = (C.c_int32 * 4)(*[int(v) for v in mlp["sizes"]])
        d.clock_hz = float(mlp.get("clock_hz", 1.5))
        d.mlp_rec = int(mlp.get("rec", 0))
    extra = getattr(w, "extra", None) or {}
    d.grad_store = GRAD_STORE[extra.get("grad_store", "auto")]
    d.grad_mem_limit = int(extra.get("grad_mem_limit", 0))
    alpha = float(getattr(w, "grad_decay", 1.0))
    d.use_grad_decay = int(alpha != 1.0)
    d.grad_decay = alpha
    if getattr(w, "restitution", None) is not None:
        d.restitution = f(w.restitution)
    d.rest_threshold = float(getattr(w, "rest_threshold", 0.5))
    if getattr(w, "servo_gain", None) is not None:
        d.servo = 1
        d.servo_gain, d.servo_torque, d.servo_vmax = f(w.servo_gain), f(w.servo_torque), f(w.servo_vmax)
    solve = extra.get("solve")
    if solve is not None:
        d.solve_mode = int(solve.get("mode", 1))
        d.tol = float(solve.get("tol", 1e-5))
        d.max_iters = int(solve.get("max_iters", 1000))
    ws = extra.get("ws")
    if ws is not None:
        d.ws_kind = 1
        d.ws_net = f(ws["w"])
        d.fb_iters = int(ws.get("fb_iters", 5))
        d.fb_tol = float(ws.get("fb_tol", 1e-3))
    return d, keep


_lib = None


def library():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.sim_abi_version.restype = C.c_int
    lib.sim_last_error.restype = C.c_char_p
    lib.sim_init.argtypes = [C.POINTER(SimDesc), C.POINTER(vp)]
    lib.sim_destroy.argtypes = [vp]
    lib.sim_get_info.argtypes = [vp, C.POINTER(SimInfo)]
    lib.sim_lambda_offsets.argtypes = [vp, _I32P]
    lib.sim_step.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int32, vp, vp]
    lib.rollout.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.rollout_grad.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp, vp]
    lib.rollout_grad_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.rollout_keep.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]
    lib.rollout_grad_kept.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp, vp]
    lib.rollout_and_grad.argtypes = [vp] * 18 + [C.c_size_t, vp, vp]
    lib.rollout_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int64, vp, C.c_int32, vp]
    lib.sim_describe_order.argtypes = [C.POINTER(SimDesc), C.c_int32, _I32P, _I32P, C.c_int32]
    lib.sim_describe_order.restype = C.c_int32
    lib.sim_step_graph.argtypes = [vp, C.c_int32, vp, vp, vp, C.c_int32, vp, C.POINTER(vp)]
    lib.sim_graph_launch.argtypes = [vp, vp]
    lib.sim_graph_destroy.argtypes = [vp]
    lib.sim_tune.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, _I32P, C.c_int32, vp]
    lib.sim_tune.restype = C.c_int32
    lib.sim_get_teams.argtypes = [vp, _I32P, C.c_int32]
    lib.sim_get_teams.restype = C.c_int32
    lib.sim_set_teams.argtypes = [vp, _I32P, C.c_int32]
    lib.wsn_to_bf16.argtypes = [vp, vp, vp]
    lib.wsn_forward.argtypes = [vp, vp, C.c_int64, C.c_int64, vp, vp]
    lib.wsn_workspace_bytes.argtypes = [C.c_int64]
    lib.wsn_workspace_bytes.restype = C.c_int64
    lib.wsn_loss_grad.argtypes = [vp, vp, C.c_int64, C.c_int64, C.c_float, C.c_int32, vp, vp, vp, C.c_size_t, vp]
    lib.wsn_adam.argtypes = [vp, vp, vp, vp, vp, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    lib.sim_adam.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float,
                             C.c_float, vp, vp, vp]
    lib.sim_time_grad.argtypes = [vp, C.POINTER(vp)]
    lib.sim_time_buckets.argtypes = [vp, C.POINTER(vp), C.c_int32]
    lib.sim_env_buckets.argtypes = [vp, _I32P]
    lib.sim_render.argtypes = [vp, vp, C.POINTER(SimCamera), C.POINTER(SimTextures), vp, vp]
    lib.sim_render_grad.argtypes = [vp, vp, C.POINTER(SimCamera), C.POINTER(SimTextures), vp, vp, vp]
    for fn in ("sim_time_grad", "sim_init", "sim_destroy", "sim_get_info", "sim_lambda_offsets", "sim_step", "rollout",
               "rollout_grad", "rollout_grad_noalloc", "rollout_keep", "rollout_grad_kept", "sim_time_buckets",
               "sim_env_buckets", "sim_step_graph", "sim_graph_launch", "sim_graph_destroy", "sim_set_teams",
               "wsn_to_bf16", "wsn_forward", "wsn_loss_grad", "wsn_adam", "rollout_solve", "sim_adam", "sim_render",
               "sim_render_grad", "rollout_and_grad"):
        getattr(lib, fn).restype = C.c_int
    if lib.sim_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH} has ABI version {lib.sim_abi_version()}, this binding expects "
                           f"{ABI_VERSION}: rebuild it (__graft_entry__.build())")
    _lib = lib
    return lib


EXPORTED = ["sim_abi_version", "sim_last_error", "sim_init", "sim_destroy", "sim_get_info",
            "sim_lambda_offsets", "sim_describe_order", "sim_step", "rollout", "rollout_grad",
            "sim_step_graph", "sim_graph_launch", "sim_graph_destroy", "sim_tune", "sim_get_teams",
            "sim_set_teams", "wsn_to_bf16", "wsn_forward", "wsn_workspace_bytes", "wsn_loss_grad", "wsn_adam",
            "rollout_solve", "sim_adam", "sim_time_grad", "rollout_grad_noalloc", "sim_time_buckets",
            "sim_env_buckets", "rollout_keep", "rollout_grad_kept", "sim_render", "sim_render_grad",
            "rollout_and_grad"]


class SimCamera(C.Structure):
    """sim_camera: pinhole at pos, axes rows (right, up, optical axis), the
    projection plane at focal, pixel pitch on it, image size."""
    _fields_ = [("pos", C.c_float * 3), ("axes", C.c_float * 9), ("focal", C.c_float), ("pitch", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


class SimTextures(C.Structure):
    _fields_ = [("sphere", C.c_void_p), ("sphere_nx", C.c_int32), ("sphere_ny", C.c_int32),
                ("ground", C.c_void_p), ("ground_nx", C.c_int32), ("ground_ny", C.c_int32),
                ("ground_cell", C.c_float)]


def camera(c):
    """A SimCamera from a dict as workloads.pinhole_camera makes."""
    s = SimCamera()
    s.pos[:] = [float(v) for v in np.asarray(c["pos"]).reshape(3)]
    s.axes[:] = [float(v) for v in np.asarray(c["axes"]).reshape(9)]
    s.focal, s.pitch, s.width, s.height = float(c["focal"]), float(c["pitch"]), int(c["width"]), int(c["height"])
    return s

# bytes of the scratch rollout_grad_noalloc uses (SIM_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20


def describe_order(w, env):
    """Canonical sweep order of one env as computed by the library (host only)."""
    lib = library()
    d, keep = make_desc(w)
    cap = 1 << 16
    codes = np.zeros(cap, np.int32)
    cols = np.zeros(cap, np.int32)
    n = lib.sim_describe_order(C.byref(d), env, codes.ctypes.data_as(_I32P), cols.ctypes.data_as(_I32P), cap)
    if n < 0:
        raise SimError(f"sim_describe_order failed ({n}): {lib.sim_last_error().decode()}")
    return codes[:n].copy(), cols[:n].copy()


class SimError(RuntimeError):
    pass


def _check(lib, st, what):
    if st != SIM_OK:
        raise SimError(f"{what} failed ({st}): {lib.sim_last_error().decode()}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def soa(x_b18):
    """[B,18] -> [18,B] (contiguous)."""
    return x_b18.transpose(0, 1).contiguous() if hasattr(x_b18, "transpose") else np.ascontiguousarray(x_b18.T)


class Simulator:
    """One model on the current HIP device.  Tensors are torch CUDA tensors."""

    def __init__(self, w):
        import torch  # device memory and streams only
        self.torch = torch
        self.lib = library()
        self.w = w
        desc, keep = make_desc(w)
        h = C.c_void_p()
        _check(self.lib, self.lib.sim_init(C.byref(desc), C.byref(h)), "sim_init")
        self.h = h
        info = SimInfo()
        _check(self.lib, self.lib.sim_get_info(h, C.byref(info)), "sim_get_info")
        self.info = info
        lo = np.zeros(w.n_envs + 1, np.int32)
        _check(self.lib, self.lib.sim_lambda_offsets(h, lo.ctypes.data_as(_I32P)), "sim_lambda_offsets")
        self.lam_off = lo
        self._graphs = []

    def close(self):
        for g in list(getattr(self, "_graphs", [])):
            g.close()
        if getattr(self, "h", None):
            self.lib.sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def _controls(self, u):
        """The control input must hold what the library reads from it: the
        controller's weights (n_params floats) or the tape [T_max][J]."""
        need = self.info.n_params if self.info.n_params else self.w.T_max * self.info.n_joints
        if need and (u is None or u.numel() < need or u.dtype != self.torch.float32 or not u.is_cuda
                     or not u.is_contiguous()):
            what = "controller weights" if self.info.n_params else "torque tape [T_max, J]"
            raise ValueError(f"the control input must be a contiguous CUDA float32 tensor of at least {need} "
                             f"floats (the {what})")
        return _ptr(u)

    def _f32(self, n):
        return self.torch.zeros(max(int(n), 1), dtype=self.torch.float32, device="cuda")

    def rollout(self, x0, u, want_ckpt=True, want_final=True, keep=None):
        """x0 [18,B] and u [T_max,J] CUDA float32 tensors.  keep: a workspace
        (trajectory mode) into which the rollout also writes every step's
        saved working set (rollout_keep), for rollout_grad(kept=...)."""
        t = self.torch
        E = self.info.n_envs
        out = dict(loss=self._f32(E), flags=t.zeros(max(E, 1), dtype=t.int32, device="cuda"))
        out["x_final"] = self._f32(18 * self.info.n_bodies).view(18, -1) if want_final else None
        out["lam_final"] = self._f32(self.info.lam_size) if want_final else None
        out["ckpt"] = self._f32(self.info.ckpt_floats) if want_ckpt else None
        if keep is not None:
            st = self.lib.rollout_keep(self.h, _ptr(x0), self._controls(u), _ptr(out["loss"]), _ptr(out["x_final"]),
                                       _ptr(out["lam_final"]), _ptr(out["ckpt"]), _ptr(out["flags"]), _ptr(keep),
                                       keep.numel() * 4, self._stream())
            _check(self.lib, st, "rollout_keep")
        else:
            st = self.lib.rollout(self.h, _ptr(x0), self._controls(u), _ptr(out["loss"]), _ptr(out["x_final"]),
                                  _ptr(out["lam_final"]), _ptr(out["ckpt"]), _ptr(out["flags"]), self._stream())
            _check(self.lib, st, "rollout")
        out["loss"] = out["loss"][:E]
        return out

    def rollout_solve(self, x0, u, rec_cap=0, rec_every=1, want_final=True):
        """Tolerance-mode rollout with sweep / fallback counts per env and, with
        rec_cap > 0, training records (a [n, 16] float32 tensor; columns 12..14
        hold int32 bit patterns of env, step, code)."""
        t = self.torch
        E = self.info.n_envs
        out = dict(loss=self._f32(E), flags=t.zeros(max(E, 1), dtype=t.int32, device="cuda"),
                   iters=t.zeros(max(E, 1), dtype=t.int32, device="cuda"),
                   fallbacks=t.zeros(max(E, 1), dtype=t.int32, device="cuda"))
        out["x_final"] = self._f32(18 * self.info.n_bodies).view(18, -1) if want_final else None
        out["lam_final"] = self._f32(self.info.lam_size) if want_final else None
        rec = t.zeros((max(int(rec_cap), 1), 16), device="cuda") if rec_cap > 0 else None
        cnt = t.zeros(1, dtype=t.int64, device="cuda")
        st = self.lib.rollout_solve(self.h, _ptr(x0), self._controls(u), _ptr(out["loss"]), _ptr(out["x_final"]),
                                    _ptr(out["lam_final"]), _ptr(out["flags"]), _ptr(out["iters"]),
                                    _ptr(out["fallbacks"]), _ptr(rec), int(rec_cap), _ptr(cnt), int(rec_every),
                                    self._stream())
        _check(self.lib, st, "rollout_solve")
        for k in ("loss", "flags", "iters", "fallbacks"):
            out[k] = out[k][:E]
        if rec is not None:
            out["n_records"] = cnt
            out["records"] = rec
        return out

    def workspace(self):
        return self.torch.empty(int(self.info.workspace_bytes) // 4 + 1, dtype=self.torch.float32, device="cuda")

    def rollout_grad(self, x0, u, ckpt, dloss, workspace=None, no_alloc=False, kept=None):
        """Reverse mode (rollout_grad), or with no_alloc the allocation-free
        entry point (rollout_grad_noalloc, the library's own scratch as the
        workspace), or with kept the workspace a rollout(keep=...) filled
        (rollout_grad_kept, no recompute).  The output tensors are allocated
        here either way."""
        ws = None
        if not no_alloc and kept is None:
            ws = workspace if workspace is not None else self.workspace()
        g, outs = self._grad_outputs()
        if kept is not None:
            st = self.lib.rollout_grad_kept(self.h, _ptr(x0), self._controls(u), _ptr(dloss), *outs, _ptr(kept),
                                            kept.numel() * 4, _ptr(g["flags"]), self._stream())
            _check(self.lib, st, "rollout_grad_kept")
        elif no_alloc:
            st = self.lib.rollout_grad_noalloc(self.h, _ptr(x0), self._controls(u), _ptr(ckpt), _ptr(dloss), *outs,
                                               _ptr(g["flags"]), self._stream())
            _check(self.lib, st, "rollout_grad_noalloc")
        else:
            st = self.lib.rollout_grad(self.h, _ptr(x0), self._controls(u), _ptr(ckpt), _ptr(dloss), *outs, _ptr(ws),
                                       ws.numel() * 4, _ptr(g["flags"]), self._stream())
            _check(self.lib, st, "rollout_grad")
        return self._grad_views(g)

    def _grad_outputs(self):
        E, B, J = self.info.n_envs, self.info.n_bodies, self.info.n_joints
        nu = self.info.n_params if self.info.n_params else self.w.T_max * J
        g = dict(g_x0=self._f32(18 * B).view(18, -1), g_u=self._f32(nu),
                 g_inv_mass=self._f32(B), g_inv_inertia=self._f32(3 * B), g_mu=self._f32(E), g_damping=self._f32(J),
                 g_anchor_p=self._f32(3 * J), g_anchor_c=self._f32(3 * J),
                 flags=self.torch.zeros(max(E, 1), dtype=self.torch.int32, device="cuda"))
        outs = [_ptr(g[k]) for k in ("g_x0", "g_u", "g_inv_mass", "g_inv_inertia", "g_mu", "g_damping",
                                     "g_anchor_p", "g_anchor_c")]
        return g, outs

    def _grad_views(self, g):
        E, B, J = self.info.n_envs, self.info.n_bodies, self.info.n_joints
        if self.info.n_params:
            g["g_u"] = g["g_u"][: self.info.n_params]
        else:
            g["g_u"] = g["g_u"][: self.w.T_max * J].view(self.w.T_max, J) if J else g["g_u"][:0]
        g["g_inv_mass"] = g["g_inv_mass"][:B]
        g["g_inv_inertia"] = g["g_inv_inertia"][: 3 * B].view(B, 3)
        g["g_mu"] = g["g_mu"][:E]
        g["flags"] = g["flags"][:E]
        g["g_damping"] = g["g_damping"][:J]
        g["g_anchor_p"] = g["g_anchor_p"][: 3 * J].view(J, 3)
        g["g_anchor_c"] = g["g_anchor_c"][: 3 * J].view(J, 3)
        return g

    def rollout_and_grad(self, x0, u, dloss, workspace, want_ckpt=False, want_final=False):
        """Forward and reverse mode in one call (rollout_and_grad, trajectory
        mode): each size bucket's reverse follows its own forward.  Returns
        (the rollout's outputs, the gradients), as rollout(keep=workspace)
        and rollout_grad(kept=workspace) would."""
        t = self.torch
        E = self.info.n_envs
        out = dict(loss=self._f32(E), flags=t.zeros(max(E, 1), dtype=t.int32, device="cuda"))
        out["x_final"] = self._f32(18 * self.info.n_bodies).view(18, -1) if want_final else None
        out["lam_final"] = self._f32(self.info.lam_size) if want_final else None
        out["ckpt"] = self._f32(self.info.ckpt_floats) if want_ckpt else None
        g, outs = self._grad_outputs()
        st = self.lib.rollout_and_grad(self.h, _ptr(x0), self._controls(u), _ptr(out["loss"]), _ptr(out["x_final"]),
                                       _ptr(out["lam_final"]), _ptr(out["ckpt"]), _ptr(out["flags"]), _ptr(dloss),
                                       *outs, _ptr(workspace), workspace.numel() * 4, _ptr(g["flags"]),
                                       self._stream())
        _check(self.lib, st, "rollout_and_grad")
        out["loss"] = out["loss"][:E]
        out["flags"] = out["flags"][:E]
        return out, self._grad_views(g)

    def render(self, x, cam, tex_sphere, tex_ground, cell, out=None):
        """Image [E, H, W] (CUDA float32) of the state x ([18, B] CUDA
        float32) seen by cam (a dict as workloads.pinhole_camera makes);
        textures are CUDA float32 [ny, nx] tensors (sim_render).  `out`, if
        given, is the image tensor to write."""
        c = camera(cam)
        t = self._textures(tex_sphere, tex_ground, cell)
        shape = (self.info.n_envs, c.height, c.width)
        img = self.torch.empty(shape, dtype=self.torch.float32, device="cuda") if out is None else out
        if tuple(img.shape) != shape or img.dtype != self.torch.float32 or not img.is_cuda or not img.is_contiguous():
            raise ValueError(f"out must be a contiguous CUDA float32 tensor of shape {shape}")
        _check(self.lib, self.lib.sim_render(self.h, _ptr(x), C.byref(c), C.byref(t), _ptr(img), self._stream()),
               "sim_render")
        return img

    def render_grad(self, x, cam, tex_sphere, tex_ground, cell, weights, out=None):
        """dL/dx [18, B] for L = sum(weights * image) (sim_render_grad);
        `out`, if given, is the tensor to write (x's shape)."""
        c = camera(cam)
        t = self._textures(tex_sphere, tex_ground, cell)
        g = self.torch.empty_like(x) if out is None else out
        if g.shape != x.shape or g.dtype != x.dtype or not g.is_cuda or not g.is_contiguous():
            raise ValueError("out must be a contiguous CUDA tensor shaped like x")
        _check(self.lib, self.lib.sim_render_grad(self.h, _ptr(x), C.byref(c), C.byref(t), _ptr(weights), _ptr(g),
                                                  self._stream()), "sim_render_grad")
        return g

    @staticmethod
    def _textures(ts, tg, cell):
        import torch
        for t in (ts, tg):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2:
                raise ValueError("textures must be contiguous 2-D CUDA float32 tensors")
        return SimTextures(ts.data_ptr(), ts.shape[1], ts.shape[0], tg.data_ptr(), tg.shape[1], tg.shape[0],
                           float(cell))

    def time_grad(self, events):
        """Record rollout_grad's phases on 4 torch.cuda.Events (recompute start
        and end, reverse start and end) in every later call; None stops it.
        The events must have been recorded once (torch creates them lazily)
        and must stay alive while set."""
        if events is None:
            st = self.lib.sim_time_grad(self.h, None)
        else:
            raw = [int(e.cuda_event) for e in events]
            if len(raw) != 4 or not all(raw):
                raise ValueError("time_grad needs 4 created events (record each once first)")
            arr = (C.c_void_p * 4)(*raw)
            st = self.lib.sim_time_grad(self.h, arr)
        _check(self.lib, st, "sim_time_grad")

    def time_buckets(self, events):
        """Record each bucket's reverse sweep kernel on events[2 i], events[2 i + 1]
        (torch.cuda.Events, recorded once first, alive while set) in every
        later rollout_grad; None stops it."""
        if events is None:
            st = self.lib.sim_time_buckets(self.h, None, 0)
        else:
            raw = [int(e.cuda_event) for e in events]
            if not all(raw):
                raise ValueError("time_buckets needs created events (record each once first)")
            arr = (C.c_void_p * len(raw))(*raw)
            st = self.lib.sim_time_buckets(self.h, arr, len(raw) // 2)
        _check(self.lib, st, "sim_time_buckets")

    def env_buckets(self):
        """Bucket index of every env ([E] numpy int32)."""
        out = np.zeros(max(self.info.n_envs, 1), np.int32)
        _check(self.lib, self.lib.sim_env_buckets(self.h, out.ctypes.data_as(_I32P)), "sim_env_buckets")
        return out[: self.info.n_envs]

    def step(self, x, u, lam, t_index=0):
        t = self.torch
        xo = t.empty_like(x)
        lo = t.empty_like(lam)
        flags = t.zeros(max(self.info.n_envs, 1), dtype=t.int32, device="cuda")
        st = self.lib.sim_step(self.h, _ptr(x), _ptr(xo), _ptr(u), _ptr(lam), _ptr(lo), int(t_index), _ptr(flags),
                               self._stream())
        _check(self.lib, st, "sim_step")
        return xo, lo, flags

    def step_graph(self, n_steps, x, u, lam, t0=0, flags=None):
        """Capture n_steps steps into a replayable HIP graph.  x is a [2, 18, B]
        CUDA tensor (step k reads x[k % 2], writes x[(k + 1) % 2]); u the
        control rows [n_steps, J] or the controller weights; lam [lam_size],
        updated in place.  The tensors must outlive the graph."""
        g = C.c_void_p()
        st = self.lib.sim_step_graph(self.h, int(n_steps), _ptr(x), _ptr(u), _ptr(lam), int(t0), _ptr(flags),
                                     C.byref(g))
        _check(self.lib, st, "sim_step_graph")
        sg = StepGraph(self, g, (x, u, lam, flags))
        self._graphs.append(sg)
        return sg

    def teams(self):
        n = self.lib.sim_get_teams(self.h, None, 0)
        _check(self.lib, min(n, 0), "sim_get_teams")
        out = np.zeros(max(n, 1), np.int32)
        self.lib.sim_get_teams(self.h, out.ctypes.data_as(_I32P), n)
        return out[:n].copy()

    def set_teams(self, teams):
        teams = np.ascontiguousarray(teams, dtype=np.int32)
        _check(self.lib, self.lib.sim_set_teams(self.h, teams.ctypes.data_as(_I32P), len(teams)), "sim_set_teams")

    def tune(self, x0, u, with_grad=True, max_candidates=3):
        """Time each bucket at its admissible team widths and keep the fastest;
        returns the chosen widths.  Results do not depend on them."""
        n = self.lib.sim_get_teams(self.h, None, 0)
        out = np.zeros(max(n, 1), np.int32)
        r = self.lib.sim_tune(self.h, _ptr(x0), self._controls(u), int(bool(with_grad)), int(max_candidates),
                              out.ctypes.data_as(_I32P), n, self._stream())
        _check(self.lib, min(r, 0), "sim_tune")
        return out[:n].copy()


class StepGraph:
    """A captured sequence of steps (see Simulator.step_graph)."""

    def __init__(self, sim, g, keep):
        self.sim, self.g, self._keep = sim, g, keep

    def launch(self):
        _check(self.sim.lib, self.sim.lib.sim_graph_launch(self.g, self.sim._stream()), "sim_graph_launch")

    def close(self):
        if self.g:
            self.sim.lib.sim_graph_destroy(self.g)
            self.g = None
            if self in self.sim._graphs:
                self.sim._graphs.remove(self)


# ---------------------------------------------------------------- warm-start network
WSN_PARAMS = 4867
REC_FLOATS = 16


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class WarmStartNet:
    """The per-contact warm-start network on the GPU: FP32 master weights, their
    bfloat16 copy used by the kernels, Adam moments.  Tensors are torch CUDA
    tensors; every step runs in the library's kernels."""

    def __init__(self, w0):
        import torch
        self.torch = torch
        self.lib = library()
        self.w = torch.tensor(np.asarray(w0, np.float32), device="cuda").contiguous()
        assert self.w.numel() == WSN_PARAMS
        self.wb = torch.empty(WSN_PARAMS, dtype=torch.int16, device="cuda")
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.grad = torch.zeros_like(self.w)
        self.loss = torch.zeros(1, device="cuda")
        self.step_count = 0
        self._ws = None
        _check(self.lib, self.lib.wsn_to_bf16(_ptr(self.w), _ptr(self.wb), _stream()), "wsn_to_bf16")

    def weights_bf16_as_float(self):
        """The bfloat16 weights the kernels use, as FP32 values (host numpy)."""
        b = self.wb.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        return b.view(np.float32).astype(np.float64)

    def forward(self, x):
        """x: [n, >= 7] CUDA float32 (features in columns 0..6) -> [n, 3]"""
        t = self.torch
        n = x.shape[0]
        y = t.empty((max(n, 1), 3), device="cuda")
        _check(self.lib, self.lib.wsn_forward(_ptr(self.wb), _ptr(x), x.stride(0), n, _ptr(y), _stream()),
               "wsn_forward")
        return y[:n]

    def loss_grad(self, rec, huber=0.0, relative=False):
        """rec: [n, >= 10] CUDA float32 records; returns (loss tensor [1], grad [4867]).
        huber > 0: Huber loss with that threshold; relative: targets are the
        corrections to the carried impulses (record columns 7..9 minus 4..6)."""
        n = rec.shape[0]
        need = int(self.lib.wsn_workspace_bytes(n))
        if self._ws is None or self._ws.numel() * 4 < need:
            self._ws = self.torch.empty(need // 4 + 1, device="cuda")
        st = self.lib.wsn_loss_grad(_ptr(self.wb), _ptr(rec), rec.stride(0), n, float(huber), int(bool(relative)),
                                    _ptr(self.loss), _ptr(self.grad), _ptr(self._ws), self._ws.numel() * 4,
                                    _stream())
        _check(self.lib, st, "wsn_loss_grad")
        return self.loss, self.grad

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        st = self.lib.wsn_adam(_ptr(self.w), _ptr(self.wb), _ptr(self.grad), _ptr(self.m), _ptr(self.v),
                               self.step_count, lr, beta1, beta2, eps, _stream())
        _check(self.lib, st, "wsn_adam")


class Adam:
    """Adam with gradient-norm clipping on a CUDA float32 parameter tensor,
    in the library's kernels."""

    def __init__(self, w, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, max_norm=0.0):
        import torch
        self.torch = torch
        self.lib = library()
        self.w = w
        self.m = torch.zeros_like(w)
        self.v = torch.zeros_like(w)
        self.scratch = torch.zeros(513, device="cuda")
        self.grad_norm = torch.zeros(1, device="cuda")
        self.lr, self.b1, self.b2, self.eps, self.max_norm = lr, beta1, beta2, eps, max_norm
        self.step_count = 0

    def step(self, grad):
        self.step_count += 1
        st = self.lib.sim_adam(_ptr(self.w), _ptr(grad), _ptr(self.m), _ptr(self.v), self.w.numel(),
                               self.step_count, self.lr, self.b1, self.b2, self.eps, self.max_norm,
                               _ptr(self.scratch), _ptr(self.grad_norm), _stream())
        _check(self.lib, st, "sim_adam")
