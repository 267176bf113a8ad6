"""Host-side checks of the HIP library (no GPU needed).

* the shared library loads and exports every function declared in include/sim.h
* descriptor validation rejects malformed models before touching a device
* the library's canonical sweep order (computed by its own host code) equals
  the oracle's, independently implemented, and every colour is race-free
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1611_01652_amd import workloads as W
from paper_1611_01652_amd import sim as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "sim.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+([a-z_][a-z0-9_]*)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = S.library()
    declared = _header_functions()
    assert set(S.EXPORTED) == set(declared), (declared, S.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name
    hdr = open(os.path.join(ROOT, "include", "sim.h")).read()
    assert lib.sim_abi_version() == S.ABI_VERSION == int(re.search(r"#define SIM_ABI_VERSION (\d+)", hdr).group(1))
    # the allocation-free entry point's scratch size, as the binding knows it
    m = re.search(r"#define SIM_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == S.NOALLOC_SCRATCH_BYTES


def _call_init(w, mutate=None):
    lib = S.library()
    d, keep = S.make_desc(w)
    if mutate:
        mutate(d, keep)
    h = C.c_void_p()
    st = lib.sim_init(C.byref(d), C.byref(h))
    msg = lib.sim_last_error().decode()
    if st == 0:
        lib.sim_destroy(h)
    return st, msg


@pytest.mark.parametrize("case,code", [
    ("dt", -1), ("iters", -1), ("ckpt", -1), ("loss_kind", -1), ("team", -1),
    ("T_env", -2), ("loss_body", -2), ("joint_child", -2), ("two_pair_spheres", -2), ("inv_mass", -1),
])
def test_init_rejects_malformed_descriptions(case, code):
    w = W.uneven_chains(n_envs=3, T=10, sizes=[3, 4, 2])

    def mutate(d, keep):
        if case == "dt":
            d.dt = 0.0
        elif case == "iters":
            d.n_iters = -1
        elif case == "ckpt":
            d.ckpt_every = 0
        elif case == "loss_kind":
            d.loss_kind = 7
        elif case == "team":
            d.min_team = 3
        elif case == "T_env":
            d.T_env[1] = 11
        elif case == "loss_body":
            d.loss_body[0] = 5   # a body of env 1
        elif case == "joint_child":
            d.joint_child[0] = 4
        elif case == "two_pair_spheres":
            d.sphere_body[1] = 0
        elif case == "inv_mass":
            d.inv_mass[2] = 0.0
    st, msg = _call_init(w, mutate)
    assert st == code, (st, msg)
    assert msg


def test_null_description_and_arguments():
    lib = S.library()
    h = C.c_void_p()
    assert lib.sim_init(None, C.byref(h)) == -1
    assert lib.sim_destroy(None) == -1
    assert lib.rollout(None, None, None, None, None, None, None, None, None) == -1


def _oracle_order(w, env):
    from oracle import Oracle
    out = []
    for kind, idx in Oracle(w).order(env):
        if kind == 2:
            a, b = idx // 65536, idx % 65536
            b0 = w.env_body_off[env]
            idx = (a - b0) | ((b - b0) << 12)
        out.append((kind << 24) | idx)
    return out


@pytest.mark.parametrize("maker", [
    lambda: W.uneven_chains(n_envs=24, T=5),
    lambda: W.planar_arms(n_envs=4, T=5),
    lambda: W.free_spheres(np.array([[0, 0, .1], [.19, 0, .1], [.095, 0, .27], [.5, .5, .1], [.6, .4, .3]]),
                           [.1] * 5, [1.0] * 5),
])
def test_sweep_order_matches_oracle_and_colours_are_disjoint(maker):
    w = maker()
    for e in range(w.n_envs):
        codes, cols = S.describe_order(w, e)
        assert list(codes) == _oracle_order(w, e), e
        # bodies of each colour are disjoint
        b0 = w.env_body_off[e]
        for c in np.unique(cols):
            seen = set()
            for code in codes[cols == c]:
                kind, idx = code >> 24, code & 0xFFFFFF
                if kind == 0:
                    bodies = {int(w.joint_parent[idx]), int(w.joint_child[idx])} - {-1}
                    bodies = {b - b0 for b in bodies}
                elif kind == 1:
                    bodies = {int(w.sphere_body[idx]) - b0}
                else:
                    bodies = {idx & 0xFFF, idx >> 12}
                assert not (bodies & seen), (e, c)
                seen |= bodies
        # round-robin pairs: each candidate exactly once
        pairs = [c & 0xFFFFFF for c in codes if (c >> 24) == 2]
        assert len(pairs) == len(set(pairs))
