"""The kernel source run on the host with whole waves of lanes.

`tests/kernel_host/kernel_lanes.cpp` compiles the library's kernel source
(step_core.h, drivers.h) for the host in FP64 and runs every lane of a wave
as a fiber, one at a time, switching at the collectives (barriers, votes,
prefix counts, team reductions, the pair exchange, the wave's controller and
warm-start network).  Each case runs under three lane schedules: lanes that
read what another lane writes between two collectives (a barrier missing, or
a read-modify-write that is right only in a wave's lockstep) give results
that depend on the schedule; lanes that reach different collectives stop the
run.  Built with AddressSanitizer, each team's LDS region is followed by a
poisoned guard and the global buffers are exact-size allocations, so an
access past either stops the run.  Every case must give the same bits under
all schedules and equal the FP64 oracle to 1e-9 (1e-8 for chains).

The cases cover the three reverse-sweep modes, contacts, the quadruped's
controller (with and without recurrent units, and a full wave of robots as
the GPU runs them), servo motors, restitution, and the tolerance mode with
the learned warm start and its training records, and the reverse with a
ring of the impulse history in LDS.
"""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
KH = os.path.join(HERE, "kernel_host")
ROOT = os.path.dirname(HERE)
SRC = os.path.join(KH, "kernel_lanes.cpp")
LIB = os.path.join(KH, "libkernel_host_lanes_asan.so")
DEPS = [SRC, os.path.join(KH, "host_common.h")] + [
    os.path.join(ROOT, "paper_1611_01652_amd", "csrc", f)
    for f in ("step_core.h", "drivers.h", "model_pack.cpp", "model_pack.h")]

TOL = {"chains": 1e-8, "chains-replay": 1e-8, "chains-segment": 1e-8, "servo-chains": 1e-8, "bouncy-chains": 1e-8}


def _asan_runtime():
    out = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.fixture(scope="module")
def lanes_lib():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime for g++ here")
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(p) for p in DEPS):
        tmp = f"{LIB}.{os.getpid()}.tmp"
        # (_longjmp between fiber stacks: the fortified longjmp check must be off)
        subprocess.check_call(["g++", "-O1", "-g", "-std=c++20", "-fPIC", "-shared", "-w", "-U_FORTIFY_SOURCE",
                               "-D_FORTIFY_SOURCE=0", "-fsanitize=address", "-fno-omit-frame-pointer", "-o", tmp,
                               SRC])
        os.replace(tmp, LIB)
    return LIB, rt


def _run(lanes_lib, teams_per_wave, cases):
    lib, rt = lanes_lib
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0")
    p = subprocess.run([sys.executable, os.path.join(KH, "lanes_run.py"), lib, "0", str(teams_per_wave)] + cases,
                       capture_output=True, text=True, env=env, timeout=900)
    assert "AddressSanitizer" not in p.stderr, p.stderr[-3000:]
    assert p.returncode == 0, p.stderr[-3000:]
    rows = [json.loads(line) for line in p.stdout.splitlines() if line.startswith("{")]
    assert [r["case"] for r in rows] == [c for c in cases if not c.startswith("--")], p.stdout
    return rows


@pytest.mark.parametrize("teams_per_wave,cases", [
    (2, ["arms", "chains", "chains-replay", "chains-segment"]),
    (2, ["quadruped", "quadruped-rec", "servo-chains", "bouncy-chains", "balls", "solve-learned"]),
    (64, ["quadruped-wave"]),
    # every env keeping only a ring of the impulse history in the reverse
    (2, ["--ring", "chains", "chains-segment", "quadruped", "servo-chains"]),
])
def test_multi_lane_waves_are_schedule_independent_and_equal_the_oracle(lanes_lib, teams_per_wave, cases):
    for r in _run(lanes_lib, teams_per_wave, cases):
        assert "error" not in r, r
        assert r["schedules_agree"], r
        assert r["counts_agree"], r
        assert r["max_rel_diff"] < TOL.get(r["case"], 1e-9), r


def test_contact_overflow_stays_in_bounds_and_schedule_independent(lanes_lib):
    # more active contacts than the env's capacity: the dropped ones get no
    # row slot and no visit entry; every access must stay inside the env's
    # (guarded) LDS region and every lane schedule give the same bits.  The
    # physics differs from the oracle's, which has no capacity, so only the
    # run itself is checked here (the GPU test checks the env's flag).
    for r in _run(lanes_lib, 2, ["overflow"]):
        assert "error" not in r, r
        assert r["schedules_agree"], r
