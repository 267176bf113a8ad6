"""Host logic of the tune cache (no GPU): the key follows what the tuned
widths depend on, and a model found in the cache gets its stored widths
without any timing."""
from __future__ import annotations

import json
import types

import numpy as np

from paper_1611_01652_amd import tune_cache as TC


class FakeSim:
    """What the cache reads of a simulator handle: its bucket structure and
    workload, and the widths it is given."""

    def __init__(self, body_counts, teams, buckets, n_iters=20, grad_store=3):
        off = np.concatenate([[0], np.cumsum(body_counts)]).astype(np.int32)
        self.w = types.SimpleNamespace(env_body_off=off, n_iters=n_iters)
        self.info = types.SimpleNamespace(grad_store=grad_store)
        self._teams = np.asarray(teams, np.int32)
        self._buckets = np.asarray(buckets, np.int32)
        self.set_calls = []

    def teams(self):
        return self._teams.copy()

    def env_buckets(self):
        return self._buckets.copy()

    def set_teams(self, t):
        self.set_calls.append(np.asarray(t).tolist())
        self._teams = np.asarray(t, np.int32)


def _sim(**kw):
    base = dict(body_counts=[2, 3, 30, 31], teams=[8, 64], buckets=[0, 0, 1, 1])
    base.update(kw)
    return FakeSim(**base)


def test_key_is_stable_and_follows_what_the_widths_depend_on():
    k = TC.cache_key(_sim())
    assert k == TC.cache_key(_sim())
    assert k != TC.cache_key(_sim(body_counts=[2, 3, 30, 32]))
    assert k != TC.cache_key(_sim(teams=[16, 64]))
    assert k != TC.cache_key(_sim(buckets=[0, 1, 1, 1]))
    assert k != TC.cache_key(_sim(n_iters=10))
    assert k != TC.cache_key(_sim(grad_store=2))


def test_a_cached_model_gets_its_stored_widths_without_timing(tmp_path):
    path = tmp_path / "tune.json"
    s = _sim()
    path.write_text(json.dumps({TC.cache_key(s) + ":call": {"teams": [16, 64], "tuned_on_steps": 500, "envs": 4}}))

    def no_controls(_w):
        raise AssertionError("a cache hit times nothing")

    teams, how = TC.tuned_teams(s, no_controls, str(path))
    assert how == "cache" and teams.tolist() == [16, 64] and s.set_calls == [[16, 64]]
    # the other objective is a different entry: a miss (which would time on
    # the device) is not taken here; a damaged file reads as empty
    path.write_text("{not json")
    assert TC._load(str(path)) == {}
