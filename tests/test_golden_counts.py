"""The stored operation counts the benchmark reads (tests/golden/flop_counts.json)
are the oracle's current counts (rewrite them with tests/golden/flop_counts.py
after a change to the oracle's step)."""
import json
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import flop_counts as FC  # noqa: E402


@pytest.mark.parametrize("name,B", [("arms", 3), ("chains", 2), ("chains", 11), ("quadruped", 9)])
def test_stored_counts_are_the_oracles(name, B):
    stored = json.load(open(FC.OUT))[name][str(B)]
    assert list(FC.count(FC.workload(name), B)) == stored
