"""Pin of the oracle's seeded generator against the published splitmix64 outputs."""
import os

import numpy as np

from oracle.rng import normal, splitmix64

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")


def test_splitmix64_reference_outputs():
    ref = [int(l, 16) for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert [int(x) for x in splitmix64(0, 3)] == ref


def test_counter_form_equals_sequential_stream():
    assert [int(x) for x in splitmix64(7, 5, start=3)] == [int(x) for x in splitmix64(7, 8)[3:]]


def test_box_muller_moments():
    z = normal(400_000, 3)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01
    assert abs(np.mean(z ** 4) - 3) < 0.05
