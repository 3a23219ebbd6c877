"""Device start-vector generator against the oracle's implementation of the same
published definitions."""
import numpy as np
import pytest

from oracle.rng import normal

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("count,seed", [(1, 0), (7, 3), (100_001, 42)])
def test_normal_fill_matches_oracle(tsk, count, seed):
    got = tsk.normal_fill(count, seed).cpu().numpy()
    want = normal(count, seed)
    assert np.max(np.abs(got - want)) <= 1e-13 * max(1.0, np.max(np.abs(want)))
