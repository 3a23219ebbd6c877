import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def _have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def tsk():
    """The HIP library binding.  Builds libtsk.so if it is missing; on a GPU
    machine a load failure is an error, never a skip."""
    import paper_1804_03859_amd.tsk as t
    if not os.path.exists(t.LIB_PATH):
        from paper_1804_03859_amd import build
        build.build()
    t.load()
    if not _have_gpu():
        pytest.skip("no GPU visible")
    return t


def match_sets(a, b):
    """Greedy one-to-one nearest matching of two complex arrays; returns the
    largest matched distance."""
    import numpy as np
    b = list(np.asarray(b))
    worst = 0.0
    for x in np.asarray(a):
        d = [abs(x - y) for y in b]
        i = int(np.argmin(d))
        worst = max(worst, d[i])
        b.pop(i)
    return worst


def golden(name):
    """A `key value` text fixture under tests/golden/ as a dict of floats."""
    out = {}
    for line in open(os.path.join(ROOT, "tests", "golden", name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out
