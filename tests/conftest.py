import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def read_golden(name):
    """Non-comment lines of a golden fixture, split into tokens."""
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(line.split())
    return out


def frac(s):
    num, den = s.split("/")
    return float(num) / float(den)


# ---------------------------------------------------------------- GPU helpers

def normwise(got, ref):
    """max |got - ref| / max |ref| (the field tolerance metric)."""
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return float(np.abs(got - ref).max() / (scale if scale > 0 else 1.0))


def within_bound(got, ref, bound):
    """Every entry satisfies |got - ref| <= abs + rel * |got|."""
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    a, r = bound
    return bool(np.all(np.abs(got - ref) <= a + r * np.abs(got)))


@pytest.fixture(scope="session")
def gpu_ctx():
    """Library context on cuda:0; fails (does not skip) if the library is missing."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1708_02845_amd import Context
    return Context(0)
