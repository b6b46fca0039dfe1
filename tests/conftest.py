import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU")
    config.addinivalue_line("markers", "slow: longer CPU oracle checks")


def read_golden(name):
    """Whitespace table under tests/golden/ with '#' comments -> list of float rows."""
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(x) for x in line.split()])
    return rows


@pytest.fixture(scope="session")
def oracle():
    import oracle as _oracle
    _oracle._load()
    return _oracle


MAX_REL_GATE = 1e-11


def fp64_err(got, ref):
    """Relative L2 error ||got - ref|| / ||ref|| of an FP64 result, after checking
    the per-element gate of the same parity bar: max|got - ref| / max|ref| must
    not exceed 1e-11 (an error confined to a few elements fails here even when
    the norm over the whole array hides it)."""
    import numpy as np
    got = np.asarray(got).ravel()
    ref = np.asarray(ref).ravel()
    d = np.abs(got - ref)
    scale = np.max(np.abs(ref))
    mx = float(np.max(d) / scale) if scale > 0 else float(np.max(d))
    assert mx <= MAX_REL_GATE, f"max|delta|/max|ref| = {mx:.3e} above {MAX_REL_GATE:g}"
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
