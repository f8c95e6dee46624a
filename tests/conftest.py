import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


def load_golden(name, dtype=float):
    import numpy as np
    return np.loadtxt(os.path.join(GOLDEN, name), dtype=dtype, comments="#")


@pytest.fixture(scope="session")
def golden():
    return load_golden


def crop_fs(cur, ref, B, R, bx, by):
    """Oracle FS of block (bx, by) from a crop that holds its whole search
    window (and the frame's own edges where the window meets them): the
    candidate set, hence the result, is the full frame's."""
    import numpy as np
    import oracle
    H, W = cur.shape
    m = (R + B - 1) // B * B  # a block-aligned margin of at least R
    x0, y0 = max(bx * B - m, 0), max(by * B - m, 0)
    x1, y1 = min(bx * B + B + m, W), min(by * B + B + m, H)
    mv, sad, nsp = oracle.fullsearch(np.ascontiguousarray(cur[y0:y1, x0:x1]),
                                     np.ascontiguousarray(ref[y0:y1, x0:x1]), B, R)
    j, i = (by * B - y0) // B, (bx * B - x0) // B
    return mv[j, i], sad[j, i], nsp[j, i]
