import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


@pytest.fixture
def rng():
    return np.random.Generator(np.random.PCG64(12345))


def dense_conv_matrix(psf, H, W, transpose=False):
    """Dense (H*W) x (H*W) matrix of the zero-boundary convolution, built entry
    by entry from the definition (H x)(i,j) = sum_{a,b} psf(a,b) x(i-a, j-b)."""
    r = (psf.shape[0] - 1) // 2
    M = np.zeros((H * W, H * W))
    for i in range(H):
        for j in range(W):
            for a in range(-r, r + 1):
                for b in range(-r, r + 1):
                    ii, jj = i - a, j - b
                    if 0 <= ii < H and 0 <= jj < W:
                        M[i * W + j, ii * W + jj] += psf[a + r, b + r]
    return M.T if transpose else M
