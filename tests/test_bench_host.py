"""Host-side pins of the benchmark's algorithmic counts (no GPU)."""
from types import SimpleNamespace

import numpy as np

import bench


def _count_householder(r, c, p):
    """Flops of an explicit Householder QR, counted operation by operation."""
    rng = np.random.default_rng(0)
    A = rng.standard_normal((r, c + p))
    flops = 0
    for q in range(min(r, c)):
        h = r - q
        if h <= 1:
            continue
        x = A[q:, q]
        flops += 2 * h                      # norm of the pivot column
        v = x.copy()
        v[0] += np.copysign(np.linalg.norm(x), x[0])
        v /= np.linalg.norm(v)
        for j in range(q + 1, c + p):       # dot product and update per column
            A[q:, j] -= 2 * v * (v @ A[q:, j])
            flops += 4 * h
        A[q:, q] = 0
        A[q, q] = -np.copysign(np.linalg.norm(x), x[0])
    return flops


def test_householder_count_matches_explicit_qr():
    for r, c, p in [(9, 6, 7), (6, 6, 1), (12, 6, 13), (72, 48, 49), (2, 1, 0)]:
        assert bench._householder_flops(r, c, p) == _count_householder(r, c, p)


def test_householder_count_leading_terms():
    r, c, p = 960, 480, 481
    approx = 2 * c * c * r - 2 * c ** 3 / 3 + 4 * r * c * p - 2 * c * c * p
    assert abs(bench._householder_flops(r, c, p) - approx) / approx < 0.01


def test_level0_bytes_count_arrays():
    p = SimpleNamespace(k=9, n=2, m=1, K_diag=False, C_diag=True, H=None)
    reads = 9 * (4 + 2 + 4) + 10 * (2 + 1 + 1)          # F, c, K per evolution; G, o, C per state
    writes = 5 * 2 * 7 + 5 * 2 * 8                       # R records and reduced columns
    assert bench.level0_forward_bytes(p) == 8 * (reads + writes)
