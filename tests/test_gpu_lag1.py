"""GPU: lag-one covariance blocks cov(u_i, u_{i+1}) = S_{i,i+1} (level-0
by-product of Algorithm 2) against the oracle's, which the CPU pins tie to
the dense inverse of A^T W A."""
import numpy as np
import pytest
import torch

from oracle import seq
from paper_2502_11686_amd import gen, ks

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,n,m,cov", [(0, 3, 3, "diag"), (1, 2, 1, "dense"), (2, 4, 2, "diag"), (37, 3, 2, "dense"),
                                       (100, 6, 3, "dense"), (333, 8, 4, "diag"), (1001, 6, 3, "dense"),
                                       (64, 16, 8, "dense"), (45, 24, 12, "dense"), (30, 32, 16, "diag"),
                                       (21, 48, 24, "diag")])
def test_lag1_blocks_match_oracle(k, n, m, cov):
    p = gen.make_problem(np.random.default_rng(3 * k + n), k, n, m, cov=cov)
    plan = ks.Plan(p.k, p.n, p.m, p.K_diag, p.C_diag)
    try:
        u, S, L1 = plan.smooth_cov_lag1(*ks.to_device(p))
        u2, S2 = plan.smooth_cov(*ks.to_device(p))
        torch.cuda.synchronize()
        u, S, L1, u2, S2 = (x.cpu().numpy() for x in (u, S, L1, u2, S2))
    finally:
        plan.close()
    assert np.array_equal(u, u2) and np.array_equal(S, S2)  # the export changes nothing else
    ref = seq.smooth(p, want_lag1=True)
    assert L1.shape == (k, n, n)
    if k:
        scale = np.sqrt(np.linalg.norm(ref["cov"][:-1], axis=(1, 2)) * np.linalg.norm(ref["cov"][1:], axis=(1, 2)))
        err = np.max(np.linalg.norm(L1 - ref["lag1"], axis=(1, 2)) / scale)
        assert err < 1e-9, err


def test_lag1_fp32_form():
    p = gen.make_problem(np.random.default_rng(11), 5000, 6, 3, cov="dense")
    plan = ks.Plan(p.k, p.n, p.m, p.K_diag, p.C_diag, fp32=True)
    try:
        u, S, L1 = plan.smooth_cov_lag1(*ks.to_device(p))
        torch.cuda.synchronize()
        L1 = L1.cpu().numpy()
    finally:
        plan.close()
    ref = seq.smooth(p, want_lag1=True)
    scale = np.sqrt(np.linalg.norm(ref["cov"][:-1], axis=(1, 2)) * np.linalg.norm(ref["cov"][1:], axis=(1, 2)))
    assert np.max(np.linalg.norm(L1 - ref["lag1"], axis=(1, 2)) / scale) < 1e-5
