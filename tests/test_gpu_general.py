"""GPU: problems with per-step dimensions (n_i, l_i, m_i varying, m_i = 0
included, rectangular H_i) through the embedding onto the uniform kernels,
against the dense definition (oracle/dense.py smooth_general, pinned on the
CPU to a per-step objective's gradient and Hessian)."""
import numpy as np
import pytest
import torch

from oracle import dense
from paper_2502_11686_amd import gen, general

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,k,n_choices,m_extra,fp32", [
    (0, 0, (3,), 1, False), (1, 1, (2, 3), 1, False), (2, 37, (2, 3, 4, 5), 1, False),
    (3, 400, (1, 2, 3, 4, 5), 1, False), (4, 300, (6, 8, 10), 1, False), (5, 60, (12, 20), 0, False),
    (6, 40, (30, 40), 0, False), (7, 400, (2, 3, 4, 5), 1, True)])
def test_general_dimensions_match_dense_definition(seed, k, n_choices, m_extra, fp32):
    gp = gen.make_general_problem(np.random.default_rng(100 + seed), k, n_choices, m_extra)
    res = general.smooth_general(gp, fp32=fp32)
    torch.cuda.synchronize()
    ref = dense.smooth_general(gp)
    # the FP64 gates of the uniform problems (states 1e-10 normwise, covariance
    # blocks 1e-9); the dense definition itself agrees with the sequential
    # oracle on these embedded problems to 6e-13
    tol_u, tol_s = (1e-5, 1e-5) if fp32 else (1e-10, 1e-9)
    scale = max(np.abs(x).max() for x in ref["u"])
    for i in range(gp.k + 1):
        u = res.u(i).cpu().numpy()
        S = res.cov(i).cpu().numpy()
        assert np.abs(u - ref["u"][i]).max() <= tol_u * scale, i
        assert np.linalg.norm(S - ref["cov"][i]) <= tol_s * np.linalg.norm(ref["cov"][i]), i
    for i in range(gp.k):
        L1 = res.lag1(i).cpu().numpy()
        den = np.sqrt(np.linalg.norm(ref["cov"][i]) * np.linalg.norm(ref["cov"][i + 1]))
        assert np.linalg.norm(L1 - ref["lag1"][i]) <= tol_s * den, i
