"""GPU: ks_smooth_cov_static (working data in the library's static device
array, no device allocation inside the call) against ks_smooth_cov on a plan
with its own workspace, through the C ABI: bitwise equal states and
covariances, both within the FP64 gates of the oracle.  Two calls in a row,
the second on a smaller problem, so the second runs on the array the first
left behind."""
import numpy as np
import pytest
import torch

from oracle import seq
from paper_2502_11686_amd import gen, ks

pytestmark = pytest.mark.gpu

TOL_U, TOL_S = 1e-10, 1e-9


def plan_pass(p, args):
    plan = ks.Plan(p.k, p.n, p.m, p.K_diag, p.C_diag)
    try:
        u, S = plan.smooth_cov(*args)
        torch.cuda.synchronize()
        return u.cpu().numpy(), S.cpu().numpy()
    finally:
        plan.close()


@pytest.mark.parametrize("first,second", [((6, 3, 20000, "dense"), (6, 3, 1501, "dense")),
                                          ((16, 8, 3000, "diag"), (4, 2, 1000, "diag")),
                                          ((48, 24, 300, "diag"), (48, 24, 37, "dense"))])
def test_static_matches_plan_two_calls(first, second):
    for seed, (n, m, k, cov) in enumerate((first, second)):
        p = gen.make_problem(np.random.default_rng(500 + 7 * seed + n), k, n, m, cov=cov)
        assert ks.workspace_bytes(k, n, m, p.K_diag, p.C_diag) <= ks.STATIC_SCRATCH_BYTES
        args = ks.to_device(p)
        print(f"static pass n={n} m={m} k={k} cov={cov}", flush=True)
        u, S = ks.smooth_cov_static((k, n, m, p.K_diag, p.C_diag, False), args)
        torch.cuda.synchronize()
        u, S = u.cpu().numpy(), S.cpu().numpy()
        u_ref, S_ref = plan_pass(p, args)
        assert np.array_equal(u, u_ref) and np.array_equal(S, S_ref)
        ref = seq.smooth(p)
        eu = np.max(np.abs(u - ref["u"])) / np.max(np.abs(ref["u"]))
        es = np.max(np.linalg.norm(S - ref["cov"], axis=(1, 2)) / np.linalg.norm(ref["cov"], axis=(1, 2)))
        assert eu <= TOL_U and es <= TOL_S, (eu, es)
