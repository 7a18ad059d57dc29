"""GPU parity at the real shapes of the batched and served workloads.

* One long problem per kernel class n in {12, 16, 24, 32} (m = n/2, per-step
  F_i, dense K_i and C_i as in the served workload), up to k = 200000 (17
  elimination levels), in FP64 and in the FP32 form -- with the switch width
  the shipped tuning table gives n and with the 1024-column default -- against
  the CPU oracle: FP64 gates 1e-10 (states, normwise) and 1e-9 (covariance
  blocks); FP32-form gate 1e-5 for both.
* The full 512-problem batched workload (k log-uniform in [64, 16384], n in
  {4, 8, 16, 32}), smoothed in one batch in FP64 and again in the FP32 form,
  every 8th problem checked against the oracle.
"""
import numpy as np
import pytest
import torch

from oracle import seq
from paper_2502_11686_amd import gen, ks

pytestmark = pytest.mark.gpu


def errs(u, S, ref):
    eu = float(np.max(np.abs(u - ref["u"])) / np.max(np.abs(ref["u"])))
    es = float(np.max(np.linalg.norm(S - ref["cov"], axis=(1, 2)) / np.linalg.norm(ref["cov"], axis=(1, 2))))
    return eu, es


def plan_pass(p, args, fp32):
    plan = ks.Plan(p.k, p.n, p.m, p.K_diag, p.C_diag, fp32=fp32)
    try:
        sched = plan.schedule()
        u, S = plan.smooth_cov(*args)
        torch.cuda.synchronize()
        return u.cpu().numpy(), S.cpu().numpy(), sched
    finally:
        plan.close()


@pytest.mark.parametrize("n,k", [(12, 200000), (16, 20000), (24, 200000), (32, 20000)])
def test_long_problem_per_class(n, k, monkeypatch):
    p = gen.make_problem(np.random.default_rng(4000 + n), k, n, n // 2, F_mode="per_step", cov="dense")
    ref = seq.smooth(p)
    args = ks.to_device(p)
    print(f"long problem n={n} k={k}: FP64", flush=True)
    u, S, _ = plan_pass(p, args, False)
    eu, es = errs(u, S, ref)
    print(f"  FP64 state {eu:.2e} cov {es:.2e}", flush=True)
    assert eu <= 1e-10 and es <= 1e-9
    for switch in (None, 1024):  # the tuning table's width, then the default
        if switch is None:
            monkeypatch.delenv("KS_FP32_SWITCH", raising=False)
        else:
            monkeypatch.setenv("KS_FP32_SWITCH", str(switch))
        u, S, sched = plan_pass(p, args, True)
        assert sched["fp32_levels"] >= 1
        eu, es = errs(u, S, ref)
        print(f"  FP32 form (switch {switch or 'table'}, {sched['fp32_levels']} FP32 levels) "
              f"state {eu:.2e} cov {es:.2e}", flush=True)
        assert eu <= 1e-5 and es <= 1e-5
    monkeypatch.delenv("KS_FP32_SWITCH", raising=False)


@pytest.mark.parametrize("fp32", [False, True])
def test_full_batched_workload(fp32):
    probs = gen.batch_workload()
    assert len(probs) == 512
    b = ks.Batch([(p.k, p.n, p.m, p.K_diag, p.C_diag, fp32) for p in probs])
    try:
        inputs = [ks.to_device(p) for p in probs]
        us, covs = b.outputs(True)
        print(f"512-problem batch, fp32 form={fp32}, {sum(p.k + 1 for p in probs)} states", flush=True)
        st = b.smooth(inputs, us, covs)
        torch.cuda.synchronize()
        assert st == [ks.KS_OK] * 512
        tol_u, tol_s = (1e-5, 1e-5) if fp32 else (1e-10, 1e-9)
        worst = [0.0, 0.0]
        for i in range(0, 512, 8):
            p = probs[i]
            eu, es = errs(us[i].cpu().numpy(), covs[i].cpu().numpy(), seq.smooth(p))
            worst = [max(worst[0], eu), max(worst[1], es)]
            assert eu <= tol_u and es <= tol_s, (i, p.n, p.k, eu, es)
        print(f"  worst of 64 checked problems: state {worst[0]:.2e} cov {worst[1]:.2e}", flush=True)
    finally:
        b.close()
