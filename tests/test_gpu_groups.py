"""GPU: level groups (several forward or backward levels in one launch, each
workgroup an aligned subtree) against one launch per level.

Every unit and block row does the same arithmetic whichever launch runs it,
so states and covariances must be bitwise those of the per-level schedule
(FP64 and FP32 form, states-only and full passes, folds of odd levels at
every depth), and within the oracle's gates."""
import numpy as np
import pytest
import torch

from oracle import seq
from paper_2502_11686_amd import gen, ks

pytestmark = pytest.mark.gpu

SETTINGS = [dict(fwd_group=2, fwd_group_from=0, bwd_group=2, bwd_group_from=0),
            dict(fwd_group=3, fwd_group_from=1, bwd_group=4, bwd_group_from=1),
            dict(fwd_group=5, fwd_group_from=0, bwd_group=3, bwd_group_from=2),
            dict(fwd_group=8, fwd_group_from=2, bwd_group=8, bwd_group_from=0, fwd_tail_passes=0,
                 bwd_tail_passes=0),
            dict(fwd_group=4, fwd_group_from=1, bwd_group=5, bwd_group_from=1, fwd_tail_passes=8,
                 bwd_tail_passes=8)]
PER_LEVEL = dict(fwd_group=1, fwd_group_from=1, bwd_group=1, bwd_group_from=1)


def passes(p, fp32):
    plan = ks.Plan(p.k, p.n, p.m, p.K_diag, p.C_diag, fp32=fp32)
    try:
        args = ks.to_device(p)
        u, S = plan.smooth_cov(*args)
        u2 = plan.smooth(*args)
        S2 = plan.covariances()
        torch.cuda.synchronize()
        return [x.cpu().numpy() for x in (u, S, u2, S2)]
    finally:
        plan.close()


@pytest.mark.parametrize("n,m", [(4, 2), (6, 3), (8, 4), (12, 6), (3, 2), (16, 8), (24, 12)])
@pytest.mark.parametrize("fp32", [False, True])
def test_groups_bitwise_equal_per_level(n, m, fp32, monkeypatch):
    for v in ("KS_FWD_GROUP", "KS_FWD_GROUP_FROM", "KS_BWD_GROUP", "KS_BWD_GROUP_FROM", "KS_TAIL_PASSES"):
        monkeypatch.delenv(v, raising=False)
    monkeypatch.setenv("KS_FP32_SWITCH", "64")  # several FP32 levels even at small k
    saved = ks.get_tuning(n, fp32)
    ks_list = [0, 1, 2, 5, 13, 31, 64, 100, 257, 1000, 4097] + ([12345] if n <= 12 else [])
    try:
        for k in ks_list:
            if (k + 1) * m < n:
                continue
            p = gen.make_problem(np.random.default_rng(31 * k + n), k, n, m, cov="dense" if k % 2 else "diag")
            ks.set_tuning(n, fp32, **dict(saved, **PER_LEVEL))
            base = passes(p, fp32)
            for st in SETTINGS:
                ks.set_tuning(n, fp32, **dict(saved, **st))
                got = passes(p, fp32)
                for b, g in zip(base, got):
                    assert np.array_equal(b, g), (k, st)
            if k in (100, 4097):
                ref = seq.smooth(p)
                u, S = base[0], base[1]
                eu = np.max(np.abs(u - ref["u"])) / np.max(np.abs(ref["u"]))
                es = np.max(np.linalg.norm(S - ref["cov"], axis=(1, 2)) / np.linalg.norm(ref["cov"], axis=(1, 2)))
                tol = (1e-5, 1e-5) if fp32 else (1e-10, 1e-9)
                assert eu <= tol[0] and es <= tol[1], (k, eu, es)
    finally:
        ks.set_tuning(n, fp32, **saved)


def test_groups_rank_status_and_static_entry(monkeypatch):
    """The rank test still sees every level's diagonal when groups replace the
    per-level launches (their slots are neutral or the group's), and the
    allocation-free entry point follows the same schedule."""
    saved = ks.get_tuning(6, False), ks.get_tuning(2, False)
    try:
        for n in (6, 2):
            ks.set_tuning(n, False, **dict(saved[0 if n == 6 else 1], fwd_group=4, fwd_group_from=0, bwd_group=4,
                                           bwd_group_from=0))
        bad = gen.make_problem(np.random.default_rng(3), 40, 2, 1)
        bad.G[:] = 0.0  # no observations: U A lacks full column rank
        plan = ks.Plan(bad.k, bad.n, bad.m, bad.K_diag, bad.C_diag)
        with pytest.raises(ks.KsError) as e:
            plan.smooth_cov(*ks.to_device(bad))
        assert e.value.status == ks.KS_E_RANK
        plan.close()
        p = gen.make_problem(np.random.default_rng(4), 20000, 6, 3, cov="dense")
        args = ks.to_device(p)
        plan = ks.Plan(p.k, p.n, p.m, p.K_diag, p.C_diag)
        plan.workspace.zero_()  # zero slots would read as rank loss unless the groups rewrite them
        u, S = plan.smooth_cov(*args)
        us, Ss = ks.smooth_cov_static((p.k, p.n, p.m, p.K_diag, p.C_diag, False), args)
        torch.cuda.synchronize()
        assert torch.equal(u, us) and torch.equal(S, Ss)
        plan.close()
    finally:
        ks.set_tuning(6, False, **saved[0])
        ks.set_tuning(2, False, **saved[1])
