"""GPU parity: libks (through its C ABI) against the CPU oracle.

Tolerances (FP64): states normwise max_i |u_i - u_i*|_inf / max_i |u_i*|_inf
<= 1e-10; covariance blocks max_i ||S_i - S_i*||_F / ||S_i*||_F <= 1e-9.
"""
import numpy as np
import pytest
import torch

from oracle import dense, seq
from paper_2502_11686_amd import gen, ks

pytestmark = pytest.mark.gpu

TOL_U, TOL_S = 1e-10, 1e-9


def rel_u(u, ref):
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


def rel_s(S, ref):
    return float(np.max(np.linalg.norm(S - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))))


def gpu(p, mode="fused"):
    plan = ks.Plan(p.k, p.n, p.m, p.K_diag, p.C_diag)
    args = ks.to_device(p)
    try:
        if mode == "fused":
            u, S = plan.smooth_cov(*args)
        elif mode == "split":
            u = plan.smooth(*args)
            S = plan.covariances()
        else:
            u, S = plan.smooth(*args), None
        torch.cuda.synchronize()
        return u.cpu().numpy(), None if S is None else S.cpu().numpy()
    finally:
        plan.close()


SHAPES = [(1, 1), (2, 1), (4, 2), (3, 3), (6, 3), (4, 5), (8, 4), (2, 4), (6, 6), (3, 1), (5, 3),
          (12, 6), (16, 8), (12, 12)]
LARGE = [(24, 12), (32, 16), (48, 24), (24, 24), (24, 5), (32, 32), (48, 48), (48, 7)]
KS = list(range(0, 20)) + [31, 32, 33, 63, 64, 100, 127, 128, 129]
KS_LARGE = [0, 1, 2, 3, 4, 5, 6, 7, 8, 15, 16, 17, 31, 33, 64]


@pytest.mark.parametrize("n,m", SHAPES + LARGE)
def test_small_sweep(n, m):
    worst = [0.0, 0.0]
    for k in (KS if n <= 16 else KS_LARGE):
        if (k + 1) * m < n:
            continue  # fewer observation rows than unknowns beyond the evolution rows: rank deficient
        for cov in ("diag", "dense"):
            for H_mode in ("identity", "random"):
                p = gen.make_problem(np.random.default_rng(97 * k + 13 * n + m), k, n, m,
                                     cov=cov, H_mode=H_mode)
                ref = seq.smooth(p)
                u, S = gpu(p)
                eu, es = rel_u(u, ref["u"]), rel_s(S, ref["cov"])
                assert eu < TOL_U and es < TOL_S, (k, cov, H_mode, eu, es)
                assert np.array_equal(S, np.swapaxes(S, 1, 2))
                worst = [max(worst[0], eu), max(worst[1], es)]
    print(f"n={n} m={m}: worst state {worst[0]:.2e}, cov {worst[1]:.2e}", flush=True)


@pytest.mark.parametrize("wid", [0, 1, 2])
def test_full_workloads(wid):
    p = gen.workload(wid)
    print(f"workload {wid}: k={p.k} n={p.n} m={p.m}", flush=True)
    ref = seq.smooth(p)
    u, S = gpu(p)
    eu, es = rel_u(u, ref["u"]), rel_s(S, ref["cov"])
    print(f"workload {wid}: state {eu:.2e} cov {es:.2e}", flush=True)
    assert eu < TOL_U and es < TOL_S


def test_split_equals_fused_and_is_deterministic():
    p = gen.workload(1, k=5000)
    u1, S1 = gpu(p, "fused")
    u2, S2 = gpu(p, "split")
    u3, S3 = gpu(p, "fused")
    u4, _ = gpu(p, "nc")
    assert np.array_equal(u1, u2) and np.array_equal(S1, S2)
    assert np.array_equal(u1, u3) and np.array_equal(S1, S3)
    assert np.array_equal(u1, u4)


def _level(i):
    return ((i + 1) & -(i + 1)).bit_length() - 1


@pytest.mark.parametrize("k,n,m", [(50, 2, 1), (37, 3, 2), (64, 4, 2)])
def test_r_factor_blocks_against_dense_qr(k, n, m):
    """Block rows of the GPU's R equal those of a dense QR of U A P, P the
    odd-even column order (up to row signs: compare R_ii^T R_ij, R_ii^T rho_i),
    and each has at most two off-diagonal blocks, at i -/+ 2^l (Fig. R-structures)."""
    p = gen.make_problem(np.random.default_rng(k), k, n, m, cov="dense", H_mode="random")
    plan = ks.Plan(k, n, m, p.K_diag, p.C_diag)
    plan.smooth(*ks.to_device(p))
    torch.cuda.synchronize()
    recs = plan.r_records().cpu().numpy()
    lay = plan.layout()
    plan.close()
    order = sorted(range(k + 1), key=lambda i: (_level(i), i))
    pos = {c: q for q, c in enumerate(order)}
    R, qtb = dense.permuted_R(p, order)
    for i in range(k + 1):
        l = _level(i)
        rec = recs[lay["level_rec_offset"][l] + ((i + 1) >> (l + 1))]
        Rii, Rp, rho, Rm = rec[:, :n], rec[:, n:2 * n], rec[:, 2 * n], rec[:, 2 * n + 1:]
        rows = slice(pos[i] * n, (pos[i] + 1) * n)
        Dii = R[rows, pos[i] * n:(pos[i] + 1) * n]
        scale = np.linalg.norm(Dii.T @ Dii)
        assert np.linalg.norm(Rii.T @ Rii - Dii.T @ Dii) < 1e-12 * scale
        assert np.linalg.norm(Rii.T @ rho - Dii.T @ qtb[rows]) < 1e-11 * max(1.0, np.linalg.norm(Dii.T @ qtb[rows]))
        nbr = {i - (1 << l): Rm, i + (1 << l): Rp}
        for c in range(k + 1):
            if c == i or pos[c] < pos[i]:
                continue
            Dic = R[rows, pos[c] * n:(pos[c] + 1) * n]
            if c in nbr:
                assert np.linalg.norm(Rii.T @ nbr[c] - Dii.T @ Dic) < 1e-11 * scale
            else:
                assert np.linalg.norm(Dic) < 1e-12 * np.sqrt(scale)
        for c, blk in nbr.items():
            if not (0 <= c <= k):
                assert not blk.any()


def test_errors():
    rng = np.random.default_rng(1)
    p = gen.make_problem(rng, 0, 3, 2)  # k = 0 with m < n
    with pytest.raises(ks.KsError) as e:
        gpu(p)
    assert e.value.status == ks.KS_E_RANK
    p = gen.make_problem(rng, 40, 2, 1)
    p.G[:] = 0.0
    with pytest.raises(ks.KsError) as e:
        gpu(p)
    assert e.value.status == ks.KS_E_RANK
    p = gen.make_problem(rng, 40, 2, 1)
    p.K[17, 1] = -1.0
    with pytest.raises(ks.KsError) as e:
        gpu(p)
    assert e.value.status == ks.KS_E_NOT_SPD
    p = gen.make_problem(rng, 40, 3, 2, cov="dense")
    p.C[5] = -np.eye(2)
    with pytest.raises(ks.KsError) as e:
        gpu(p)
    assert e.value.status == ks.KS_E_NOT_SPD
    p = gen.make_problem(rng, 40, 3, 2)
    p.F[9, 0, 0] = np.nan
    with pytest.raises(ks.KsError) as e:
        gpu(p)
    assert e.value.status == ks.KS_E_NONFINITE
    p = gen.make_problem(rng, 10, 3, 2)
    plan = ks.Plan(p.k, p.n, p.m, p.K_diag, p.C_diag)
    with pytest.raises(ks.KsError) as e:
        plan.covariances()
    assert e.value.status == ks.KS_E_ORDER
    plan.close()


@pytest.mark.parametrize("k,n,m,cov", [(100, 6, 3, "dense"), (5000, 6, 3, "dense"), (777, 4, 2, "diag"),
                                       (3000, 8, 4, "diag"), (1, 2, 1, "diag"), (201, 24, 12, "dense"),
                                       (334, 32, 16, "diag"), (45, 48, 24, "dense")])
def test_tail_kernels_equal_per_level_kernels(k, n, m, cov, monkeypatch):
    """The single-workgroup tail (top levels in one launch) computes exactly
    what one launch per level computes."""
    p = gen.make_problem(np.random.default_rng(k + n), k, n, m, cov=cov)
    monkeypatch.setenv("KS_TAIL_PASSES", "0")
    u0, S0 = gpu(p)
    monkeypatch.setenv("KS_TAIL_PASSES", "1000000")
    u1, S1 = gpu(p)
    monkeypatch.delenv("KS_TAIL_PASSES")
    u2, S2 = gpu(p)
    assert np.array_equal(u0, u1) and np.array_equal(S0, S1)
    assert np.array_equal(u0, u2) and np.array_equal(S0, S2)
    ref = seq.smooth(p)
    assert rel_u(u0, ref["u"]) < TOL_U and rel_s(S0, ref["cov"]) < TOL_S
