"""GPU: the forward elimination on FP64 matrix cores (forward variant 1 of
n = 32 and 48: blocked Householder QR with compact-WY trailing updates).

* Single plans, FP64 and the FP32 form (whose FP64 levels run it), over k
  that cover every level count, odd and even column counts and folds, with
  diagonal covariances, identity and general H, and observation counts below,
  at and above the class of n/2, against the CPU oracle (1e-10 states, 1e-9
  covariance blocks; FP32 form 1e-5).
* A problem with dense covariances under the same variant takes variant 0
  (this forward whitens diagonal covariances only) and still matches.
* Levels with at least 512 units run it above level 0 as well (narrower
  levels run the workgroup family), checked at k long enough for that.
* A batch of such problems equals, bitwise, each problem smoothed alone with
  the same variant (the batched launches run the same kernels per level).
* The kernel's R rows: sign-invariant products against a dense QR are covered
  by the oracle comparison of states and covariances, which use every R row.
"""
import numpy as np
import pytest
import torch

from oracle import seq
from paper_2502_11686_amd import gen, ks

pytestmark = pytest.mark.gpu

KS = [0, 1, 2, 3, 4, 5, 6, 7, 8, 15, 16, 17, 31, 33, 64, 100, 257]


def errs(u, S, ref):
    eu = float(np.max(np.abs(u - ref["u"])) / np.max(np.abs(ref["u"])))
    es = float(np.max(np.linalg.norm(S - ref["cov"], axis=(1, 2)) / np.linalg.norm(ref["cov"], axis=(1, 2))))
    return eu, es


def smooth(p, fp32=False):
    u, S = ks.smooth_problem(p, fp32=fp32)
    torch.cuda.synchronize()
    return u.cpu().numpy(), S.cpu().numpy()


@pytest.fixture
def variant1(monkeypatch):
    monkeypatch.setenv("KS_FWD_VARIANT", "1")
    monkeypatch.setenv("KS_FP32_SWITCH", "16")  # several FP32 levels at these k


@pytest.mark.parametrize("n,m", [(32, 16), (32, 9), (32, 32), (48, 24), (48, 7), (48, 48)])
def test_mfma_forward_matches_oracle(n, m, variant1):
    assert ks.kernel_variants(n, m, False) >= 2
    worst = [0.0, 0.0, 0.0, 0.0]
    for k in KS:
        if (k + 1) * m < n:
            continue  # rank deficient
        for H_mode in ("identity", "random"):
            p = gen.make_problem(np.random.default_rng(31 * k + n + m), k, n, m, cov="diag", H_mode=H_mode)
            ref = seq.smooth(p)
            for fp32 in (False, True):
                u, S = smooth(p, fp32)
                eu, es = errs(u, S, ref)
                tol = (1e-5, 1e-5) if fp32 else (1e-10, 1e-9)
                assert eu < tol[0] and es < tol[1], (k, H_mode, fp32, eu, es)
                i = 2 if fp32 else 0
                worst[i], worst[i + 1] = max(worst[i], eu), max(worst[i + 1], es)
    print(f"n={n} m={m}: FP64 {worst[0]:.1e} / {worst[1]:.1e}, FP32 form {worst[2]:.1e} / {worst[3]:.1e}",
          flush=True)


@pytest.mark.parametrize("n,m,k", [(32, 16, 2100), (48, 24, 2100), (48, 48, 2060)])
def test_mfma_forward_wide_levels(n, m, k, variant1):
    """Levels with at least 512 units run the MFMA forward above level 0 too
    (narrower ones the workgroup family): k long enough for level 1 to be
    that wide."""
    p = gen.make_problem(np.random.default_rng(900 + n + m), k, n, m, cov="diag", H_mode="random")
    ref = seq.smooth(p)
    for fp32 in (False, True):
        u, S = smooth(p, fp32)
        eu, es = errs(u, S, ref)
        tol = (1e-5, 1e-5) if fp32 else (1e-10, 1e-9)
        assert eu < tol[0] and es < tol[1], (fp32, eu, es)


@pytest.mark.parametrize("n,m", [(32, 16), (48, 24)])
def test_dense_covariances_take_variant_0(n, m, variant1):
    p = gen.make_problem(np.random.default_rng(3 + n), 40, n, m, cov="dense")
    u, S = smooth(p)
    eu, es = errs(u, S, seq.smooth(p))
    assert eu < 1e-10 and es < 1e-9


def test_batch_equals_alone_with_variant_1(variant1):
    shapes = [(32, 16, 90), (48, 24, 41), (32, 16, 7), (48, 24, 200), (32, 32, 64), (32, 16, 2100), (48, 24, 1100)]
    probs = [gen.make_problem(np.random.default_rng(70 + i), k, n, m, cov="diag") for i, (n, m, k) in
             enumerate(shapes)]
    b = ks.Batch([(p.k, p.n, p.m, p.K_diag, p.C_diag, False) for p in probs])
    try:
        us, covs = b.outputs(True)
        b.smooth([ks.to_device(p) for p in probs], us, covs)
        torch.cuda.synchronize()
        for p, u, S in zip(probs, us, covs):
            ua, Sa = smooth(p)
            assert np.array_equal(u.cpu().numpy(), ua) and np.array_equal(S.cpu().numpy(), Sa), (p.n, p.k)
    finally:
        b.close()


def test_fp32_form_with_a_wide_fp64_level(monkeypatch):
    """The FP32 form where the first FP64 level above the switch level has at
    least 512 units (k = 8200, switch 4096: levels 0, 1 in FP32, level 2 reads
    FP32 records, level 3 with 512 units runs the matrix-core forward)."""
    monkeypatch.setenv("KS_FWD_VARIANT", "1")
    monkeypatch.setenv("KS_FP32_SWITCH", "4096")
    p = gen.make_problem(np.random.default_rng(44), 8200, 32, 16, cov="diag")
    u, S = smooth(p, fp32=True)
    eu, es = errs(u, S, seq.smooth(p))
    assert eu < 1e-5 and es < 1e-5, (eu, es)
