"""GPU: the autotuner, the compiled shape variants and the committed tuning
table.

The tuner times each candidate on the device and keeps the fastest by its
noise rule.  Schedule choices (tail passes, level groups) leave FP64 results
bitwise unchanged; compiled shape variants are different kernels, whose
instruction selection (fused multiply-adds) may round differently, so every
variant of every n is checked against the oracle instead."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import seq
from paper_2502_11686_amd import autotune, gen, ks

pytestmark = pytest.mark.gpu


def smooth(p, fp32=False):
    u, S = ks.smooth_problem(p, fp32=fp32)
    torch.cuda.synchronize()
    return u.cpu().numpy(), S.cpu().numpy()


def errs(u, S, ref):
    eu = float(np.max(np.abs(u - ref["u"])) / np.max(np.abs(ref["u"])))
    es = float(np.max(np.linalg.norm(S - ref["cov"], axis=(1, 2)) / np.linalg.norm(ref["cov"], axis=(1, 2))))
    return eu, es


def test_tune_one_entry_keeps_results(monkeypatch):
    n = 6
    monkeypatch.setattr(autotune, "problem_k", lambda n: 5000)
    p = gen.make_problem(np.random.default_rng(5), 3000, n, 3, cov="dense")
    saved = ks.get_tuning(n, False)
    try:
        ks.set_tuning(n, False, **ks.TUNING_DEFAULTS)
        u0, S0 = smooth(p)
        e = autotune.tune_one(n, False, reps=2)
        assert e["fwd_tail_passes"] in autotune.PASSES and e["bwd_tail_passes"] in autotune.PASSES
        assert e["bwd_variant"] < ks.kernel_variants(n, 3, True)
        assert e["fwd_variant"] < ks.kernel_variants(n, 3, False)
        assert {k: ks.get_tuning(n, False)[k] for k in ks.TUNING_KEYS} == {k: e[k] for k in ks.TUNING_KEYS}
        u1, S1 = smooth(p)
        if e["fwd_variant"] == 0 and e["bwd_variant"] == 0:
            assert np.array_equal(u0, u1) and np.array_equal(S0, S1)
        ref = seq.smooth(p)
        eu, es = errs(u1, S1, ref)
        assert eu < 1e-10 and es < 1e-9
    finally:
        ks.set_tuning(n, False, **saved)


@pytest.mark.parametrize("n,m", [(2, 1), (3, 2), (4, 2), (5, 3), (6, 3), (8, 4), (12, 6), (16, 8), (24, 12),
                                 (32, 16), (48, 24)])
def test_every_variant_matches_oracle(n, m, monkeypatch):
    """Every compiled forward x backward variant, FP64 and the FP32 form, on a
    problem with several levels, folds and FP32 levels, against the oracle."""
    monkeypatch.setenv("KS_FP32_SWITCH", "64")
    k = 700 if n <= 12 else 90
    p = gen.make_problem(np.random.default_rng(17 * n + m), k, n, m, cov="dense")
    ref = seq.smooth(p)
    nfv, nbv = ks.kernel_variants(n, m, False), ks.kernel_variants(n, m, True)
    assert nfv >= 1 and nbv >= 1
    for fp32 in (False, True):
        for fv in range(nfv):
            for bv in range(nbv):
                monkeypatch.setenv("KS_FWD_VARIANT", str(fv))
                monkeypatch.setenv("KS_BWD_VARIANT", str(bv))
                u, S = smooth(p, fp32)
                eu, es = errs(u, S, ref)
                tol = (1e-5, 1e-5) if fp32 else (1e-10, 1e-9)
                assert eu <= tol[0] and es <= tol[1], (fv, bv, fp32, eu, es)
                print(f"n={n} fv={fv} bv={bv} fp32={fp32}: state {eu:.1e} cov {es:.1e}", flush=True)


def test_committed_table_is_complete_and_loads():
    if not os.path.exists(ks.TUNE_PATH):
        pytest.skip("no tuning table next to the library")
    table = json.load(open(ks.TUNE_PATH))
    got = {(e["n"], e["form"]): e for e in table["entries"]}
    for n in autotune.ALL_N:
        for form in ("fp64", "fp32"):
            e = got[(n, form)]
            m = max(1, n // 2)
            assert e.get("fwd_variant", 0) < ks.kernel_variants(n, m, False)
            assert e.get("bwd_variant", 0) < ks.kernel_variants(n, m, True)
    assert ks.load_tuning(ks.TUNE_PATH) == len(table["entries"])
