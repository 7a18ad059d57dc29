"""GPU: the schedule autotuner and the committed tuning table.

The tuner times each candidate on the device and keeps the fastest; whatever
it picks, results stay those of the default schedule bitwise in FP64 (tail
and per-level kernels do the same arithmetic) and match the oracle."""
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


def test_tune_one_entry_keeps_results():
    n = 6
    p = gen.make_problem(np.random.default_rng(5), 3000, n, 3, cov="dense")
    saved = ks.get_tuning(n, False)
    try:
        ks.set_tuning(n, False, **ks.TUNING_DEFAULTS)
        u0, S0 = smooth(p)
        e = autotune.tune_one(n, False, reps=2)
        assert e["fwd_tail_passes"] in autotune.PASSES and e["bwd_tail_passes"] in autotune.PASSES
        assert set(e["fwd_ms"]) == {str(q) for q in autotune.PASSES}
        assert ks.get_tuning(n, False)["fwd_tail_passes"] == e["fwd_tail_passes"]
        u1, S1 = smooth(p)
        assert np.array_equal(u0, u1) and np.array_equal(S0, S1)
        ref = seq.smooth(p)
        assert np.max(np.abs(u1 - ref["u"])) / np.max(np.abs(ref["u"])) < 1e-10
    finally:
        ks.set_tuning(n, False, **saved)


def test_committed_table_is_complete_and_loads():
    if not os.path.exists(ks.TUNE_PATH):
        pytest.skip("no tuning table next to the library")
    table = json.load(open(ks.TUNE_PATH))
    got = {(e["n"], e["form"]) for e in table["entries"]}
    for n in autotune.ALL_N:
        assert (n, "fp64") in got and (n, "fp32") in got
    assert ks.load_tuning(ks.TUNE_PATH) == len(table["entries"])
