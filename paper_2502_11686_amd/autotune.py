"""Autotuner of the schedule's free choices, per state dimension and form.

For each (n, form) it smooths one synthetic problem of that n (long enough
that the top levels of any longer problem look the same: their unit counts
do not depend on k) with every candidate setting and keeps the fastest:

* forward tail passes: how many unit passes of the single-workgroup forward
  tail kernel the top levels may take instead of one launch each (timed over
  the forward launches, KS_TIME_FWD_ALL);
* backward tail passes: the same for the backward tail (KS_TIME_BWD_ALL);
* FP32 form: the column count above which a level runs in FP32 (timed over
  whole passes).

The choice depends only on (n, form), never on what a batch holds, and none
of the choices changes an FP64 result (tail and per-level kernels do the same
arithmetic).  The table is JSON; ks.load_tuning applies it, and the binding
loads tune_mi355x.json next to the library by default.

    python -m paper_2502_11686_amd.autotune [--out FILE] [--n 6 12 ...] [--reps R]
"""
from __future__ import annotations

import argparse
import json
import statistics
import sys
import time

import numpy as np
import torch

from . import gen, ks

PASSES = (0, 1, 2, 3, 4, 6, 8, 12)
SWITCHES = (256, 512, 1024, 2048, 4096)
ALL_N = (1, 2, 3, 4, 5, 6, 8, 12, 16, 24, 32, 48)


def _problem(n: int):
    k = 32768 if n <= 8 else (16384 if n <= 16 else 4096)
    return gen.make_problem(np.random.default_rng(7000 + n), k, n, max(1, n // 2), F_mode="per_step", cov="diag")


def _timed(p, args, fp32: bool, kind: int, reps: int) -> float:
    plan = ks.Plan(p.k, p.n, p.m, p.K_diag, p.C_diag, fp32=fp32)
    try:
        u = torch.empty((p.k + 1, p.n), dtype=torch.float64, device="cuda")
        S = torch.empty((p.k + 1, p.n, p.n), dtype=torch.float64, device="cuda")
        plan.smooth_cov(*args, u_out=u, cov_out=S)  # warm-up
        if kind is None:
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                plan.smooth_cov(*args, u_out=u, cov_out=S)
                ts.append(time.perf_counter() - t0)
            return statistics.median(ts) * 1e3
        plan.time_kernels(kind)
        ms = []
        for _ in range(reps):
            plan.time_kernels(kind)
            plan.smooth_cov(*args, u_out=u, cov_out=S)
            t, cnt = plan.kernel_time()
            ms.append(t / max(cnt, 1))
        plan.time_kernels(ks.KS_TIME_OFF)
        return statistics.median(ms)
    finally:
        plan.close()


def tune_one(n: int, fp32: bool, reps: int = 7) -> dict:
    p = _problem(n)
    args = ks.to_device(p)
    base = ks.get_tuning(n, fp32)
    sw = base["fp32_switch_columns"]
    fwd = {}
    for q in PASSES:
        ks.set_tuning(n, fp32, fwd_tail_passes=q, bwd_tail_passes=base["bwd_tail_passes"], fp32_switch_columns=sw)
        fwd[q] = _timed(p, args, fp32, ks.KS_TIME_FWD_ALL, reps)
    best_f = min(fwd, key=fwd.get)
    bwd = {}
    for q in PASSES:
        ks.set_tuning(n, fp32, fwd_tail_passes=best_f, bwd_tail_passes=q, fp32_switch_columns=sw)
        bwd[q] = _timed(p, args, fp32, ks.KS_TIME_BWD_ALL, reps)
    best_b = min(bwd, key=bwd.get)
    best_s, sws = sw, {}
    if fp32:
        for s in SWITCHES:
            ks.set_tuning(n, fp32, fwd_tail_passes=best_f, bwd_tail_passes=best_b, fp32_switch_columns=s)
            sws[s] = _timed(p, args, fp32, None, reps)
        best_s = min(sws, key=sws.get)
    ks.set_tuning(n, fp32, fwd_tail_passes=best_f, bwd_tail_passes=best_b, fp32_switch_columns=best_s)
    return dict(n=n, form="fp32" if fp32 else "fp64", fwd_tail_passes=best_f, bwd_tail_passes=best_b,
                fp32_switch_columns=best_s, k=p.k,
                fwd_ms={str(q): round(v, 4) for q, v in fwd.items()},
                bwd_ms={str(q): round(v, 4) for q, v in bwd.items()},
                pass_ms_by_switch={str(q): round(v, 4) for q, v in sws.items()})


def tune(ns=ALL_N, forms=(False, True), reps: int = 7, log=sys.stderr) -> dict:
    entries = []
    for n in ns:
        for fp32 in forms:
            e = tune_one(n, fp32, reps)
            entries.append(e)
            print(f"tuned n={n} {e['form']}: fwd passes {e['fwd_tail_passes']}, bwd passes "
                  f"{e['bwd_tail_passes']}, switch {e['fp32_switch_columns']}", file=log, flush=True)
    return dict(version=1, device=torch.cuda.get_device_name(0), entries=entries)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=ks.TUNE_PATH)
    ap.add_argument("--n", type=int, nargs="*", default=list(ALL_N))
    ap.add_argument("--reps", type=int, default=7)
    args = ap.parse_args()
    import os
    os.environ["KS_NO_TUNE"] = "1"  # start from the defaults, not a previous table
    table = tune(args.n, reps=args.reps)
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1)
    print(json.dumps({"entries": len(table["entries"]), "out": args.out}), flush=True)


if __name__ == "__main__":
    main()
