"""Autotuner of the kernels' shape variants and the schedule's free choices,
per state dimension and precision form.

For each (n, form) it smooths one synthetic problem of that n and times the
candidates of each choice in turn, keeping the best so far for the next:

* backward variant: the compiled shapes of the backward kernels (records per
  MFMA workgroup; for n = 1, 2, 3, 5 the MFMA family instead of the wavefront
  family), timed over the backward launches (KS_TIME_BWD_ALL);
* forward variant: level 0 with or without its inputs staged in LDS, timed
  over the forward launches (KS_TIME_FWD_ALL);
* forward and backward tail passes: how many unit passes of the
  single-workgroup tail kernels the top levels may take instead of one launch
  each;
* level groups: several consecutive levels per launch from a given level on
  (forward: where the kernel family has group kernels; backward);
* FP32 form: the column count above which a level runs in FP32.  A width is
  admissible only if the FP32-form errors against the FP64 path of the same
  problem stay within 1e-5 (states normwise, covariance blocks per block).

A candidate replaces the current choice only if its median beats the current
median by more than 2 % and by more than the spread (median absolute
deviation) of the current choice's repeats, so timing noise never moves a
choice.  Variants and schedule choices change launch shapes, not what is
computed (apart from the FP32 switch, and the wavefront / MFMA choice at
n <= 5, which change rounding); the choice depends only on (n, form), never
on what a batch holds.  The table is JSON; ks.load_tuning applies it, and the
binding loads tune_mi355x.json next to the library by default.

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
GROUP_SIZES = (2, 3, 4)
GROUP_FROM = (1, 3, 5, 7, 9, 11)
ALL_N = (1, 2, 3, 4, 5, 6, 8, 12, 16, 24, 32, 48)
FP32_GATE = 1e-5


def problem_k(n: int) -> int:
    """Trajectory length the table is tuned at: the single-problem workloads'
    lengths (k = 1e5 at small n, 2e4 for the large blocks), so that both the
    wide levels (where the shape variants differ most) and the top levels
    (what the tail and group choices act on) are there."""
    return 100000 if n <= 8 else (50000 if n <= 12 else 20000)


def _problem(n: int):
    return gen.make_problem(np.random.default_rng(7000 + n), problem_k(n), n, max(1, n // 2),
                            F_mode="per_step", cov="diag")


def _mad(xs):
    m = statistics.median(xs)
    return statistics.median([abs(x - m) for x in xs])


def _timed(p, args, fp32: bool, kind, reps: int):
    """Repeats of one timing: milliseconds of the selected launches per call
    (kind) or of whole calls (kind None); and the outputs."""
    plan = ks.Plan(p.k, p.n, p.m, p.K_diag, p.C_diag, fp32=fp32)
    try:
        u = torch.empty((p.k + 1, p.n), dtype=torch.float64, device="cuda")
        S = torch.empty((p.k + 1, p.n, p.n), dtype=torch.float64, device="cuda")
        plan.smooth_cov(*args, u_out=u, cov_out=S)  # warm-up (and graph capture)
        plan.smooth_cov(*args, u_out=u, cov_out=S)
        out = []
        if kind is None:
            torch.cuda.synchronize()
            for _ in range(reps):
                t0 = time.perf_counter()
                plan.smooth_cov(*args, u_out=u, cov_out=S)
                out.append((time.perf_counter() - t0) * 1e3)
        else:
            for _ in range(reps):
                plan.time_kernels(kind)
                plan.smooth_cov(*args, u_out=u, cov_out=S)
                t, cnt = plan.kernel_time()
                out.append(t / max(cnt, 1))
            plan.time_kernels(ks.KS_TIME_OFF)
        return out, u, S
    finally:
        plan.close()


def _choose(n, fp32, keys, candidates, p, args, kind, reps, cur, log, admissible=None):
    """Time every candidate value of the tuning keys and move the current
    choice to the fastest by the noise rule; returns the new choice and the
    median milliseconds per candidate."""
    times = {}
    for c in candidates:
        ks.set_tuning(n, fp32, **dict(cur, **dict(zip(keys, c))))
        ts, u, S = _timed(p, args, fp32, kind, reps)
        if admissible is not None and not admissible(u, S):
            print(f"  n={n} {keys}={c}: outside the FP32-form gate, not admissible", file=log, flush=True)
            continue
        times[c] = (statistics.median(ts), _mad(ts))
    base = tuple(cur[k] for k in keys)
    if base not in times:  # the current choice itself, timed the same way
        ks.set_tuning(n, fp32, **cur)
        ts, _u, _S = _timed(p, args, fp32, kind, reps)
        times[base] = (statistics.median(ts), _mad(ts))
    best = min(times, key=lambda c: times[c][0])
    m0, d0 = times[base]
    if best != base and times[best][0] < m0 * 0.98 and m0 - times[best][0] > d0:
        cur = dict(cur, **dict(zip(keys, best)))
    ks.set_tuning(n, fp32, **cur)
    return cur, {"/".join(map(str, c)): round(v[0], 4) for c, v in times.items()}


def tune_one(n: int, fp32: bool, reps: int = 7, log=sys.stderr) -> dict:
    p = _problem(n)
    args = ks.to_device(p)
    cur = dict(ks.TUNING_DEFAULTS)
    ks.set_tuning(n, fp32, **cur)
    rec = {}
    nbv = ks.kernel_variants(n, p.m, True)
    nfv = ks.kernel_variants(n, p.m, False)
    cur, rec["bwd_variant_ms"] = _choose(n, fp32, ("bwd_variant",), [(v,) for v in range(nbv)], p, args,
                                         ks.KS_TIME_BWD_ALL, reps, cur, log)
    cur, rec["fwd_variant_ms"] = _choose(n, fp32, ("fwd_variant",), [(v,) for v in range(nfv)], p, args,
                                         ks.KS_TIME_FWD_ALL, reps, cur, log)
    cur, rec["fwd_ms"] = _choose(n, fp32, ("fwd_tail_passes",), [(q,) for q in PASSES], p, args,
                                 ks.KS_TIME_FWD_ALL, reps, cur, log)
    cur, rec["bwd_ms"] = _choose(n, fp32, ("bwd_tail_passes",), [(q,) for q in PASSES], p, args,
                                 ks.KS_TIME_BWD_ALL, reps, cur, log)
    groups = [(g, f) for g in GROUP_SIZES for f in GROUP_FROM]
    if n <= 12:  # forward group kernels exist for the wavefront family
        cur, rec["fwd_group_ms"] = _choose(n, fp32, ("fwd_group", "fwd_group_from"), groups, p, args,
                                           ks.KS_TIME_FWD_ALL, reps, cur, log)
    cur, rec["bwd_group_ms"] = _choose(n, fp32, ("bwd_group", "bwd_group_from"), groups, p, args,
                                       ks.KS_TIME_BWD_ALL, reps, cur, log)
    if fp32:
        saved64 = ks.get_tuning(n, False)
        ks.set_tuning(n, False, **ks.TUNING_DEFAULTS)
        _ts, u64, S64 = _timed(p, args, False, None, 1)
        ks.set_tuning(n, False, **saved64)
        s_norm = torch.linalg.matrix_norm(S64)
        u_max = u64.abs().max()

        def admissible(u, S):
            eu = float((u - u64).abs().max() / u_max)
            es = float((torch.linalg.matrix_norm(S - S64) / s_norm).max())
            return eu <= FP32_GATE and es <= FP32_GATE

        cur, rec["pass_ms_by_switch"] = _choose(n, fp32, ("fp32_switch_columns",), [(s,) for s in SWITCHES], p,
                                                args, None, reps, cur, log, admissible)
    ks.set_tuning(n, fp32, **cur)
    entry = dict(n=n, form="fp32" if fp32 else "fp64", k=p.k, **cur, **rec)
    print(f"tuned n={n} {entry['form']}: " + ", ".join(f"{k}={cur[k]}" for k in ks.TUNING_KEYS), file=log,
          flush=True)
    return entry


def tune(ns=ALL_N, forms=(False, True), reps: int = 7, log=sys.stderr) -> dict:
    entries = [tune_one(n, fp32, reps, log) for n in ns for fp32 in forms]
    return dict(version=2, device=torch.cuda.get_device_name(0), entries=entries)


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
