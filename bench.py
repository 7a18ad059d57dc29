"""Throughput benchmark of the odd-even Kalman smoother on one MI355X.

One step = one full smoothing pass (states and covariance blocks) of the
single-trajectory workload: n = 6, m = 3, k = 100000 (100001 states), per-step
F_i, dense SPD K_i and C_i, synthetic seeded data already resident in HBM.
Prints one JSON line:
  value        smoothed time steps per second (k+1 per step / wall time)
  roofline     the level-0 forward kernel (loads raw inputs, whitens, first
               elimination level): algorithmic bytes (below the FP64 ridge
               point, "hbm") or flops (above it, "alu") per launch / its
               average duration from hipEvents recorded on its own stream
  cpu_baseline the CPU oracle (sequential FP64 Paige-Saunders + Algorithm 1,
               compiled -O3 -march=native on this host, one thread pinned to
               one core) timed on a bounded sample
  large_blocks the large-block workload (n = 48, m = 24, k = 20000) in FP64
               and in the FP32 form: pass rate, the level-0 forward launch's
               FLOP/s against the FP64 / FP32 peak, errors against the oracle
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 FP64 lanes x 2 flops per FMA x 2.4 GHz
FP64_VALU_PEAK_TFS = 78.6
# FP32 vector (non-packed: 32 lanes per SIMD per clock)
FP32_VALU_PEAK_TFS = 157.3
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fwd_level0_n6_k100000.json")
# sources of the level-0 forward kernel of the benchmark workload (n = 6): a
# traffic summary taken on other sources is not used
KERNEL_SRCS = [os.path.join(ROOT, "paper_2502_11686_amd", "csrc", f)
               for f in ("ks_device.h", "ks_internal.h", "ks_inst_n6.hip")]


WORKLOAD_NAMES = {
    0: "one trajectory, n=4, m=2, k={k}, constant F, diagonal K and C, states and covariances",
    1: "one trajectory, n=6, m=3, k={k}, per-step F, dense K and C, states and covariances",
    2: "one trajectory, n=48, m=24, k={k}, per-step F, diagonal K and C, states and covariances",
}


def level0_forward_bytes(p, record_bytes: int = 8) -> int:
    """Algorithmic HBM bytes of the level-0 forward launch.

    Reads every raw input once (F, c, K for k steps, G, o, C for k+1 steps; H is
    the identity and not read; FP64) and writes ceil((k+1)/2) R-factor records
    of n(3n+1) values and floor((k+1)/2) reduced-system columns of n(3n+2)
    values (record_bytes each: 8, or 4 for an FP32 level of the FP32 form)."""
    k, n, m = p.k, p.n, p.m
    kk = n if p.K_diag else n * n
    cc = m if p.C_diag else m * m
    reads = k * (n * n + n + kk) + (k + 1) * (m * n + m + cc)
    if p.H is not None:
        reads += k * n * n
    writes = ((k + 2) // 2) * n * (3 * n + 1) + ((k + 1) // 2) * n * (3 * n + 2)
    return 8 * reads + record_bytes * writes


def state_model_bytes(n: int, m: int, K_diag: bool, C_diag: bool, fp32: bool = False) -> int:
    """Bytes one smoothed state moves in the whole pass by the per-state work
    model: s (18 n^2 + 9 n) for the levels' records, reduced systems, S blocks
    and outputs (s = 8, or 4 in the FP32 form whose wide levels store FP32),
    plus the FP64 inputs 2 n^2 + n + cov(n) + m n + m + cov(m)."""
    s = 4 if fp32 else 8
    cov_n = n if K_diag else n * n
    cov_m = m if C_diag else m * m
    return s * (18 * n * n + 9 * n) + 8 * (2 * n * n + n + cov_n + m * n + m + cov_m)


def _householder_flops(r: int, c: int, p: int) -> int:
    """Flops of a Householder QR of an r x c stack whose reflectors are also
    applied to p further columns: for pivot q (h = r - q rows below and on the
    diagonal, h > 1) the norm takes 2h and each of the c - q - 1 + p columns to
    its right a dot product and an update of 2h each (Section II's QR steps)."""
    f = 0
    for q in range(min(r, c)):
        h = r - q
        if h > 1:
            f += 2 * h + 4 * h * (c - q - 1 + p)
    return f


def level0_forward_flops(p) -> int:
    """Algorithmic flops of the level-0 forward launch, from the implemented
    stack shapes (Section III steps 1-3 with whitening fused in).

    Per unit (even column j and its right neighbour j+1): whitening of two
    evolution blocks [F | H | c] and two observation blocks [G | o] (Cholesky
    plus triangular solves for dense covariances, a scaling for diagonal ones);
    step 1, QR of the (m+n) x n stack [O_j; E-_{j+1}] applied to E+_{j+1} and
    the right-hand side; step 3, QR of the 2m x n stack [D~_{j+1}; O_{j+1}]
    with its right-hand side; step 2, QR of the 2n x n stack [E+_j; R~_j]
    applied to the left neighbour, right neighbour and right-hand side."""
    k, n, m = p.k, p.n, p.m
    units = (k + 1) // 2
    ev = n * (2 * n + 1) if p.K_diag else n ** 3 // 3 + n * n * (2 * n + 1)
    ob = m * (n + 1) if p.C_diag else m ** 3 // 3 + m * m * (n + 1)
    per_unit = (2 * ev + 2 * ob + _householder_flops(m + n, n, n + 1) + _householder_flops(2 * m, n, 1)
                + _householder_flops(2 * n, n, 2 * n + 1))
    return units * per_unit


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(per_launch_algo: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on a different kernel source."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if d.get("algorithmic_bytes_per_launch") != per_launch_algo:  # another workload's launch
        return None
    return d.get("bytes_per_launch")


_NATIVE_ORACLE = None


def native_oracle():
    """The oracle compiled on this host with -O3 -march=native (in a
    temporary directory) and loaded: the CPU baseline runs what a user of this
    machine would build."""
    global _NATIVE_ORACLE
    if _NATIVE_ORACLE is None:
        import tempfile
        from oracle import build as oracle_build, seq
        d = tempfile.mkdtemp(prefix="ks_oracle_")
        path = oracle_build.build(out=os.path.join(d, "libks_oracle_native.so"), native=True)
        _NATIVE_ORACLE = seq.load(path)
    return _NATIVE_ORACLE


def cpu_baseline(p, budget_s: float = 10.0):
    """The oracle on one core (the process pinned to its first allowed CPU
    while timed): the whole problem solved repeatedly for about budget_s."""
    from oracle import seq
    lib = native_oracle()
    allowed = os.sched_getaffinity(0)
    cpu = min(allowed)
    os.sched_setaffinity(0, {cpu})
    try:
        reps, t0 = 0, time.perf_counter()
        while True:
            seq.smooth(p, lib=lib)
            reps += 1
            el = time.perf_counter() - t0
            if el >= budget_s:
                break
    finally:
        os.sched_setaffinity(0, allowed)
    return dict(value=(p.k + 1) * reps / el, unit="steps/s", cores=1, kind="oracle",
                sample=f"the full workload (k={p.k}, n={p.n}, m={p.m}) solved {reps} times "
                       f"in {el:.1f} s, one thread pinned to CPU {cpu}, C FP64 built -O3 -march=native",
                host=host_cpu())


def cpu_baseline_many(probs, budget_s: float = 10.0):
    """The oracle on every allowed core, one problem per thread (the C code
    runs outside the GIL): problems taken in order until budget_s has passed,
    the ones started finished; rate = their states / wall time."""
    from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor, wait
    from oracle import seq
    lib = native_oracle()
    cores = len(os.sched_getaffinity(0))
    states, done = 0, 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        running, nxt = set(), 0
        while nxt < len(probs) or running:
            while nxt < len(probs) and len(running) < cores and time.perf_counter() - t0 < budget_s:
                running.add(ex.submit(lambda q: (seq.smooth(q, lib=lib), q.k + 1)[1], probs[nxt]))
                nxt += 1
            if not running:
                break
            fin, running = wait(running, return_when=FIRST_COMPLETED)
            for f in fin:
                states += f.result()
                done += 1
    el = time.perf_counter() - t0
    return dict(value=states / el, unit="steps/s", cores=cores, kind="oracle",
                sample=f"{done} of the {len(probs)} problems ({states} states) in {el:.1f} s, one problem per "
                       f"thread on {cores} threads, C FP64 built -O3 -march=native",
                host=host_cpu())


def host_cpu() -> str:
    """CPU model name and logical CPU count of this host."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical CPUs"



def large_block_leg(check: bool, dev):
    """The large-block workload (n = 48, m = 24, k = 20000, per-step F,
    diagonal covariances) in FP64 and in the FP32 form: whole-pass rate, the
    level-0 forward launch's FLOP/s against the peak of the precision it
    computes in (its arithmetic intensity is above the FP64 ridge point), and
    the errors against the oracle."""
    import numpy as np
    import torch

    from paper_2502_11686_amd import gen, ks

    p = gen.workload(2)
    tens = ks.to_device(p, dev)
    u = torch.empty((p.k + 1, p.n), dtype=torch.float64, device=dev)
    S = torch.empty((p.k + 1, p.n, p.n), dtype=torch.float64, device=dev)
    ref = None
    if check:
        from oracle import seq
        ref = seq.smooth(p)
    flops = level0_forward_flops(p)
    out = {"workload": WORKLOAD_NAMES[2].format(k=p.k)}
    for fp32 in (False, True):
        plan = ks.Plan(p.k, p.n, p.m, p.K_diag, p.C_diag, device=dev, fp32=fp32)
        for _ in range(3):
            plan.smooth_cov(*tens, u_out=u, cov_out=S)
        steps = 10
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.smooth_cov(*tens, u_out=u, cov_out=S)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        plan.time_kernels(ks.KS_TIME_FWD_LEVEL0)
        for _ in range(5):
            plan.smooth_cov(*tens, u_out=u, cov_out=S)
        ms, cnt = plan.kernel_time()
        plan.time_kernels(ks.KS_TIME_OFF)
        level0_fp32 = fp32 and plan.schedule()["fp32_levels"] >= 1
        plan.close()
        avg_s = ms / max(cnt, 1) / 1e3
        peak = FP32_VALU_PEAK_TFS if level0_fp32 else FP64_VALU_PEAK_TFS
        # FP64 level 0 of forward variant 1 (diagonal covariances): the blocked
        # QR whose trailing updates run on the FP64 matrix cores (their dense
        # peak equals the FP64 vector peak, 78.6 TFLOP/s)
        on_mfma = (not level0_fp32 and p.K_diag and p.C_diag
                   and ks.get_tuning(p.n, False)["fwd_variant"] == 1 and ks.kernel_variants(p.n, p.m, False) >= 2)
        algo = level0_forward_bytes(p, 4 if level0_fp32 else 8)
        err = None
        if ref is not None:
            uu, SS = u.cpu().numpy(), S.cpu().numpy()
            err = dict(state=float(np.max(np.abs(uu - ref["u"])) / np.max(np.abs(ref["u"]))),
                       cov=float(np.max(np.linalg.norm(SS - ref["cov"], axis=(1, 2)) /
                                        np.linalg.norm(ref["cov"], axis=(1, 2)))))
        model_flops = 40 * p.n ** 3 * (p.k + 1)
        out["fp32_form" if fp32 else "fp64"] = {
            "value": (p.k + 1) * steps / el, "unit": "steps/s", "ms_per_step": el / steps * 1e3,
            "err_vs_oracle": err,
            "pass_model_tflops": model_flops / (el / steps) / 1e12,
            "roofline": {"bound": "mfma" if on_mfma else "alu", "achieved": flops / avg_s / 1e12, "peak": peak,
                         "unit": "TFLOP/s", "frac": flops / avg_s / 1e12 / peak, "traffic": None,
                         "kernel": f"level-0 forward (n={p.n}, m={p.m}, {'FP32' if level0_fp32 else 'FP64'}"
                                   f"{', blocked QR on FP64 matrix cores' if on_mfma else ''})",
                         "algo_flops_per_launch": flops, "algo_bytes_per_launch": algo,
                         "avg_launch_ms": avg_s * 1e3, "launches_timed": cnt,
                         "hbm_frac": algo / avg_s / 1e9 / HBM_PEAK_GBS}}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", type=int, default=1, choices=(0, 1, 2, 3, 4))
    ap.add_argument("--problems", type=int, default=512, help="batched workload: number of problems")
    ap.add_argument("--requests", type=int, default=2000, help="serving workload: number of requests")
    ap.add_argument("--pool", type=int, default=48, help="serving workload: distinct problems the requests cycle over")
    ap.add_argument("--rate", type=float, default=None,
                    help="serving workload: Poisson arrival rate (1/s); default 0.7 x the measured capacity")
    ap.add_argument("--hbm-gb", type=float, default=96.0,
                    help="serving workload: engine workspace (request regions) in GB; inputs and outputs "
                         "are admitted against the same amount again")
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device copy of 1 GiB (5 launches) for HBM-counter calibration")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="default line: leave out the large-block (n = 48) FP64 / FP32-form leg")
    ap.add_argument("--no-check", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (independent problems "
              "would shard with no communication, one long trajectory by time chunks with one exchange of "
              "the chunk-top reduced columns)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2502_11686_amd import gen, ks

    if args.calibrate_copy:
        # a plain copy kernel of known size: 1 GiB read and 1 GiB written per launch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": src.numel() * 8, "launches": 5}), flush=True)
        return
    if args.workload == 3:
        return batch_bench(args)
    if args.workload == 4:
        return serve_bench(args)
    p = gen.workload(args.workload, k=args.k)
    dev = torch.device("cuda", 0)
    tens = ks.to_device(p, dev)
    plan = ks.Plan(p.k, p.n, p.m, p.K_diag, p.C_diag, device=dev)
    u = torch.empty((p.k + 1, p.n), dtype=torch.float64, device=dev)
    S = torch.empty((p.k + 1, p.n, p.n), dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        plan.smooth_cov(*tens, u_out=u, cov_out=S)

    # timed region: K full passes, each a synchronous library call
    plan.time_kernels(ks.KS_TIME_FWD_LEVEL0)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        plan.smooth_cov(*tens, u_out=u, cov_out=S)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    k_ms, k_cnt = plan.kernel_time()

    # states-only (NC) rate and the phase split, outside the timed region
    plan.time_kernels(ks.KS_TIME_OFF)
    nc_steps = max(10, args.steps // 4)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(nc_steps):
        plan.smooth(*tens, u_out=u)
    torch.cuda.synchronize()
    nc_el = time.perf_counter() - t1
    phases = {}
    for name, kind in (("forward_all", ks.KS_TIME_FWD_ALL), ("backward_all", ks.KS_TIME_BWD_ALL),
                       ("backward_level0", ks.KS_TIME_BWD_LEVEL0)):
        plan.time_kernels(kind)
        for _ in range(10):
            plan.smooth_cov(*tens, u_out=u, cov_out=S)
        ms, cnt = plan.kernel_time()
        phases[name] = round(ms / max(cnt, 1), 4)
    plan.time_kernels(ks.KS_TIME_OFF)

    def errors(ref):
        uu, SS = u.cpu().numpy(), S.cpu().numpy()
        return dict(state=float(np.max(np.abs(uu - ref["u"])) / np.max(np.abs(ref["u"]))),
                    cov=float(np.max(np.linalg.norm(SS - ref["cov"], axis=(1, 2)) /
                                     np.linalg.norm(ref["cov"], axis=(1, 2)))))

    ref = None
    err = None
    if not args.no_check:
        from oracle import seq
        ref = seq.smooth(p)
        plan.smooth_cov(*tens, u_out=u, cov_out=S)
        err = errors(ref)

    # the FP32 form on the same inputs (FP32 wide levels, FP64 top levels and SelInv)
    plan32 = ks.Plan(p.k, p.n, p.m, p.K_diag, p.C_diag, device=dev, fp32=True)
    for _ in range(max(1, args.warmup // 2)):
        plan32.smooth_cov(*tens, u_out=u, cov_out=S)
    steps32 = max(10, args.steps // 2)
    lat32 = []
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps32):
        ts = time.perf_counter()
        plan32.smooth_cov(*tens, u_out=u, cov_out=S)
        lat32.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    el32 = time.perf_counter() - t2
    fp32_form = dict(value=(p.k + 1) * steps32 / el32, unit="steps/s",
                     ms_per_step=el32 / steps32 * 1e3,
                     p50_ms=float(np.percentile(np.array(lat32) * 1e3, 50)),
                     p99_ms=float(np.percentile(np.array(lat32) * 1e3, 99)),
                     err_vs_oracle=errors(ref) if ref is not None else None)
    plan32.close()

    algo = level0_forward_bytes(p)
    flops = level0_forward_flops(p)
    avg_s = (k_ms / max(k_cnt, 1)) / 1e3
    # the bound is the resource the kernel's arithmetic intensity saturates
    # first: HBM below the FP64 ridge point (peak flops / peak bytes), the FP64
    # vector units above it (the level kernels do their FP64 arithmetic on VALU)
    hbm_bound = flops / algo <= FP64_VALU_PEAK_TFS * 1e3 / HBM_PEAK_GBS
    if hbm_bound:
        achieved, peak, unit = algo / avg_s / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        achieved, peak, unit = flops / avg_s / 1e12, FP64_VALU_PEAK_TFS, "TFLOP/s"
    traffic = measured_traffic(algo)
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": "smoothed time steps/s incl. covariances, FP64 vs FP32 form; p50/p99 latency",
        "value": (p.k + 1) * args.steps / el,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generator; per-step Haar-based F, Gaussian G, dense SPD K and C)",
        "config": {"workload": WORKLOAD_NAMES[args.workload].format(k=p.k), "problems": 1,
                   "k": p.k, "n": p.n, "m": p.m},
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "nc_value": (p.k + 1) * nc_steps / nc_el,
        "phase_ms": phases,
        "err_vs_oracle": err,
        "fp32_form": fp32_form,
        "roofline": {"bound": "hbm" if hbm_bound else "alu", "achieved": achieved, "peak": peak,
                     "unit": unit, "frac": achieved / peak, "traffic": traffic,
                     "kernel": f"level-0 forward (n={p.n}, m={p.m})", "algo_bytes_per_launch": algo,
                     "algo_flops_per_launch": flops, "avg_launch_ms": avg_s * 1e3, "launches_timed": k_cnt,
                     "hbm_frac": algo / avg_s / 1e9 / HBM_PEAK_GBS,
                     "fp64_frac": flops / avg_s / 1e12 / FP64_VALU_PEAK_TFS},
    }
    plan.close()
    if args.workload == 1 and not args.no_large:
        out["large_blocks"] = large_block_leg(not args.no_check, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out), flush=True)


def batch_bench(args):
    """512 uneven problems (k log-uniform in [64, 16384], n in {4, 8, 16, 32},
    m = n/2, diagonal covariances): one batched pass per step, FP64 and the
    FP32 form; value = smoothed states of all problems per second."""
    import numpy as np
    import torch

    from paper_2502_11686_amd import gen, ks

    dev = torch.device("cuda", 0)
    probs = gen.batch_workload(args.problems)
    steps_total = sum(p.k + 1 for p in probs)
    inputs = [ks.to_device(p, dev) for p in probs]
    out = {}
    for fp32 in (False, True):
        b = ks.Batch([(p.k, p.n, p.m, p.K_diag, p.C_diag, fp32) for p in probs], device=dev)
        us, covs = b.outputs(True)
        for _ in range(max(1, args.warmup)):
            b.smooth(inputs, us, covs)
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            b.smooth(inputs, us, covs)
            lat.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        err = None
        if not args.no_check:
            from oracle import seq
            eu = es = 0.0
            for i in range(0, len(probs), max(1, len(probs) // 16)):
                ref = seq.smooth(probs[i])
                u, S = us[i].cpu().numpy(), covs[i].cpu().numpy()
                eu = max(eu, float(np.max(np.abs(u - ref["u"])) / np.max(np.abs(ref["u"]))))
                es = max(es, float(np.max(np.linalg.norm(S - ref["cov"], axis=(1, 2)) /
                                          np.linalg.norm(ref["cov"], axis=(1, 2)))))
            err = dict(state=eu, cov=es, problems_checked=len(range(0, len(probs), max(1, len(probs) // 16))))
        out["fp32_form" if fp32 else "fp64"] = dict(
            value=steps_total * args.steps / el, ms_per_step=el / args.steps * 1e3,
            p50_ms=float(np.percentile(np.array(lat) * 1e3, 50)),
            p99_ms=float(np.percentile(np.array(lat) * 1e3, 99)), err_vs_oracle=err)
        b.close()
    # whole-pass roofline by the per-state work model (bytes each state moves)
    for name, fp32 in (("fp64", False), ("fp32_form", True)):
        bytes_pass = sum((p.k + 1) * state_model_bytes(p.n, p.m, p.K_diag, p.C_diag, fp32) for p in probs)
        ach = bytes_pass / (out[name]["ms_per_step"] / 1e3) / 1e9
        out[name]["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": ach / HBM_PEAK_GBS, "traffic": None,
                                 "kernel": "whole batched pass (per-state work model bytes)",
                                 "model_bytes_per_pass": bytes_pass}
    line = {
        "metric": "smoothed time steps/s incl. covariances, FP64 vs FP32 form; p50/p99 latency",
        "value": out["fp64"]["value"], "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": out["fp64"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generator; per-step F and G, diagonal covariances)",
        "config": {"workload": f"{len(probs)} uneven problems, k log-uniform [64,16384], n in {{4,8,16,32}}, "
                               "m=n/2, one batched pass (hipGraph)", "problems": len(probs),
                   "states": steps_total},
        "p50_ms": out["fp64"]["p50_ms"], "p99_ms": out["fp64"]["p99_ms"],
        "err_vs_oracle": out["fp64"]["err_vs_oracle"], "fp32_form": out["fp32_form"],
        "roofline": out["fp64"]["roofline"],
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_many(probs)
    print(json.dumps(line), flush=True)


def _make_request(req):
    from paper_2502_11686_amd import gen
    p = gen.request_problem(req)
    return p


def _oracle_result(p):
    from oracle import seq
    r = seq.smooth(p, lib=native_oracle())
    return r["u"], r["cov"]


def serve_bench(args):
    """Serving: Poisson arrivals of requests (k log-uniform in [100, 2e5],
    n in {6, 12, 24}, m = n/2, per-step F, dense K and C, half of them in the
    FP32 form) into the continuous-batching engine.  Request i smooths problem
    i mod P of a pool of P generated problems (drawn from the same
    distribution), which keeps host memory bounded at thousands of requests;
    arrival, precision form, admission, inputs copy and outputs are per
    request.  Two runs over the same requests: all arriving at once (the
    engine's capacity: value = smoothed states per second of makespan), then
    Poisson arrivals at 0.7 of the capacity's request rate (or --rate), whose
    p50/p99 latency is reported.  A request's latency runs from its arrival to
    its outputs being final, including the copy of its inputs from pinned host
    memory.  Every 10th request's outputs are compared on the device with the
    oracle's solution of its problem; a failed request ends the run."""
    import numpy as np
    import torch
    from concurrent.futures import ProcessPoolExecutor, ThreadPoolExecutor

    from paper_2502_11686_amd import gen, ks

    dev = torch.device("cuda", 0)
    reqs = gen.serving_requests(args.requests, 1.0)
    P = max(1, min(args.pool, len(reqs)))
    t_gen = time.perf_counter()
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        pool = list(ex.map(_make_request, reqs[:P]))
    host = []
    for p in pool:
        host.append([None if a is None else torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
                     for a in (p.H, p.F, p.c, p.K, p.G, p.o, p.C)])
    probs = [pool[i % P] for i in range(len(reqs))]
    t_gen = time.perf_counter() - t_gen
    print(f"serving: {len(reqs)} requests over a pool of {P} problems generated in {t_gen:.1f} s",
          file=sys.stderr, flush=True)

    # the oracle's solutions of the pool problems the checked requests use, on the device
    checked = list(range(0, len(reqs), 10)) if not args.no_check else []
    refs = {}
    if checked:
        need = sorted({i % P for i in checked})
        t_or = time.perf_counter()
        with ThreadPoolExecutor(max_workers=len(os.sched_getaffinity(0))) as ex:
            for q, (u, S) in zip(need, ex.map(lambda q: _oracle_result(pool[q]), need)):
                refs[q] = (torch.from_numpy(u).to(dev), torch.from_numpy(S).to(dev),
                           float(np.max(np.abs(u))), torch.from_numpy(np.linalg.norm(S, axis=(1, 2))).to(dev))
        print(f"serving: oracle solutions of {len(need)} pool problems in {time.perf_counter() - t_or:.1f} s",
              file=sys.stderr, flush=True)

    ws = int(args.hbm_gb * 1e9) // 256 * 256
    io_budget = ws
    main_stream = torch.cuda.current_stream(dev)
    copy_stream = torch.cuda.Stream(dev)
    eng = ks.Engine(ws, device=dev, stream=main_stream)

    def io_bytes(p):
        per = sum(0 if a is None else a.nbytes for a in (p.H, p.F, p.c, p.K, p.G, p.o, p.C))
        return per + 8 * (p.k + 1) * p.n * (p.n + 1)

    # warm-up: one small request of each (n, form) through the engine
    for n in (6, 12, 24):
        for f32 in (False, True):
            wp = gen.make_problem(np.random.default_rng(n), 300, n, n // 2, cov="dense")
            u = torch.empty((wp.k + 1, n), dtype=torch.float64, device=dev)
            S = torch.empty((wp.k + 1, n, n), dtype=torch.float64, device=dev)
            eng.submit((wp.k, n, n // 2, False, False, f32), ks.to_device(wp, dev), u, S)
    while eng.stats()["inflight"]:
        eng.step()
    eng.wait()
    torch.cuda.synchronize()

    def run(arrival, check):
        """Serve every request, request i arriving at arrival[i] seconds
        (sorted); with check, the errors of the checked requests (device
        scalars, read at the end)."""
        queue, nxt = [], 0
        inflight, lat, io_used, statuses = {}, {}, 0, {}
        errs = []
        ticks = 0
        t0 = time.perf_counter()
        while nxt < len(reqs) or queue or inflight:
            now = time.perf_counter() - t0
            while nxt < len(reqs) and arrival[nxt] <= now:
                queue.append(nxt)
                nxt += 1
            # FIFO admission: stop at the first request that does not fit
            while queue:
                i = queue[0]
                p, r = probs[i], reqs[i]
                need = io_bytes(p)
                if io_used + need > io_budget:
                    break
                # the inputs travel on a copy stream, overlapping the ticks already
                # enqueued; the engine's stream waits for them before its next tick
                with torch.cuda.stream(copy_stream):
                    dargs = tuple(None if a is None else a.to(dev, non_blocking=True) for a in host[i % P])
                for a in dargs:
                    if a is not None:
                        a.record_stream(main_stream)
                main_stream.wait_event(copy_stream.record_event())
                u = torch.empty((p.k + 1, p.n), dtype=torch.float64, device=dev)
                S = torch.empty((p.k + 1, p.n, p.n), dtype=torch.float64, device=dev)
                t = eng.submit((p.k, p.n, p.m, p.K_diag, p.C_diag, r["fp32"]), dargs, u, S)
                if t is None:
                    break
                queue.pop(0)
                io_used += need
                inflight[t] = (i, u, S, need)
            if not inflight:
                if queue:
                    raise RuntimeError(f"request {queue[0]} does not fit the HBM budget")
                if nxt < len(reqs):
                    time.sleep(max(0.0, arrival[nxt] - (time.perf_counter() - t0)))
                continue
            for t, st in eng.step():
                i, u, S, need = inflight.pop(t)
                lat[i] = time.perf_counter() - t0 - arrival[i]
                io_used -= need
                statuses[i] = st
                if st != ks.KS_OK:
                    raise RuntimeError(f"request {i} failed with status {st}")
                if check and i % 10 == 0:
                    ru, rS, umax, snorm = refs[i % P]
                    eu = (u - ru).abs().max() / umax
                    es = (torch.linalg.matrix_norm(S - rS) / snorm).max()
                    errs.append((i, eu, es))
            ticks += 1
        torch.cuda.synchronize()
        makespan = time.perf_counter() - t0 - arrival[0]
        return lat, makespan, ticks, errs

    steps_total = sum(p.k + 1 for p in probs)
    # capacity: every request queued at t = 0
    _lat_sat, span_sat, ticks_sat, _e = run([0.0] * len(reqs), False)
    capacity = steps_total / span_sat
    rate = args.rate if args.rate else 0.7 * len(reqs) / span_sat
    print(f"serving: capacity {capacity:.3e} states/s ({len(reqs) / span_sat:.1f} requests/s); "
          f"paced run at {rate:.1f} requests/s", file=sys.stderr, flush=True)
    gaps = np.diff([0.0] + [r["arrival_s"] for r in reqs])  # Poisson gaps at rate 1
    arrival = list(np.cumsum(gaps) / rate)
    lat, makespan, ticks, errs = run(arrival, bool(checked))
    lat_ms = np.array([lat[i] for i in range(len(reqs))]) * 1e3
    by_form = {}
    for name, f in (("fp64", False), ("fp32_form", True)):
        idx = [i for i, r in enumerate(reqs) if r["fp32"] == f]
        if idx:
            by_form[name] = dict(requests=len(idx), p50_ms=float(np.percentile(lat_ms[idx], 50)),
                                 p99_ms=float(np.percentile(lat_ms[idx], 99)),
                                 states=int(sum(probs[i].k + 1 for i in idx)))
    err = None
    if checked:
        err = {}
        for name, f in (("fp64", False), ("fp32_form", True)):
            sel = [(float(eu), float(es)) for i, eu, es in errs if reqs[i]["fp32"] == f]
            if sel:
                err[name] = dict(state=max(a for a, _b in sel), cov=max(b for _a, b in sel),
                                 requests_checked=len(sel))
        gate = {"fp64": (1e-10, 1e-9), "fp32_form": (1e-5, 1e-5)}
        for name, e in err.items():
            e["within_gate"] = e["state"] <= gate[name][0] and e["cov"] <= gate[name][1]
    bytes_total = sum((p.k + 1) * state_model_bytes(p.n, p.m, p.K_diag, p.C_diag, r["fp32"])
                      for p, r in zip(probs, reqs))
    ach = bytes_total / span_sat / 1e9
    line = {
        "metric": "smoothed time steps/s incl. covariances, FP64 vs FP32 form; p50/p99 latency",
        "value": capacity, "unit": "steps/s", "n_gpus": 1, "steps": len(reqs),
        "warmup": 6, "ms_per_step": span_sat * 1e3 / len(reqs), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
        "data": "synthetic (seeded generator; per-step F and G, dense K and C, Poisson arrivals)",
        "config": {"workload": f"serving: {len(reqs)} requests (a pool of {P} problems), k log-uniform "
                               "[100,200000], n in {6,12,24}, m=n/2, half FP32 form, continuous batching; value = "
                               "capacity (all queued at t=0), latency at Poisson arrivals of 0.7x the capacity "
                               "request rate", "requests": len(reqs), "pool": P, "states": steps_total,
                   "hbm_budget_gb": args.hbm_gb},
        "capacity_requests_per_s": len(reqs) / span_sat, "ticks_saturated": ticks_sat,
        "paced": {"rate_per_s": rate, "throughput_steps_per_s": steps_total / makespan,
                  "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
                  "ticks": ticks, "by_form": by_form},
        "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
        "err_vs_oracle": err,
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole capacity run (per-state work model bytes)", "model_bytes": bytes_total},
    }
    eng.close()
    if not args.no_cpu_baseline:
        # the oracle's single-core rate on the pool problems of the checked requests (its time per request)
        line["cpu_baseline"] = cpu_baseline_many([pool[q] for q in sorted({i % P for i in range(0, len(reqs), 10)})],
                                                 budget_s=10.0)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
