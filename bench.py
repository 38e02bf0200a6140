"""Benchmark: sketched TT-GMRES time to a 1e-6 true relative residual on one MI355X.

Workload: convection-diffusion, d = 10, n = 64 per mode: Laplacian (h = 1/65)
plus 0.1 x upwind convection in mode 1 as a rank-3 TT-matrix; right-hand side a
seeded random rank-4 TT with Gaussian cores; basis ranks capped at 64; Khatri-Rao
sketch with s = 1000 rows; STTA target ranks 64 and left ranks 84; q = 1;
basis rounding tolerance 1e-7; stop on the FP64 true residual <= 1e-6.

One step = one complete solve (every Krylov step of the hot path: Khatri-Rao
sketch of A v_k, orthogonalization coefficients, STTA sketch and streaming
combination, STTA recovery + TT-SVD rounding, sketch of v_{k+1}, sketched least
squares; then the final solution and its FP64 true residual).  Inputs are
resident on the GPU before the timed region.

Prints one JSON line.  Only N = 1 is supported (one GPU).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TT-SGMRES time to 1e-6 residual + rounding GFLOP/s, mixed vs FP64 GPU"
PEAK = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2.5e15}
# FP64 vector ALU peak (256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz)
PEAK_F64_VECTOR = 78.6e12
HBM_PEAK = 8.0e12


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["mixed", "f64"], default="mixed")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="wall-clock budget of the oracle sample")
    ap.add_argument("--no-fp64-leg", action="store_true", help="skip timing the FP64 path beside the mixed one")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default contraction tiles (no tuned table, no tuning)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy a 256 MiB buffer with a plain device copy (reference for HBM byte counters)")
    return ap.parse_args()


def build_inputs(dev):
    import synthetic as syn
    from paper_2409_09471_amd import ttsg
    w = syn.config_c2()
    t = dict(
        A=ttsg.kron_sum_operator(w.terms, dev), b=ttsg.to_device(w.b, dev), S=ttsg.to_device(w.S, dev),
        X=ttsg.to_device(w.X, dev), Y=ttsg.to_device(w.Y, dev),
    )
    return w, t


def solve(w, t, precision, phase_timing=False):
    from paper_2409_09471_amd import ttsg
    return ttsg.sgmres_solve(t["A"], t["b"], t["S"], t["X"], t["Y"], w.rx, w.rho, maxit=w.maxit, tol=w.tol,
                             q=w.q, round_tol=w.round_tol, maxrank=w.cap, stop_safety=w.stop_safety,
                             precision=precision, phase_timing=phase_timing)


def timed_solves(w, t, precision, steps, warmup, measure=True, tune=False):
    """Wall-clock time of `steps` solves (measurement off), then (measure=True)
    one more solve with the per-launch device timers on for the kernel figures.
    With tune=True the first warmup solve runs with the tile autotuner on."""
    import torch
    from paper_2409_09471_amd import ttsg
    for i in range(warmup):
        ttsg.autotune(tune and i == 0)
        r = solve(w, t, precision)
        ttsg.autotune(False)
        print(f"# warmup {i}: its={r.iterations} true_res={r.true_residual:.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(steps):
        results.append(solve(w, t, precision))
        print(f"# step {i}: its={results[-1].iterations} true_res={results[-1].true_residual:.3e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stats = {}
    if measure:
        ttsg.stats_enable(True)
        solve(w, t, precision)
        stats = ttsg.stats_read()
        ttsg.stats_enable(False)
    return elapsed, results, stats


def rounding_gflops(w, t):
    """ttsg_round_rand on a materialized A v (rank 3 x 64 -> 64) at the workload's shapes."""
    import numpy as np
    import torch
    import synthetic as syn
    from paper_2409_09471_amd import ttsg
    rng = np.random.default_rng(7)
    v = ttsg.to_device(syn.gaussian_tt(rng, w.ns, [1] + [w.cap] * (w.d - 1) + [1]), "cuda:0")
    av = ttsg.matvec(t["A"], v)
    ttsg.round_rand(av, t["X"], t["Y"], w.rx, w.rho, w.round_tol, w.cap)
    torch.cuda.synchronize()
    ttsg.stats_enable(True)
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        ttsg.round_rand(av, t["X"], t["Y"], w.rx, w.rho, w.round_tol, w.cap)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    st = ttsg.stats_read()
    ttsg.stats_enable(False)
    fl = sum(v["flops"] for v in st.values()) / reps
    return dict(seconds=el, gflop=fl / 1e9, gflops_per_s=fl / el / 1e9)


# HBM counter summaries per kernel class: (file under profiles/, kernel source
# whose SHA-256 the summary records)
COUNTER_SUMMARIES = {
    "contract_f64": ("contract_kernel_f64_hbm_counters_convdiff_d10_n64.md", "contract.hip"),
    "contract_f32": ("contract_kernel_f32_hbm_counters_convdiff_d10_n64.md", "contract.hip"),
    "svd_jacobi": ("k_jacobi_lds_hbm_counters_convdiff_d10_n64.md", "la_lds.hip"),
}
TILE_TABLE = os.path.join(ROOT, "paper_2409_09471_amd", "tiles_gfx950.txt")


def counter_traffic(cls):
    """HBM bytes per launch of the kernel class `cls` from its committed
    FETCH_SIZE / WRITE_SIZE summary, or None when there is none for the class or
    it was taken on a different version of the kernel's source."""
    ent = COUNTER_SUMMARIES.get(cls)
    if ent is None:
        return None
    path = os.path.join(ROOT, "profiles", ent[0])
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        m = re.match(r"^- (\w+): (\S+)", line.strip())
        if m:
            fields[m.group(1)] = m.group(2)
    src = os.path.join(ROOT, "paper_2409_09471_amd", "csrc", ent[1])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != sha or fields.get("class") != cls:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, gpu_iterations, budget_s):
    """The oracle's TT-sGMRES on the same inputs, timed for a bounded number of
    iterations (k = 1, 2, 4, ... while the next run fits in the budget); the
    rest of the GPU's iteration count is extrapolated at the incremental rate of
    the last two samples.  Early iterations have lower ranks, so this estimate
    is a lower bound on the oracle's full solve."""
    from oracle import operators as oops
    from oracle import solvers as osol
    A = oops.tt_kron_sum(w.terms)
    times = []
    spent = 0.0
    k = 1
    while True:
        s = time.perf_counter()
        osol.tt_sgmres(A, w.b, w.S, w.X, w.Y, maxit=k, tol=w.tol, q=w.q, round_tol=w.round_tol, maxrank=w.cap,
                       stop_safety=w.stop_safety, fixed_iterations=k)
        el = time.perf_counter() - s
        spent += el
        times.append((k, el))
        if k >= gpu_iterations or spent + 2.5 * el > budget_s:
            break
        k = min(2 * k, gpu_iterations)
    kmax, tmax = times[-1]
    k_prev, t_prev = times[-2] if len(times) > 1 else (0, 0.0)
    per_it = (tmax - t_prev) / max(kmax - k_prev, 1)
    est = tmax + max(gpu_iterations - kmax, 0) * per_it
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return dict(value=est, unit="s", cores=cores, kind="oracle",
                sample=f"oracle TT-sGMRES (numpy float64, {cores} threads) on the same inputs: runs of "
                       f"{', '.join(str(a) for a, _ in times)} iterations ({spent:.1f} s in total); the last "
                       f"run took {tmax:.1f} s for {kmax} iterations, the remaining "
                       f"{max(gpu_iterations - kmax, 0)} of the GPU's {gpu_iterations} iterations are "
                       f"extrapolated at {per_it:.2f} s/iteration",
                extrapolated=gpu_iterations > kmax)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is a "
              f"design note, not a measured path.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2409_09471_amd import ttsg
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("# calibration copy: 268435456 bytes read, 268435456 bytes written", file=sys.stderr, flush=True)
        del src, dst
    w, t = build_inputs("cuda:0")
    prec = ttsg.PREC_MIXED if args.precision == "mixed" else ttsg.PREC_F64
    # contraction tiles: the committed table from the tile tuner, else tune
    # during the first warmup solve
    tune = False
    if not args.no_autotune:
        if os.path.exists(TILE_TABLE):
            ttsg.autotune_load(TILE_TABLE)
        else:
            tune = True
    el, results, stats = timed_solves(w, t, prec, args.steps, max(args.warmup, 1 if tune else 0), tune=tune)
    per = el / args.steps
    last = results[-1]
    converged = all(r.status == ttsg.OK for r in results)
    out = {
        "metric": METRIC, "value": per, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": per * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == ttsg.PREC_MIXED else "f64", "data": "synthetic",
        "config": {"workload": "convection-diffusion d=10 n=64, rank-3 TT operator, rank-4 rhs, ranks<=64, "
                               "s=1000, q=1, tol 1e-6 (true residual)",
                   "d": w.d, "n": w.ns[0], "op_rank": w.op_rank, "rhs_rank": 4, "maxrank": w.cap, "s": w.s,
                   "rho": max(w.rho), "rx": max(w.rx), "q": w.q, "round_tol": w.round_tol, "tol": w.tol},
        "converged": converged, "iterations": last.iterations, "true_residual": last.true_residual,
        "sketched_residual": last.sketched_residual, "max_rank": last.max_rank,
    }
    # per-class kernel figures of one measured solve (device wall-clock per launch)
    kern = {}
    for k, v in stats.items():
        kern[k] = dict(launches=v["launches"], seconds=round(v["seconds"], 6),
                       tflops=round(v["flops"] / max(v["seconds"], 1e-12) / 1e12, 4),
                       gbs=round(v["bytes"] / max(v["seconds"], 1e-12) / 1e9, 2))
    out["kernels"] = kern
    # roofline of the dominant kernel class (summed device time of the measured
    # solve); when that is not a contraction, the leading contraction class is
    # reported beside it
    def roofline(cls):
        v = stats[cls]
        ach = v["flops"] / v["launches"] / (v["seconds"] / v["launches"])
        if cls.startswith("contract"):
            dt = cls.split("_")[1]
            name = f"contract_kernel<{ {'f64': 'double', 'f32': 'float', 'bf16': 'bf16'}[dt]}>"
            bound, peak, traffic = "mfma", PEAK[dt], counter_traffic(cls)
        else:
            # single-workgroup FP64 factorizations: vector ALU work
            name = {"svd_jacobi": "k_jacobi_lds", "qr": "k_chol_inv + k_qr_small"}.get(cls, cls)
            bound, peak, traffic = "alu", PEAK_F64_VECTOR, counter_traffic(cls)
        return {"kernel": name, "bound": bound, "achieved": ach / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": traffic, "flop_per_launch": v["flops"] / v["launches"],
                "avg_launch_us": v["seconds"] / v["launches"] * 1e6}
    timed = [k for k in stats if stats[k]["launches"] > 0 and stats[k]["seconds"] > 0 and k != "qr_redo"]
    dom = max(timed, key=lambda k: stats[k]["seconds"], default=None)
    if dom is not None:
        out["roofline"] = roofline(dom)
        top_c = max((k for k in timed if k.startswith("contract")), key=lambda k: stats[k]["seconds"], default=None)
        if top_c is not None and top_c != dom:
            out["roofline_contraction"] = roofline(top_c)
    if prec == ttsg.PREC_MIXED and not args.no_fp64_leg:
        el64, res64, _ = timed_solves(w, t, ttsg.PREC_F64, 1, 1 if tune else 0, measure=False, tune=tune)
        out["fp64_seconds"] = el64
        out["fp64_iterations"] = res64[-1].iterations
        out["fp64_true_residual"] = res64[-1].true_residual
        out["speedup_vs_fp64"] = el64 / per
    out["rounding"] = rounding_gflops(w, t)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, last.iterations, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
