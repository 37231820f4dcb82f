#!/usr/bin/env python3
"""RT-TDA propagation throughput on one MI355X: sigma GFLOP/s, % of the MFMA roofline and fs/hour.

A step is one classic RK4 step (4 sigma evaluations with the Coulomb GEMV pair, the exchange
contraction, the field/trace product and the FP64 epilogue) for all right-hand sides of the
workload, inputs resident in HBM.  Default workload: o=60, v=400, N_Q=1500, x/y/z delta kicks as
3 right-hand sides, dt = 0.05 au, FP32 factors (synthetic, seeded).

    python bench.py [--steps K] [--warmup W] [--workload cfg2|cfg1|cfg3|cfg4]
                    [--precision fp32|mixed] [--integrator rk4|sso] [--graph-compare]

cfg1: o10 v40 N_Q120, z kick; cfg3: o240 v1800 N_Q5000, x/y/z kicks, split BF16; cfg4: o40
v300 N_Q1000, 64 Gaussian-pulse carriers.  With --integrator sso a step is one split-operator
step (2 real sigma).  The default run adds the FP64 oracle timed on the host cores on a bounded
sample (cpu_baseline) and the batched-mixed against plain-FP32-single comparison.

Prints one JSON line.  The timed region brackets exactly K steps with device synchronisation;
per-kernel-class durations come from HIP events recorded by the library on its stream inside
that region.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2601_16949_amd import inputs as I  # noqa: E402

AU_FS = 0.02418884326585747

# HBM bytes per exchange launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (KiB per dispatch,
# scaled by the counters' readings for a plain 1 GiB copy: factors 2.0 and 1.0), keyed by
# (variant, workload, splits); valid only while the kernel's source file hashes to `src`.
TRAFFIC = {
    # HBM bytes per exchange launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per dispatch),
    # scaled by what the same counters read for a plain device copy (2.0 and 1.0), keyed by
    # (variant, workload, Q splits, real slices per launch: 2 per RHS for RK4, 1 for the split
    # operator) and tied to the kernel source they were taken on
    ("f32dlq_o64_ws1_wc2", "o60_v400_nq1500_kick_xyz", 357, 6):
        {"file": "exchange_f32_dl.hip", "src": "f238a7e6c53d48d8",
         "fetch_bytes": 666078.92 * 1024 * 2.0, "write_bytes": 210662.2 * 1024 * 1.0},
    ("f32dlp_p40_ws1_wc2", "o40_v300_nq1000_gauss_cos_scan64", 40, 128):
        {"file": "exchange_f32_dl.hip", "src": "f238a7e6c53d48d8",
         "fetch_bytes": 6595093.2 * 1024 * 2.0, "write_bytes": 257260.6 * 1024 * 1.0},
    ("f32dlp_o64_ws1_wc1_s1", "o60_v400_nq1500_kick_xyz", 466, 3):
        {"file": "exchange_f32_dl.hip", "src": "f238a7e6c53d48d8",
         "fetch_bytes": 507626.11 * 1024 * 2.0, "write_bytes": 139579.3 * 1024 * 1.0},
    ("bf16x2k64_o64_wc2_w8", "o60_v400_nq1500_kick_xyz", 220, 6):
        {"file": "exchange_bf16_dl.hip", "src": "f90b2171f434b93d",
         "fetch_bytes": 264290.89 * 1024 * 2.0, "write_bytes": 125895.47 * 1024 * 1.0},
    # the GEMM path: one exchange stage is 25 chunks of 200 Q, each a k_xgemm_w + k_boo_w pair
    ("bf16x2gemm_a256x256w8_b256x128w8", "o240_v1800_nq5000_kick_xyz_mixed", 8, 6):
        {"file": "exchange_bf16_gemm.hip", "src": "7dc7d8bb3f4ee411",
         "fetch_bytes": 25 * (8459398.4 + 1347847.4) * 1024 * 2.0,
         "write_bytes": 25 * (2257817.4 + 96479.69) * 1024 * 1.0},
}
PEAK = {"fp32": 157.3, "mixed": 2516.6}  # dense MFMA TFLOP/s: FP32, BF16
HBM_PEAK_GBS = 8000.0


def flops_per_sigma(o, v, nq):
    """Algorithmic flops of one complex sigma for one RHS: (Coulomb, exchange)."""
    ov = o * v
    return 8.0 * nq * ov, 4.0 * nq * ov * (o + v)


def make_workload(name: str):
    if name == "cfg1":
        return I.workload(1)
    if name == "cfg2":
        return I.workload(2)
    if name == "cfg3":
        return I.workload(3)
    if name == "cfg4":
        wl = I.workload(4)
        # carriers span 0.5x..1.2x the lowest excitation; the bench uses a fixed nominal
        # lowest excitation (the shape's orbital-gap scale) since no eigen-solve runs here
        wl.pulses = I.gauss_cos_scan(0.39, 0.05)
        return wl
    raise SystemExit(f"unknown workload {name}")


def traffic_for(variant: str, workload: str, splits: int, slices: int):
    import hashlib

    e = TRAFFIC.get((variant, workload, splits, slices))
    if not e:
        return None
    src = os.path.join(ROOT, "paper_2601_16949_amd", "csrc", e["file"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != e["src"]:
        return None  # kernel changed since the counters were taken
    return e["fetch_bytes"] + e["write_bytes"]


def oracle_run(wl, prob, pulses, budget_s: float, max_steps: int = 1000):
    """The FP64 oracle's direct route from the ground state (after the kicks) for as many RK4 steps
    of all RHS as fit in budget_s: (trace [steps+1, R], steps, seconds, BLAS threads)."""
    from oracle import rttda64 as O

    try:
        from threadpoolctl import threadpool_info

        cores = max((d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"), default=1)
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    op = O.Operator.from_problem(prob)
    states, trace = [], [[]]
    t0 = time.perf_counter()
    for p in pulses:
        blocks = O.dipole_blocks(op, p.direction)
        c0, C = O.apply_kick(op, blocks, p, 1.0 + 0j, np.zeros((prob.o, prob.v), complex))
        states.append([blocks, c0, C])
        trace[0].append(O.dipole_expectation(blocks, c0, C))
    steps = 0
    while True:
        row = []
        for r, p in enumerate(pulses):
            blocks, c0, C = states[r]
            states[r][1], states[r][2] = O.rk4_step(op, blocks, p, wl.dt, steps, c0, C)
            row.append(O.dipole_expectation(blocks, states[r][1], states[r][2]))
        trace.append(row)
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s or steps >= max_steps:
            break
    return np.array(trace), steps, el, int(cores)


def cpu_baseline(wl, prob, budget_s: float):
    """The FP64 oracle (direct route) timed on this host's cores on a bounded sample; its trace is
    kept for the error of the GPU result against it."""
    R = len(wl.pulses)
    tr, steps, el, cores = oracle_run(wl, prob, wl.pulses, budget_s)
    fc, fx = flops_per_sigma(prob.o, prob.v, prob.nq)
    gflops = steps * R * 4 * (fc + fx) / el / 1e9
    fs_h = steps * wl.dt * AU_FS * R / (el / 3600.0)
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        nproc = os.cpu_count() or 1
    return {"value": round(gflops, 3), "unit": "sigma GFLOP/s (FP64)", "cores": int(cores), "kind": "oracle",
            "nproc": nproc,
            "sample": f"{steps} RK4 steps x {R} RHS of {wl.name} ({el:.1f} s, NumPy FP64 over {cores} BLAS threads)",
            "fs_per_hour": round(fs_h, 4)}, tr


def trace_error(ctx, wl, pulses, ref):
    """max |mu_gpu - mu_oracle| / max |mu_oracle| over the oracle's steps, the GPU run from a fresh
    ground state on the same context (the launch configuration of the timed run)."""
    import torch
    from paper_2601_16949_amd import rttda

    n = ref.shape[0] - 1
    c0, c = rttda.ground_state(len(pulses), ctx.o, ctx.v)
    got = ctx.propagate(pulses, wl.dt, n, c0, c)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def short_leg(wl, precision: str, pulses, steps: int, warmup: int = 5, oracle_s: float = 0.0):
    """Aggregate fs/hour and sigma GFLOP/s of a short timed run (comparison legs); with oracle_s > 0
    also its trace error against the FP64 oracle over the oracle steps that fit in oracle_s."""
    import torch
    from paper_2601_16949_amd import rttda

    shape = I.Shape(wl.shape.o, wl.shape.v, wl.shape.nq, wl.shape.b_scale,
                    storage="f32" if precision == "fp32" else "bf16")
    prob = I.make_problem(shape, wl.seed)
    R = len(pulses)
    ctx = rttda.Context(rttda.DeviceProblem(prob, precision), max_rhs=R)
    tuned = ctx.use_tuned(R)
    c0, c = rttda.ground_state(R, prob.o, prob.v)
    ctx.propagate(pulses, wl.dt, warmup, c0, c, want_trace=False)
    torch.cuda.synchronize()
    ctx.set_profiling(True)  # per-kernel-class HIP events inside the timed region, as in the main run
    t0 = time.perf_counter()
    ctx.propagate(pulses, wl.dt, steps, c0, c, step0=warmup)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = ctx.get_profile()
    ctx.set_profiling(False)
    fc, fx = flops_per_sigma(prob.o, prob.v, prob.nq)
    tun = ctx.get_tuning()
    ex_us = 1e3 * prof["exchange"]["ms"] / max(prof["exchange"]["launches"], 1)
    peak = PEAK[precision]
    out = {"precision": precision, "nrhs": R, "steps": steps, "ms_per_step": round(1e3 * el / steps, 4),
           "fs_per_hour": round(steps * wl.dt * AU_FS * R / (el / 3600.0), 3),
           "sigma_gflops": round(steps * 4 * R * (fc + fx) / el / 1e9, 2),
           "exchange_variant": ctx.variant_name(tun["exchange_variant"]), "autotuned": tuned,
           # the exchange launch of this leg: algorithmic flops over its average event-timed duration
           "roofline": {"bound": "mfma", "kernel": "exchange", "avg_launch_us": round(ex_us, 2),
                        "achieved": round(R * fx / (ex_us * 1e-6) / 1e12, 3), "peak": peak, "unit": "TFLOP/s",
                        "frac": round(R * fx / (ex_us * 1e-6) / 1e12 / peak, 4)}}
    if oracle_s > 0:
        ref, k, _, _ = oracle_run(wl, prob, pulses, oracle_s)
        out["error_vs_oracle"] = {"rel_trace_err": trace_error(ctx, wl, pulses, ref), "steps": k,
                                  "bar": 1e-5 if precision == "fp32" else 1e-4}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the mixed vs FP32 single-solve legs")
    ap.add_argument("--graph-compare", action="store_true",
                    help="also time the same number of steps replayed from the captured HIP graph (no events)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--splits", type=int, default=0)
    ap.add_argument("--overlap", type=int, default=0, choices=(0, 1, 2),
                    help="1: the Coulomb pair on a second stream beside the exchange, 2: in order on one "
                         "stream (times each kernel alone), 0: the library's choice")
    ap.add_argument("--precision", default=None, help="override the workload's precision (fp32 | mixed)")
    ap.add_argument("--integrator", default="rk4", choices=("rk4", "sso"),
                    help="rk4 (4 complex sigma per step) or the split operator sso (2 real sigma per step)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; --gpus must be 1 (multi-GPU sharding is a design "
                                   "note only)"}))
        sys.exit(2)

    import torch
    from paper_2601_16949_amd import rttda

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4, "dispatches": 5}))
        return
    rttda.load()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    wl = make_workload(args.workload)
    if args.precision and args.precision != wl.precision:
        wl.precision = args.precision
        wl.shape = I.Shape(wl.shape.o, wl.shape.v, wl.shape.nq, wl.shape.b_scale,
                           storage="f32" if args.precision == "fp32" else "bf16")
    if args.workload == "cfg3":
        # 37 GB of factors: the per-Q host streams, uploaded a range of Q at a time (the values the
        # oracle's cached reference read)
        print("# drawing the o240 factors on the host", file=sys.stderr, flush=True)
        t = I.upload_factors_streamed(wl.shape, wl.seed, threads=16)
        dev = rttda.DeviceProblem.from_tensors(wl.shape, t, wl.precision)
        prob = None
        args.no_cpu_baseline = True
    else:
        prob = I.make_problem(wl.shape, wl.seed)
        dev = rttda.DeviceProblem(prob, wl.precision)
    R = len(wl.pulses)
    ctx = rttda.Context(dev, max_rhs=R)
    tuned = False
    if args.variant or args.splits:
        ctx.set_tuning(exchange_variant=args.variant, exchange_splits=args.splits)
    else:
        tuned = ctx.use_tuned(R, args.integrator)
    if args.overlap:
        ctx.set_tuning(overlap=args.overlap)
    # time-step guard: Lanczos bound on rho(A) against the integrator's stability limit
    rho, rho_bound = ctx.spectral_radius(30)
    limit = 2.5 if args.integrator == "rk4" else 2.0
    if rho_bound * wl.dt > limit:
        raise SystemExit(f"refused: rho(A) dt <= {rho_bound * wl.dt:.3f} exceeds the stability limit {limit}")
    tun = ctx.get_tuning()
    c0, c = rttda.ground_state(R, dev.o, dev.v)
    ctx.propagate(wl.pulses, wl.dt, args.warmup, c0, c, integrator=args.integrator)
    torch.cuda.synchronize()
    print(f"# warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    ctx.set_profiling(True)
    trace = torch.empty((args.steps + 1, R), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.propagate(wl.pulses, wl.dt, args.steps, c0, c, step0=args.warmup, trace=trace, integrator=args.integrator)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.get_profile()
    ctx.set_profiling(False)
    bad = ctx.guard()
    elapsed = t1 - t0
    print(f"# timed {args.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    o, v, nq = dev.o, dev.v, dev.nq
    fc, fx = flops_per_sigma(o, v, nq)
    # RK4: 4 complex sigma per step; split operator: 2 real sigma (= 1 complex) per step
    sigmas_per_step = 4 if args.integrator == "rk4" else 1
    sigma_flops = args.steps * sigmas_per_step * R * (fc + fx)
    value = sigma_flops / elapsed / 1e9
    fs_h = args.steps * wl.dt * AU_FS * R / (elapsed / 3600.0)
    ex = prof["exchange"]
    ex_avg_ms = ex["ms"] / max(ex["launches"], 1)
    # one launch covers all slices of one stage: 2R (complex RK4 stage) or R (real half step);
    # on the small-problem path that launch also carries the Coulomb partial sums
    small = tun.get("small_path") == 1
    ex_flops = R * (fx + (fc if small else 0.0))
    if args.integrator != "rk4":
        ex_flops /= 2
    achieved = ex_flops / (ex_avg_ms * 1e-3) / 1e12
    peak = PEAK[wl.precision]
    breakdown = {k: {"launches": d["launches"], "avg_us": round(1e3 * d["ms"] / max(d["launches"], 1), 2),
                     "share": round(d["ms"] / (elapsed * 1e3), 4)} for k, d in prof.items()}
    traffic = traffic_for(ctx.variant_name(tun["exchange_variant"]), wl.name, tun["exchange_splits"],
                          2 * R if args.integrator == "rk4" else R)
    out = {
        "metric": "sigma GFLOP/s (% MFMA peak) + fs/hour",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if wl.precision == "fp32" else "bf16x2+f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "o": o, "v": v, "n_aux": nq, "nrhs": R, "dt": wl.dt,
                   "integrator": args.integrator,
                   "precision": wl.precision, "exchange_variant": ctx.variant_name(tun["exchange_variant"]),
                   "exchange_splits": tun["exchange_splits"], "coulomb_splits": tun["coulomb_splits"],
                   "autotuned": tuned, "small_path": bool(tun.get("small_path") == 1),
                   "parallelism": "single GPU, RHS batched"},
        "fs_per_hour": round(fs_h, 3),
        "mfma_frac_step": round(value / 1e3 / peak, 4),
        "roofline": {"bound": "mfma", "kernel": "coulomb+exchange partial sums" if small else "exchange",
                     "achieved": round(achieved, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
                     # counter bytes over the same launch time, against the 8 TB/s of HBM
                     "traffic_gbs": round(traffic / (ex_avg_ms * 1e-3) / 1e9, 1) if traffic else None,
                     "avg_launch_us": round(ex_avg_ms * 1e3, 2), "algorithmic_flops_per_launch": ex_flops},
        "kernels": breakdown,
        "guard_bad_step": bad,
        "stability": {"rho_bound": round(rho_bound, 6), "rho_dt": round(rho_bound * wl.dt, 4), "limit": limit,
                      "lanczos_steps": 30},
        "trace_finite": bool(torch.isfinite(trace).all().item()),
    }
    if args.graph_compare or args.workload in ("cfg1", "cfg2"):
        # the same K steps with the step captured once in a HIP graph and replayed, against
        # direct launches (no profiling events in either; at the launch-bound o10 v40 shape the
        # per-kernel events of the timed run above cost as much as the kernels)
        times = {}
        for mode, tag in ((1, "graph"), (2, "direct")):
            ctx.set_tuning(use_graph=mode)
            ctx.propagate(wl.pulses, wl.dt, 16, c0, c, step0=args.warmup + args.steps, want_trace=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.propagate(wl.pulses, wl.dt, args.steps, c0, c, step0=args.warmup + args.steps + 16, want_trace=False)
            torch.cuda.synchronize()
            times[tag] = round(1e3 * (time.perf_counter() - t0) / args.steps, 4)
        ctx.set_tuning(use_graph=1)
        out["ms_per_step_graph_vs_direct"] = times
    if not args.no_compare and args.workload == "cfg2":
        # batched mixed precision (3 RHS, BF16 factors, split exchange) against the plain FP32
        # single solve (1 RHS) on the same shape; the accuracy of the mixed path against the FP64
        # oracle (trace <= 1e-4) is checked by the parity tests
        del ctx, dev
        ctx = None
        torch.cuda.empty_cache()
        single = short_leg(wl, "fp32", wl.pulses[:1], 100)
        mixed = short_leg(wl, "mixed", wl.pulses, 200, oracle_s=0.0 if args.no_cpu_baseline else 8.0)
        out["mixed_vs_fp32_single"] = {"fp32_single": single, "mixed_batched": mixed,
                                       "ratio_fs_per_hour": round(mixed["fs_per_hour"] / single["fs_per_hour"], 3)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"], ref = cpu_baseline(wl, prob, args.cpu_budget)
        if ctx is not None:
            err = trace_error(ctx, wl, wl.pulses, ref)
        else:  # the comparison legs freed the timed context: a fresh one in the same configuration
            ctx2 = rttda.Context(rttda.DeviceProblem(prob, wl.precision), max_rhs=R)
            if args.variant or args.splits:
                ctx2.set_tuning(exchange_variant=args.variant, exchange_splits=args.splits)
            else:
                ctx2.use_tuned(R, args.integrator)
            err = trace_error(ctx2, wl, wl.pulses, ref)
        out["error_vs_oracle"] = {"rel_trace_err": err, "steps": int(ref.shape[0] - 1),
                                  "bar": 1e-5 if wl.precision == "fp32" else 1e-4}
    elif args.workload == "cfg3" and ctx is not None:
        # the oracle's direct route costs minutes per step here: compare with its cached first steps
        gold = os.path.join(ROOT, "tests", "golden", "cfg3_trace_z.npz")
        if os.path.exists(gold):
            ref = np.load(gold, allow_pickle=False)["trace"]
            c0r, cr = rttda.ground_state(R, dev.o, dev.v)
            got = ctx.propagate(wl.pulses, wl.dt, ref.size - 1, c0r, cr).cpu().numpy()[:, 2]
            out["error_vs_oracle"] = {"rel_trace_err": float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))),
                                      "steps": int(ref.size - 1), "rhs": "z", "bar": 1e-4,
                                      "reference": "cached oracle trace (tests/golden/cfg3_trace_z.npz)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
