"""Benchmark: ADMM inner iterations per second and time to a 1e-4 primal/dual
residual on the seeded 2000-bus, 3200-line, 500-unit, 24-period workload (one
MI355X, FP64), plain flat-start Newton vs previous-iterate warm start.

A "step" is one inner ADMM iteration over every component and period (UC DP,
generator and line subproblems, relaxed commitments, bus projection, multiplier
and residual updates, inner/outer control).  `value` = steps/s of the captured
iteration graph with the instance resident in HBM.  A second pass of the same
number of iterations launches the kernels one by one with HIP events on the
library's stream; it gives each kernel's mean device time, from which the line
kernel's roofline fraction is computed.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 vector peak of MI355X: 256 CU x 2.4 GHz x 128 flop/clk (64 FMA lanes per CU).
FP64_VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0

# Algorithmic flops of the line kernel, counted from its source (one flop per
# +, -, *, /, sqrt, sin, cos; an FMA counts two; compile-time zero terms dropped):
FLOP_EVAL = 349      # value + gradient + 10-entry Hessian at one point (inactive line limits)
FLOP_TRIAL = 75      # value only at a trial point
FLOP_CG = 80         # one Steihaug-Toint CG iteration on the 4x4 system
FLOP_NEWTON = 80     # per trust-region iteration: projection, predicted reduction, ratio, radius
FLOP_LANE = 70       # per solve: targets from duplicates/multipliers, start, final flows, nu update

# Algorithmic HBM bytes per item, counted from the kernels' loads and stores (8 B per
# double, each state array touched once per item; per-line/per-unit constants omitted):
BYTES_BRANCH = 8 * 36 + 4   # x-bar (8), z, y (16), nu (2) in; x (4), flows (4), nu (2) out; iteration count
BYTES_GEN = 8 * 29          # duplicates (5), z, y (16) in; p, q, six slacks out
BYTES_UBAR = 8 * 40
BYTES_GEN_DUAL = 8 * 66
BYTES_BUS_PER_END = 8 * 28  # per incident line end; plus per unit 24 and per bus 6 doubles


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--config", type=int, default=2, help="synthetic workload id (2 = 2000-bus T=24)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-tolerance runs")
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--max-iters", type=int, default=20000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def cpu_baseline(inst, seconds):
    """The FP64 oracle as it stands, single-threaded, on the same workload; a bounded
    sample of iterations from the cold start."""
    import oracle
    o = oracle.Oracle(inst)
    n, t0 = 0, time.perf_counter()
    while True:
        o.step(1)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= 200:
            break
    return dict(value=n / el, unit="iters/s", cores=1, kind="oracle",
                sample=f"first {n} inner iterations from the cold start of the same workload, {el:.1f} s, one thread")


def time_to_tol(ucac, torch, inst, args):
    """Solve from the cold start to r_p, r_d <= tol with the flat and the previous-iterate
    Newton start; the device records the first iteration under 1e-2, 1e-3 and 1e-4."""
    res = {}
    for label, ws in (("plain", 0), ("prev_iterate", 1)):
        s = ucac.Solver(inst, warm_start=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, iters = s.solve(args.tol, args.max_iters)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rp, rd, zinf, obj = s.residuals()
        ms = s.milestones()
        per_it = el / max(iters, 1)
        res[label] = {"converged": rc == 0, "iters": iters, "seconds": el, "r_p": rp, "r_d": rd, "objective": obj,
                      "first_iter_below": ms,
                      "seconds_to": {k: (v * per_it if v > 0 else None) for k, v in ms.items()}}
        s.close()
    if res["plain"]["converged"] and res["prev_iterate"]["converged"]:
        res["speedup_prev_iterate"] = res["plain"]["seconds"] / res["prev_iterate"]["seconds"]
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the workload is one "
              "instance on one MI355X; see DESIGN.md for how it would shard", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2310_13145_amd import synth, ucac

    inst = synth.config_instance(args.config)
    name = synth.CONFIGS[args.config]["name"] if args.config in synth.CONFIGS else f"cfg{args.config}"
    N, L, G, T = inst["n_bus"], inst["n_line"], inst["n_gen"], inst["T"]

    solver = ucac.Solver(inst)
    solver.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.steps

    # the same timed region with the previous-iterate Newton start (warm start)
    warm = ucac.Solver(inst, warm_start=1)
    warm.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    warm.step(args.steps)
    torch.cuda.synchronize()
    dt_warm = time.perf_counter() - t0
    warm.close()

    # profiled pass: the same iterations kernel by kernel, HIP events on the library stream
    solver.branch_counters(reset=True)
    ktimes = solver.kernel_times(args.steps)
    cnt = solver.branch_counters(reset=True)
    prof_ms_per_step = sum(ktimes.values())
    lanes = T * L
    flops_per_launch = (cnt["evals"] * FLOP_EVAL + cnt["trials"] * FLOP_TRIAL + cnt["cg"] * FLOP_CG +
                        cnt["newton"] * FLOP_NEWTON) / args.steps + lanes * FLOP_LANE
    br_s = ktimes["branch"] * 1e-3
    achieved = flops_per_launch / br_s / 1e12
    n_ends = 2 * L
    bytes_bus = n_ends * T * BYTES_BUS_PER_END + G * T * 8 * 24 + N * T * 8 * 6
    hbm = {
        "gen": {"bytes": G * T * BYTES_GEN, "ms": ktimes["gen"]},
        "ubar": {"bytes": G * T * BYTES_UBAR, "ms": ktimes["ubar"]},
        "bus": {"bytes": bytes_bus, "ms": ktimes["bus"]},
        "gen_dual": {"bytes": G * T * BYTES_GEN_DUAL, "ms": ktimes["gen_dual"]},
        "branch": {"bytes": lanes * BYTES_BRANCH, "ms": ktimes["branch"]},
    }
    for v in hbm.values():
        v["GB_s"] = v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 else None
        v["frac"] = v["GB_s"] / HBM_PEAK_GBS if v["GB_s"] else None

    out = {
        "metric": "ADMM iters/sec and time-to-1e-4 residual, 2000-bus T=24; warm-start vs plain",
        "value": args.steps / dt,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": name, "n_bus": N, "n_line": L, "n_gen": G, "T": T,
                   "branch_solves_per_step": lanes, "newton_start": "flat (plain method)"},
        "roofline": {"bound": "alu", "kernel": "branch (trust-region Newton, one lane per line-period)",
                     "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "flops_per_launch": flops_per_launch, "launch_ms": ktimes["branch"],
                     "newton_iters_per_solve": cnt["newton"] / args.steps / lanes},
        "warm_start_prev_iterate": {"value": args.steps / dt_warm, "ms_per_step": 1e3 * dt_warm / args.steps},
        "kernels_ms": ktimes,
        "profiled_ms_per_step": prof_ms_per_step,
        "hbm": hbm,
    }

    if not args.no_solve:
        out["time_to_tol"] = time_to_tol(ucac, torch, inst, args)
        out["time_to_tol_mesh118_T24"] = time_to_tol(ucac, torch, synth.config_instance(1), args)

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
        out["cpu_baseline"]["gpu_over_cpu"] = out["value"] / out["cpu_baseline"]["value"]

    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
