"""Benchmark: ADMM inner iterations per second and time to a 1e-4 primal/dual
residual on the seeded 2000-bus, 3200-line, 500-unit, 24-period workload (one
MI355X, FP64), plain flat-start Newton vs previous-iterate warm start.

A "step" is one inner ADMM iteration over every component and period (UC DP,
generator and line subproblems, relaxed commitments, bus projection, multiplier
and residual updates, inner/outer control).  `value` = steps/s of the captured
iteration graph with the instance resident in HBM.  A second pass, from the
iterate after 200 iterations and after one untimed launch of every kernel, runs
100 iterations with the kernels launched one by one and HIP events on the
library's stream; it gives each kernel's mean device time.  The line kernel of
that pass also carries its own start/stop events (the dispatch's begin and end
timestamps, what a kernel trace reports); its roofline fraction uses that
duration.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 vector peak of MI355X: 256 CU x 2.4 GHz x 128 flop/clk (64 FMA lanes per CU).
FP64_VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0

# Algorithmic flops of the line kernel, counted from its source (one flop per
# +, -, *, /, sqrt, sin, cos; an FMA counts two; compile-time zero terms dropped):
FLOP_EVAL = 349      # value + gradient + 10-entry Hessian at one point (inactive line limits)
FLOP_TRIAL = 75      # value only at a trial point (what a rejected trial needs)
FLOP_CG = 80         # one Steihaug-Toint CG iteration on the 4x4 system
FLOP_DIRECT = 83     # one direct Newton step in its usual reduced form: the angle sum decouples, so a
                     # 3x3 LDL^T (free-set assembly, 3 refined reciprocals, elimination, triangular
                     # solves) plus one product for the sum, back to the angles, length test (the 4x4
                     # form, 110, runs only with an angle on its +-2 pi bound and is counted as 83)
FLOP_NEWTON = 80     # per trust-region iteration: projection, predicted reduction, ratio, radius
FLOP_SEARCH = 64     # one projected search: four break points, the new trial point and step, and the
                     # model value at it (Hessian product, two dot products)
FLOP_LANE = 94       # per solve: targets from duplicates/multipliers, start, final flows, nu update,
                     # the bus QP's per-end sums

# The profiled (kernel-by-kernel) pass starts from the iterate after PROF_FROM iterations and
# times PROF_ITERS iterations, whatever --steps and --warmup are.
PROF_FROM = 200
# Residual balancing of the time_to_tol section: a decision after every ADAPT_EVERY-th
# iteration, with the library's default factors (mu = 3, tau = 1.5)
ADAPT_EVERY = 20
PROF_ITERS = 100

# Algorithmic HBM bytes per item, counted from the kernels' loads and stores (8 B per
# double, each state array touched once per item; per-line/per-unit constants omitted):
BYTES_BRANCH = 8 * 52 + 12  # x-bar (8), z, y (16), nu (2) in; x (4), flows (4), nu (2) out; iteration count;
                            # then the bus QP's per-end sums: z, y of 8 rows again (16 in, 8 out) and 2 positions
BYTES_GEN = 8 * 29          # duplicates (5), z, y (16) in; p, q, six slacks out
BYTES_DP = 8 * 12           # relaxed commitments (3), z, y of U1..U3 (6) in; u_on, u_su, u_sd out
BYTES_UBAR = 8 * 40
BYTES_UNITS = BYTES_GEN + BYTES_DP + BYTES_UBAR  # the unit kernel per (unit, t)
BYTES_GEN_DUAL = 8 * 66
BYTES_BUS_END = 8 * 4       # bus QP: the 4 sums of each incident line end
BYTES_BUS_BUS = 8 * 8       # bus QP per (bus, t): wbar, thetabar in/out, 2 multipliers out, loads
BYTES_BUS_GEN = 8 * 30      # bus QP per (unit, t): consensus and next-period ramp rows, duplicates out
BYTES_BUS_POST = 8 * 64     # per (line, t), both ends: flows, targets, bus results, old duplicates, y/lambda of
                            # 4 rows in; duplicates and z/y of 4 rows out


# HBM bytes per dispatch of the plain-start line kernel, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch averaged over the dispatches of the
# mesh2000_T24 bench command), each scaled by the ratio of true to counted bytes of a
# plain copy kernel of known size.  They describe the kernel source they were taken
# on (hash below) and are reported as null once that source has changed.
BRANCH_COUNTERS = {"source_sha256": "ac60767bd3d45dabcba876e849f58e61594b6cff320b9e816cd68ca240190983",
                   "fetch_kib": 8049.0, "write_kib": 11196.4, "fetch_scale": 2.0, "write_scale": 1.0}
# the line kernel's translation unit and every header it includes
BRANCH_SOURCES = ('k_branch.hip', 'ucac_mlp.hpp', 'ucac_dev.hpp', 'ucac_launch.hpp', 'ucac_units.hpp', 'ucac_ctl.hpp',
                  'ucac_pwl.hpp', 'ucac_rows.hpp')


def branch_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in BRANCH_SOURCES:
        with open(os.path.join(ROOT, "paper_2310_13145_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def branch_traffic():
    c = BRANCH_COUNTERS
    if not c or c["source_sha256"] != branch_source_hash():
        return None
    return 1024.0 * (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"])


def line_roofline(solver, inst, from_iter):
    """The line kernel's roofline from the solver's current iterate: one untimed
    kernel-by-kernel iteration (every kernel's first launch in the process), then
    PROF_ITERS timed ones from the same iterate; algorithmic flops from the device work
    counters over the dispatch-timestamp mean.  Returns it and the kernel means."""
    state = solver.get_state()
    solver.kernel_times(1)
    solver.set_state(state)
    solver.branch_counters(reset=True)
    ktimes = solver.kernel_times(PROF_ITERS)
    cnt = solver.branch_counters(reset=True)
    dispatch = {k: ktimes.pop(f"{k}_dispatch") for k in list(ktimes) if not k.endswith("_dispatch")}
    branch_dispatch_ms = dispatch["branch"]
    lanes = inst["T"] * inst["n_line"]
    # the kernel evaluates value, gradient and Hessian at the start and at every trial
    # point; the method needs the full evaluation at the start and at accepted points and
    # only the value at rejected ones, which is what is counted
    full = cnt["evals"] - cnt["rejected"]
    flops_per_launch = (full * FLOP_EVAL + cnt["rejected"] * FLOP_TRIAL + cnt["cg"] * FLOP_CG +
                        cnt["direct"] * FLOP_DIRECT + cnt["newton"] * FLOP_NEWTON +
                        cnt["searches"] * FLOP_SEARCH) / PROF_ITERS + lanes * FLOP_LANE
    achieved = flops_per_launch / (branch_dispatch_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "kernel": "branch (trust-region Newton, one lane per line-period)",
            "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
            "flops_per_launch": flops_per_launch, "launch_ms": branch_dispatch_ms,
            "launch_ms_between_events": ktimes["branch"], "line_solves_per_launch": lanes,
            "newton_iters_per_solve": cnt["newton"] / PROF_ITERS / lanes,
            "projected_searches_per_launch": cnt["searches"] / PROF_ITERS,
            "profiled_iterations": f"{PROF_ITERS} kernel-by-kernel iterations from the iterate after "
                                   f"{from_iter}, after one untimed iteration"}
    return roof, ktimes, dispatch


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
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start evaluation")
    ap.add_argument("--train-instances", type=int, default=2)
    ap.add_argument("--log-iters", type=int, default=300)
    ap.add_argument("--log-stride", type=int, default=10)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--learned-steps", type=int, default=200)
    ap.add_argument("--learned-max-iters", type=int, default=4000)
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batch")
    ap.add_argument("--no-dp", action="store_true", help="skip the standalone DP benchmark")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--no-large", action="store_true",
                    help="skip the line-kernel roofline on the 10,000-bus T = 48 workload")
    ap.add_argument("--hbm-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB five times (reads and writes exactly 1 GiB per "
                         "dispatch), the known-size kernel the HBM byte counters are scaled by")
    return ap.parse_args()


def hbm_calibration(nbytes=1 << 30, reps=5):
    """A multiply-by-one over 1 GiB of FP32: each dispatch reads and writes exactly nbytes.
    Profiled with --pmc FETCH_SIZE (then WRITE_SIZE), it gives the ratio of true to counted
    bytes that the line kernel's counters are scaled by."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    return {"read_bytes_per_dispatch": 4 * n, "write_bytes_per_dispatch": 4 * n, "dispatches": reps}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(inst, seconds, state0=None):
    """The FP64 oracle as it stands on the host: its parallel loops on every thread
    OpenMP gives it (the host's share of cores) and on one thread, each for about
    `seconds` of inner iterations of the same workload from the iterate the GPU's
    timed region starts from (cold start if none)."""
    import oracle
    legs = {}
    for label, n_thr in (("all_cores", 0), ("one_core", 1)):
        oracle.set_threads(n_thr)
        threads = oracle.max_threads()
        o = oracle.Oracle(inst)
        if state0 is not None:
            o.set_state(state0)
        n, t0 = 0, time.perf_counter()
        while True:
            o.step(1)
            n += 1
            el = time.perf_counter() - t0
            if el >= seconds or n >= 400:
                break
        legs[label] = {"value": n / el, "threads": threads, "iters": n, "seconds": el}
        del o
    oracle.set_threads(0)
    a = legs["all_cores"]
    res = dict(value=a["value"], unit="iters/s", cores=a["threads"], kind="oracle",
               sample=f"{a['iters']} inner iterations of the same workload from the iterate the timed region starts "
                      f"from, {a['seconds']:.1f} s on {a['threads']} threads (OpenMP parallel for over each block's "
                      f"items); the same on one thread: {legs['one_core']['value']:.2f} iters/s",
               one_core=legs["one_core"], nproc=os.cpu_count(),
               affinity=len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
               cpu_model=_cpu_model())
    # the oracle's DP alone on the tables of the standalone DP benchmark (200 units per shape)
    dp = {}
    for G, T in DP_SHAPES:
        tab, (tu, td, u0, lon, loff) = _dp_case(G, T, 7 + G + T)
        k = min(G, 200)
        t0 = time.perf_counter()
        for g in range(k):
            oracle.dp(tab[g], u0[g], lon[g], loff[g], tu[g], td[g])
        dp[f"G{G}_T{T}"] = {"dp_per_s": k / (time.perf_counter() - t0), "sample": f"{k} units, one thread"}
    res["dp"] = dp
    return res


def time_to_tol(ucac, torch, inst, args):
    """Solve from the cold start to r_p, r_d <= tol with the flat and the previous-iterate
    Newton start, each with fixed penalties and with residual balancing of the penalty
    classes (a decision after every 20th iteration); the device records the first
    iteration under 1e-2, 1e-3 and 1e-4."""
    res = {}
    for label, ws, adapt in (("plain", 0, 0), ("prev_iterate", 1, 0), ("plain_balanced", 0, ADAPT_EVERY),
                             ("prev_iterate_balanced", 1, ADAPT_EVERY)):
        s = ucac.Solver(inst, warm_start=ws, adapt_every=adapt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, iters = s.solve(args.tol, args.max_iters)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rp, rd, zinf, obj = s.residuals()
        ms = s.milestones()
        per_it = el / max(iters, 1)
        if adapt:
            S = ucac.split_state(s.get_state(), inst["n_bus"], inst["n_line"], inst["n_gen"], inst["T"])
            pen = {k: S[k] for k in ("rho_pq", "rho_va", "rho_cpl", "rho_uc")}
        else:
            pen = None
        res[label] = {"converged": rc == 0, "iters": iters, "seconds": el, "r_p": rp, "r_d": rd, "objective": obj,
                      "final_penalties": pen,
                      "first_iter_below": ms,
                      "seconds_to": {k: (v * per_it if v > 0 else None) for k, v in ms.items()}}
        s.close()
    # the UC warm start of the paper's experiments: the multiperiod ACOPF first (to 1e-3),
    # commitments from its generation levels, then the plain method from them; the
    # seconds count both solves
    s = ucac.Solver(inst)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc0, it0 = s.uc_warmstart(1e-3, args.max_iters)
    t_relax = time.perf_counter() - t0
    S = ucac.split_state(s.get_state(), inst["n_bus"], inst["n_line"], inst["n_gen"], inst["T"])
    committed = float(S["uon"].sum()) / max(1, S["uon"].size)
    rc, iters = s.solve(args.tol, args.max_iters)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rp, rd, zinf, obj = s.residuals()
    res["uc_warmstart"] = {"converged": rc == 0, "relaxed_iters": it0, "relaxed_converged": rc0 == 0,
                           "relaxed_seconds": t_relax, "committed_fraction": committed, "iters": iters,
                           "seconds": el, "r_p": rp, "r_d": rd, "objective": obj,
                           "first_iter_below": s.milestones()}
    s.close()
    for label in ("prev_iterate", "plain_balanced", "prev_iterate_balanced", "uc_warmstart"):
        if res["plain"]["converged"] and res[label]["converged"]:
            res[f"speedup_{label}"] = res["plain"]["seconds"] / res[label]["seconds"]
    return res


def _timed_steps(solver, torch, warmup, steps):
    solver.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(steps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def learned_start(ucac, synth, torch, args):
    """Learned Newton start: pairs logged by the method on 2000-bus T=24 instances of
    other seeds, the network trained on the GPU, then plain (flat start) against
    learned start on the 2000-bus and the 10000-bus T=48 workloads: iteration rate,
    Newton work per solve, and time to the residual milestones from the cold start."""
    out = {}
    t0 = time.perf_counter()
    X, Y = [], []
    for k in range(args.train_instances):
        s = ucac.Solver(synth.training_instance(2, k))
        f, t = s.log_pairs(args.log_iters, stride=args.log_stride)
        X.append(f), Y.append(t)
        s.close()
    X, Y = np.vstack(X), np.vstack(Y)
    t_log = time.perf_counter() - t0
    net = ucac.WarmStartNet(seed=0)
    _, loss0 = net.grad(X[:65536], Y[:65536])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = net.train(X, Y, epochs=args.epochs, batch=4096, lr=2e-3, seed=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    w = net.get_weights()
    net.close()
    out["training"] = {"pairs": int(X.shape[0]), "instances": args.train_instances,
                       "source": f"2000-bus T=24 instances of other seeds, {args.log_iters} iterations, every "
                                 f"{args.log_stride}th solve", "log_seconds": t_log, "train_seconds": t_train,
                       "epochs": args.epochs, "batch": 4096, "mse_before": loss0, "mse_last_epoch": loss}
    del X, Y
    for cfg in (2, 4):
        inst = synth.config_instance(cfg)
        name = synth.CONFIGS[cfg]["name"]
        lanes = inst["n_line"] * inst["T"]
        res = {}
        for label in ("plain", "learned"):
            s = ucac.Solver(inst)
            if label == "learned":
                s.set_warmstart(w)
            s.branch_counters(reset=True)
            sec = _timed_steps(s, torch, 20, args.learned_steps)
            cnt = s.branch_counters(reset=True)
            kt = s.kernel_times(20)
            n_it = 20 + 20 + args.learned_steps
            res[label] = {"iters_per_s": 1.0 / sec, "ms_per_iter": 1e3 * sec, "branch_ms": kt["branch"],
                          "newton_per_solve": cnt["newton"] / (n_it - 20) / lanes,
                          "fallbacks_per_iter": cnt["fallbacks"] / (n_it - 20)}
            s.close()
            # time to the milestones from the cold start, same stopping rule
            s = ucac.Solver(inst)
            if label == "learned":
                s.set_warmstart(w)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, iters = s.solve(args.tol, args.learned_max_iters)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            ms = s.milestones()
            rp, rd, zinf, obj = s.residuals()
            res[label].update({"solve_iters": iters, "solve_seconds": el, "converged": rc == 0, "r_p": rp, "r_d": rd,
                               "objective": obj, "first_iter_below": ms,
                               "seconds_to": {k: (v * el / max(iters, 1) if v > 0 else None) for k, v in ms.items()}})
            s.close()
        p, l = res["plain"], res["learned"]
        res["speedup_per_iter"] = p["ms_per_iter"] / l["ms_per_iter"]
        res["speedup_branch_kernel"] = p["branch_ms"] / l["branch_ms"]
        res["speedup_time_to"] = {k: (p["seconds_to"][k] / l["seconds_to"][k]
                                      if p["seconds_to"][k] and l["seconds_to"][k] else None)
                                  for k in p["seconds_to"]}
        res["same_trajectory"] = p["first_iter_below"] == l["first_iter_below"]
        out[name] = res
    return out


DP_SHAPES = [(g, t) for g in (1000, 10000) for t in (24, 48, 96, 168)]


def _dp_case(G, T, seed):
    rng = np.random.default_rng(seed)
    tab = rng.normal(0.0, 1.0, size=(G, T, 2, 2))
    ints = [rng.integers(1, 5, G), rng.integers(1, 5, G), rng.integers(0, 2, G), np.zeros(G), np.zeros(G)]
    return tab, [x.astype(np.int32) for x in ints]


def dp_standalone(ucac, torch, reps=20):
    """The UC dynamic program alone at the shapes of the paper's DP experiment
    (1,000 and 10,000 units, T = 24 ... 168; seeded random tables resident on the
    GPU): DPs per second with the faster of 64 and 16 lanes per unit."""
    out = {}
    dev = torch.device("cuda:0")
    for G, T in DP_SHAPES:
        tab, ints = _dp_case(G, T, 7 + G + T)
        args = [torch.from_numpy(tab).to(dev)] + [torch.from_numpy(x).to(dev) for x in ints]
        best = None
        for lanes in (64, 16):
            try:
                ucac.ucac_dp_batch(*args, lanes_per_unit=lanes)
            except ucac.UcacError:
                continue  # horizon too long for 4 units per block
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ucac.ucac_dp_batch(*args, lanes_per_unit=lanes)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / reps
            if best is None or sec < best[0]:
                best = (sec, lanes)
        out[f"G{G}_T{T}"] = {"ms_per_batch": 1e3 * best[0], "dp_per_s": G / best[0], "lanes_per_unit": best[1]}
    return out


def batching(ucac, synth, torch, args):
    """64 independent instances of uneven size (30 to 2000 buses, T in {12, 24, 48}):
    one grouped launch per kernel with the tuned mapping, against running the same
    instances one at a time (each with its own captured graph)."""
    insts = synth.batch_instances(64)
    solves = sum(i["n_line"] * i["T"] for i in insts)
    b = ucac.Batch(insts)
    chosen, cand = b.autotune(iters=10)
    sec = _timed_steps(b, torch, 10, args.batch_steps)
    b.close()
    seq = 0.0
    for inst in insts:
        s = ucac.Solver(inst)
        seq += _timed_steps(s, torch, 10, args.batch_steps)
        s.close()
    return {"instances": len(insts), "buses": sum(i["n_bus"] for i in insts),
            "branch_solves_per_iter": solves, "tuned_mapping": {"dp_lanes": chosen[0], "branch_block": chosen[1],
                                                                "order": ["given", "largest_first"][chosen[2]]},
            "candidates_ms_per_iter": {f"dp{k[0]}_bb{k[1]}_o{k[2]}": v for k, v in cand.items()},
            "batched": {"ms_per_iter": 1e3 * sec, "branch_solves_per_s": solves / sec},
            "one_at_a_time": {"ms_per_iter": 1e3 * seq, "branch_solves_per_s": solves / seq},
            "speedup": seq / sec}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the workload is one "
              "instance on one MI355X; multi-GPU execution is not built", file=sys.stderr)
        sys.exit(2)
    if args.hbm_calibration:
        print(json.dumps(hbm_calibration()), flush=True)
        return

    import torch
    from paper_2310_13145_amd import synth, ucac

    inst = synth.config_instance(args.config)
    name = synth.CONFIGS[args.config]["name"] if args.config in synth.CONFIGS else f"cfg{args.config}"
    N, L, G, T = inst["n_bus"], inst["n_line"], inst["n_gen"], inst["T"]

    solver = ucac.Solver(inst)
    solver.step(args.warmup)
    state0 = solver.get_state()
    solver.branch_counters(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.steps
    newton_plain = solver.branch_counters(reset=True)["newton"] / (args.steps * T * L)

    # the same timed region with the previous-iterate Newton start (warm start)
    warm = ucac.Solver(inst, warm_start=1)
    warm.step(args.warmup)
    warm.branch_counters(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    warm.step(args.steps)
    torch.cuda.synchronize()
    dt_warm = time.perf_counter() - t0
    newton_warm = warm.branch_counters(reset=True)["newton"] / (args.steps * T * L)
    warm.close()

    # profiled pass, independent of --steps/--warmup: from the iterate after
    # PROF_FROM iterations (past the cold-start transient), one untimed kernel-by-kernel
    # iteration (every kernel's first launch in the process), then PROF_ITERS iterations
    # kernel by kernel with HIP events on the library's stream; the line kernel's mean is
    # taken from its dispatch timestamps, what a kernel trace of the same run reports
    solver.set_state(state0)
    solver.step(max(0, PROF_FROM - args.warmup))
    roof, ktimes, dispatch = line_roofline(solver, inst, max(PROF_FROM, args.warmup))
    roof["traffic"] = branch_traffic()
    prof_ms_per_step = sum(dispatch.values())
    lanes = T * L
    bytes_bus = 2 * L * T * BYTES_BUS_END + N * T * BYTES_BUS_BUS + G * T * BYTES_BUS_GEN
    # algorithmic bytes over each kernel's dispatch-timestamp mean (the event pairs
    # around a kernel also count the dispatch latency; kept as ms_between_events)
    hbm = {
        "post": {"bytes": lanes * BYTES_BUS_POST + G * T * BYTES_GEN_DUAL, "ms": dispatch["post"],
                 "ms_between_events": ktimes["post"]},
        "units": {"bytes": G * T * BYTES_UNITS, "ms": dispatch["units"], "ms_between_events": ktimes["units"]},
        "bus": {"bytes": bytes_bus, "ms": dispatch["bus"], "ms_between_events": ktimes["bus"]},
        "branch": {"bytes": lanes * BYTES_BRANCH, "ms": dispatch["branch"], "ms_between_events": ktimes["branch"]},
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
        "roofline": roof,
        "warm_start_prev_iterate": {"value": args.steps / dt_warm, "ms_per_step": 1e3 * dt_warm / args.steps,
                                    "newton_per_solve": newton_warm, "newton_per_solve_flat": newton_plain},
        "kernels_ms": ktimes,
        "kernels_dispatch_ms": dispatch,
        "profiled_ms_per_step": prof_ms_per_step,
        "hbm": hbm,
    }

    if not args.no_large:
        # the same line-kernel roofline on the 10,000-bus T = 48 workload (624,000 line
        # solves per launch, several waves per SIMD): from its iterate after PROF_FROM
        # iterations, PROF_ITERS kernel-by-kernel iterations
        big = synth.config_instance(4)
        s4 = ucac.Solver(big)
        s4.step(PROF_FROM)
        out["roofline_" + synth.CONFIGS[4]["name"]], _, _ = line_roofline(s4, big, PROF_FROM)
        s4.close()

    if not args.no_solve:
        out["time_to_tol"] = time_to_tol(ucac, torch, inst, args)
        out["time_to_tol_mesh118_T24"] = time_to_tol(ucac, torch, synth.config_instance(1), args)

    if not args.no_batch:
        out["batching"] = batching(ucac, synth, torch, args)

    if not args.no_dp:
        out["dp_standalone"] = dp_standalone(ucac, torch)

    if not args.no_learned:
        out["learned_start"] = learned_start(ucac, synth, torch, args)

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds, state0)
        out["cpu_baseline"]["gpu_over_cpu"] = out["value"] / out["cpu_baseline"]["value"]
        if "dp_standalone" in out:
            for k, v in out["dp_standalone"].items():
                v["gpu_over_cpu"] = v["dp_per_s"] / out["cpu_baseline"]["dp"][k]["dp_per_s"]

    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
