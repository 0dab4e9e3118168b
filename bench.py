#!/usr/bin/env python3
"""Benchmark: wall time of plain MLMC to RMSE 1e-3 on the config-2 workload, on one MI355X.

One step = one complete run of Algorithm 1 (dk_mlmc_estimate) from a fresh context: level
setup and discrete mean field on the device, then rounds of batched level pairs (Philox +
Box--Muller noise, fused fine/coarse EM stepping, observables, ordered FP64 moment sums)
until the bias test passes.  Each step uses its own seed.

Workload (synthetic, defined by formulas): unit torus, levels h = 1/8 .. 1/128,
tau_l = 0.1 h_l^2, T = 0.05, rho0 = 1 + 0.5 cos 2 pi x cos 2 pi y, N = 1e4, primary observable
(sqrt(N)(rho_T - rho_bar_T, sin 2 pi x + sin 2 pi y)_h)^2, eps = 1e-3.

The JSON line carries the roofline of the dominant kernel (the finest level pair, bound by
vector ALU issue) measured with HIP events inside the library over the timed region, and
the CPU oracle's projected time for the same run from a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLMC wall-time to RMSE 1e-3 (plain vs learned CV); cell-updates/s and HBM %"

# Algorithmic vector-ALU operations per fine cell update of a coupled pair (see the design doc,
# "Measurement"): half a Philox4x32-10 call (40), one binary32 Box--Muller pair (60), the
# explicit EM update with central flux and compensated increment (18), the NN restriction
# and the amortised coarse step (3).
OPS_PER_CELL_UPDATE = 121.0
# MI355X vector FP32 rate: 157.3 TFLOP/s counts an FMA as 2 flops, i.e. 78.6e12 32-bit
# vector lane-operations per second (256 CUs x 128 lanes x 2.4 GHz).
VALU_PEAK_OPS = 256 * 128 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--warmup-eps", type=float, default=1e-2, help="accuracy of the untimed warmup runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle sampling")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 256 MiB buffer 4 times (reference for HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(problem, M, budget):
    """Oracle per-sample cost on the host cores for levels 0..L, projected to the sample
    counts M of the GPU run.  Levels whose sample would not fit the budget are extrapolated
    from the last measured level by the cell-update count."""
    import numpy as np
    import oracle

    threads = oracle.default_threads()
    op = oracle.OracleProblem(problem)
    for l in range(len(M)):
        op.centre(l)
    per_sample = []
    measured = []
    measured_cells = []
    spent = 0.0
    for l in range(len(M)):
        cells = problem.n(l) ** 2 * problem.steps(l) * (1 + (l > 0) / 16)
        if measured:
            # predicted wall time of `threads` samples on `threads` cores
            pred = per_sample[-1] / measured_cells[-1] * cells
            if spent + pred > budget:
                per_sample.append(pred)
                continue
        n = threads
        t0 = time.perf_counter()
        oracle.run_range(op, l, 0, n, threads=threads)
        wall = time.perf_counter() - t0
        spent += wall
        per_sample.append(wall * threads / n)          # core-seconds per sample
        measured_cells.append(cells)
        measured.append(l)
    core_s = sum(m * c for m, c in zip(M, per_sample))
    return {"value": core_s / threads, "unit": "s", "cores": threads, "kind": "oracle",
            "sample": (f"{threads} oracle samples on each of levels {measured} ({spent:.1f} s wall on "
                       f"{threads} threads); per-sample cost of levels {[l for l in range(len(M)) if l not in measured]} "
                       "extrapolated by cell updates; projected to the GPU run's M_l"),
            "per_sample_core_s": per_sample}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the path shards by "
                                   "sample range across GPUs, see DESIGN.md)"}))
        sys.exit(2)
    import torch

    import dk_workloads as W
    import paper_2311_08872_amd as dk

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_launch": 2 * src.numel() * 4, "launches": 4}), flush=True)
        return
    base = W.config2(N=1e4)

    os.environ.setdefault("DK_LOG", "1")     # progress lines on stderr (per round and per long launch)

    def one(seed, ctx, eps):
        p = base.with_(seed=seed)
        return dk.estimate(p, eps, ctx=ctx, level_moments=True)

    for w in range(args.warmup):
        ctx = dk.Context(0)
        one(1000 + w, ctx, args.warmup_eps)
        ctx.close()

    torch.cuda.synchronize()
    results = []
    stats = {}
    t0 = time.perf_counter()
    for k in range(args.steps):
        ctx = dk.Context(0)            # fresh context: level tables and mean field are rebuilt
        r = one(k, ctx, args.eps)
        print(f"[bench] step {k}: {time.perf_counter() - t0:.1f} s, L={r['L']} M={r['M']}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        for s in ctx.stats():
            key = (s["level"], s["coupled"])
            acc = stats.setdefault(key, {"launches": 0, "samples": 0, "kernel_ms": 0.0, "cell_updates": 0.0})
            for f in acc:
                acc[f] += s[f]
            acc["rows"] = s["rows"]
        ctx.close()
        results.append(r)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_step = wall / args.steps

    cells = sum(r["cell_updates"] for r in results)
    kernel_ms = sum(v["kernel_ms"] for v in stats.values())
    (dl, dc), dom = max(stats.items(), key=lambda kv: kv[1]["kernel_ms"])
    avg_launch_s = dom["kernel_ms"] / 1e3 / dom["launches"]
    ops_per_launch = OPS_PER_CELL_UPDATE * dom["cell_updates"] / dom["launches"]
    achieved = ops_per_launch / avg_launch_s
    last = results[-1]
    # plain MC on the finest level reached: M_MC = 2 Var(P_L) / eps^2, time from the measured
    # per-sample kernel cost of that level (projected, as the paper did for its smallest eps)
    Lr = last["L"]
    lm = last["level_moments"][Lr][base.primary]
    varPL = max(0.0, (lm.sums[3] - lm.sums[2] ** 2 / lm.count) / (lm.count - 1))
    pair_stat = stats.get((Lr, True))
    mc_sample_s = (pair_stat["kernel_ms"] / 1e3 / pair_stat["samples"]) / (1 + 1 / 16) if pair_stat else float("nan")
    mc_M = math.ceil(2 * varPL / args.eps ** 2)
    out = {
        "metric": METRIC,
        "value": per_step,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per_step * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "config-2 plain MLMC: unit torus, h=1/8..1/128, tau=0.1h^2, T=0.05, "
                               "rho0=1+0.5cos2pix cos2piy, N=1e4, psi=x^2 of the centred sqrt(N)-scaled "
                               "<rho_T, sin2pix+sin2piy>, Algorithm 1, eps=1e-3",
                   "eps": args.eps, "levels": base.levels, "N": base.N, "state": "fp32 (compensated)",
                   "seeds": list(range(args.steps))},
        "cell_updates_per_s": cells / wall,
        "kernel_fraction_of_wall": kernel_ms / 1e3 / wall,
        "mlmc": {"L": last["L"], "converged": last["converged"], "M": last["M"],
                 "Yhat": last["Yhat"], "Vhat": last["Vhat"], "estimate": last["estimate"][base.primary],
                 "rmse_est": last["rmse_est"], "rounds": last["rounds"], "cell_updates": last["cell_updates"]},
        "plain_mc_projected": {"level": Lr, "var_P": varPL, "samples": mc_M, "per_sample_s": mc_sample_s,
                               "wall_s": mc_M * mc_sample_s,
                               "speedup_vs_mlmc": mc_M * mc_sample_s / per_step if per_step > 0 else None},
        "roofline": {"bound": "alu", "kernel": f"level_kernel pair={dc} level={dl} ({base.n(dl)}^2)",
                     "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12, "unit": "Top/s",
                     "frac": achieved / VALU_PEAK_OPS, "traffic": None,
                     "ops_per_cell_update": OPS_PER_CELL_UPDATE,
                     "cell_updates_per_launch": dom["cell_updates"] / dom["launches"],
                     "avg_launch_ms": avg_launch_s * 1e3,
                     "kernel_cell_updates_per_s": dom["cell_updates"] / (dom["kernel_ms"] / 1e3)},
        "kernels": {f"L{l}{'p' if c else 's'}": v for (l, c), v in sorted(stats.items())},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(base, last["M"], args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
