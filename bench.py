#!/usr/bin/env python3
"""Benchmark: wall time of plain MLMC at eps = 1e-3 on the config-2 workload, on one MI355X.

One step = one complete run of Algorithm 1 (dk_mlmc_estimate) from a fresh context: level
setup and discrete mean field on the device, then rounds of batched level pairs (Philox +
Box--Muller noise, fused fine/coarse EM stepping, observables, ordered FP64 moment sums)
until the bias test passes or the finest level is reached with the variance target eps^2/2
met.  Each step uses its own seed.  One step takes minutes, so the loop is wall-budgeted:
warm-ups (at a loose eps) stop once --warmup-budget seconds are spent, and a further timed
step starts only while the time since start plus the longest step so far stays within
--time-budget; "steps" reports the steps actually timed, "steps_requested" the request.  A
step is never cut short.

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

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLMC wall-time to RMSE 1e-3 (plain vs learned CV); cell-updates/s and HBM %"

# Algorithmic vector-ALU operations per FINE cell update of a coupled pair: half a
# Philox4x32-10 call (40), one binary32 Box--Muller pair (60), the explicit EM update with
# central flux and compensated increment (18), the NN restriction and the amortised coarse
# step (3).  The coarse step is included here, so the count it multiplies is fine updates only
# (the library's per-level statistics count a pair's coarse updates too, 1/16 of the fine ones).
OPS_PER_CELL_UPDATE = 121.0
COARSE_SHARE = 1.0 / 16.0
# MI355X vector FP32 rate: 157.3 TFLOP/s counts an FMA as 2 flops, i.e. 78.6e12 32-bit
# vector lane-operations per second (256 CUs x 128 lanes x 2.4 GHz).
VALU_PEAK_OPS = 256 * 128 * 2.4e9

# HBM traffic of the dominant kernel (the 128^2 pair level kernel), from rocprofv3 --pmc runs of
# `bench.py --workload counters` (one production launch of 14024 pairs): read bytes from the
# size-resolved request counters (32/64/128-B requests to EA), written bytes from WRITE_SIZE; both
# read 1.000 x the bytes of a 256 MiB copy (FETCH_SIZE reads 0.5 x on gfx950).  A constant per
# dispatch (the level tables, fetched once per compute die) plus bytes per pair (the outputs).  It is
# reported only while the kernel sources hash to the value the counters were taken on.
TRAFFIC = {"sha256": "2a2bd19999f3c5d39d4cba75ea02557a0ee6622b52665fb312e8e485c3d47994",
           "read_bytes_per_dispatch": 3320.5 * 1024, "write_bytes_per_pair": 32.0,
           "profile": "profiles/level_kernel_128_pair_counters_workload_hbm.md"}
KERNEL_SOURCES = ["dk_level.h", "dk_rng.h", "dk_kernels.hip", "dk_internal.h"]


def kernel_source_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_08872_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--warmup-eps", type=float, default=1e-2, help="accuracy of the untimed warmup runs")
    ap.add_argument("--warmup-budget", type=float, default=30.0,
                    help="no further warmup run starts after this many seconds of warmups")
    ap.add_argument("--time-budget", type=float, default=450.0,
                    help="a further timed step starts only if the seconds since start plus the longest "
                         "step so far stay within this budget (the first timed step always runs)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle sampling")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 256 MiB buffer 4 times (reference for HBM byte counters)")
    ap.add_argument("--workload", default="config2",
                    choices=["config2", "config2-mc", "config3", "config4", "config5", "paper-type1", "paper-type2",
                             "paper-couplings", "paper-theta", "counters"],
                    help="config2 (default): the bench line; the others print a report line: config2-mc "
                         "plain Monte Carlo on the finest config-2 level to the same eps, config3 "
                         "low-density MLMC with persistent rounds, config4 learned control variate, "
                         "config5 streaming-kernel throughput at 256^2..1024^2, paper-type1 the paper's own "
                         "Type-1 experiment (MLMC and MC at its accuracies, speed-ups against its table), "
                         "paper-type2 its variance-reduction factor against h_min, paper-couplings the "
                         "symmetric NN and the Fourier coupling against the NN coupling, paper-theta "
                         "explicit against Crank-Nicolson and implicit Euler time stepping, counters one "
                         "production-size launch of each hot kernel and a 256 MiB copy (for rocprofv3 --pmc runs)")
    ap.add_argument("--N", type=float, default=None, help="particle number (config3: 1e5, config5: 1e6)")
    ap.add_argument("--samples", type=int, default=32, help="config5: finest-level pairs to time")
    ap.add_argument("--depth-only", action="store_true",
                    help="config5: only the temporal-depth study (4 x --samples pairs, 128 x --samples steps)")
    ap.add_argument("--cv-levels", default=None, help="config4: comma-separated levels that use the control "
                                                        "variate (default: those where it lowers variance x cost)")
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
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the path would shard "
                                   "by sample range across GPUs, with one all-reduce of the level moments "
                                   "per Algorithm-1 round)"}))
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
    os.environ.setdefault("DK_LOG", "1")     # progress lines on stderr (per round and per long launch)
    if args.workload != "config2":
        {"config2-mc": bench_config2_mc, "config3": bench_config3, "config4": bench_config4,
         "config5": bench_config5, "paper-type1": bench_paper_type1,
         "paper-type2": bench_paper_type2, "paper-couplings": bench_paper_couplings, "paper-theta": bench_paper_theta,
         "counters": bench_counters}[args.workload](args)
        return
    base = W.config2(N=1e4)

    def one(seed, ctx, eps):
        p = base.with_(seed=seed)
        return dk.estimate(p, eps, ctx=ctx, level_moments=True)

    warmups = 0
    t_w = time.perf_counter()
    for w in range(args.warmup):
        if w > 0 and time.perf_counter() - t_w > args.warmup_budget:
            break
        ctx = dk.Context(0)
        one(1000 + w, ctx, args.warmup_eps)
        ctx.close()
        warmups += 1
    print(f"[bench] {warmups} warmup run(s) at eps={args.warmup_eps:g}: {time.perf_counter() - t_w:.1f} s",
          file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    results = []
    step_s = []
    stats = {}
    t0 = time.perf_counter()
    for k in range(args.steps):
        if k > 0 and (time.perf_counter() - T_START) + max(step_s) > args.time_budget:
            print(f"[bench] stopping after {k} timed step(s): another ({max(step_s):.0f} s) would end past the "
                  f"{args.time_budget:.0f} s budget", file=sys.stderr, flush=True)
            break
        ts = time.perf_counter()
        ctx = dk.Context(0)            # fresh context: level tables and mean field are rebuilt
        r = one(k, ctx, args.eps)
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - ts)
        print(f"[bench] step {k}: {step_s[-1]:.1f} s, L={r['L']} M={r['M']} converged={r['converged']} "
              f"rmse_est={r['rmse_est']:.3g}", file=sys.stderr, flush=True)
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
    steps = len(results)
    per_step = wall / steps

    cells = sum(r["cell_updates"] for r in results)
    kernel_ms = sum(v["kernel_ms"] for v in stats.values())
    (dl, dc), dom = max(stats.items(), key=lambda kv: kv[1]["kernel_ms"])
    avg_launch_s = dom["kernel_ms"] / 1e3 / dom["launches"]
    traffic = None
    if (TRAFFIC["sha256"] and TRAFFIC["sha256"] == kernel_source_sha256() and (dl, dc) == (base.levels - 1, True)):
        traffic = TRAFFIC["read_bytes_per_dispatch"] + TRAFFIC["write_bytes_per_pair"] * dom["samples"] / dom["launches"]
    fine_per_launch = dom["cell_updates"] / dom["launches"] / (1.0 + COARSE_SHARE if dc else 1.0)
    ops_per_launch = OPS_PER_CELL_UPDATE * fine_per_launch
    achieved = ops_per_launch / avg_launch_s
    last = results[-1]
    # plain MC on the finest level reached: M_MC = 2 Var(P_L) / eps^2, time from the measured
    # per-sample kernel cost of that level (projected, as the paper did for its smallest eps)
    Lr = last["L"]
    lm = last["level_moments"][Lr][base.primary]
    varPL = lm.stats(1)[1]
    pair_stat = stats.get((Lr, True))
    mc_sample_s = (pair_stat["kernel_ms"] / 1e3 / pair_stat["samples"]) / (1 + 1 / 16) if pair_stat else float("nan")
    mc_M = math.ceil(2 * varPL / args.eps ** 2)
    out = {
        "metric": METRIC,
        "value": per_step,
        "unit": "s",
        "n_gpus": 1,
        "steps": steps,
        "steps_requested": args.steps,
        "warmup": warmups,
        "warmup_requested": args.warmup,
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
                   "seeds": list(range(steps))},
        "reached": {"converged": last["converged"], "rmse_est": last["rmse_est"], "bias_est": last["bias_est"],
                    "var_est": last["var_est"][base.primary], "eps": args.eps,
                    "value_is": ("wall time of Algorithm 1 to RMSE eps (bias test passed)" if last["converged"] else
                                 "wall time of Algorithm 1 to the variance target eps^2/2 on the finest level "
                                 f"allowed (L={last['L']}); the bias test was not passed, so the estimated RMSE "
                                 f"is {last['rmse_est']:.3g}, not eps")},
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
                     "frac": achieved / VALU_PEAK_OPS, "traffic": traffic,
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 counters)",
                     "ops_per_fine_cell_update": OPS_PER_CELL_UPDATE,
                     "fine_cell_updates_per_launch": fine_per_launch,
                     "avg_launch_ms": avg_launch_s * 1e3,
                     "launches": dom["launches"],
                     "fine_cell_updates_per_s": fine_per_launch / avg_launch_s},
        "kernels": {f"L{l}{'p' if c else 's'}": v for (l, c), v in sorted(stats.items())},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(base, last["M"], args.cpu_budget)
    print(json.dumps(out), flush=True)



def _report(workload, value, unit, extra):
    line = {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "data": "synthetic",
            "config": {"workload": workload}, "report_only": True}
    line.update(extra)
    print(json.dumps(line), flush=True)


def bench_config2_mc(args):
    """Plain Monte Carlo (the paper's comparison estimator) on the finest config-2 level (128^2,
    8192 steps, single paths from their own noise stream) to RMSE args.eps: a pilot of 1000 paths,
    then M = ceil(2 Var / eps^2) paths, so that the variance term meets eps^2 / 2 as in the MLMC
    run.  Measured, not projected."""
    import torch
    import dk_workloads as W
    import paper_2311_08872_amd as dk
    p = W.config2(N=1e4)
    L = p.levels - 1
    ctx = dk.Context(0)
    dk.estimate(p.with_(seed=1000), 5e-2, ctx=ctx, plain_mc_level=L)       # warm-up (untimed)
    ctx.close()
    ctx = dk.Context(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = dk.estimate(p, args.eps, ctx=ctx, plain_mc_level=L)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.stats()
    ctx.close()
    _report(f"config-2 plain MC on the finest level (128^2, 8192 steps), eps={args.eps:g}", wall, "s",
            {"mc": {"level": L, "M": r["M"][L], "estimate": r["estimate"][p.primary], "var_est": r["var_est"][0],
                    "rmse_est": r["rmse_est"], "rounds": r["rounds"], "cell_updates": r["cell_updates"]},
             "cell_updates_per_s": r["cell_updates"] / wall,
             "kernels": [{k: s_[k] for k in ("level", "coupled", "launches", "samples", "kernel_ms", "cell_updates", "rows")}
                         for s_ in st]})


def bench_paper_type1(args):
    """The paper's Type-1 experiment (Sec. 7) in its own setting: the 2 pi torus, h_l = 2 pi
    2^-(2+l) (4^2 .. 128^2), tau_l = 1e-3 4^(5-l), T = 1.024, phi = sin x + sin y, psi = x^2, the
    regular datum at N = 2e9 and 2e5 and the irregular one at N = 2e9.  For every accuracy of its
    list, Algorithm 1, then plain MC on the finest level that run reached, to the same variance
    target (eps^2 / 2).  Both are measured (not extrapolated).  Speed-ups are reported as the ratio
    of wall times on this GPU and as the ratio of work (fine + coarse cell updates), the latter
    comparable with the paper's CPU timings; the paper's table gives 5.6, 5.4 and 22.8 at the
    smallest accuracies."""
    import torch
    import dk_workloads as W
    import paper_2311_08872_amd as dk
    reg = [10 ** -1.4, 10 ** -1.7, 10 ** -2.0, 10 ** -2.2, 10 ** -2.4, 10 ** -2.6]
    irreg = reg[:-1] + [10 ** -2.75]
    settings = [("reg", 2e9, W.paper_reg, reg, 5.6), ("reg", 2e5, W.paper_reg, reg, 5.4),
                ("irreg", 2e9, W.paper_irreg, irreg, 22.8)]
    ctx = dk.Context(0)
    dk.estimate(W.paper_reg(2e9).with_(seed=1000), 10 ** -1.4, ctx=ctx)         # warm-up (untimed)
    ctx.close()
    for name, N, make, eps_list, paper_speedup in settings:
        p = make(N)
        rows = []
        for eps in eps_list:
            ctx = dk.Context(0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = dk.estimate(p, eps, ctx=ctx)
            torch.cuda.synchronize()
            t_mlmc = time.perf_counter() - t0
            L = r["L"]
            t0 = time.perf_counter()
            mc = dk.estimate(p.with_(seed=p.seed + 1), eps, ctx=ctx, plain_mc_level=L)
            torch.cuda.synchronize()
            t_mc = time.perf_counter() - t0
            ctx.close()
            rows.append({"eps": eps, "L": L, "converged": r["converged"], "M": r["M"], "estimate": r["estimate"][0],
                         "Yhat": r["Yhat"], "Vhat": r["Vhat"], "mlmc_s": t_mlmc, "mlmc_cell_updates": r["cell_updates"],
                         "mc_M": mc["M"][L], "mc_s": t_mc, "mc_cell_updates": mc["cell_updates"],
                         "speedup_wall": t_mc / t_mlmc, "speedup_work": mc["cell_updates"] / r["cell_updates"]})
            print(f"[bench] paper {name} N={N:g} eps={eps:.3g}: L={L} MLMC {t_mlmc:.3f} s, MC {t_mc:.3f} s, "
                  f"work ratio {rows[-1]['speedup_work']:.2f}", file=sys.stderr, flush=True)
        last = rows[-1]
        _report(f"paper Sec. 7 Type-1 experiment: rho0_{name}, N={N:g}, 2 pi torus, h=2pi/4..2pi/128, "
                f"tau_l=1e-3*4^(5-l), T=1.024", last["speedup_work"], "MC/MLMC work ratio at the smallest eps",
                {"paper_speedup_at_smallest_eps": paper_speedup, "smallest_eps": last["eps"], "L_reached": last["L"],
                 "speedup_wall_at_smallest_eps": last["speedup_wall"], "runs": rows})


def bench_paper_couplings(args):
    """The couplings of Sec. 3 in the paper's Sec. 7 setting (regular datum): the NN coupling of
    Sec. 3.2 on the vertex grid (the paper's runs), its symmetric variant on cell centres (the
    remark after Sec. 3.2) and the Fourier coupling of Sec. 3.1 (the paper's proposed next step).
    NN: 4^2 .. 128^2 (ratio 2); Fourier: 4^2, 12^2, 36^2, 108^2 (ratio 3, similar h_min).  Per N
    in {2e9, 2e5}:
    1. level profile: args.samples * 125 samples per level (P = X^2, the paper's observable):
       V_l, |Y_l|, cell updates and kernel time per sample, and the observed variance rate
       beta_l = log(V_(l-1) / V_l) / log(ratio) (the paper predicts 4 for Fourier, 2 for NN);
    2. Algorithm 1 at the paper's accuracies 10^-1.4 .. 10^-2.6 with either coupling: levels,
       work (cell updates) and GPU wall time."""
    import math
    import torch
    import dk_workloads as W
    import paper_2311_08872_amd as dk
    eps_list = [10 ** -1.4, 10 ** -1.7, 10 ** -2.0, 10 ** -2.2, 10 ** -2.4, 10 ** -2.6]
    per_level = args.samples * 125
    out = {}
    ctx = dk.Context(0)
    dk.estimate(W.paper_fourier(2e9).with_(seed=1000), 10 ** -1.4, ctx=ctx)      # warm-up (untimed)
    dk.estimate(W.paper_reg(2e9).with_(seed=1000), 10 ** -1.4, ctx=ctx)
    ctx.close()
    for N in (2e9, 2e5):
        res = {}
        for name, p in (("nn", W.paper_reg(N)), ("nn_cell", W.paper_reg(N).with_(grid=W.GRID_CELL)),
                        ("fourier", W.paper_fourier(N))):
            ctx = dk.Context(0)
            prof = []
            for l in range(p.levels):
                ctx.reset()
                mom = dk.level_pair(p, l, 0, per_level, ctx=ctx)[0]
                torch.cuda.synchronize()
                st = [s_ for s_ in ctx.stats() if s_["level"] == l][0]
                prof.append({"level": l, "n": p.n(l), "steps": p.steps(l), "V": mom.var, "Y": mom.mean,
                             "cell_updates_per_sample": st["cell_updates"] / per_level,
                             "kernel_s_per_sample": st["kernel_ms"] / 1e3 / per_level,
                             "cell_updates_per_s": st["cell_updates"] / (st["kernel_ms"] / 1e3)})
            for l in range(2, p.levels):
                prof[l]["beta"] = math.log(prof[l - 1]["V"] / prof[l]["V"]) / math.log(p.ratio)
            vs = ", ".join("%.3g" % r_["V"] for r_ in prof)
            bs = ", ".join("%.2f" % r_["beta"] for r_ in prof if "beta" in r_)
            print(f"[bench] paper {name} N={N:g}: V_l = [{vs}], beta = [{bs}]", file=sys.stderr, flush=True)
            runs = []
            for eps in eps_list:
                ctx.reset(drop_tables=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = dk.estimate(p, eps, ctx=ctx)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                runs.append({"eps": eps, "L": r["L"], "n_finest": p.n(r["L"]), "converged": r["converged"], "M": r["M"],
                             "estimate": r["estimate"][0], "rmse_est": r["rmse_est"], "cell_updates": r["cell_updates"],
                             "wall_s": wall})
                print(f"[bench] paper {name} N={N:g} eps={eps:.3g}: L={r['L']} ({p.n(r['L'])}^2) work "
                      f"{r['cell_updates']:.3g} cell updates, {wall:.3f} s, estimate {r['estimate'][0]:.5f}",
                      file=sys.stderr, flush=True)
            ctx.close()
            res[name] = {"profile": prof, "alg1": runs}
        res["work_ratio_nn_over_fourier"] = [a["cell_updates"] / b["cell_updates"]
                                             for a, b in zip(res["nn"]["alg1"], res["fourier"]["alg1"])]
        res["wall_ratio_nn_over_fourier"] = [a["wall_s"] / b["wall_s"] for a, b in zip(res["nn"]["alg1"], res["fourier"]["alg1"])]
        res["work_ratio_nn_over_nn_cell"] = [a["cell_updates"] / b["cell_updates"]
                                             for a, b in zip(res["nn"]["alg1"], res["nn_cell"]["alg1"])]
        out[f"N={N:g}"] = res
    last = out["N=2e+09"]
    _report("couplings in the paper's Sec. 7 setting (NN vertex, NN cell-centred, Fourier; regular datum, N=2e9 "
            "and 2e5): level variances and Algorithm 1 at eps=10^-1.4..10^-2.6", last["work_ratio_nn_over_fourier"][-1],
            "NN/Fourier MLMC work ratio at eps=10^-2.6, N=2e9", out)


def bench_paper_theta(args):
    """Time stepping with the implicit weight b0 of eq. (FullyDiscreteDK) in the paper's Sec. 7
    setting (regular datum, N = 2e9, grids 4^2 .. 64^2): the explicit scheme of the paper
    (b0 = 0), Crank--Nicolson (b0 = 1/2) and implicit Euler (b0 = 1) at the paper's tau/h^2, and
    implicit Euler with four times the time step (tau/h^2 = 4 x 0.415, beyond the explicit limit
    1/2; hierarchy 8^2 .. 64^2).  Per scheme: level profile (args.samples * 125 samples per level: V_l, E[Y_l], kernel
    rate) and Algorithm 1 at the paper's accuracies 10^-1.4 .. 10^-2.4 (work, wall time,
    estimate)."""
    import math
    import torch
    import dk_workloads as W
    import paper_2311_08872_amd as dk
    eps_list = [10 ** -1.4, 10 ** -1.7, 10 ** -2.0, 10 ** -2.2, 10 ** -2.4]
    per_level = args.samples * 125
    base = W.paper_reg(2e9).with_(levels=5)
    # four times the step: tau_0 = 4 mu h_0^2 equals T on the 8 x 8 grid, so that hierarchy is
    # 8^2 .. 64^2 with 1, 4, 16, 64 steps (a quarter of the explicit scheme's on each grid)
    schemes = [("explicit", base), ("crank_nicolson", base.with_(b0=0.5)), ("implicit_euler", base.with_(b0=1.0)),
               ("implicit_euler_4tau", base.with_(b0=1.0, mu=4 * base.mu, n0=8, levels=4))]
    out = {}
    ctx = dk.Context(0)
    dk.estimate(base.with_(b0=0.5, seed=1000), 10 ** -1.4, ctx=ctx)          # warm-up (untimed)
    ctx.close()
    for name, p in schemes:
        ctx = dk.Context(0)
        prof = []
        try:
            for l in range(p.levels):
                ctx.reset()
                mom = dk.level_pair(p, l, 0, per_level, ctx=ctx)[0]
                torch.cuda.synchronize()
                st = [s_ for s_ in ctx.stats() if s_["level"] == l][0]
                prof.append({"level": l, "n": p.n(l), "steps": p.steps(l), "V": mom.var, "Y": mom.mean,
                             "cell_updates_per_s": st["cell_updates"] / (st["kernel_ms"] / 1e3)})
        except dk.DKError as e:
            print(f"[bench] paper theta {name}: {e}", file=sys.stderr, flush=True)
            ctx.close()
            continue
        for l in range(2, p.levels):
            prof[l]["beta"] = math.log(prof[l - 1]["V"] / prof[l]["V"]) / math.log(2.0)
        vs = ", ".join("%.3g" % r_["V"] for r_ in prof)
        ys = ", ".join("%.3g" % r_["Y"] for r_ in prof)
        print(f"[bench] paper theta {name}: V_l = [{vs}], E[Y_l] = [{ys}]", file=sys.stderr, flush=True)
        runs = []
        for eps in eps_list:
            ctx.reset(drop_tables=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = dk.estimate(p, eps, ctx=ctx)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            runs.append({"eps": eps, "L": r["L"], "converged": r["converged"], "M": r["M"], "estimate": r["estimate"][0],
                         "cell_updates": r["cell_updates"], "wall_s": wall})
            print(f"[bench] paper theta {name} eps={eps:.3g}: L={r['L']} converged={r['converged']} work "
                  f"{r['cell_updates']:.3g}, {wall:.3f} s, estimate {r['estimate'][0]:.5f}", file=sys.stderr, flush=True)
        ctx.close()
        out[name] = {"b0": p.b0, "mu": p.mu, "steps": [p.steps(l) for l in range(p.levels)], "profile": prof, "alg1": runs}
    _report("time stepping with implicit weight b0 in the paper's Sec. 7 setting (regular datum, N=2e9, 4^2..64^2): "
            "explicit, Crank-Nicolson, implicit Euler, implicit Euler with 4x tau", out["crank_nicolson"]["alg1"][-1]["estimate"],
            "Crank-Nicolson MLMC estimate at eps=10^-2.4", out)


def bench_paper_type2(args):
    """The paper's Type-2 experiment (Sec. 7, Prop. PropVarFactor): MLMC with the fixed geometric
    schedule M_(l-1) = 4 M_l (M_L = args.samples * 32 on the finest level) for h_min = 2 pi 2^-(2+L),
    L = 1..5.  From the per-level moments: the MLMC estimator's variance sum_l V_l / M_l and cost
    sum_l M_l C_l, and the variance of plain MC on the finest level at the same cost,
    Var(P_L) C_L / cost.  Their ratio F is compared with the proposition's NN rate
    [(N h_min^2)^-1 + h_min^2]^-1 |log h_min|^-1 (up to a constant, reported normalised to L = 1)."""
    import torch
    import dk_workloads as W
    import paper_2311_08872_amd as dk
    settings = [("reg", 2e9, W.paper_reg), ("reg", 2e5, W.paper_reg), ("irreg", 2e9, W.paper_irreg)]
    m_top = args.samples * 32
    for name, N, make in settings:
        p = make(N)
        rows = []
        for L in range(1, p.levels):
            count = [m_top * 4 ** (L - l) for l in range(L + 1)]
            ctx = dk.Context(0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mom = dk.round_sums(p.with_(seed=p.seed + L), L, [0] * (L + 1), count, ctx=ctx)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ctx.close()
            V, C = [], []
            for l in range(L + 1):
                m = mom[l][p.primary]
                n = m.count
                V.append(m.var)
                C.append(p.n(l) ** 2 * p.steps(l) * (1.0 + (l > 0) / 16.0))
            mL = mom[L][p.primary]
            var_PL = mL.stats(1)[1]
            var_ml = sum(V[l] / count[l] for l in range(L + 1))
            cost = sum(count[l] * C[l] for l in range(L + 1))
            c_single = p.n(L) ** 2 * p.steps(L)
            var_mc = var_PL * c_single / cost
            h = p.box / p.n(L)
            rate = 1.0 / ((1.0 / (N * h * h) + h * h) * abs(math.log(h)))
            rows.append({"L": L, "h_min": h, "M": count, "V": V, "var_P_L": var_PL, "var_mlmc": var_ml,
                         "var_mc_same_cost": var_mc, "F": var_mc / var_ml, "rate": rate, "wall_s": wall})
        for r in rows:
            r["rate_normalised"] = r["rate"] / rows[0]["rate"] * rows[0]["F"]
        print(f"[bench] paper type2 {name} N={N:g}: F = {[round(r['F'], 2) for r in rows]}", file=sys.stderr, flush=True)
        _report(f"paper Sec. 7 Type-2 experiment: rho0_{name}, N={N:g}, M_(l-1) = 4 M_l, M_L = {m_top}",
                rows[-1]["F"], "variance-reduction factor F at h_min = 2 pi/128", {"rows": rows})


def bench_config3(args):
    """Low-density MLMC (config 3): rho0 = max(0, cos 2 pi x) + 0.05, levels 8^2..256^2, 29
    observables (Fourier modes |k| <= 3 and the primary, a squared bump), N = 1e5 and 1e3.
    1. Variance profile: one round of 1000 samples on every level (the resident levels in one
       persistent launch, the 256^2 pairs on the streaming kernel): Y_l and V_l per level show
       the low-density behaviour (V_l stops decreasing once N h^2 rho is small).
    2. Algorithm 1 with persistent rounds.  The primary observable is uncentred and unscaled
       (about 1.5e-4), so the accuracy is relative to its magnitude, estimated by a 1000-sample
       level-0 pilot from another noise stream: 1e-3 at N = 1e5 (reaches 256^2) and 1.5e-2 at
       N = 1e3 (there the level means grow from 32^2 on, so the bias test does not pass and the run
       ends on 256^2 with the variance target met, in about 4 minutes; a looser 3e-2 passes the
       bias test on 16^2 by chance); --N with --eps overrides.
    Reports wall times, the share of wall time outside kernels, the tuner's choices and the
    per-level statistics."""
    import torch
    import dk_workloads as W
    import paper_2311_08872_amd as dk
    runs = [(args.N, args.eps)] if args.N else [(1e5, 1e-3), (1e3, 1.5e-2)]
    for N, rel in runs:
        p = W.config3(N=N)
        L = p.levels - 1
        ctx = dk.Context(0)
        dk.round_sums(p, L, [0] * (L + 1), [64] * (L + 1), tag=W.TAG_MC, round_mode=3, ctx=ctx)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prof = dk.round_sums(p, L, [0] * (L + 1), [1000] * (L + 1), round_mode=3, ctx=ctx)
        torch.cuda.synchronize()
        t_prof = time.perf_counter() - t0
        Y, V = [], []
        for l in range(L + 1):
            m = prof[l][p.primary]
            Y.append(m.mean)
            V.append(m.var)
        pilot = dk.round_sums(p, 0, [0], [1000], tag=W.TAG_MC, round_mode=3, ctx=ctx)[0][p.primary]
        scale = abs(pilot.stats(1)[0])
        eps = rel * scale
        ctx.close()
        ctx = dk.Context(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = dk.estimate(p, eps, ctx=ctx, round_mode=3)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = ctx.stats()
        kernel_ms = sum(s["kernel_ms"] for s in st)
        tuned = json.loads(ctx.tuning_json())
        ctx.close()
        _report(f"config-3 low-density MLMC: rho0=max(0,cos2pix)+0.05, h=1/8..1/256, N={N:g}, 29 observables, "
                f"eps={rel:g} relative ({eps:.3g} absolute), persistent rounds", wall, "s",
                {"eps_abs": eps, "kernel_fraction_of_wall": kernel_ms / 1e3 / wall,
                 "variance_profile": {"samples_per_level": 1000, "wall_s": t_prof, "Y": Y, "V": V,
                                      "N_h2_min_density": [N * 0.05 / p.n(l) ** 2 for l in range(L + 1)]},
                 "mlmc": {k: r[k] for k in ("L", "converged", "M", "Yhat", "Vhat", "rmse_est", "rounds",
                                            "cell_updates", "estimate")},
                 "cell_updates_per_s": r["cell_updates"] / wall, "tuned_shapes": tuned["shapes"],
                 "kernels": [{k: s[k] for k in ("level", "coupled", "launches", "samples", "kernel_ms",
                                                "cell_updates", "rows")} for s in st]})


def bench_config4(args):
    """Learned control variate (config 4): for every pair l >= 1 of config 2, a network trained on
    2^16 pairs from its own noise stream; its held-out statistics decide whether level l uses it:
    the control-variate sample Z = (Y - r) + mean of r over k = 4 independent coarse-only paths has
    variance Var(Y - r) + Var(r) / k and costs (1 + k / 17) pairs, so the level uses it only if
    (Var(Y - r) + Var(r) / k) (1 + k / 17) < Var(Y) (--cv-levels forces a set).  Then Algorithm
    1 to args.eps.  Wall time includes the training."""
    import numpy as np
    import torch
    import dk_workloads as W
    import paper_2311_08872_amd as dk
    p = W.config2(N=1e4)
    kappa = 4
    ctx = dk.Context(0)
    dk.estimate(p.with_(seed=1000), 2e-2, ctx=ctx)                      # warm-up (untimed)
    ctx.close()
    ctx = dk.Context(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    params = np.zeros((p.levels, dk.L.DK_CNN_NPARAM), np.float32)
    train = {}
    use = []
    for l in range(1, p.levels):
        t1 = time.perf_counter()
        res = dk.cv_train(p, l, n_train=1 << 16, epochs=6, batch=256, lr=1e-3, n_val=1 << 13, seed=l, ctx=ctx)
        params[l] = res["params"]
        var_z = res["var_Y_minus_r"] + res["var_r"] / kappa
        gain = res["var_Y"] / (var_z * (1 + kappa / 17))
        train[l] = {"s": time.perf_counter() - t1, "var_Y": res["var_Y"], "var_Y_minus_r": res["var_Y_minus_r"],
                    "var_r": res["var_r"], "explained": 1 - res["var_Y_minus_r"] / res["var_Y"],
                    "variance_cost_gain": gain}
        if gain > 1:
            use.append(l)
        print(f"[bench] config4 level {l} trained: explained {train[l]['explained']:.4f}, gain {gain:.3f}",
              file=sys.stderr, flush=True)
    if args.cv_levels is not None:
        use = [int(v) for v in args.cv_levels.split(",") if v]
    mask = sum(1 << l for l in use)
    t_train = time.perf_counter() - t0
    r = dk.estimate(p, args.eps, ctx=ctx, cv_params=params, cv_level_mask=mask, cv_ratio=kappa)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    _report(f"config-4 learned control variate on config-2 pairs l=1..4 (2^16 training pairs per level, "
            f"used on levels {use}), eps={args.eps:g}", wall, "s",
            {"train_s": t_train, "train": train, "cv_levels": use,
             "mlmc": {k: r[k] for k in ("L", "converged", "M", "Yhat", "Vhat", "rmse_est", "rounds", "cell_updates")}})


def bench_config5(args):
    """Throughput scale (config 5): finest grids 256^2, 512^2 and 1024^2 (levels 4..6 of h = 1/16 ..
    1/1024, N = 1e6, T = 26 tau_0), coupled pairs on the streaming kernel (state in HBM, depth
    chosen by the tuner); args.samples pairs at 1024^2 and correspondingly more at the smaller
    grids.  Then every temporal depth (1, 2, 4, 8 fine steps per launch) at 1024^2, pairs and
    single paths, with the algorithmic HBM rate.  Also the noise-free FP32 stencil, which is
    bound by HBM bandwidth."""
    import torch
    import dk_workloads as W
    import paper_2311_08872_amd as dk
    N = args.N or 1e6
    p = W.config5(N=N)
    out = {}
    ctx = dk.Context(0)
    if not args.depth_only:
        dk.level_pair(p, 4, 0, 64, ctx=ctx)                             # warm-up (untimed)
    for l in (() if args.depth_only else (4, 5, 6)):
        cnt = args.samples * 4 ** (6 - l)
        ctx.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dk.level_pair(p, l, 0, cnt, ctx=ctx)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = [s for s in ctx.stats() if s["level"] == l][0]
        cells = st["cell_updates"]
        out[f"{p.n(l)}"] = {"pairs": cnt, "wall_s": wall, "kernel_ms": st["kernel_ms"],
                            "cell_updates_per_s": cells / (st["kernel_ms"] / 1e3),
                            "algorithmic_GB_per_s": 5.0 * cells / (st["kernel_ms"] / 1e3) / 1e9}
        print(f"[bench] config5 {p.n(l)}^2: {out[str(p.n(l))]['cell_updates_per_s']:.3g} cell updates/s",
              file=sys.stderr, flush=True)
    # temporal depth: 128 pairs (and 128 single paths) at 1024^2 over 4096 fine steps per depth.
    # Algorithmic HBM bytes per fine cell update (halo re-reads excluded): single paths 16/D (FP32
    # value and compensation, read and written once per launch); pairs add the coarse state and,
    # at D != 4, the restricted-noise sums that go through HBM: per 4 fine steps D = 1: 64 + 14 + 6,
    # D = 2: 32 + 6 + 6, D = 4: 16 + 4; per 8 fine steps D = 8: 16 + 4 + 12.
    pair_bytes = {1: 84 / 4, 2: 44 / 4, 4: 20 / 4, 8: 32 / 8}
    dsteps = min(4096, 128 * args.samples)              # 4096 at the default --samples 32
    dcount = 4 * args.samples                           # 128 pairs at the default
    ps = p.with_(n0=512, levels=2)                      # the 1024^2 / 512^2 pair as level 1
    ps = ps.with_(T=ps.tau(1) * dsteps, steps_policy=W.STEPS_EXACT)
    assert ps.n(1) == 1024 and ps.steps(1) == dsteps
    depths = {}
    for coupled in (True, False):
        for d in (1, 2, 4, 8):
            ctx.set_stream_depth(d)
            ctx.reset()
            if coupled:
                dk.level_pair(ps, 1, 0, dcount, ctx=ctx)
            else:
                dk.mc_level(ps, 1, 0, dcount, ctx=ctx)
            torch.cuda.synchronize()
            st = [s for s in ctx.stats() if s["level"] == 1][0]
            assert st["rows"] == -d
            fine = st["cell_updates"] / (1 + 1 / 16 if coupled else 1.0)
            rate = st["cell_updates"] / (st["kernel_ms"] / 1e3)
            by = (pair_bytes[d] if coupled else 16.0 / d) * fine / (st["kernel_ms"] / 1e3)
            depths[f"{'pair' if coupled else 'single'}_D{d}"] = {
                "cell_updates_per_s": rate, "algorithmic_bytes_per_fine_update": pair_bytes[d] if coupled else 16.0 / d,
                "algorithmic_GB_per_s": by / 1e9, "frac_of_8TBps": by / 8e12, "kernel_ms": st["kernel_ms"]}
            print(f"[bench] config5 1024^2 {'pair' if coupled else 'single'} depth {d}: {rate:.3g} cell updates/s, "
                  f"{by / 1e9:.0f} GB/s algorithmic ({100 * by / 8e12:.1f} % of 8 TB/s)", file=sys.stderr, flush=True)
    ctx.set_stream_depth(0)
    heat = {}
    for n, batch in (() if args.depth_only else ((256, 4096), (1024, 256))):
        x = torch.ones((batch, n, n), dtype=torch.float32, device="cuda")
        dk.heat_steps(x, 4, p.mu, ctx=ctx)
        dt = dk.heat_steps(x, 64, p.mu, ctx=ctx) / 1e3      # kernel time of the 64 steps
        heat[f"{n}"] = {"batch": batch, "GB_per_s": 8.0 * batch * n * n * 64 / dt / 1e9,
                        "frac_of_8TBps": 8.0 * batch * n * n * 64 / dt / 8e12}
        del x
    ctx.close()
    if args.depth_only:
        _report(f"config-5 streaming depths at 1024^2 ({dcount} pairs / paths, {dsteps} fine steps)",
                depths["pair_D4"]["cell_updates_per_s"], "cell updates/s (pairs, depth 4)", {"depths_1024": depths})
        return
    fin = out[f"{p.n(6)}"]
    _report(f"config-5 throughput: coupled pairs at 256^2, 512^2, 1024^2 (N={N:g}, tau=0.1h^2, "
            f"{args.samples} pairs at 1024^2), streaming kernel", fin["cell_updates_per_s"], "cell updates/s",
            {"grids": out, "depths_1024": depths, "noise_free_stencil": heat})

def bench_counters(args):
    """One launch of each hot kernel at the size it runs in production, for HBM byte counters
    (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE / request sizes, one pass per counter set):
      1. a 256 MiB device copy, twice (the calibration: 256 MiB read and 256 MiB written per launch);
      2. the noise-free FP32 stencil (heat_f32_kernel), 8 steps at 256^2 x 4096 and at 1024^2 x 256
         (one launch per step: 1 GiB read and 1 GiB written algorithmically);
      3. the streaming kernel on 4 pairs and 4 single paths of the 1024^2 / 512^2 pair over 128 fine
         steps at each depth D = 1, 2, 4, 8;
      4. the resident 128^2 pair kernel: one launch of 14024 pairs (the production chunk of the
         config-2 finest level, 8192 fine steps, about 3.3 s).
    Prints one report line with the HIP-event kernel times."""
    import torch
    import dk_workloads as W
    import paper_2311_08872_amd as dk
    out = {}
    src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    ctx = dk.Context(0)
    heat = {}
    for n, batch in ((256, 4096), (1024, 256)):
        x = torch.ones((batch, n, n), dtype=torch.float32, device="cuda")
        ms = dk.heat_steps(x, 8, 0.1, ctx=ctx)
        heat[str(n)] = {"batch": batch, "steps": 8, "kernel_ms": ms, "GB_per_s": 8.0 * batch * n * n * 8 / (ms / 1e3) / 1e9}
        del x
    out["heat_f32"] = heat
    p = W.config5(N=1e6)
    ps = p.with_(n0=512, levels=2)
    ps = ps.with_(T=ps.tau(1) * 128, steps_policy=W.STEPS_EXACT)
    st = {}
    for coupled in (True, False):
        for d in (1, 2, 4, 8):
            ctx.set_stream_depth(d)
            ctx.reset()
            (dk.level_pair if coupled else dk.mc_level)(ps, 1, 0, 4, ctx=ctx)
            torch.cuda.synchronize()
            s_ = [s for s in ctx.stats() if s["level"] == 1][0]
            st[f"{'pair' if coupled else 'single'}_D{d}"] = {"kernel_ms": s_["kernel_ms"], "cell_updates": s_["cell_updates"]}
    ctx.set_stream_depth(0)
    out["stream_1024"] = st
    c2 = W.config2(N=1e4)
    ctx.set_shape(128, 0)
    ctx.reset()
    dk.level_pair(c2, 4, 0, 14024, ctx=ctx)
    torch.cuda.synchronize()
    s_ = [s for s in ctx.stats() if s["level"] == 4][0]
    out["level_128_pair"] = {"pairs": 14024, "launches": s_["launches"], "kernel_ms": s_["kernel_ms"],
                             "fine_cell_updates_per_s": s_["cell_updates"] / (1 + 1 / 16) / (s_["kernel_ms"] / 1e3)}
    ctx.close()
    _report("one production-size launch of each hot kernel (copy calibration, heat_f32, stream, 128^2 pair)",
            out["level_128_pair"]["fine_cell_updates_per_s"], "fine cell updates/s (128^2 pair launch)", out)


if __name__ == "__main__":
    main()
