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

# Algorithmic vector-ALU operations per fine cell update of a coupled pair: half a
# Philox4x32-10 call (40), one binary32 Box--Muller pair (60), the explicit EM update with
# central flux and compensated increment (18), the NN restriction and the amortised coarse
# step (3).
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
    ap.add_argument("--workload", default="config2", choices=["config2", "config3", "config4", "config5"],
                    help="config2 (default): the bench line; the others print a report line: config3 "
                         "low-density MLMC with persistent rounds, config4 learned control variate, "
                         "config5 streaming-kernel throughput at 256^2..1024^2")
    ap.add_argument("--N", type=float, default=None, help="particle number (config3: 1e5, config5: 1e6)")
    ap.add_argument("--samples", type=int, default=32, help="config5: finest-level pairs to time")
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
        {"config3": bench_config3, "config4": bench_config4, "config5": bench_config5}[args.workload](args)
        return
    base = W.config2(N=1e4)

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



def _report(workload, value, unit, extra):
    line = {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "data": "synthetic",
            "config": {"workload": workload}, "report_only": True}
    line.update(extra)
    print(json.dumps(line), flush=True)


def bench_config3(args):
    """Low-density MLMC (config 3): rho0 = max(0, cos 2 pi x) + 0.05, levels 8^2..256^2, 29
    observables (Fourier modes |k| <= 3 and the primary, a squared bump), N = 1e5 and 1e3.
    1. Variance profile: one round of 1000 samples on every level (the resident levels in one
       persistent launch, the 256^2 pairs on the streaming kernel): Y_l and V_l per level show
       the low-density behaviour (V_l stops decreasing once N h^2 rho is small).
    2. Algorithm 1 with persistent rounds.  The primary observable is uncentred and unscaled
       (about 1.5e-4), so the accuracy is relative to its magnitude, estimated by a 1000-sample
       level-0 pilot from another noise stream: 1e-3 at N = 1e5 (reaches 256^2) and 3e-2 at
       N = 1e3 (where the growing V_l make tighter targets cost hours); --N with --eps overrides.
    Reports wall times, the share of wall time outside kernels, the tuner's choices and the
    per-level statistics."""
    import torch
    import dk_workloads as W
    import paper_2311_08872_amd as dk
    runs = [(args.N, args.eps)] if args.N else [(1e5, 1e-3), (1e3, 3e-2)]
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
            Y.append(m.sums[0] / m.count)
            V.append(max(0.0, (m.sums[1] - m.sums[0] ** 2 / m.count) / (m.count - 1)))
        pilot = dk.round_sums(p, 0, [0], [1000], tag=W.TAG_MC, round_mode=3, ctx=ctx)[0][p.primary]
        scale = abs(pilot.sums[2] / pilot.count)
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
    2^16 pairs from its own noise stream, then Algorithm 1 to args.eps with the control variate on
    levels 1..4 (4 independent coarse-only paths per pair).  Wall time includes the training.
    Reports each network's held-out variance ratio Var(Y - r) / Var(Y)."""
    import numpy as np
    import torch
    import dk_workloads as W
    import paper_2311_08872_amd as dk
    p = W.config2(N=1e4)
    ctx = dk.Context(0)
    dk.estimate(p.with_(seed=1000), 2e-2, ctx=ctx)                      # warm-up (untimed)
    ctx.close()
    ctx = dk.Context(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    params = np.zeros((p.levels, dk.L.DK_CNN_NPARAM), np.float32)
    train = {}
    for l in range(1, p.levels):
        t1 = time.perf_counter()
        res = dk.cv_train(p, l, n_train=1 << 16, epochs=6, batch=256, lr=1e-3, n_val=1 << 13, seed=l, ctx=ctx)
        params[l] = res["params"]
        train[l] = {"s": time.perf_counter() - t1, "var_Y": res["var_Y"], "var_Y_minus_r": res["var_Y_minus_r"],
                    "var_r": res["var_r"], "ratio": res["var_Y_minus_r"] / res["var_Y"]}
        print(f"[bench] config4 level {l} trained: ratio {train[l]['ratio']:.4f}", file=sys.stderr, flush=True)
    t_train = time.perf_counter() - t0
    r = dk.estimate(p, args.eps, ctx=ctx, cv_params=params, cv_level_mask=0b11110, cv_ratio=4)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    _report(f"config-4 learned control variate on config-2 pairs l=1..4 (2^16 training pairs per level), "
            f"eps={args.eps:g}", wall, "s",
            {"train_s": t_train, "train": train,
             "mlmc": {k: r[k] for k in ("L", "converged", "M", "Yhat", "Vhat", "rmse_est", "rounds", "cell_updates")}})


def bench_config5(args):
    """Throughput scale (config 5): finest grids 256^2, 512^2 and 1024^2 (levels 4..6 of h = 1/16 ..
    1/1024, N = 1e6, T = 26 tau_0), coupled pairs on the streaming kernel (state in HBM, 4 fine
    steps per launch); args.samples pairs at 1024^2 and correspondingly more at the smaller grids.
    Also the noise-free FP32 stencil, which is bound by HBM bandwidth."""
    import torch
    import dk_workloads as W
    import paper_2311_08872_amd as dk
    N = args.N or 1e6
    p = W.config5(N=N)
    out = {}
    ctx = dk.Context(0)
    dk.level_pair(p, 4, 0, 64, ctx=ctx)                                 # warm-up (untimed)
    for l in (4, 5, 6):
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
    heat = {}
    for n, batch in ((256, 4096), (1024, 256)):
        x = torch.ones((batch, n, n), dtype=torch.float32, device="cuda")
        dk.heat_steps(x, 4, p.mu, ctx=ctx)
        dt = dk.heat_steps(x, 64, p.mu, ctx=ctx) / 1e3      # kernel time of the 64 steps
        heat[f"{n}"] = {"batch": batch, "GB_per_s": 8.0 * batch * n * n * 64 / dt / 1e9,
                        "frac_of_8TBps": 8.0 * batch * n * n * 64 / dt / 8e12}
        del x
    ctx.close()
    fin = out[f"{p.n(6)}"]
    _report(f"config-5 throughput: coupled pairs at 256^2, 512^2, 1024^2 (N={N:g}, tau=0.1h^2, "
            f"{args.samples} pairs at 1024^2), streaming kernel", fin["cell_updates_per_s"], "cell updates/s",
            {"grids": out, "noise_free_stencil": heat})

if __name__ == "__main__":
    main()
