"""Benchmark of the smoothing-step hot path on one MI355X.

Workload (2D, 256 x 256 quadrilaterals, Q2 / P1disc x dG(1), one slab with
tau = 0.01; p = 1.2, delta = 1e-4, nu = 1, nu_inf = 1e-4, Nitsche
gamma1 = gamma2 = 40, sigma_max = 1): the surrogate-tangent (modified Newton)
Jacobian action and one 4-level V-cycle (256^2 -> 32^2, 2 pre + 2 post Vanka
steps, omega = 0.5, dense FP64 coarsest solve).  Linearisation state: smooth
sin-series velocity with 8 random modes plus U[-0.01, 0.01] noise (seed 201),
input vector U[-1, 1] (seed 202).  All inputs are synthetic and resident in
HBM before timing.

One step = one Jacobian action + one V-cycle (every row of the hot path).
Reported value: Jacobian-action throughput in GDoF/s (space-time unknowns per
second) in FP64; FP32 figures and V-cycle seconds alongside.  Kernel time of
the action is measured with HIP events on the stream the kernels run on.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256]
       [--levels 4] [--no-cpu] [--apply-only]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Jacobian-apply GDoF/s + V-cycle s, FP64 vs FP32; p50/p99 solve latency @1e-8"
HBM_PEAK_GBS = 8000.0
MODEL = dict(p=1.2, delta=1e-4, nu=1.0, nu_inf=1e-4, gamma1=40.0, gamma2=40.0, sigma_max=1.0,
             convection=1, qsign=1)


def algorithmic_bytes(sizes, elem):
    """x read + y written + u_k (both Radau nodes) read, per Jacobian action."""
    return (2 * sizes["nst"] + 2 * sizes["nv"]) * elem


def cpu_baseline(n_sample=128, reps=2):
    """The oracle (plain per-cell quadrature C code, one thread) on the same
    parameters and input recipe, on an n_sample^2 mesh."""
    import numpy as np

    from oracle import oracle as O
    from paper_2603_28706_amd import inputs

    n = (n_sample, n_sample)
    prob = O.Problem(n=n, tau=0.01, lin=O.MODIFIED_NEWTON, **{k: v for k, v in MODEL.items()
                                                                if k not in ("qsign",)})
    uk = inputs.sin_series_velocity(n, seed=201, t_nodes=[0.01 / 3, 0.01])
    x = inputs.uniform(202, prob.nst)
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        O.apply(prob, uk, x)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    return {"value": prob.nst / t / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": f"one surrogate-tangent Jacobian action on a {n_sample}x{n_sample} mesh "
                      f"({prob.nst} space-time DoF), same parameters and input recipe, median of "
                      f"{reps}, {t:.2f} s each"}


def run(args):
    import numpy as np
    import torch

    from paper_2603_28706_amd import inputs, pnsmg

    dev = torch.device("cuda:0")
    n = (args.n, args.n)
    uk_np = inputs.sin_series_velocity(n, seed=201, t_nodes=[0.01 / 3, 0.01])
    uk = torch.tensor(uk_np, dtype=torch.float64, device=dev)
    results = {}
    stream = torch.cuda.current_stream(dev)
    for prec, name in ((pnsmg.FP64, "fp64"), (pnsmg.FP32, "fp32")):
        levels = 1 if args.apply_only else args.levels
        ctx = pnsmg.Context(n, n_levels=levels, precision=prec, tau=0.01, device="cuda:0")
        sz = ctx.sizes(0)
        ctx.pns_set_state(dict(MODEL, lin=args.lin), uk)
        x = torch.tensor(inputs.uniform(202, sz["nst"]), dtype=ctx.dtype, device=dev)
        r = torch.tensor(inputs.uniform(203, sz["nst"]), dtype=ctx.dtype, device=dev)
        y = ctx.vector()
        d = ctx.vector()
        t_setup = None
        if not args.apply_only:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.pns_vanka_setup()
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            print(f"[bench] {name}: smoother setup {t_setup:.2f} s", file=sys.stderr, flush=True)

        def step(ev=None):
            if ev is not None:
                ev[0].record(stream)
            ctx.pns_cell_apply(x, y)
            if ev is not None:
                ev[1].record(stream)
            if not args.apply_only:
                ctx.pns_vcycle(2, 2, 0.5, r, d)
            if ev is not None:
                ev[2].record(stream)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
        t0 = time.perf_counter()
        for k in range(args.steps):
            step(evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        t_apply = np.array([e[0].elapsed_time(e[1]) for e in evs]) * 1e-3
        t_vc = np.array([e[1].elapsed_time(e[2]) for e in evs]) * 1e-3
        # dense runs of back-to-back applies for the kernel average, both apply modes
        n_rep = max(50, args.steps)
        t_rep = {}
        for mode in (pnsmg.APPLY_RECOMPUTE, pnsmg.APPLY_CACHED):
            ctx.pns_set_apply_mode(mode)
            ctx.pns_cell_apply(x, y)
            ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ea.record(stream)
            for _ in range(n_rep):
                ctx.pns_cell_apply(x, y)
            eb.record(stream)
            torch.cuda.synchronize()
            t_rep[mode] = ea.elapsed_time(eb) * 1e-3 / n_rep
        t_apply_rep = t_rep[pnsmg.APPLY_CACHED]
        elem = 8 if prec == pnsmg.FP64 else 4
        results[name] = dict(
            nst=sz["nst"], wall_s=wall, ms_per_step=wall / args.steps * 1e3,
            apply_s_median=float(np.median(t_apply)), apply_s_p10=float(np.percentile(t_apply, 10)),
            apply_s_p90=float(np.percentile(t_apply, 90)), apply_s_backtoback=t_apply_rep,
            apply_s_recompute=t_rep[pnsmg.APPLY_RECOMPUTE],
            vcycle_s_median=float(np.median(t_vc)) if not args.apply_only else None,
            setup_s=t_setup, bytes=algorithmic_bytes(sz, elem))
        print(f"[bench] {name}: apply {t_apply_rep * 1e6:.1f} us back-to-back (recompute "
              f"{t_rep[pnsmg.APPLY_RECOMPUTE] * 1e6:.1f} us), "
              f"median in step {np.median(t_apply) * 1e6:.1f} us; V-cycle "
              f"{(np.median(t_vc) * 1e3) if not args.apply_only else 0:.3f} ms",
              file=sys.stderr, flush=True)
        del ctx
        torch.cuda.empty_cache()
    return results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--apply-only", action="store_true")
    ap.add_argument("--lin", type=int, default=2, help="0 Picard, 1 exact Newton, 2 modified Newton")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    res = run(args)
    f64, f32 = res["fp64"], res["fp32"]
    t_ap = f64["apply_s_median"]
    value = f64["nst"] / t_ap / 1e9
    achieved = f64["bytes"] / t_ap / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f64["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"2D {args.n}x{args.n} Q2/P1disc x dG(1) slab, p=1.2 delta=1e-4 "
                         f"nu_inf=1e-4, surrogate-tangent Jacobian action + "
                         f"{args.levels}-level V-cycle (2+2 Vanka, omega=0.5)"),
            "space_time_dof": f64["nst"],
            "levels": args.levels,
        },
        "apply_gdofs_fp64": round(value, 4),
        "apply_gdofs_fp32": round(f32["nst"] / f32["apply_s_median"] / 1e9, 4),
        "apply_us_fp64": round(t_ap * 1e6, 3),
        "apply_us_fp32": round(f32["apply_s_median"] * 1e6, 3),
        "apply_us_back_to_back_fp64_fp32": [round(f64["apply_s_backtoback"] * 1e6, 3),
                                            round(f32["apply_s_backtoback"] * 1e6, 3)],
        "apply_us_recompute_tangent_fp64_fp32": [round(f64["apply_s_recompute"] * 1e6, 3),
                                                 round(f32["apply_s_recompute"] * 1e6, 3)],
        "apply_us_in_step_p10_p50_p90_fp64": [round(f64[k] * 1e6, 2) for k in
                                              ("apply_s_p10", "apply_s_median", "apply_s_p90")],
        "vcycle_s_fp64": f64["vcycle_s_median"],
        "vcycle_s_fp32": f32["vcycle_s_median"],
        "setup_s_fp64": f64["setup_s"],
        "setup_s_fp32": f32["setup_s"],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "cell_apply_kernel<double, modified Newton>"},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
