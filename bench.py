"""Benchmark of the smoothing-step hot path on one MI355X.

Workload (2D, 256 x 256 quadrilaterals, Q2 / P1disc x dG(1), one slab with
tau = 0.01; p = 1.2, delta = 1e-4, nu = 1, nu_inf = 1e-4, Nitsche
gamma1 = gamma2 = 40, sigma_max = 1): the surrogate-tangent (modified Newton)
Jacobian action and one 4-level V-cycle (256^2 -> 32^2, 2 pre + 2 post Vanka
steps, omega = 0.1, dense FP64 coarsest solve).  Linearisation state: smooth
sin-series velocity with 8 random modes plus U[-0.01, 0.01] noise (seed 201),
input vector U[-1, 1] (seed 202).  All inputs are synthetic and resident in
HBM before timing.

One step = a block of four Jacobian actions + one V-cycle (every row of the
hot path).  Reported value: Jacobian-action throughput in GDoF/s (space-time
unknowns per second) in FP64 with the tangent recomputed at every point
(nothing cached), from the mean in-step duration of the action (HIP events on
the stream the kernels run on around the block of four); FP32 figures, the cached-tangent variant and the
V-cycle seconds alongside.  The action's roofline is the FP64 vector ALU
(its arithmetic intensity, ~14 flop/B, is above the FP64 ridge of ~9.8 flop/B).

Beside the step: on 32^3 hexahedra the 3D action, Vanka setup and sweep, a
4-level V-cycle and the 3D slab solve's time to 1e-8 (FP64 and FP32 / mixed);
the 2D slab solve's time to 1e-8, the batched
finest-level Vanka at 512^2 and the request server's latencies, each as a
field of its own in the JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256]
       [--levels 4] [--no-cpu] [--apply-only] [--lin 2] [--calib-copy]
       [--apply3d-n 32] [--solve3d-n 32] [--solve-n 256] [--vanka-n 512]
       [--serve-requests 256]
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
sys.path.insert(0, ROOT)

METRIC = "Jacobian-apply GDoF/s + V-cycle s, FP64 vs FP32; p50/p99 solve latency @1e-8"
HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CUs x 2.4 GHz x 128 FP64 flop / clock
# Jacobian actions per step, timed as one block: as many level-0 operator
# evaluations as a 2 + 2 V-cycle makes (one defect per Vanka step); the block
# also spreads the event overhead so that the per-launch mean is the kernel's
APPLIES_PER_STEP = 4
MODEL = dict(p=1.2, delta=1e-4, nu=1.0, nu_inf=1e-4, gamma1=40.0, gamma2=40.0, sigma_max=1.0,
             convection=1, qsign=1)
OMEGA = 0.1   # Vanka damping of the V-cycle (its cost does not depend on it)
# slab solves on the model of the 256^2 workload (p = 1.2, delta = 1e-4,
# nu_inf = 1e-4, nu = 1): exact finest-level patches, omega 0.2, refresh 0.9
SOLVE_MODEL = dict(MODEL, lin=2)
SOLVE_SEEDS = (201, 202, 203)


def algorithmic_bytes(sizes, elem):
    """x read + y written + u_k (both Radau nodes) read, per Jacobian action."""
    return (2 * sizes["nst"] + 2 * sizes["nv"]) * elem


# FETCH_SIZE / WRITE_SIZE of the FP64 action (mean over its launches), each
# scaled by the counter's reading for a plain streaming kernel of known size,
# with the hash of the kernel source the counters were taken on; one summary
# per mesh size
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "cell_apply_{n}x{n}_fp64_counters.md")
# the action kernel's own source and its elementary functions (the element
# constants it includes are fixed by the discretisation)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2603_28706_amd", "csrc", f)
                  for f in ("apply.hip", "devmath.h")]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(n):
    """HBM bytes per launch of the action on the n x n mesh from the committed
    counter summary; None if there is none for that size or the kernel source
    changed since it was taken."""
    try:
        with open(TRAFFIC_SUMMARY.format(n=n)) as fh:
            txt = fh.read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", txt, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("traffic_bytes_per_launch")


def tangent_flops(lin):
    """FP64 operations of the tangent scalars at one point (FMA = 2; the
    elementary functions at the operation counts of their evaluation:
    log 39, exp 33, plus |A|^2 6, Delta^2 1, mu 2, eta 1; exact Newton adds
    the reciprocal of Delta^2 and kappa (11), modified Newton also the clip
    sigma_max / |A| and the min (13))."""
    return {0: 82, 1: 93, 2: 106}[lin]


def apply_flops_per_cell(lin):
    """Algorithmic operations of the sum-factorised volume action per cell
    (both Radau nodes; the O(N) boundary faces and the halo recomputation of
    the tiles are not counted).  Per Radau node and Gauss row: contraction of
    x and u_k along y (9 nodes x 8 FMA = 144), three points, the transposed
    contraction onto the 9 nodes (2 x 9 x 2 FMA = 72) and its summation (18).
    Per point: contraction along x (72), temporal mass coupling (6), gradient
    scalings and symmetric parts (12), weights (3), pressure value (4),
    tangent, rank-one part and T(B) (18 Newton / 5 Picard), convection
    (16 Newton / 8 Picard), quadrature scalings (8), mass values (2),
    divergence and pressure rows (7), test-coefficient sums (36)."""
    newton = lin != 0
    point = (72 + 6 + 12 + 3 + 4 + tangent_flops(lin) + (18 if newton else 5)
             + (16 if newton else 8) + 8 + 2 + 7 + 36)
    return 2 * 3 * (144 + 3 * point + 72 + 18)


def apply3d_flops_per_cell(lin):
    """Algorithmic operations of the sum-factorised 3D volume action per
    hexahedron (both Radau nodes; the boundary faces and the gather over cells
    are not counted).  Forward contractions of 12 fields (x and u_k, 3
    components, 2 Radau nodes) on 9 lines each: along x 2 outputs, along y 3,
    along z 4, at 3 points with 3 FMA each (3888 + 5832 + 7776).  Per point
    and Radau node (54): gradient scalings (18), symmetric parts (36), tangent
    scalars (those of the 2D count plus 12 for the longer |A|^2), A:B (18),
    kappa A:B (1), pressure value (6), temporal mass coupling (12), test
    coefficients of the 9 gradient entries (84 Newton / 66 Picard), divergence
    and pressure-row terms (7), weights (4); pressure-row sums over the 27
    points (216).  Transposed contractions onto the 81 velocity tests per
    Radau node: along z 12 FMA, along y 9, along x 6 per line and node
    (3888 + 2916 + 1944)."""
    newton = lin != 0
    point = 18 + 36 + tangent_flops(lin) + 12 + 18 + 1 + 6 + 12 + (84 if newton else 66) + 7 + 4
    return 3888 + 5832 + 7776 + 54 * point + 216 + 3888 + 2916 + 1944


MODEL3D = dict(p=1.3, delta=1e-3, nu=1.0, nu_inf=1e-3, gamma1=40.0, gamma2=40.0, sigma_max=1.0,
               convection=1, qsign=1)


OMEGA3D = 0.15


def apply3d(n=32, reps=50, lin=2, smoother=True, sweeps=20, vcycles=10, levels3d=4):
    """3D action on n^3 hexahedra (Q2 / P1disc x dG(1), tau = 0.01) with
    p = 1.3, delta = 1e-3, nu = 1, nu_inf = 1e-3; state: 3D sin-series
    velocity (8 modes, seed 301, O(tau) time variation), input U[-1, 1]
    (seed 302).  Mean duration of `reps` back-to-back actions (HIP events on
    the stream the kernels run on), BF16 storage (x and u_k, FP32 arithmetic,
    FP32 y), FP64 and FP32; then the finest-level
    Vanka smoother: setup wall time (all levels of the `levels3d`-level
    hierarchy) and the mean of `sweeps` sweeps (residual U[-1, 1], seed 303,
    omega = 0.5); then the mean of `vcycles` V-cycles (2 + 2 sweeps, omega
    0.15)."""
    import torch

    from paper_2603_28706_amd import inputs, pnsmg

    uk = torch.tensor(inputs.sin_series_velocity((n, n, n), seed=301, t_nodes=[0.01 / 3, 0.01]),
                      device="cuda")
    out = {}
    # BF16 storage of x and u_k, FP32 arithmetic: the action only
    ctx = pnsmg.Context((n, n, n), precision=pnsmg.BF16)
    ctx.pns_set_state(dict(MODEL3D, lin=lin), uk)
    sz = ctx.sizes()
    xb = torch.tensor(inputs.uniform(302, sz["nst"]), device="cuda").to(torch.bfloat16)
    y = ctx.vector()
    for _ in range(3):
        ctx.pns_cell_apply(xb, y)
    stream = torch.cuda.current_stream()
    ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ea.record(stream)
    for _ in range(reps):
        ctx.pns_cell_apply(xb, y)
    eb.record(stream)
    torch.cuda.synchronize()
    t = ea.elapsed_time(eb) * 1e-3 / reps
    bytes_bf16 = 2 * sz["nst"] + 4 * sz["nst"] + 2 * 2 * sz["nv"]
    out["bf16"] = dict(us_mean=t * 1e6, gdofs=sz["nst"] / t / 1e9,
                       tflops=apply3d_flops_per_cell(lin) * sz["cells"] / t / 1e12,
                       hbm_gbs=bytes_bf16 / t / 1e9)
    print(f"[bench] 3D action {n}^3 bf16 storage: {t * 1e6:.1f} us, {sz['nst'] / t / 1e9:.2f} GDoF/s",
          file=sys.stderr, flush=True)
    del ctx
    for prec, name in ((pnsmg.FP64, "fp64"), (pnsmg.FP32, "fp32")):
        ctx = pnsmg.Context((n, n, n), precision=prec, n_levels=levels3d if smoother else 1)
        ctx.pns_set_state(dict(MODEL3D, lin=lin), uk)
        sz = ctx.sizes()
        x = torch.tensor(inputs.uniform(302, sz["nst"]), dtype=ctx.dtype, device="cuda")
        y = ctx.vector()
        for _ in range(3):
            ctx.pns_cell_apply(x, y)
        stream = torch.cuda.current_stream()
        ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ea.record(stream)
        for _ in range(reps):
            ctx.pns_cell_apply(x, y)
        eb.record(stream)
        torch.cuda.synchronize()
        t = ea.elapsed_time(eb) * 1e-3 / reps
        flops = apply3d_flops_per_cell(lin) * sz["cells"]
        # tflops: the volume-term operation count over the whole action's time
        out[name] = dict(us_mean=t * 1e6, gdofs=sz["nst"] / t / 1e9,
                         tflops=flops / t / 1e12,
                         hbm_gbs=algorithmic_bytes(sz, 8 if prec == pnsmg.FP64 else 4) / t / 1e9)
        out["space_time_dof"] = sz["nst"]
        out["flop_per_apply"] = flops
        print(f"[bench] 3D action {n}^3 {name}: {t * 1e6:.1f} us, {sz['nst'] / t / 1e9:.2f} GDoF/s",
              file=sys.stderr, flush=True)
        if smoother:
            # finest-level Vanka smoother: setup (cell matrices at the midpoint
            # state + batched complex 85 x 85 inversions), then sweeps
            # (defect by the action + 8 colour launches of patch solves)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.pns_vanka_setup()
            torch.cuda.synchronize()
            setup_s = time.perf_counter() - t0
            r = torch.tensor(inputs.uniform(303, sz["nst"]), dtype=ctx.dtype, device="cuda")
            d = ctx.vector()
            for _ in range(2):
                ctx.pns_vanka_smooth(0, 1, 0.5, r, d)
            torch.cuda.synchronize()
            ea.record(stream)
            for _ in range(sweeps):
                ctx.pns_vanka_smooth(0, 1, 0.5, r, d)
            eb.record(stream)
            torch.cuda.synchronize()
            ts = ea.elapsed_time(eb) * 1e-3 / sweeps
            es = 8 if prec == pnsmg.FP64 else 4
            factor_bytes = sz["cells"] * 2 * 85 * 85 * es
            # the patch part: sweep time less one action (the defect)
            tp = max(ts - t, 1e-9)
            out[name].update(vanka_setup_s=setup_s, sweep_us=ts * 1e6, patch_part_us=tp * 1e6,
                             factor_bytes=factor_bytes, factor_gbs=factor_bytes / tp / 1e9)
            print(f"[bench] 3D Vanka {n}^3 {name}: setup {setup_s:.3f} s (all {levels3d} levels), "
                  f"sweep {ts * 1e6:.1f} us (patch part {tp * 1e6:.1f} us, "
                  f"{factor_bytes / tp / 1e9:.0f} GB/s on factors)", file=sys.stderr, flush=True)
            # V-cycle over the hierarchy (2 + 2 sweeps, damping 0.15: a vertex lies
            # in 8 cell patches)
            for _ in range(2):
                ctx.pns_vcycle(2, 2, OMEGA3D, r, d)
            torch.cuda.synchronize()
            ea.record(stream)
            for _ in range(vcycles):
                ctx.pns_vcycle(2, 2, OMEGA3D, r, d)
            eb.record(stream)
            torch.cuda.synchronize()
            tv = ea.elapsed_time(eb) * 1e-3 / vcycles
            # the same V-cycle replayed from one captured HIP graph
            ctx.pns_set_vcycle_graph(1)
            for _ in range(2):
                ctx.pns_vcycle(2, 2, OMEGA3D, r, d)  # capture, then one replay
            torch.cuda.synchronize()
            ea.record(stream)
            for _ in range(vcycles):
                ctx.pns_vcycle(2, 2, OMEGA3D, r, d)
            eb.record(stream)
            torch.cuda.synchronize()
            tg = ea.elapsed_time(eb) * 1e-3 / vcycles
            ctx.pns_set_vcycle_graph(0)
            out[name].update(vcycle_ms=tv * 1e3, vcycle_graph_ms=tg * 1e3)
            out["levels"] = levels3d
            out["omega"] = OMEGA3D
            print(f"[bench] 3D V-cycle {n}^3 {name}: {tv * 1e3:.3f} ms (graph-replayed "
                  f"{tg * 1e3:.3f} ms)", file=sys.stderr, flush=True)
        del ctx
        torch.cuda.empty_cache()
    return out


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_sample=256, reps_all=3):
    """The oracle (plain per-cell quadrature C code, no sum factorisation) on the
    benchmark's own parameters, input recipe and mesh: one action on one thread,
    and the median of `reps_all` actions on every core this process may run on
    (the same per-cell code over the cells in parity classes).  A correctness
    baseline, not a tuned CPU code."""
    import numpy as np

    from oracle import oracle as O
    from paper_2603_28706_amd import inputs

    n = (n_sample, n_sample)
    prob = O.Problem(n=n, tau=0.01, lin=O.MODIFIED_NEWTON, **{k: v for k, v in MODEL.items()
                                                                if k not in ("qsign",)})
    uk = inputs.sin_series_velocity(n, seed=201, t_nodes=[0.01 / 3, 0.01])
    x = inputs.uniform(202, prob.nst)
    cores = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit():
        cores = min(cores, int(omp))
    t0 = time.perf_counter()
    O.apply(prob, uk, x)
    t1 = time.perf_counter() - t0
    times = []
    for _ in range(reps_all):
        t0 = time.perf_counter()
        O.apply_threads(prob, uk, x, cores)
        times.append(time.perf_counter() - t0)
    tn = float(np.median(times))
    print(f"[bench] oracle action {n_sample}^2: 1 thread {t1:.2f} s, {cores} threads {tn:.2f} s",
          file=sys.stderr, flush=True)
    return {"value": prob.nst / tn / 1e9, "unit": "GDoF/s", "cores": cores, "kind": "oracle",
            "sample": f"one surrogate-tangent Jacobian action on the benchmark's {n_sample}x"
                      f"{n_sample} mesh ({prob.nst} space-time DoF), same parameters and input "
                      f"recipe; {cores} threads: median of {reps_all}, {tn:.2f} s each",
            "single_core": {"value": prob.nst / t1 / 1e9, "cores": 1, "seconds": round(t1, 3)},
            "cpu_model": host_cpu_model()}


def measured_copy_gbs(nbytes=2 << 30, reps=10):
    """HBM bandwidth of a plain device-to-device copy (read + write bytes per
    second), the measured counterpart of the nominal 8 TB/s."""
    import torch

    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    b.record(stream)
    torch.cuda.synchronize()
    t = a.elapsed_time(b) * 1e-3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / t / 1e9


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

        if args.calib_copy:
            # plain streaming kernel of known size (reads and writes nst values)
            # for the calibration of the memory-traffic counters
            scratch = torch.empty_like(x)
            for _ in range(3):
                torch.neg(x, out=scratch)
            torch.cuda.synchronize()
            del scratch

        def step(ev=None):
            if ev is not None:
                ev[0].record(stream)
            for _ in range(APPLIES_PER_STEP):
                ctx.pns_cell_apply(x, y)
            if ev is not None:
                ev[1].record(stream)
            if not args.apply_only:
                ctx.pns_vcycle(2, 2, OMEGA, r, d)
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
        t_apply = np.array([e[0].elapsed_time(e[1]) for e in evs]) * 1e-3 / APPLIES_PER_STEP
        t_vc = np.array([e[1].elapsed_time(e[2]) for e in evs]) * 1e-3
        # back-to-back applies with the cached-tangent variant (reported alongside)
        n_rep = max(50, args.steps)
        ctx.pns_set_apply_mode(pnsmg.APPLY_CACHED)
        ctx.pns_cell_apply(x, y)
        ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ea.record(stream)
        for _ in range(n_rep):
            ctx.pns_cell_apply(x, y)
        eb.record(stream)
        torch.cuda.synchronize()
        t_cached = ea.elapsed_time(eb) * 1e-3 / n_rep
        ctx.pns_set_apply_mode(pnsmg.APPLY_RECOMPUTE)
        # back-to-back applies in the fixed summation order (reported alongside)
        ctx.pns_set_reproducible(1)
        ctx.pns_cell_apply(x, y)
        ea.record(stream)
        for _ in range(n_rep):
            ctx.pns_cell_apply(x, y)
        eb.record(stream)
        torch.cuda.synchronize()
        t_ordered = ea.elapsed_time(eb) * 1e-3 / n_rep
        ctx.pns_set_reproducible(0)
        # the same V-cycle replayed from one captured HIP graph (reported alongside)
        t_vc_graph = None
        if not args.apply_only:
            ctx.pns_set_vcycle_graph(1)
            ctx.pns_vcycle(2, 2, OMEGA, r, d)   # capture
            torch.cuda.synchronize()
            tg = []
            for _ in range(max(20, args.steps // 2)):
                ga, gb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ga.record(stream)
                ctx.pns_vcycle(2, 2, OMEGA, r, d)
                gb.record(stream)
                tg.append((ga, gb))
            torch.cuda.synchronize()
            t_vc_graph = float(np.median([a.elapsed_time(b) for a, b in tg])) * 1e-3
            ctx.pns_set_vcycle_graph(0)
        # the benchmarked V-cycle as a stationary iteration x <- x + V(b - A x) on a
        # consistent system b = A x_true from x = 0 (the operator has the constant
        # pressure as null vector, so b is taken in its range): geometric mean of
        # the residual reduction per V-cycle over 10 V-cycles, and the last ratio
        rho_vc = None
        if not args.apply_only:
            xt = torch.tensor(inputs.uniform(204, sz["nst"]), dtype=ctx.dtype, device=dev)
            bt, xs, res = ctx.vector(), ctx.vector(), ctx.vector()
            ctx.pns_cell_apply(xt, bt)
            res.copy_(bt)
            norms = [float(torch.linalg.vector_norm(res.double()))]
            for _ in range(10):
                ctx.pns_vcycle(2, 2, OMEGA, res, d)
                xs += d
                ctx.pns_cell_defect(bt, xs, res)
                norms.append(float(torch.linalg.vector_norm(res.double())))
            rho_vc = dict(mean=(norms[-1] / norms[0]) ** 0.1, last=norms[-1] / norms[-2])
            del xt, bt, xs, res
        elem = 8 if prec == pnsmg.FP64 else 4
        results[name] = dict(
            nst=sz["nst"], cells=sz["cells"], wall_s=wall, ms_per_step=wall / args.steps * 1e3,
            apply_s_mean=float(np.mean(t_apply)), apply_s_median=float(np.median(t_apply)),
            apply_s_p10=float(np.percentile(t_apply, 10)),
            apply_s_p90=float(np.percentile(t_apply, 90)), apply_s_cached=t_cached,
            apply_s_ordered=t_ordered,
            vcycle_s_median=float(np.median(t_vc)) if not args.apply_only else None,
            vcycle_s_graph=t_vc_graph, setup_s=t_setup, bytes=algorithmic_bytes(sz, elem),
            vcycle_rho=rho_vc)
        print(f"[bench] {name}: apply {np.mean(t_apply) * 1e6:.1f} us mean in step "
              f"(p50 {np.median(t_apply) * 1e6:.1f}), cached tangent {t_cached * 1e6:.1f} us "
              f"back-to-back; V-cycle "
              f"{(np.median(t_vc) * 1e3) if not args.apply_only else 0:.3f} ms (graph-replayed "
              f"{(t_vc_graph or 0) * 1e3:.3f} ms)", file=sys.stderr, flush=True)
        del ctx
        torch.cuda.empty_cache()
    return results


def vcycle_marked(args):
    """The benchmarked V-cycle alone (FP64, then FP32): smoother setup, 5
    warm-up V-cycles, then args.steps V-cycles between two launches of
    torch.flip, which mark them in a kernel trace.  Returns the event-timed
    median per V-cycle and precision."""
    import numpy as np
    import torch

    from paper_2603_28706_amd import inputs, pnsmg

    dev = torch.device("cuda:0")
    n = (args.n, args.n)
    uk = torch.tensor(inputs.sin_series_velocity(n, seed=201, t_nodes=[0.01 / 3, 0.01]),
                      dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    out = {}
    for prec, name in ((pnsmg.FP64, "fp64"), (pnsmg.FP32, "fp32")):
        ctx = pnsmg.Context(n, n_levels=args.levels, precision=prec, tau=0.01, device="cuda:0")
        ctx.pns_set_state(dict(MODEL, lin=args.lin), uk)
        ctx.pns_vanka_setup()
        sz = ctx.sizes(0)
        r = torch.tensor(inputs.uniform(203, sz["nst"]), dtype=ctx.dtype, device=dev)
        d = ctx.vector()
        for _ in range(5):
            ctx.pns_vcycle(2, 2, OMEGA, r, d)
        mark = torch.arange(8, device=dev)
        torch.cuda.synchronize()
        torch.flip(mark, dims=[0])
        evs = []
        for _ in range(args.steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ctx.pns_vcycle(2, 2, OMEGA, r, d)
            b.record(stream)
            evs.append((a, b))
        torch.flip(mark, dims=[0])
        torch.cuda.synchronize()
        out[name] = {"vcycles": args.steps,
                     "median_ms": float(np.median([a.elapsed_time(b) for a, b in evs]))}
        print(f"[bench] marked V-cycles {name}: {out[name]}", file=sys.stderr, flush=True)
        del ctx
        torch.cuda.empty_cache()
    return out


def solve_latency(n, seeds, rtol=1e-8):
    """Time-to-rtol of independent slab solves (Newton-FGMRES, one V-cycle per
    Krylov step) at n x n, one per seed of the left-trace velocity, in FP64
    and mixed precision (FP32 action and V-cycle inside FP64 Newton/FGMRES)."""
    import numpy as np
    import torch

    from paper_2603_28706_amd import inputs, pnsmg

    levels = max(1, int(np.log2(n // 8)) + 1)   # coarsest level 8 x 8
    out = {}
    for prec, name in ((pnsmg.FP64, "fp64"), (pnsmg.FP32, "mixed")):
        ctx = pnsmg.Context((n, n), n_levels=levels, precision=prec, patch_kind=pnsmg.PATCH_EXACT)
        sz = ctx.sizes(0)
        lat, newton, krylov, ok = [], [], [], 0
        for seed in seeds:
            vprev = inputs.sin_series_velocity((n, n), seed=seed, t_nodes=[0.0])
            U0 = np.zeros(sz["nst"])
            U0[:sz["nv"]] = vprev
            U0[sz["ns"]:sz["ns"] + sz["nv"]] = vprev
            U = torch.tensor(U0, device="cuda")
            vp = torch.tensor(vprev, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, info = ctx.pns_solve(SOLVE_MODEL, vp, U, rtol=rtol, omega=SERVE_OMEGA,
                                     rho=SERVE_RHO, max_newton=80, max_krylov=150)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
            ok += rc == pnsmg.PNS_OK
            newton.append(info["newton_iterations"])
            krylov.append(info["krylov_iterations"])
        out[name] = dict(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                         converged=f"{ok}/{len(seeds)}", newton_mean=float(np.mean(newton)),
                         krylov_mean=float(np.mean(krylov)))
        print(f"[bench] solve {name} {n}x{n}: p50 {out[name]['p50_s']:.3f} s, p99 "
              f"{out[name]['p99_s']:.3f} s, converged {out[name]['converged']}, Newton "
              f"{np.mean(newton):.1f}, FGMRES {np.mean(krylov):.1f}", file=sys.stderr, flush=True)
        del ctx
        torch.cuda.empty_cache()
    return out


def exact_setup3d(n=32, reps=3):
    """Time of the FP64 smoother setup with exact finest-level patches on n^3
    hexahedra, 4 levels (the setup a 3D slab-solve refresh repeats): cell
    matrices, n^3 level-0 170 x 170 patch inversions (blocked Gauss-Jordan on
    the FP64 matrix cores), Galerkin products, coarse patches, the dense
    coarsest inverse.  State: the 3D sin-series velocity (seed 301)."""
    import torch

    from paper_2603_28706_amd import inputs, pnsmg

    ctx = pnsmg.Context((n, n, n), n_levels=4, precision=pnsmg.FP64, patch_kind=pnsmg.PATCH_EXACT)
    uk = torch.tensor(inputs.sin_series_velocity((n, n, n), seed=301,
                                                 t_nodes=[0.01 / 3, 0.01]), device="cuda")
    ctx.pns_set_state(dict(MODEL3D, lin=2), uk)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.pns_vanka_setup()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    print(f"[bench] exact 3D setup {n}^3: {[round(t * 1e3, 1) for t in ts]} ms", file=sys.stderr,
          flush=True)
    del ctx
    torch.cuda.empty_cache()
    return dict(patches_level0=n ** 3, setup_ms_median=round(1e3 * sorted(ts)[len(ts) // 2], 2))


def solve3d_latency(n=32, rtol=1e-8, max_newton=60, rho=0.9):
    """Time to rtol of the 3D slab solve on n^3 hexahedra (the 3D workload:
    p = 1.3, delta = 1e-3, nu = 1, nu_inf = 1e-3, modified Newton, left trace
    = 3D sin-series velocity, seed 301), 4-level V-cycle (coarsest n/8 cubed)
    with exact finest-level patches (the two Radau velocities of the iterates
    differ by O(1) in this regime, where midpoint-frozen patches stall the
    Krylov solves), damping 0.15, smoother rebuilt when a Newton step reduces
    the residual by less than rho = 0.9 (the clipped tangent contracts by
    ~0.55 per step, so rho = 0.5 would rebuild at every step); FP64 and mixed
    precision, and mixed precision whose FGMRES applies the Jacobian with x and
    u_k stored in BF16 (FP32 arithmetic)."""
    import torch

    from paper_2603_28706_amd import inputs, pnsmg

    model = dict(MODEL3D, lin=2)
    vprev = torch.tensor(inputs.sin_series_velocity((n, n, n), seed=301, t_nodes=[0.0]),
                         device="cuda")
    out = {}
    for prec, name, jac in ((pnsmg.FP64, "fp64", None), (pnsmg.FP32, "mixed", None),
                            (pnsmg.FP32, "mixed_bf16_jacobian", pnsmg.BF16)):
        ctx = pnsmg.Context((n, n, n), n_levels=4, precision=prec, patch_kind=pnsmg.PATCH_EXACT)
        if jac is not None:
            ctx.pns_set_jacobian_precision(jac)
        sz = ctx.sizes()
        U = torch.zeros(sz["nst"], dtype=torch.float64, device="cuda")
        U[:sz["nv"]] = vprev
        U[sz["ns"]:sz["ns"] + sz["nv"]] = vprev
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, info = ctx.pns_solve(model, vprev, U, rtol=rtol, omega=OMEGA3D, max_newton=max_newton,
                                 rho=rho)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out[name] = dict(time_s=t, converged=bool(rc == pnsmg.PNS_OK), **info)
        print(f"[bench] 3D solve {n}^3 {name}: {t:.2f} s, rc {rc}, {info}", file=sys.stderr,
              flush=True)
        del ctx
        torch.cuda.empty_cache()
    return out


# serving workload: the request distribution of the serving configuration
# (p ~ U[1.1, 1.9], delta ~ logU[1e-5, 1e-1], nu_inf ~ logU[1e-4, 1e-2]) with
# nu = 1; exact finest-level patches and omega = 0.2, the smoother setting that
# converges on the most requests of this distribution (low p needs up to ~45
# Newton steps of the clipped tangent)
SERVE_MODEL = dict(nu=1.0, gamma1=40.0, gamma2=40.0, sigma_max=1.0, convection=1, qsign=1, lin=2)
SERVE_OMEGA = 0.2
# smoother refresh threshold of the 2D solves: a smoother from an earlier
# iterate preconditions the quadrilateral solves poorly (rho = 0.9 measured
# 4.5x more FGMRES iterations at 256^2), so the default 0.5 is kept
SERVE_RHO = 0.5


def serve_latency(n_req=256, rate=20.0, slots=8, seed=501):
    """Poisson stream of independent slab-solve requests through the native
    request server: meshes from {32^2, 64^2, 128^2, 256^2}, p ~ U[1.1, 1.9],
    delta ~ logU[1e-5, 1e-1], nu_inf ~ logU[1e-4, 1e-2], nu = 1, left traces
    from the sin-series recipe (seed 501 + i), each solved to 1e-8 (modified
    Newton, FGMRES / V-cycle with exact finest patches, omega 0.2, at most 60
    Newton steps).  Two runs of the same stream with `slots` concurrent
    requests: FP64 and mixed precision.  Every request counts: latency is
    completion - submission whether it converged or stopped with
    PNS_ENOTCONV, and the converged count is reported."""
    import numpy as np

    from paper_2603_28706_amd import inputs, pnsmg

    rng = inputs.rng(seed)
    sizes = [32, 64, 128, 256]
    reqs = []
    for i in range(n_req):
        n = int(sizes[rng.integers(0, 4)])
        model = dict(SERVE_MODEL, p=float(rng.uniform(1.1, 1.9)),
                     delta=float(10 ** rng.uniform(-5, -1)),
                     nu_inf=float(10 ** rng.uniform(-4, -2)))
        reqs.append((n, model, seed + i))
    gaps = rng.exponential(1.0 / rate, n_req)
    arrivals = np.cumsum(gaps) - gaps[0]
    vps = [inputs.sin_series_velocity((n, n), seed=sd, t_nodes=[0.0]) for n, _, sd in reqs]
    out = {}
    for name, prec in (("fp64", pnsmg.FP64), ("mixed", pnsmg.FP32)):
        srv = pnsmg.Server(slots=slots, arena_bytes=48 << 30)
        tickets = []
        t0 = time.perf_counter()
        for (n, model, _), vp, ta in zip(reqs, vps, arrivals):
            dt = t0 + ta - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            U = np.zeros(2 * (2 * (2 * n + 1) ** 2 + 3 * n * n))
            levels = max(1, int(np.log2(n // 8)) + 1)
            q = pnsmg.make_request((n, n), model, vp, U, levels, precision=prec,
                                   patch_kind=pnsmg.PATCH_EXACT, omega=SERVE_OMEGA, max_newton=60,
                                   max_krylov=150, rho=SERVE_RHO)
            tickets.append(srv.submit(q, keep=(vp, U)))
        res = [srv.wait(t) for t in tickets]
        srv.close()
        lat = np.array([r["t_done"] - r["t_submit"] for r in res])
        span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
        dof = sum(2 * (2 * (2 * n + 1) ** 2 + 3 * n * n) for n, _, _ in reqs)
        ok = sum(r["status"] == pnsmg.PNS_OK for r in res)
        failed = [dict(n=n, p=round(m["p"], 3), delta=float(f"{m['delta']:.2e}"),
                       nu_inf=float(f"{m['nu_inf']:.2e}"), status=r["status"],
                       newton=r["newton_iterations"])
                  for (n, m, _), r in zip(reqs, res) if r["status"] != pnsmg.PNS_OK]
        out[name] = dict(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                         solves_per_s=n_req / span, mdof_per_s=dof / span / 1e6,
                         converged=f"{ok}/{n_req}", slots=slots,
                         newton_mean=float(np.mean([r["newton_iterations"] for r in res])),
                         not_converged=failed)
        print(f"[bench] serve {name}: p50 {out[name]['p50_s']:.3f} s, p99 "
              f"{out[name]['p99_s']:.3f} s, {out[name]['solves_per_s']:.2f} solves/s, "
              f"converged {ok}/{n_req}", file=sys.stderr, flush=True)
    return out


def batched_vanka(n=512, sweeps=20):
    """Finest-level smoother alone at n x n in FP32 with boundary-truncated
    (uneven) patches: patch entries from the surrogate tangent at p = 1.1,
    delta = 1e-5, nu_inf = 1e-4 (state: sin-series, seed 401; masks seed 402).
    Setup (element matrices + batched patch factorisation + sweep autotuning)
    and one additive Vanka step (global defect + all patch solves), for the
    midpoint-frozen surrogate patches (complex 21x21 time-diagonal factors)
    and the exact 42x42 patches.  Factor GB/s = factor bytes / (step -
    defect).  The step is timed with the autotuned sweep shape and again with
    variant 0 (the fixed shape: three complex patches or one real patch per
    wave, four waves per workgroup)."""
    import numpy as np
    import torch

    from paper_2603_28706_amd import inputs, pnsmg

    model = dict(MODEL, p=1.1, delta=1e-5, nu_inf=1e-4, lin=2)
    uk = torch.tensor(inputs.sin_series_velocity((n, n), seed=401, t_nodes=[0.01 / 3, 0.01]),
                      device="cuda")
    masks = pnsmg.masks_to_bits(inputs.truncation_masks((n, n), seed=402))
    out = {}
    for kind, name, vals in ((pnsmg.PATCH_SURROGATE, "surrogate_complex21", 2 * 21 * 21),
                             (pnsmg.PATCH_EXACT, "exact_real42", 42 * 42)):
        ctx = pnsmg.Context((n, n), n_levels=1, precision=pnsmg.FP32)
        ctx.pns_set_patch_kind(kind)
        ctx.pns_set_state(model, uk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.pns_vanka_setup(masks)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        r = torch.tensor(inputs.uniform(403, ctx.sizes()["nst"]), dtype=torch.float32, device="cuda")
        d = ctx.vector()
        y = ctx.vector()
        ctx.pns_vanka_smooth(0, 1, OMEGA, r, d)
        ea, eb, ec = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        stream = torch.cuda.current_stream()
        ea.record(stream)
        for _ in range(sweeps):
            ctx.pns_vanka_smooth(0, 1, OMEGA, r, d)
        eb.record(stream)
        for _ in range(sweeps):
            ctx.pns_cell_defect(r, d, y)
        ec.record(stream)
        torch.cuda.synchronize()
        t_step = ea.elapsed_time(eb) * 1e-3 / sweeps
        t_def = eb.elapsed_time(ec) * 1e-3 / sweeps
        # the autotuned sweep shape against variant 0 (the fixed shape it replaces)
        tuned = ctx.pns_sweep_variant(0)
        times = [ctx.pns_sweep_variant_time(0, v) for v in range(tuned["count"])]
        ctx.pns_set_sweep_variant(0, 0)
        ctx.pns_vanka_smooth(0, 1, OMEGA, r, d)
        ea.record(stream)
        for _ in range(sweeps):
            ctx.pns_vanka_smooth(0, 1, OMEGA, r, d)
        eb.record(stream)
        torch.cuda.synchronize()
        t_step0 = ea.elapsed_time(eb) * 1e-3 / sweeps
        fbytes = n * n * vals * 4
        out[name] = dict(setup_s=t_setup, step_ms=t_step * 1e3, defect_ms=t_def * 1e3,
                         factor_mb=fbytes / 1e6, factor_gbs=fbytes / max(t_step - t_def, 1e-9) / 1e9,
                         step_ms_variant0=t_step0 * 1e3,
                         autotuned_variant=tuned["variant"], waves_per_workgroup=tuned["waves"],
                         loads_in_flight=tuned["unroll"], rows_per_lane=tuned["rows"],
                         variant_step_ms=[round(t, 4) for t in times])
        print(f"[bench] batched Vanka {n}x{n} {name}: setup {t_setup:.3f} s, step "
              f"{t_step * 1e3:.3f} ms (defect {t_def * 1e3:.3f} ms), factors "
              f"{fbytes / 1e6:.0f} MB at {out[name]['factor_gbs']:.0f} GB/s; autotuned {tuned}, "
              f"variant 0 step {t_step0 * 1e3:.3f} ms", file=sys.stderr, flush=True)
        del ctx
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--apply-only", action="store_true")
    ap.add_argument("--solve-n", type=int, default=256,
                    help="mesh of the slab-solve latency measurement (0: skip)")
    ap.add_argument("--vanka-n", type=int, default=512,
                    help="mesh of the batched-Vanka measurement (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests of the serving measurement (0: skip)")
    ap.add_argument("--solve3d-n", type=int, default=32,
                    help="3D slab solve to 1e-8 on n^3 (0 skips it)")
    ap.add_argument("--apply3d-n", type=int, default=32,
                    help="mesh of the 3D action measurement, n^3 hexahedra (0: skip)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain streaming kernel of known size (counter calibration)")
    ap.add_argument("--lin", type=int, default=2, help="0 Picard, 1 exact Newton, 2 modified Newton")
    ap.add_argument("--setup3d-only", action="store_true",
                    help="only time --steps exact-patch 3D setups (profiling runs)")
    ap.add_argument("--vcycle-only", action="store_true",
                    help="only the 256^2 4-level V-cycles, FP64 then FP32: setup, 5 warm-up "
                         "V-cycles, then --steps V-cycles between two torch.flip launches "
                         "that mark them in a kernel trace (per-phase breakdown runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.setup3d_only:
        print(json.dumps({"exact_setup3d": exact_setup3d(32, max(1, args.steps))}), flush=True)
        return
    if args.vcycle_only:
        print(json.dumps({"vcycle_marked": vcycle_marked(args)}), flush=True)
        return
    res = run(args)
    f64, f32 = res["fp64"], res["fp32"]
    t_ap = f64["apply_s_mean"]
    value = f64["nst"] / t_ap / 1e9
    flops = apply_flops_per_cell(args.lin) * f64["cells"]
    achieved = flops / t_ap / 1e12
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
                         f"{args.levels}-level V-cycle (2+2 Vanka, omega={OMEGA})"),
            "space_time_dof": f64["nst"],
            "levels": args.levels,
        },
        "apply_gdofs_fp64": round(value, 4),
        "apply_gdofs_fp32": round(f32["nst"] / f32["apply_s_mean"] / 1e9, 4),
        "apply_us_mean_fp64_fp32": [round(t_ap * 1e6, 3), round(f32["apply_s_mean"] * 1e6, 3)],
        "apply_us_p10_p50_p90_fp64": [round(f64[k] * 1e6, 2) for k in
                                      ("apply_s_p10", "apply_s_median", "apply_s_p90")],
        "apply_us_cached_tangent_fp64_fp32": [round(f64["apply_s_cached"] * 1e6, 3),
                                              round(f32["apply_s_cached"] * 1e6, 3)],
        "apply_us_reproducible_fp64_fp32": [round(f64["apply_s_ordered"] * 1e6, 3),
                                            round(f32["apply_s_ordered"] * 1e6, 3)],
        "apply_hbm_gbs_fp64": round(f64["bytes"] / t_ap / 1e9, 1),
        "vcycle_s_fp64": f64["vcycle_s_median"],
        "vcycle_s_fp32": f32["vcycle_s_median"],
        "vcycle_s_graph_fp64_fp32": [f64["vcycle_s_graph"], f32["vcycle_s_graph"]],
        "setup_s_fp64": f64["setup_s"],
        "setup_s_fp32": f32["setup_s"],
        # residual reduction per V-cycle used as a stationary iteration on a
        # consistent system (geometric mean over 10, last ratio), FP64 / FP32
        "vcycle_residual_reduction": None if args.apply_only else {
            "mean_fp64_fp32": [round(f64["vcycle_rho"]["mean"], 4),
                               round(f32["vcycle_rho"]["mean"], 4)],
            "last_fp64_fp32": [round(f64["vcycle_rho"]["last"], 4),
                               round(f32["vcycle_rho"]["last"], 4)]},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_VALU_PEAK_TFLOPS, 4),
                     "traffic": measured_traffic(args.n),
                     "kernel": "cell_apply_kernel<double, modified Newton, recompute>",
                     "flop_per_launch": flops, "algorithmic_bytes": f64["bytes"],
                     "hbm_copy_measured_gbs": round(measured_copy_gbs(), 1),
                     "hbm_nominal_gbs": HBM_PEAK_GBS},
    }
    if args.apply3d_n and not args.apply_only:
        a3 = apply3d(args.apply3d_n, lin=args.lin)
        line["apply3d"] = {
            "workload": (f"3D {args.apply3d_n}^3 hexahedra Q2/P1disc x dG(1), p=1.3 delta=1e-3 "
                         f"nu_inf=1e-3, modified-Newton Jacobian action (bf16: x and u_k stored "
                         f"in BF16, FP32 arithmetic), 3D sin-series state"),
            **{k: ({kk: round(vv, 4) for kk, vv in v.items()} if isinstance(v, dict) else v)
               for k, v in a3.items()}}
    if args.solve3d_n and not args.apply_only:
        line["exact_setup3d"] = {
            "workload": (f"FP64 4-level smoother setup with exact finest-level patches on "
                         f"{args.solve3d_n}^3 hexahedra (170 x 170 patch inversions on the "
                         f"FP64 matrix cores), the 3D workload's state"),
            **exact_setup3d(args.solve3d_n)}
        s3 = solve3d_latency(args.solve3d_n)
        line["solve3d_time_to_1e-8_s"] = {
            "workload": (f"3D {args.solve3d_n}^3 slab solve, p=1.3 delta=1e-3 nu0=1 nu_inf=1e-3, "
                         f"modified Newton + FGMRES(30) / 4-level V-cycle (exact finest "
                         f"patches, omega 0.15, refresh rho 0.9) to ||R||_M <= 1e-8 ||R0||_M; "
                         f"FP64, mixed (FP32 action and V-cycle), mixed with the BF16-storage "
                         f"Jacobian in FGMRES"),
            **{k: {kk: (float(f"{vv:.5g}") if isinstance(vv, float) else vv)
                   for kk, vv in v.items()}
               for k, v in s3.items()},
            "mixed_speedup": round(s3["fp64"]["time_s"] / s3["mixed"]["time_s"], 3),
            "mixed_bf16_jacobian_speedup": round(s3["fp64"]["time_s"] /
                                                 s3["mixed_bf16_jacobian"]["time_s"], 3)}
    if args.solve_n and not args.apply_only:
        sl = solve_latency(args.solve_n, SOLVE_SEEDS)
        line["solve_time_to_1e-8_s"] = {
            "workload": (f"2D {args.solve_n}x{args.solve_n} slab solve, p=1.2 delta=1e-4 nu0=1 "
                         f"nu_inf=1e-4 (the 256^2 model), modified Newton + FGMRES(30) / V-cycle "
                         f"(exact finest patches, omega {SERVE_OMEGA}, refresh rho {SERVE_RHO}) to "
                         f"||R||_M <= 1e-8 ||R0||_M, {len(SOLVE_SEEDS)} seeded left traces"),
            **{k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
               for k, v in sl.items()},
            "mixed_speedup_p50": round(sl["fp64"]["p50_s"] / sl["mixed"]["p50_s"], 3)}
    if args.vanka_n and not args.apply_only:
        bv = batched_vanka(args.vanka_n)
        line["batched_vanka"] = {
            "workload": (f"{args.vanka_n}x{args.vanka_n} finest-level additive Vanka, FP32, "
                         f"boundary-truncated patches (30-42 unknowns), surrogate tangent "
                         f"p=1.1 delta=1e-5"),
            **{k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
               for k, v in bv.items()}}
    if args.serve_requests and not args.apply_only:
        sv = serve_latency(args.serve_requests)
        line["serving"] = {
            "workload": (f"{args.serve_requests} slab solves to 1e-8, Poisson arrivals 20/s (seed "
                         f"501), meshes U{{32,64,128,256}}^2, p~U[1.1,1.9], delta~logU[1e-5,1e-1], "
                         f"nu_inf~logU[1e-4,1e-2], nu=1; modified Newton + FGMRES / V-cycle "
                         f"(exact finest patches, omega {SERVE_OMEGA}); native server, 8 slots, "
                         f"arena-admitted; non-converged requests counted in the latencies"),
            **{k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
               for k, v in sv.items()}}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
