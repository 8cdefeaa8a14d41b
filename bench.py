#!/usr/bin/env python3
"""Benchmark of the space-time heat BEM hot path on one MI355X.

One step = one pass of the whole path over the workload (icosphere, 1280 triangles / 642
vertices, 64 uniform steps on (0, 1], alpha = 1):
  1. fused assembly of all V_h^d and K_h^d blocks (FP64),
  2. Dirichlet right-hand side (1/2 M_h + K_h) g,
  3. solve of V_h w = b to relative residual 1e-8 taken with the double-precision operator, by
     the fastest solver measured on this workload: time marching in FP64 (the inverse of the
     freshly assembled V_h^0 by blocked Gauss-Jordan, then block forward substitution with the
     history subtracted in chunks),
  4. representation formula at 10^4 interior space-time points.
After the timed steps every solver is timed on the same b: plain double GMRES (the reference),
time marching, mixed-precision refinement, learned GMRES and learned + mixed, each to 1e-8.  The
learned preconditioner's MLP is trained on random ellipsoids (the learned-preconditioner
workload), never on this mesh.
Inputs (mesh, data, points) are synthetic and seeded and already resident on the device when the
timed region starts.  value = pair-block integrals per second of the whole step:
E_x^2 * E_t units (one unit = one (test panel, trial panel, d) triple with its V entry and its
three K contributions) divided by the step time.

Prints one JSON line.  --gpus N > 1 is refused: this build runs on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6e12  # MI355X FP64 vector FLOP/s

# Counters of the separated-pair assembly (k_separated + k_fold_KT, one launch each) on this
# workload, from rocprofv3 --pmc runs of `bench.py --assembly-only`: FETCH_SIZE and WRITE_SIZE,
# each scaled by the reading of the same counter for a plain 256 MiB device copy taken in the same
# run (FETCH_SIZE reads 0.500x, WRITE_SIZE 1.000x of the copied bytes), and the FP64 VALU
# instruction counts (wave instructions; 64 lanes each, an FMA is 2 FLOP).  Valid only for the
# assembly sources they were taken on (sha256 prefix of COUNTER_SOURCES below); reported as null
# otherwise.
COUNTERS = {"source_sha256": "08cfbc323ac7b64f",
            "fetch_kib": 13657.1875 + 460173.0625, "fetch_scale": 262144.0 / 131086.125,
            "write_kib": 2950251.34375 + 424960.0, "write_scale": 262144.0 / 262144.0,
            "fma_f64": 1.35706111e9, "mul_f64": 2.7930831e8, "add_f64": 1.449856e8}
COUNTER_SOURCES = ("hb_assemble.hip", "hb_sep.h", "hb_device.h", "hb_closed.h", "hb_internal.h")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_flops_separated(n_sep_pairs, n_t):
    """FLOPs the semi-analytic method needs for the separated pairs: per (pair, point pair) 15 FLOP
    of geometry (r, rho, 1/rho, r.n) and per (pair, point pair, level delta = i h, i = 0..E_t) one
    erf and one exp (60 FLOP together) plus 25 FLOP of bracket arithmetic and accumulation; 49
    point pairs of the 7-point rule.  n_sep_pairs counts ordered pairs (the unit count of the
    metric); since V^d and the kernel values are symmetric in the pair, the algorithm needs the
    work of the unordered pairs only, n_sep_pairs / 2, and that is what the roofline counts."""
    return n_sep_pairs * 49.0 * (15.0 + 85.0 * (n_t + 1))


def counter_source_sha():
    import hashlib
    h = hashlib.sha256()
    for name in COUNTER_SOURCES:
        with open(os.path.join(ROOT, "paper_2102_09811_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _counters_valid():
    return COUNTERS["source_sha256"] is not None and counter_source_sha() == COUNTERS["source_sha256"]


def assembly_traffic_bytes():
    """HBM bytes per separated-pair assembly launch from the committed counter runs, or None when
    the assembly source has changed since they were taken."""
    if not _counters_valid():
        return None
    return 1024.0 * (COUNTERS["fetch_kib"] * COUNTERS["fetch_scale"] +
                     COUNTERS["write_kib"] * COUNTERS["write_scale"])


def executed_flops():
    """FP64 FLOP the separated-pair kernel executes per launch (counters of k_separated; k_fold_KT
    adds 0.06 %), or None."""
    if not _counters_valid():
        return None
    return 64.0 * (2.0 * COUNTERS["fma_f64"] + COUNTERS["mul_f64"] + COUNTERS["add_f64"])


def assembly_only(args):
    """Counter runs: two assemblies of the benchmarked workload, then a plain 256 MiB device copy
    (the calibration of the HBM byte counters)."""
    import torch
    from paper_2102_09811_amd import Context, HB_OP_K, HB_OP_V
    from synthetic import icosphere
    verts, tris = icosphere(3)
    ctx = Context(verts, tris, 1.0, 1.0, 64)
    for _ in range(2):
        ctx.assemble(HB_OP_V | HB_OP_K)
    torch.cuda.synchronize()
    log("assembly kernels ms: separated+fold %.3f, touching %.3f" % tuple(ctx.last_assembly_ms()[:2]))
    a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ctx.close()
    log("calibration copy: 256 MiB read, 256 MiB written")
    return 0


def apply_only(args):
    """Counter runs of the block-Toeplitz products of the benchmarked workload: 1 + 10 products with
    the double V_h blocks, 1 + 10 with K_h, 1 + 10 with the V_h blocks in float storage (the kernel
    of the mixed solve's inner products), then the 256 MiB calibration copy."""
    import torch
    from paper_2102_09811_amd import HB_DTYPE_F32, HB_OP_K, HB_OP_V, Context
    from synthetic import icosphere
    verts, tris = icosphere(3)
    ne, nv, nt = len(tris), len(verts), 64
    gen = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn(nt, ne, dtype=torch.float64, device="cuda", generator=gen)
    xg = torch.randn(nt, nv, dtype=torch.float64, device="cuda", generator=gen)
    y = torch.empty_like(x)
    for storage in (None, HB_DTYPE_F32):
        ctx = Context(verts, tris, 1.0, 1.0, nt) if storage is None else \
            Context(verts, tris, 1.0, 1.0, nt, storage=storage)
        ctx.assemble(HB_OP_V | HB_OP_K)
        ops = ((HB_OP_V, x), (HB_OP_K, xg)) if storage is None else ((HB_OP_V, x),)
        for op, xx in ops:
            ctx.apply(op, xx, y)  # first call allocates the partial sums
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(10):
                ctx.apply(op, xx, y)
            e1.record()
            torch.cuda.synchronize()
            log("apply %s %s: %.1f us per product" % ("V" if op == HB_OP_V else "K",
                                                     "float" if storage else "double",
                                                     e0.elapsed_time(e1) * 100.0))
        ctx.close()
    a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    log("calibration copy: 256 MiB read, 256 MiB written")
    return 0


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(verts, tris, alpha, T, n_t):
    """The oracle's plain double-precision mode -- the method as the paper runs it on a CPU
    (level order, one erf and one exp per point and level, OpenMP dynamic over test rows) -- on
    bounded samples of test rows of the same workload: 16 rows on 1 thread, then 32 rows per
    thread on every thread of the host share."""
    import numpy as np
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    ne = len(tris)
    oracle.assemble_plain(verts, tris, alpha, T, n_t, rows=np.array([0], np.int32), threads=1)
    res = {}
    for nth, nrows in ((1, 16), (threads, min(32 * threads, ne))):
        rows = np.linspace(0, ne - 1, nrows).astype(np.int32)
        t0 = time.perf_counter()
        oracle.assemble_plain(verts, tris, alpha, T, n_t, rows=rows, threads=nth)
        dt = time.perf_counter() - t0
        res[nth] = (nrows * ne * n_t / dt, nrows, dt)
        log("cpu baseline: %d thread(s), %d rows, %.1f s, %.3g units/s" % (nth, nrows, dt, res[nth][0]))
    v1, vn = res[1], res[threads]
    return {"value": vn[0], "unit": "pair-block integrals/s", "cores": threads,
            "kind": "oracle", "mode": "plain double, the paper's level order (V and K fused)",
            "value_1_thread": v1[0], "nproc": os.cpu_count(), "cpu": _cpu_model(),
            "sample": "%d test rows x %d trial panels x %d blocks on %d threads (%.1f s); "
                      "%d rows on 1 thread (%.1f s)" % (vn[1], ne, n_t, threads, vn[2], v1[1], v1[2])}


def mixed_block_errors(ctx, mixed):
    """Per-block error of the mixed-precision assembly against the double one, for every d and
    for V_h and K_h: max |A_mixed^d - A^d| / max |A^d| (device; the blocks below the first float
    block are double in both and equal)."""
    from paper_2102_09811_amd import HB_OP_K, HB_OP_V
    res = {}
    for op, name in ((HB_OP_V, "V"), (HB_OP_K, "K")):
        ref = ctx.blocks(op)
        err = (mixed[op] - ref).abs().amax(dim=(1, 2)) / ref.abs().amax(dim=(1, 2))
        e = err.cpu().tolist()
        res["max_block_rel_err_" + name] = max(e)
        res["block_rel_err_" + name] = [float("%.3g" % x) for x in e]
        del ref
    return res


def compare_solvers(ctx, b, net):
    """Every solver on the same right-hand side, each to relative residual 1e-8 measured with the
    double operator; wall time of the whole call (median of 3)."""
    import numpy as np
    from paper_2102_09811_amd import HB_SOLVE_GMRES, HB_SOLVE_MIXED_IR, HB_SOLVE_TIMEMARCH, learned
    cases = [("gmres_fp64", HB_SOLVE_GMRES, False), ("time_marching", HB_SOLVE_TIMEMARCH, False),
             ("mixed_ir", HB_SOLVE_MIXED_IR, False), ("learned_gmres", HB_SOLVE_GMRES, True),
             ("learned_mixed_ir", HB_SOLVE_MIXED_IR, True)]
    learned.install(net, ctx)
    res = {}
    for name, method, pc in cases:
        ctx.solve(b, method=method, tol=1e-8, precond=pc)  # warm (time marching: inverse of V^0)
        times, info = [], None
        for _ in range(3):
            _, info = ctx.solve(b, method=method, tol=1e-8, precond=pc)
            times.append(1e3 * info["seconds"])
        res[name] = {"ms": float(np.median(times)), "iterations": info["iterations"],
                     "refinements": info["refinements"], "rel_residual": info["rel_residual"],
                     "converged": info["converged"]}
        log("solve %-16s %8.2f ms  it=%d res=%.2e" % (name, res[name]["ms"], info["iterations"],
                                                      info["rel_residual"]))
    # time marching including the Gauss-Jordan inverse of V^0 (needed once per assembled V^0)
    from paper_2102_09811_amd import HB_OP_V
    ctx.assemble(HB_OP_V)
    _, info = ctx.solve(b, method=HB_SOLVE_TIMEMARCH, tol=1e-8)
    res["time_marching_with_inverse"] = {"ms": 1e3 * info["seconds"], "iterations": 0,
                                         "refinements": 0, "rel_residual": info["rel_residual"],
                                         "converged": info["converged"]}
    log("solve %-16s %8.2f ms (first call after assembly)" % ("time_marching+inv",
                                                               res["time_marching_with_inverse"]["ms"]))
    learned.install(net, ctx)
    base = res["gmres_fp64"]["ms"]
    for name in res:
        res[name]["speedup_vs_gmres_fp64"] = base / res[name]["ms"]
    return res


def neumann_timings(ctx, stream):
    """Hypersingular side of the same workload (outside the timed step): assembly of D_h and
    V_h^{11} (p1 x p1 blocks) from the assembled V_h, and GMRES on D_h u = (1/2 M_h^T - K_h^T) psi
    for a synthetic Neumann datum psi, plain and with the operator preconditioner."""
    import numpy as np
    import torch
    from paper_2102_09811_amd import HB_OP_D, HB_OP_V11
    res = {}
    for name, op in (("assemble_D_ms", HB_OP_D), ("assemble_V11_ms", HB_OP_V11)):
        ctx.assemble(op)                       # first call allocates
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.assemble(op)
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1)
    psi = torch.from_numpy(np.random.default_rng(5).standard_normal((ctx.n_t, ctx.n_tris))).cuda()
    b = ctx.rhs_neumann(psi)
    ctx.solve_neumann(b, precond=True)        # inverts the mass matrix once
    for key, pc in (("gmres", False), ("gmres_operator_precond", True)):
        u, info = ctx.solve_neumann(b, tol=1e-8, precond=pc)
        res[key] = {"ms": info["seconds"] * 1e3, "iterations": info["iterations"],
                    "rel_residual": info["rel_residual"]}
        log("neumann %-24s %7.2f ms  it=%d res=%.2e" % (key, info["seconds"] * 1e3,
                                                       info["iterations"], info["rel_residual"]))
    log("assembly D %.2f ms, V11 %.2f ms" % (res["assemble_D_ms"], res["assemble_V11_ms"]))
    return res


def nearfield_timings(ctx, stream, radius=0.35):
    """Near-field assembly (outside the timed step): the per-pair blocks of V_h and K_h for the
    pairs within `radius` (centroid distance) plus the touching ones."""
    import torch
    start, cols = ctx.nearfield_pattern(radius)
    ctx.assemble_nearfield()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.assemble_nearfield()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    units = len(cols) * ctx.n_t
    log("near field r=%g: %d pairs (%.1f per row), %.2f ms, %.3g pair-blocks/s" % (
        radius, len(cols), len(cols) / ctx.n_tris, ms, units / (ms * 1e-3)))
    return {"radius": radius, "pairs": int(len(cols)), "ms": ms, "pair_blocks_per_s": units / (ms * 1e-3)}


def nonuniform_timings(verts, tris, alpha, n_t, stream, gamma=1.5):
    """Non-uniform time grid (outside the timed step): the same mesh on the graded nodes
    t_j = (j / E_t)^gamma, assembly of all E_t (E_t + 1) / 2 blocks V^{k,i}, K^{k,i}, the
    block-triangular product, GMRES to 1e-8 and time marching (its first call inverts every
    V^{k,k}) on the same right-hand side."""
    import numpy as np
    import torch
    from paper_2102_09811_amd import HB_OP_K, HB_OP_V, HB_SOLVE_TIMEMARCH, NonuniformContext
    tn = (np.arange(n_t + 1) / n_t) ** gamma
    ctx = NonuniformContext(verts, tris, alpha, tn)
    ctx.assemble(HB_OP_V | HB_OP_K)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ctx.assemble(HB_OP_V | HB_OP_K)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    units = float(len(tris)) ** 2 * n_t * (n_t + 1) / 2
    x = torch.from_numpy(np.random.default_rng(7).standard_normal((n_t, len(tris)))).cuda()
    ctx.apply(HB_OP_V, x)
    e0.record(stream)
    y = ctx.apply(HB_OP_V, x)
    e1.record(stream)
    torch.cuda.synchronize()
    apply_ms = e0.elapsed_time(e1)
    w, info = ctx.solve(y, tol=1e-8)
    _, tm1 = ctx.solve(y, method=HB_SOLVE_TIMEMARCH, tol=1e-8)
    _, tm2 = ctx.solve(y, method=HB_SOLVE_TIMEMARCH, tol=1e-8)
    ctx.close()
    log("non-uniform grid (t_j = (j/%d)^%g): assembly %.2f ms (%.3g pair-block integrals/s), "
        "product %.3f ms, GMRES %d it %.2f ms, time marching %.2f ms (with the inverses %.2f ms)"
        % (n_t, gamma, ms, units / (ms * 1e-3), apply_ms, info["iterations"],
           info["seconds"] * 1e3, tm2["seconds"] * 1e3, tm1["seconds"] * 1e3))
    return {"grid": "t_j = (j / %d)^%g" % (n_t, gamma), "blocks": n_t * (n_t + 1) // 2,
            "assemble_ms": ms, "units_per_s": units / (ms * 1e-3), "apply_V_ms": apply_ms,
            "gmres": {"ms": info["seconds"] * 1e3, "iterations": info["iterations"],
                      "rel_residual": info["rel_residual"]},
            "time_marching": {"ms": tm2["seconds"] * 1e3, "ms_with_inverses": tm1["seconds"] * 1e3,
                              "rel_residual": tm2["rel_residual"]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--points", type=int, default=10000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the solver comparison")
    ap.add_argument("--train-meshes", type=int, default=16)
    ap.add_argument("--assembly-only", action="store_true",
                    help="two assemblies and a 256 MiB calibration copy (for counter runs)")
    ap.add_argument("--apply-only", action="store_true",
                    help="block-Toeplitz products and a 256 MiB calibration copy (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        return 2

    if args.assembly_only:
        return assembly_only(args)
    if args.apply_only:
        return apply_only(args)

    import numpy as np
    import torch
    from paper_2102_09811_amd import measure_peaks
    from paper_2102_09811_amd import (Context, HB_OP_K, HB_OP_V, HB_PREC_MIXED, HB_SOLVE_GMRES,
                                      HB_SOLVE_MIXED_IR, HB_SOLVE_TIMEMARCH, check_mesh, learned)
    from synthetic import ball_points, exp_solution, icosphere, nodal_samples, space_time_points

    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    alpha, T, n_t = 1.0, 1.0, 64
    verts, tris = icosphere(3)
    ne, nv = len(tris), len(verts)
    rc, counts, _ = check_mesh(verts, tris)
    n_sep = int(counts[0])
    g = nodal_samples(verts, n_t, T, lambda x, t: exp_solution(x, t, alpha))
    pts = space_time_points(ball_points(args.points, 0.5, seed=0), 0.25, 0.75, seed=0)
    log("training the learned preconditioner on %d ellipsoids" % args.train_meshes)
    t_train = time.perf_counter()
    net, hist = learned.train(learned.ellipsoid_set(range(args.train_meshes)), epochs=30)
    t_train = time.perf_counter() - t_train
    log("trained in %.1f s, loss %.3e -> %.3e" % (t_train, hist[0], hist[-1]))
    ctx = Context(verts, tris, alpha, T, n_t)
    gd = torch.from_numpy(g).cuda()
    ptsd = torch.from_numpy(pts).cuda()
    b = torch.empty((n_t, ne), dtype=torch.float64, device="cuda")
    w = torch.empty((n_t, ne), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step(record):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record(stream)
        ctx.assemble(HB_OP_V | HB_OP_K)
        ev[1].record(stream)
        ctx.rhs_dirichlet(gd, b)
        ev[2].record(stream)
        _, info = ctx.solve(b, method=HB_SOLVE_TIMEMARCH, tol=1e-8, w=w)
        ev[3].record(stream)
        u = ctx.eval_repr(ptsd, w, gd)
        ev[4].record(stream)
        if record is not None:
            torch.cuda.synchronize()
            record.append({"assemble_ms": ev[0].elapsed_time(ev[1]),
                           "rhs_ms": ev[1].elapsed_time(ev[2]),
                           "solve_ms": ev[2].elapsed_time(ev[3]),
                           "repr_ms": ev[3].elapsed_time(ev[4]),
                           "kernels_ms": ctx.last_assembly_ms(),
                           "iterations": info["iterations"],
                           "rel_residual": info["rel_residual"]})
        return u

    for i in range(args.warmup):
        log("warmup %d" % i)
        step(None)
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(rec)
        log("step %d: %.2f ms (assemble %.2f, solve %.2f, repr %.2f)" % (
            i, sum(rec[-1][k] for k in ("assemble_ms", "rhs_ms", "solve_ms", "repr_ms")),
            rec[-1]["assemble_ms"], rec[-1]["solve_ms"], rec[-1]["repr_ms"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1000.0 * wall / args.steps
    units = float(ne) * ne * n_t
    avg = lambda k: float(np.mean([r[k] for r in rec]))
    sep_ms = float(np.mean([r["kernels_ms"][0] for r in rec]))
    touch_ms = float(np.mean([r["kernels_ms"][1] for r in rec]))
    flops_ordered = algorithmic_flops_separated(n_sep, n_t)
    flops = 0.5 * flops_ordered  # unordered pairs
    achieved = flops / (sep_ms * 1e-3) / 1e12
    out = {
        "metric": "V_d+K_d pair-block integrals/sec & % VALU peak; solve time to 1e-8 vs FP64",
        "value": units / (ms_per_step * 1e-3),
        "unit": "pair-block integrals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "icosphere r=1, 1280 triangles / 642 vertices, E_t=64 on (0,1], "
                               "alpha=1; assemble V+K, RHS, solve to 1e-8 (FP64 time marching), "
                               "repr at %d points"
                               % args.points,
                   "E_x": ne, "N_x": nv, "E_t": n_t, "alpha": alpha, "T": T,
                   "repr_points": args.points, "solve_tol": 1e-8},
        "phases_ms": {"assemble": avg("assemble_ms"), "rhs": avg("rhs_ms"),
                      "solve": avg("solve_ms"), "repr": avg("repr_ms"),
                      "assemble_separated_kernel": sep_ms, "assemble_touching_kernels": touch_ms},
        "assembly_units_per_s": units / (avg("assemble_ms") * 1e-3),
        "solve": {"method": "time marching in FP64 (Gauss-Jordan inverse of the assembled V_h^0, "
                            "block forward substitution), residual recomputed with the double "
                            "operator",
                  "iterations": int(rec[-1]["iterations"]),
                  "rel_residual": rec[-1]["rel_residual"], "ms": avg("solve_ms")},
        "learned_training_s": t_train,
        "roofline": {"bound": "alu",
                     "kernel": "k_separated + k_fold_KT (separated-pair assembly)",
                     "achieved": achieved, "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / (PEAK_FP64_VALU / 1e12),
                     "frac_kind": "algorithmic: the method's work on the unordered separated pairs "
                                  "(one erf and one exp per level) over the launch time; "
                                  "frac_executed is the FP64 work the kernel issues (counters); "
                                  "frac_ordered_effective counts both orders of every pair, the "
                                  "work of an evaluation without the pair symmetry, so it can "
                                  "exceed 1 and is no hardware fraction",
                     "traffic": assembly_traffic_bytes(),
                     "algorithmic_flops_per_launch": flops,
                     "frac_ordered_effective": 2.0 * achieved / (PEAK_FP64_VALU / 1e12),
                     "executed_flops_per_launch": executed_flops(),
                     "frac_executed": (None if executed_flops() is None else
                                       executed_flops() / (sep_ms * 1e-3) / PEAK_FP64_VALU)},
    }
    # the chip's vector-ALU ceilings measured on this device (microbenchmarks of the library): the
    # roofline above is quoted against the published FP64 figure, these check it
    out["alu_peaks_measured"] = measure_peaks()
    log("measured peaks: FP64 FMA %(fp64_fma_tflops).1f TFLOP/s, v_rsq_f64 %(fp64_rsq_gops).0f G/s, "
        "FP32 FMA (no packed FP32) %(fp32_fma_tflops).1f TFLOP/s" % out["alu_peaks_measured"])
    if not args.no_compare:
        log("solver comparison")
        out["solve_comparison"] = compare_solvers(ctx, b, net)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ctx.assemble(HB_OP_V | HB_OP_K, precision=HB_PREC_MIXED)
        ev0.record(stream)
        ctx.assemble(HB_OP_V | HB_OP_K, precision=HB_PREC_MIXED)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_mixed = ev0.elapsed_time(ev1)
        out["mixed_assembly"] = {"ms": ms_mixed, "units_per_s": units / (ms_mixed * 1e-3),
                                 "separated_kernel_ms": ctx.last_assembly_ms()[0]}
        mixed = {op: ctx.blocks(op) for op in (HB_OP_V, HB_OP_K)}
        ctx.assemble(HB_OP_V | HB_OP_K)
        out["mixed_assembly"].update(mixed_block_errors(ctx, mixed))
        del mixed
        out["neumann"] = neumann_timings(ctx, stream)
        out["nearfield"] = nearfield_timings(ctx, stream)
        out["nonuniform"] = nonuniform_timings(verts, tris, alpha, n_t, stream)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(verts, tris, alpha, T, n_t)
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
