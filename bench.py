#!/usr/bin/env python3
"""Benchmark: compressed-VIE solves on one MI355X.

Workload (default): the 32 x 32 array of dielectric disks (1024 particles,
147,456 unknowns), radii U[0.15, 0.25] from seed 0, eps_r = 12 + 0.1i, compression
tolerance 1e-6, one TM plane wave at 10 degrees, left-preconditioned GMRES to a
true relative residual of 1e-6, complex128 throughout.

GMRES(50) stagnates on this strongly coupled array (the true residual stalls near
1e-1; the line's forms.gmres50 leg measures it), so the solver runs unrestarted (the
paper's setting, §6) with at most 5000 iterations.  The far factors are stored once per pair
(transpose sharing, Z = Z^T), so each product streams a pair's Q twice and its R once.  A
step is one full solve on the resident compressed operator (inputs in HBM when the timed
region starts).  The operator build (assembly + compression + preconditioner
factorisation) runs once before the timed region; its time is reported as setup_s.

Reported: value = compressed-matvec HBM GB/s (algorithmic bytes of every product executed
in the timed solves, the self-block inverse of the fused preconditioner included, over
their device time, HIP events on the library stream), solves/s, the roofline of the
dominant product kernel, the other forms on the same array (block GMRES over 64 waves,
mixed-precision refinement, GMRES(50)), a bounded serving stream whose arrival-to-result
p50/p99 are the line's latencies, and the FP64 oracle's compressed product on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "compressed-VIE matvec HBM GB/s; GMRES solves/s at 1e-6; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


# product kernels by stage, as rocprofv3 names them: per-block storage, and shared factors
KERNEL_SYMBOL = {"rphase": "k_rphase<4>", "qphase": "k_qphase<4>", "final": "k_final"}
KERNEL_SYMBOL_C64 = {"rphase": "k_rphase_c64<4>", "qphase": "k_qphase_c64<4>", "final": "k_final"}
KERNEL_SYMBOL_SH = {"qtphase": "k_qtphase<HIP_vector_type<double, 2u> >",
                    "rphase": "k_rphase_sh<HIP_vector_type<double, 2u>, 4>",
                    "qphase": "k_qphase_sh<HIP_vector_type<double, 2u>, 4>", "final": "k_final"}
KERNEL_SYMBOL_SH_C64 = {"qtphase": "k_qtphase<HIP_vector_type<float, 2u> >",
                        "rphase": "k_rphase_sh<HIP_vector_type<float, 2u>, 4>",
                        "qphase": "k_qphase_sh<HIP_vector_type<float, 2u>, 4>", "final": "k_final"}
COUNTERS = os.path.join(ROOT, "profiles", "product_shared_mid32x32_counters.txt")
PRODUCT_SOURCES = [os.path.join(ROOT, "paper_2603_10586_amd", "csrc", f) for f in ("k_apply.hip", "stream.h", "op.cpp")]


def source_hash() -> str:
    import hashlib
    return hashlib.sha256(b"".join(open(p, "rb").read() for p in PRODUCT_SOURCES)).hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per dispatch of a product kernel from the committed rocprofv3 counter
    summary (keyed by the kernel's rocprofv3 name), or None if the product sources changed
    since those counters were taken."""
    try:
        kv = dict(line.rstrip("\n").split("=", 1) for line in open(COUNTERS) if "=" in line and not line.startswith("#"))
    except OSError:
        return None
    if kv.get("source_sha256_16") != source_hash():
        return None
    v = kv.get(f"{kernel}.traffic_bytes")
    return int(float(v)) if v else None


def cpu_solve_extrapolation(arr, iterations: int, product_bytes: float, cpu_gbs: float, seconds: float = 6.0,
                            seed: int = 1) -> dict:
    """Per-solve CPU figures of the same workload from bounded samples, all stated as
    extrapolated: the oracle's matrix-free dense product (every entry regenerated, §3) timed
    over whole particle rows and scaled to all rows; and one solve at the GPU's iteration
    count, iterations x (compressed product + block-diagonal preconditioner, §4) plus the
    Arnoldi projections (two passes over a basis that grows by one vector per step), with the
    product at the oracle's measured compressed-product rate, the preconditioner timed on a
    sample of particles and the projections on a 32-vector basis of the full length."""
    from oracle import discretise, greens, solvers
    rng = np.random.default_rng(seed)
    disc = discretise.Discretisation(arr)
    N = disc.n_particles
    n = N * 144
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    order = rng.permutation(N)
    k, t0 = 0, time.perf_counter()
    while k == 0 or (k < N and time.perf_counter() - t0 < 0.5 * seconds):
        greens.matvec_free(disc, x, rows=order[k:k + 1])
        k += 1
    dense_s = (time.perf_counter() - t0) / k * N
    ns = min(N, 32)
    pre = solvers.BlockDiagPreconditioner(np.stack([greens.particle_self_block(disc, int(p)) for p in order[:ns]]))
    y = x[:ns * 144]
    reps, t0 = 0, time.perf_counter()
    while reps == 0 or time.perf_counter() - t0 < 0.1 * seconds:
        pre.apply(y)
        reps += 1
    prec_s = (time.perf_counter() - t0) / reps * N / ns
    m = 32
    V = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    reps, t0 = 0, time.perf_counter()
    while reps == 0 or time.perf_counter() - t0 < 0.2 * seconds:
        h = (x.conj() @ V).conj()                  # V^H w
        x - V @ h                                  # w - V h
        reps += 1
    per_vector_s = (time.perf_counter() - t0) / reps / m
    arnoldi_s = per_vector_s * iterations * (iterations + 1) / 2
    product_s = product_bytes / (cpu_gbs * 1e9)

    def sig(v: float) -> float:
        return float(f"{v:.4g}")
    return {"matrix_free_dense_product": {"particle_rows_timed": k, "s_extrapolated": sig(dense_s)},
            "solve_extrapolated": {"iterations": iterations, "compressed_product_s": sig(product_s),
                                   "preconditioner_s": sig(prec_s), "arnoldi_s": sig(arnoldi_s),
                                   "solve_s": sig(iterations * (product_s + prec_s) + arnoldi_s),
                                   "note": "extrapolated from timed samples, not a measured solve"}}


def cpu_baseline(op, geom, seconds: float = 15.0, seed: int = 0, arr=None, iterations: int = 0,
                 product_bytes: float = 0.0) -> dict:
    """The oracle's compressed product (Q (R x) per block, §5.2) on the host cores,
    timed on a bounded stratified sample of the exported blocks; with the array, the GPU's
    iteration count and the product's bytes, also the extrapolated per-solve figures."""
    from oracle import compressed
    rng = np.random.default_rng(seed)
    order = geom.order()
    nb = op.num_blocks()
    infos = [op.export_block(b, factors=False)[0] for b in range(nb)]
    by_level: dict = {}
    for b, inf in enumerate(infos):
        by_level.setdefault(inf["level"], []).append(b)
    pick = []
    for lev, ids in sorted(by_level.items()):
        pick += list(rng.choice(ids, size=min(len(ids), 160), replace=False))
    factors, fbytes = [], 0
    for b in pick:
        inf, Q, R = op.export_block(int(b))
        if Q is None:
            continue
        rows = order[inf["row_first"]:inf["row_first"] + inf["row_count"]]
        cols = order[inf["col_first"]:inf["col_first"] + inf["col_count"]]
        factors.append((rows, cols, Q, R))
        fbytes += (Q.size + R.size) * 16
    x = (rng.standard_normal(geom.ndof) + 1j * rng.standard_normal(geom.ndof)).reshape(-1, 1)
    y = np.zeros_like(x)
    reps, t = 0, 0.0
    t0 = time.perf_counter()
    while t < seconds or reps == 0:
        compressed.factor_apply(factors, x, y)
        reps += 1
        t = time.perf_counter() - t0
    gbs = fbytes * reps / t / 1e9
    out = {"value": round(gbs, 3), "unit": "GB/s", "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
           "sample": f"oracle compressed product over {len(factors)} exported blocks stratified by level "
                     f"({fbytes / 1e9:.2f} GB of factors), {reps} passes in {t:.1f} s; CPU {cpu_model()}",
           "tiny_dense_context_s": oracle_tiny_timings()}
    if arr is not None and iterations > 0 and product_bytes > 0:
        out["per_solve_context"] = cpu_solve_extrapolation(arr, iterations, product_bytes, gbs)
    return out


def oracle_tiny_timings() -> dict:
    """The oracle's dense path on the 4 x 4 array (2304 unknowns) on the host cores: dense
    assembly, one dense product and preconditioned GMRES(30) on the dense matrix to 1e-8
    (seconds each), as context for the compressed GPU path.  The oracle's loop LU (about
    30 s here) is left out to keep the run short."""
    import workloads as W
    from oracle import discretise, greens, solvers
    disc = discretise.Discretisation(W.tiny())
    out = {}
    t = time.perf_counter()
    Z = greens.assemble_dense(disc)
    out["dense_assembly"] = time.perf_counter() - t
    v = greens.plane_wave_rhs(disc, [0.0], [0.0], [1])[:, 0]
    t = time.perf_counter()
    Z @ v
    out["dense_product"] = time.perf_counter() - t
    pre = solvers.BlockDiagPreconditioner(greens.self_blocks(disc))
    t = time.perf_counter()
    _, info = solvers.gmres(lambda x: Z @ x, v, apply_M=pre.apply, restart=30, tol=1e-8)
    out["gmres30_dense"] = time.perf_counter() - t
    out["gmres_iterations"] = info.iterations
    return {k: (round(x, 3) if isinstance(x, float) else x) for k, x in out.items()}


def serving(args) -> int:
    """Continuous batching through the library's native server: Poisson arrivals of arrays with
    side U{lo..hi}, random radii, 1-16 plane waves each, tolerance 1e-6; every request's waves
    share one block Krylov space.  Latency is arrival (submission) to completion."""
    import workloads as W
    from paper_2603_10586_amd.server import Server, ServerOpts, replay
    reqs = W.serving_requests(n=args.serving, seed=0, rate_per_s=args.serving_rate,
                              side_lo=args.serving_side[0], side_hi=args.serving_side[1])
    opts = ServerOpts(slots=args.serving_slots, hbm_budget=200 << 30, eps=args.eps, restart=args.block_basis,
                      max_iter=args.max_iter)
    srv = Server(opts)
    t0 = time.perf_counter()
    res = replay(srv, reqs, report=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
    wall = time.perf_counter() - t0
    st = srv.stats()
    last_error = srv.last_error() if any(r.status not in (0, 5) for r in res) else ""
    srv.close()
    ok = all(r.status == 0 for r in res)
    worst = max(i["rel_res_true"] for r in res for i in r.info)
    print(json.dumps({
        "metric": METRIC, "value": round(st["rhs_solves_per_s"], 4), "unit": "RHS solves/s", "n_gpus": 1,
        "steps": len(res), "warmup": 0, "ms_per_step": round(wall / len(res) * 1e3, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"serving: {len(res)} requests, Poisson {args.serving_rate}/s, side "
                               f"U{{{args.serving_side[0]}..{args.serving_side[1]}}}, radii U[0.15, 0.25], "
                               f"1-16 RHS, tol 1e-6, {args.serving_slots} slots, block GMRES per request"},
        "latency_ms_p50": round(st["latency_p50_s"] * 1e3, 1), "latency_ms_p99": round(st["latency_p99_s"] * 1e3, 1),
        "requests_per_s": round(st["requests_per_s"], 4), "queue_wait_ms_p50": round(st["queue_wait_p50_s"] * 1e3, 1),
        "peak_admitted_bytes": st["peak_bytes"], "operators_built": st["ops_built"], "cache_hits": st["cache_hits"],
        "all_converged": ok, "worst_true_residual": worst, "rhs_solved": st["rhs_solved"], "wall_s": round(wall, 1),
        "last_error": last_error,
        "requests": {"fields": ["particles", "waves", "status", "latency_s", "queue_s", "block_steps"],
                     "rows": [[q.array.n_particles, len(q.incidence.theta_deg), r.status, round(r.latency, 2),
                               round(r.admitted - r.arrival, 2), max(i["iterations"] for i in r.info)]
                              for q, r in zip(reqs, res)]}}))
    return 0


def vogel_leg(args) -> int:
    """The paper's own test arrays (§6.1): Vogel spirals of n gold spheres, voxelised, grouped
    on the paper's grid, compressed by cross approximation at eps, and solved by GMRES without
    restart (at most 5000 iterations) to 1e-4 for one normally incident plane wave, with the
    stage counters of the paper's performance table (products, preconditioner applications,
    their times, Krylov time, total) and its build table (assembly + compression).  Up to
    --vogel-dense-max particles the dense product Z x (assembled Z, rocBLAS) is timed beside
    the compressed one for the product speed-up."""
    import torch
    import paper_2603_10586_amd as q
    import workloads as W
    ctx = q.Context(0)
    rows = []
    for n in args.vogel_n:
        arr = W.vogel(n)
        geom = q.Geometry(ctx, arr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op = q.Operator(ctx, geom, eps=args.eps, compression=args.compression, verbose=n >= 1000)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        st = op.stats()
        v = q.rhs_plane_waves(ctx, geom, [0.0], [0.0], [1])
        x, info, status = op.solve(v, restart=5000, max_iter=5000, tol=args.vogel_tol)
        i = info[0]
        prof = op.profile_apply(reps=20)
        row = {"meta_atoms": n, "dofs": geom.ndof, "levels": geom.n_levels, "blocks": st["n_blocks"],
               "build_s": round(build_s, 2), "t_compression_s": round(st["t_compression_s"], 2),
               "operator_bytes": st["device_bytes"], "gain": round(st["gain"], 2),
               "converged": bool(i["converged"]), "iterations": i["iterations"], "restarts": i["restarts"],
               "rel_res_true": i["rel_res_true"],
               "N_prd": i["n_apply"], "N_Pcnd": i["n_prec"], "t_prd_s": round(i["t_apply_s"], 4),
               "t_Pcnd_s": round(i["t_prec_s"], 4), "t_Kryl_s": round(i["t_krylov_s"], 4),
               "t_tot_s": round(i["t_total_s"], 4), "product_ms": round(prof["product"]["ms"], 4)}
        if n <= args.vogel_dense_max:
            allp = np.arange(n)
            Z = q.assemble(ctx, geom, allp, allp).t()            # the column-major buffer: Z^T by rows
            xd = torch.randn(geom.ndof, dtype=torch.complex128, device="cuda")
            for _ in range(3):
                yd = torch.matmul(xd, Z)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            for _ in range(10):
                yd = torch.matmul(xd, Z)
            ev[1].record()
            torch.cuda.synchronize()
            row["dense_product_ms"] = round(ev[0].elapsed_time(ev[1]) / 10, 4)
            row["product_speedup"] = round(row["dense_product_ms"] / row["product_ms"], 2)
            del Z, yd
            torch.cuda.empty_cache()
        rows.append(row)
        print(f"[bench] vogel {n}: {json.dumps(row)}", file=sys.stderr, flush=True)
        op.close()
        geom.close()
    total = sum(r["t_tot_s"] for r in rows)
    print(json.dumps({
        "metric": "unrestarted GMRES to 1e-4 on the paper's Vogel arrays (s per solve)", "value": round(total, 3),
        "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(total * 1e3, 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "vogel spirals of voxelised gold spheres (R = 100 nm, 600 nm wavelength), paper grid, "
                               f"eps {args.eps:g}, {args.compression} compression, one plane wave, tol {args.vogel_tol:g}",
                   "meta_atoms": args.vogel_n},
        "arrays": rows}))
    return 0


def build_leg(args) -> int:
    """One operator build (untimed elsewhere): wall time, compression time, blocks, ranks and
    device bytes, for the sketch or the cross-approximation compression."""
    import torch
    import paper_2603_10586_amd as q
    import workloads as W
    arr = W.batching() if args.graded else (W.mid(0) if args.side == 32 else W.random_lattice(args.side, seed=0))
    far = q.PREC_C64_ONLY if args.c64_only else q.PREC_C128
    ctx = q.Context(0)
    geom = q.Geometry(ctx, arr)
    est = q.Operator.footprint_estimate(geom, eps=args.eps, max_block_rows=args.max_block_rows, far_prec=far,
                                        compression=args.compression)
    print(f"[bench] build: {arr.name}, {geom.ndof} unknowns, {args.compression}, cap {args.max_block_rows}, "
          f"footprint estimate {est / 1e9:.1f} GB", file=sys.stderr, flush=True)
    walls = []
    for r in range(args.build_reps):          # repeated builds in one process (the last is kept)
        if r:
            op.close()
        ctx.peak_bytes(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op = q.Operator(ctx, geom, eps=args.eps, far_prec=far, max_block_rows=args.max_block_rows,
                        verbose=True, share_transpose=args.share, compression=args.compression,
                        aca_start=args.aca_start, aca_stop=args.aca_stop)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
    wall = float(np.median(walls))
    st = op.stats()
    sizes = {}
    for b in range(op.num_blocks()):
        i = op.export_block(b, factors=False)[0]
        sizes[i["m"]] = max(sizes.get(i["m"], 0), i["rank"])
    print(json.dumps({
        "metric": "operator build s", "value": round(wall, 2), "unit": "s", "n_gpus": 1, "steps": len(walls),
        "warmup": 0, "build_s_each": [round(w, 2) for w in walls],
        "ms_per_step": round(wall * 1e3, 1), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{arr.name}: {arr.n_particles} disks, {geom.ndof} unknowns, eps {args.eps:g}",
                   "compression": args.compression, "max_block_rows": args.max_block_rows,
                   "far_prec": "c64" if args.c64_only else "c128", "share_transpose": bool(args.share)},
        "t_compression_s": round(st["t_compression_s"], 2), "blocks": st["n_blocks"],
        "max_block_rows_built": max(sizes), "max_rank_by_rows": {str(k): v for k, v in sorted(sizes.items())},
        "mean_rank_level": [round(x, 1) for x in st["mean_rank_level"][:st["n_levels"] + 2]],
        "max_block_rel_err": st["max_block_rel_err"], "operator_device_bytes": st["device_bytes"],
        "build_peak_bytes": ctx.peak_bytes(), "footprint_estimate": est,
        "cross_approximation": {k: st[k] for k in ("n_aca", "n_aca_resumed", "n_aca_retried", "n_aca_sketch")}}))
    return 0


def block(args) -> int:
    """Block GMRES: 64 plane waves (32 angles x TE/TM) share one block Krylov space; the
    product runs on FP64 matrix cores.  A step is one solve of all right-hand sides."""
    import torch
    import paper_2603_10586_amd as q
    import workloads as W
    if args.graded:
        arr = W.batching()
    else:
        arr = W.mid(0) if args.side == 32 else W.random_lattice(args.side, seed=0)
    nrhs = args.nrhs if args.nrhs > 1 else 64
    far = q.PREC_C64_ONLY if args.c64_only else q.PREC_C128
    ctx = q.Context(0)
    t0 = time.perf_counter()
    geom = q.Geometry(ctx, arr)
    est = q.Operator.footprint_estimate(geom, eps=args.eps, max_block_rows=args.max_block_rows)
    print(f"[bench] block: {arr.name}, {geom.ndof} unknowns, operator footprint estimate {est / 1e9:.1f} GB "
          f"(complex128 form)", file=sys.stderr, flush=True)
    op = q.Operator(ctx, geom, eps=args.eps, far_prec=far, max_block_rows=args.max_block_rows, verbose=True,
                    share_transpose=args.share, compression=args.compression)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    sw = W.sweep((nrhs + 1) // 2)
    v = q.rhs_plane_waves(ctx, geom, sw.theta_deg[:nrhs], sw.phi_deg[:nrhs], sw.pol[:nrhs])
    print(f"[bench] block: {arr.name}, {nrhs} right-hand sides, setup {setup_s:.1f} s", file=sys.stderr, flush=True)
    tiles = None if (args.no_tune or args.share) else tune_tiles(op)
    restart = args.block_basis
    for _ in range(args.warmup):
        op.solve(v, restart=restart, tol=args.tol, max_iter=args.max_iter, mode=q.SOLVE_BLOCK)
    torch.cuda.synchronize()
    lat, infos = [], []
    t_start = time.perf_counter()
    for k in range(args.steps):
        t = time.perf_counter()
        x, info, status = op.solve(v, restart=restart, tol=args.tol, max_iter=args.max_iter, mode=q.SOLVE_BLOCK,
                                   verbose=True, block_width=args.block_width)
        lat.append(time.perf_counter() - t)
        infos.append(info)
        print(f"[bench] step {k}: {lat[-1]:.2f} s, block steps {info[0]['iterations']}, "
              f"worst true res {max(i['rel_res_true'] for i in info):.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_start
    if not all(i["converged"] for inf in infos for i in inf):
        print("[bench] a timed block solve did not converge", file=sys.stderr, flush=True)
    single = None
    if args.single_compare:
        t = time.perf_counter()
        xs, inf1, _ = op.solve(v[:1].contiguous(), restart=args.max_iter, tol=args.tol, max_iter=args.max_iter)
        single = {"s_per_solve": round(time.perf_counter() - t, 2), "iterations": inf1[0]["iterations"],
                  "converged": bool(inf1[0]["converged"]), "rel_res_true": inf1[0]["rel_res_true"]}
        print(f"[bench] single-vector FP64 solve: {single}", file=sys.stderr, flush=True)
    if args.share:      # the stage profiler takes per-block storage only
        prof = {"product": {"ms": last_product_ms(infos), "flops": 0}}
    else:
        prof = op.profile_block(nrhs=min(nrhs, args.block_width or 64), reps=5)
    dom = max(prof, key=lambda k: prof[k]["ms"])
    ach = prof[dom]["flops"] / (prof[dom]["ms"] * 1e-3) / 1e12
    pt = sum(p["ms"] for p in prof.values())
    last = infos[-1][0]
    print(json.dumps({
        "metric": METRIC, "value": round(args.steps * nrhs / total_s, 3), "unit": "RHS solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(total_s / args.steps * 1e3, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 factors, f64 accumulation" if args.c64_only else "f64", "data": "synthetic",
        "config": {"workload": f"{arr.name}: {arr.n_particles} disks, {geom.ndof} unknowns, eps {args.eps:g}, "
                               f"block GMRES on {nrhs} plane waves ({(nrhs + 1) // 2} angles x TE/TM) to {args.tol:g}"
                               + (", complex64 far factors" if args.c64_only else ""),
                   "particles": arr.n_particles, "unknowns": geom.ndof, "nrhs": nrhs, "tol": args.tol,
                   "basis_vectors_per_cycle": restart, "max_block_rows": args.max_block_rows},
        "operator_device_bytes": op.stats()["device_bytes"], "block_width": args.block_width or 64,
        "single_vector_fp64": single,
        "block_steps": last["iterations"], "cycles": last["restarts"], "block_products": last["n_apply"],
        "worst_true_residual": max(i["rel_res_true"] for i in infos[-1]),
        "solve_split_s": {"block_products": round(last["t_apply_s"], 3),
                          "krylov_and_host": round(lat[-1] - last["t_apply_s"], 3)},
        "setup_s": round(setup_s, 2),
        "block_product_ms": round(pt, 3), "block_product_stage_ms": {k: round(p["ms"], 3) for k, p in prof.items()},
        "tile_tuning": tiles,
        "roofline": {"bound": "mfma", "achieved": round(ach, 2), "peak": FP64_MFMA_PEAK_TFS, "unit": "TF/s",
                     "frac": round(ach / FP64_MFMA_PEAK_TFS, 4), "traffic": None, "kernel": "k_strip_mfma<4>",
                     "stage": dom, "algorithmic_flops": prof[dom]["flops"]},
    }))
    return 0


def precision_pattern(args) -> int:
    """The precision workload: far factors in BF16 split-complex (with the complex64 factors they
    were rounded from, stored once per pair), corrections by block GMRES with the BF16 factors on
    FP32 matrix cores and complex64 self blocks, FP64-accumulated residuals of the complex64
    operator, 8 plane waves (4 angles in [-30, 30] deg x TE/TM; --nrhs N > 1: the batching sweep of N
    waves, solved in blocks of --block-width).  With --ir-reference the same
    right-hand sides are then solved by FP64 block GMRES on the complex128 factors of the same
    array (another operator, built after this one is freed) and each wave's relative difference
    is reported."""
    import torch
    import paper_2603_10586_amd as q
    import workloads as W
    if args.graded:
        arr = W.batching()
    else:
        arr = W.precision(0) if args.side == 96 else W.random_lattice(args.side, seed=0)
    ctx = q.Context(0)
    geom = q.Geometry(ctx, arr)
    cap = args.max_block_rows
    est = q.Operator.footprint_estimate(geom, eps=args.eps, max_block_rows=cap, far_prec=q.PREC_BF16X2,
                                        share_transpose=True)
    print(f"[bench] precision: {arr.name}, {geom.ndof} unknowns, footprint estimate {est / 1e9:.1f} GB",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    op = q.Operator(ctx, geom, eps=args.eps, far_prec=q.PREC_BF16X2, max_block_rows=cap, share_transpose=True,
                    compression=args.compression,
                    verbose=True)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    st = op.stats()
    print(f"[bench] precision: operator {st['device_bytes'] / 1e9:.1f} GB built in {setup:.1f} s", file=sys.stderr,
          flush=True)
    if args.nrhs > 1:                          # the batching sweep: nrhs waves, nrhs / 2 angles x TE/TM
        sw = W.sweep((args.nrhs + 1) // 2)
        thetas, phis, pols = sw.theta_deg[:args.nrhs], sw.phi_deg[:args.nrhs], sw.pol[:args.nrhs]
    else:
        th = np.linspace(-30.0, 30.0, 4)
        thetas, pols = np.concatenate([th, th]), np.array([0] * 4 + [1] * 4, dtype=np.int32)
        phis = np.zeros(8)
    nrhs = len(thetas)
    v = q.rhs_plane_waves(ctx, geom, thetas, phis, pols)
    torch.cuda.synchronize()
    t = time.perf_counter()
    x, info, status = op.solve(v, restart=args.block_basis, tol=args.tol, max_iter=args.max_iter,
                               mode=q.SOLVE_BLOCK_IR, verbose=True, block_width=args.block_width)
    torch.cuda.synchronize()
    t_ir = time.perf_counter() - t
    print(f"[bench] precision: BF16 refinement {t_ir:.1f} s, {info[0]['iterations']} block steps, "
          f"{info[0]['n_refine']} corrections, true residuals {max(i['rel_res_true'] for i in info):.2e}",
          file=sys.stderr, flush=True)
    out = {"metric": METRIC, "value": round(nrhs / t_ir, 4) if all(i["converged"] for i in info) else None,
           "unit": "RHS solves/s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(t_ir * 1e3, 1),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16 far factors on f32 MFMA (inner), f64-accumulated c64 residuals", "data": "synthetic",
           "config": {"workload": f"{arr.name}: {arr.n_particles} disks, {geom.ndof} unknowns, eps {args.eps:g}, "
                                  f"{nrhs} plane waves, BF16 split-complex far factors, mixed-precision block refinement "
                                  f"to {args.tol:g}, transpose-shared factors, block rows <= {cap}",
                      "particles": arr.n_particles, "unknowns": geom.ndof, "basis_vectors": args.block_basis,
                      "max_block_steps": args.max_iter},
           "operator_device_bytes": st["device_bytes"], "footprint_estimate": est, "setup_s": round(setup, 1),
           "mean_rank_level": [round(r, 1) for r in st["mean_rank_level"]],
           "converged": [bool(i["converged"]) for i in info], "rel_res_true": [i["rel_res_true"] for i in info],
           "block_steps": info[0]["iterations"], "corrections": info[0]["n_refine"]}
    if args.ir_reference:
        xh = x.cpu()
        del x
        op.close()
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        op64 = q.Operator(ctx, geom, eps=args.eps, max_block_rows=cap, share_transpose=True, verbose=True,
                          compression=args.compression)
        t = time.perf_counter()
        x64, i64, _ = op64.solve(v, restart=args.block_basis, tol=args.tol, max_iter=args.max_iter,
                                 mode=q.SOLVE_BLOCK, verbose=True, block_width=args.block_width)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t
        x64h = x64.cpu()
        out["fp64_reference"] = {
            "s": round(t64, 2), "build_s": round(t - t0, 1), "block_steps": i64[0]["iterations"],
            "converged": [bool(i["converged"]) for i in i64], "rel_res_true": [i["rel_res_true"] for i in i64],
            "rel_diff_per_rhs": [float(torch.linalg.norm(xh[r] - x64h[r]) / torch.linalg.norm(x64h[r]))
                                 for r in range(nrhs)]}
        print(f"[bench] precision: FP64 reference {t64:.1f} s, per-RHS differences "
              f"{max(out['fp64_reference']['rel_diff_per_rhs']):.2e}", file=sys.stderr, flush=True)
    print(json.dumps(out))
    return 0


def last_product_ms(infos) -> float:
    i = infos[-1][0]
    return i["t_apply_s"] / max(i["n_apply"], 1) * 1e3


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--side", type=int, default=32)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--restart", type=int, default=5000)
    ap.add_argument("--max-iter", type=int, default=5000)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--nrhs", type=int, default=1,
                    help="right-hand sides per solve (plane waves at angles spread over [-30, 30] deg)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--product-only", action="store_true",
                    help="build the operator and time products only (for hardware-counter runs)")
    ap.add_argument("--read-probe-mib", type=int, default=0,
                    help="time the library's streaming-read probe over this many MiB and its FP64/FP32 "
                         "matrix-core probes, then exit")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device copy of this many MiB five times (counter calibration)")
    ap.add_argument("--serving", type=int, default=0,
                    help="run the serving workload with this many Poisson-arriving requests instead")
    ap.add_argument("--serving-rate", type=float, default=1.0, help="request arrival rate (1/s)")
    ap.add_argument("--serving-side", type=int, nargs=2, default=[8, 48], help="array side range")
    ap.add_argument("--serving-slots", type=int, default=3)
    ap.add_argument("--block", action="store_true",
                    help="block GMRES on 64 plane waves (FP64 matrix-core products)")
    ap.add_argument("--no-tune", action="store_true", help="block mode without the tile autotuner")
    ap.add_argument("--block-ir", action="store_true",
                    help="with --mixed-ir: block GMRES corrections on the complex64 factors (all RHS together)")
    ap.add_argument("--ir-reference", action="store_true",
                    help="with --mixed-ir: also solve in plain FP64 and report per-RHS differences")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the block and mixed-precision forms in the default line")
    ap.add_argument("--graded", action="store_true",
                    help="block and precision modes on the 64 x 64 graded metalens array")
    ap.add_argument("--c64-only", action="store_true", help="block mode with complex64 far factors only")
    ap.add_argument("--block-basis", type=int, default=16384, help="block mode: basis vectors per cycle")
    ap.add_argument("--max-block-rows", type=int, default=0, help="split far blocks taller than this")
    ap.add_argument("--compression", choices=["aca", "sketch"], default="aca",
                    help="far-block compression: cross approximation, or assembled blocks and a randomised sketch")
    ap.add_argument("--vogel", action="store_true",
                    help="the paper's Vogel-spiral arrays: unrestarted GMRES to 1e-4 with stage timers")
    ap.add_argument("--vogel-n", type=int, nargs="+", default=[100, 500, 1000, 2000])
    ap.add_argument("--vogel-tol", type=float, default=1e-4)
    ap.add_argument("--vogel-dense-max", type=int, default=500,
                    help="time the dense product for arrays up to this many particles")
    ap.add_argument("--build-reps", type=int, default=1, help="build leg: builds in one process (median reported)")
    ap.add_argument("--aca-start", type=int, default=0, help="build leg: crosses per block at first (0 = library default)")
    ap.add_argument("--aca-stop", type=float, default=0.0, help="build leg: crosses' stopping tolerance / eps (0 = default)")
    ap.add_argument("--build", action="store_true",
                    help="operator build leg: build time, ranks and memory of one operator (--side / --graded)")
    ap.add_argument("--block-width", type=int, default=0, help="block mode: right-hand sides per block (0 = 64)")
    ap.add_argument("--single-compare", action="store_true",
                    help="block mode: also time one single-vector FP64 solve of the first wave")
    ap.add_argument("--mixed-ir", action="store_true",
                    help="iterative refinement: complex64 far factors inside, complex128 residuals outside")
    ap.add_argument("--precision", action="store_true",
                    help="the precision workload (96 x 96 random array by default, --side to change): BF16 "
                         "corrections on FP32 matrix cores, 8 plane waves")
    ap.add_argument("--share", action="store_true", help="block mode: transpose-shared far factors")
    ap.add_argument("--no-share", action="store_true",
                    help="store every ordered far block's factors (no transpose sharing) for the single-vector line")
    ap.add_argument("--gmres50-steps", type=int, default=2000,
                    help="default line: Arnoldi steps of the GMRES(50) leg (0 skips it)")
    ap.add_argument("--no-batching64", dest="batching64_leg", action="store_false",
                    help="default line: skip the 64 x 64 batching form (about 80 s)")
    ap.add_argument("--serving-leg", type=int, default=24,
                    help="default line: requests of the bounded serving leg (0 skips it)")
    ap.add_argument("--serving-leg-rate", type=float, default=0.9, help="serving leg arrival rate (1/s)")
    ap.add_argument("--serving-leg-side", type=int, nargs=2, default=[8, 24], help="serving leg array sides")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: multi-GPU execution is not implemented (asked for --gpus {args.gpus})",
              file=sys.stderr)
        return 2

    import torch

    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(5):
            dst.copy_(src)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / 5
        print(json.dumps({"copy_probe_bytes_each_way": src.numel() * 8, "launches": 10, "ms_per_copy": round(ms, 4),
                          "read_plus_write_gbs": round(2 * src.numel() * 8 / (ms * 1e-3) / 1e9, 1)}))
        return 0

    import paper_2603_10586_amd as q

    if args.read_probe_mib:
        buf = torch.ones(args.read_probe_mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        gbs = q.Context(0).probe_read(buf, reps=10)
        ctx = q.Context(0)
        f64, f32 = ctx.probe_mfma(True), ctx.probe_mfma(False)
        print(json.dumps({"read_probe_bytes": buf.numel() * 8, "best_read_gbs": round(gbs, 1),
                          "of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                          "mfma_f64_16x16x4_tfs": round(f64, 1), "mfma_f32_16x16x4_tfs": round(f32, 1)}))
        return 0
    import workloads as W

    if args.serving:
        return serving(args)
    if args.build:
        return build_leg(args)
    if args.vogel:
        return vogel_leg(args)
    if args.block:
        return block(args)
    if args.precision:
        return precision_pattern(args)

    arr = W.mid(0) if args.side == 32 else W.random_lattice(args.side, seed=0)
    inc = W.mid_incidence()
    print(f"[bench] {arr.name}: {arr.n_particles} particles, {arr.ndof} unknowns", file=sys.stderr, flush=True)
    ctx = q.Context(0)
    t0 = time.perf_counter()
    geom = q.Geometry(ctx, arr)
    # the complex64 copy of the far factors serves the mixed-precision line; the FP64 solves
    # and products read only the complex128 panels.  Block corrections need per-block storage.
    share = not args.no_share and not args.block_ir
    op = q.Operator(ctx, geom, eps=args.eps, far_prec=q.PREC_C64 if (args.mixed_ir or not args.no_forms) else q.PREC_C128,
                    max_block_rows=args.max_block_rows, verbose=arr.n_particles > 1024, share_transpose=share,
                    compression=args.compression)
    mode = q.SOLVE_BLOCK_IR if args.block_ir else (q.SOLVE_MIXED_IR if args.mixed_ir else q.SOLVE_FP64)
    restart = args.block_basis if args.block_ir else args.restart
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    st = op.stats()
    print(f"[bench] setup {setup_s:.2f} s, gain {st['gain']:.2f}, product bytes {st['apply_bytes'] / 1e9:.2f} GB",
          file=sys.stderr, flush=True)
    if args.nrhs > 1:
        sw = W.sweep((args.nrhs + 1) // 2)          # TE angles then TM angles
        v = q.rhs_plane_waves(ctx, geom, sw.theta_deg[:args.nrhs], sw.phi_deg[:args.nrhs], sw.pol[:args.nrhs])
    else:
        v = q.rhs_plane_waves(ctx, geom, inc.theta_deg, inc.phi_deg, inc.pol)
    n = geom.ndof
    prec_bytes = st["apply_bytes"] + st["n_self_types"] * 144 * 144 * 16
    if args.product_only:
        for prec in ((q.PREC_C128, q.PREC_C64) if args.mixed_ir else (q.PREC_C128,)):
            prof = op.profile_apply(reps=20, prec=prec)
            # (stages the operator does not run, the Q^T pass of per-block storage, report 0 ms)
            print(json.dumps({"prec": "c64" if prec == q.PREC_C64 else "c128",
                              **{k: dict(ms=round(p["ms"], 4), bytes=p["bytes"],
                                         gbs=round(p["bytes"] / (p["ms"] * 1e-3) / 1e9, 1) if p["ms"] > 0 else None)
                                 for k, p in prof.items()}}))
        return 0

    for _ in range(args.warmup):
        op.solve(v, restart=restart, tol=args.tol, max_iter=args.max_iter, mode=mode)
    torch.cuda.synchronize()
    lat, infos = [], []
    t_start = time.perf_counter()
    for k in range(args.steps):
        t = time.perf_counter()
        x, info, status = op.solve(v, restart=restart, tol=args.tol, max_iter=args.max_iter, mode=mode)
        lat.append(time.perf_counter() - t)
        infos.extend(info)
        print(f"[bench] step {k}: {lat[-1] * 1e3:.1f} ms, iterations {[i['iterations'] for i in info]}, "
              f"true res {max(i['rel_res_true'] for i in info):.2e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_start
    if not all(i["converged"] for i in infos):
        raise SystemExit("a timed solve did not converge: no throughput is reported")

    n_apply = sum(i["n_apply"] for i in infos)
    t_apply = sum(i["t_apply_s"] for i in infos)
    if args.block_ir:
        value = args.steps * args.nrhs / total_s    # block products have their own roofline (--block)
    elif args.mixed_ir:
        # outer residuals (complex128 factors): one per refinement plus the final check
        n_hi = sum(i["n_refine"] + 1 for i in infos)
        lo_bytes = st["apply_bytes_c64"] + st["n_self_types"] * 144 * 144 * 16
        value = (prec_bytes * n_hi + lo_bytes * (n_apply - n_hi)) / t_apply / 1e9
    else:
        value = prec_bytes * n_apply / t_apply / 1e9

    prof = op.profile_apply(reps=20, prec=q.PREC_C64 if args.mixed_ir else q.PREC_C128)
    stages = ("qtphase", "rphase", "qphase", "final") if share else ("rphase", "qphase", "final")
    dom = max(stages, key=lambda k: prof[k]["ms"])
    ach = prof[dom]["bytes"] / (prof[dom]["ms"] * 1e-3) / 1e9
    symbols = (KERNEL_SYMBOL_SH_C64 if args.mixed_ir else KERNEL_SYMBOL_SH) if share else \
        (KERNEL_SYMBOL_C64 if args.mixed_ir else KERNEL_SYMBOL)
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(symbols[dom]) if share else None,
                "algorithmic_bytes": prof[dom]["bytes"], "kernel": symbols[dom],
                "timing": "HIP events around the kernel's own launch, averaged over 20 products",
                "stages_ms": {k: round(prof[k]["ms"], 4) for k in stages + ("product",)},
                "stages_gbs": {k: round(prof[k]["bytes"] / (prof[k]["ms"] * 1e-3) / 1e9, 1)
                               for k in stages + ("product",)}}
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC, "value": round(value, 3 if args.block_ir else 1),
        "unit": "RHS solves/s" if args.block_ir else "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total_s / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 factors, f64 accumulation" if args.mixed_ir else "f64",
        "data": "synthetic",
        "config": {"workload": f"{arr.name}: {arr.n_particles} disks, {n} unknowns, eps {args.eps:g}, "
                               + ("transpose-shared far factors, " if share else "")
                               + (f"GMRES({args.restart})" if args.restart < args.max_iter else "unrestarted GMRES")
                               + f" to {args.tol:g}, "
                               + ("one TM plane wave at 10 deg" if args.nrhs == 1 else
                                  f"{args.nrhs} plane waves ({(args.nrhs + 1) // 2} angles in [-30, 30] deg x TE/TM)")
                               + (", mixed-precision refinement (complex64 inner)" if args.mixed_ir else "")
                               + (", block corrections" if args.block_ir else ""),
                   "particles": arr.n_particles, "unknowns": n, "eps": args.eps, "restart": args.restart,
                   "tol": args.tol},
        "value_bytes": "each product's algorithmic bytes: far factors as streamed (shared: a pair's Q twice, "
                       "its R once), self blocks, the self-block inverses of the fused preconditioner, x, y and the "
                       "rank-space vectors",
        "solves_per_s": round(args.steps * args.nrhs / total_s, 3),
        "rhs_per_solve_call": args.nrhs,
        "solve_ms_p50": round(float(np.percentile(lat_ms, 50)), 2),
        "solve_ms_p99": round(float(np.percentile(lat_ms, 99)), 2),
        "iterations": infos[-1]["iterations"], "rel_res_true": infos[-1]["rel_res_true"],
        "basis_orthogonality": infos[-1]["basis_ortho"], "refinements": infos[-1]["n_refine"],
        "solve_split_s": {"products": round(infos[-1]["t_apply_s"], 3),
                          "krylov_and_host": round(lat[-1] - infos[-1]["t_apply_s"], 3)},
        "setup_s": round(setup_s, 2), "gain": round(st["gain"], 3), "product_bytes": st["apply_bytes"],
        "operator_device_bytes": st["device_bytes"], "share_transpose": share,
        "product_ms": round(prof["product"]["ms"], 4),
        "product_gbs": round(prof["product"]["bytes"] / (prof["product"]["ms"] * 1e-3) / 1e9, 1),
        "mean_rank_level": [round(r, 1) for r in st["mean_rank_level"]],
        "roofline": roofline,
    }
    if not args.mixed_ir and not args.no_forms and args.nrhs == 1:
        out["forms"] = other_forms(q, W, ctx, geom, op, v, args, out["solves_per_s"], share)
        if args.batching64_leg:
            try:
                out["forms"]["batching64"] = batching64_leg(args)
            except Exception as e:                 # the line is still reported without this form
                out["forms"]["batching64"] = {"error": str(e)[:300]}
        if args.serving_leg > 0:
            leg = serving_leg(args)
            out["forms"]["serving"] = leg
            out["latency_ms_p50"], out["latency_ms_p99"] = leg["latency_ms_p50"], leg["latency_ms_p99"]
            out["latency_source"] = "forms.serving: arrival to result over the bounded serving stream"
    if args.mixed_ir and args.ir_reference:
        out["fp64_reference"] = ir_reference(q, op, v, x, args, total_s / args.steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(op, geom, seconds=args.cpu_seconds, arr=arr, iterations=out["iterations"],
                                           product_bytes=st["apply_bytes"])
    print(json.dumps(out))
    return 0


def ir_reference(q, op, v, x_ir, args, s_ir: float) -> dict:
    """The plain FP64 solve of the same right-hand sides on the same operator (complex128
    factors), its time, and each right-hand side's relative difference between the
    mixed-precision and the FP64 solutions."""
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    x64, info, _ = op.solve(v, restart=args.block_basis if args.block_ir else args.restart, tol=args.tol,
                            max_iter=args.max_iter, mode=q.SOLVE_BLOCK if args.block_ir else q.SOLVE_FP64)
    torch.cuda.synchronize()
    s64 = time.perf_counter() - t
    err = [float(torch.linalg.norm(x_ir[r] - x64[r]) / torch.linalg.norm(x64[r])) for r in range(x64.shape[0])]
    print(f"[bench] FP64 reference: {s64:.2f} s, per-RHS difference {max(err):.2e}", file=sys.stderr, flush=True)
    return {"s_per_solve": round(s64, 3), "iterations": [i["iterations"] for i in info],
            "rel_res_true": [i["rel_res_true"] for i in info], "converged": all(i["converged"] for i in info),
            "rel_diff_per_rhs": err, "mixed_precision_speedup": round(s64 / s_ir, 2)}


def tune_tiles(op, prec=None) -> dict:
    """Autotune the block product's tile shapes for 16, 32, 48 and 64 right-hand sides (the
    widths a block solve uses before and after deflation); per width and strip group the
    kept shape and the default/kept launch times."""
    out = {}
    for w in (16, 32, 48, 64):
        t = op.tune_block(nrhs=w, reps=3, prec=prec)
        g = {}
        for k, ms in t["ms"].items():
            c = t["chosen"][k]
            g[k] = {"u": t["variants"][c]["u"], "rows_per_wave": t["variants"][c]["rows_per_wave"],
                    "default_ms": round(ms[0], 4), "tuned_ms": round(ms[c], 4),
                    "all_ms": [round(m, 4) for m in ms]}
        out[str(w)] = g
    print(f"[bench] tile tuning (64 RHS): " + ", ".join(
        f"{k} u{v['u']}/r{v['rows_per_wave']} {v['default_ms']:.3f}->{v['tuned_ms']:.3f} ms"
        for k, v in out["64"].items()), file=sys.stderr, flush=True)
    return out


def other_forms(q, W, ctx, geom, op, v, args, plain_solves_per_s: float, share: bool) -> dict:
    """On the same array and tolerance, beside the plain single-solve FP64 form timed above: block
    GMRES over 64 plane waves (per-block storage, FP64 matrix cores), mixed-precision refinement
    (complex64 inner products) and the configured GMRES(50) for a bounded step budget."""
    import torch
    sw = W.sweep(32)
    vb = q.rhs_plane_waves(ctx, geom, sw.theta_deg, sw.phi_deg, sw.pol)
    opb = q.Operator(ctx, geom, eps=args.eps, max_block_rows=args.max_block_rows) if share else op
    tiles = tune_tiles(opb)
    opb.solve(vb, restart=16384, tol=args.tol, max_iter=args.max_iter, mode=q.SOLVE_BLOCK)     # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, ib, sb = opb.solve(vb, restart=16384, tol=args.tol, max_iter=args.max_iter, mode=q.SOLVE_BLOCK)
    tb = time.perf_counter() - t
    if opb is not op:
        opb.close()
    print(f"[bench] block form: {tb:.2f} s for 64 waves, {ib[0]['iterations']} block steps", file=sys.stderr,
          flush=True)
    t = time.perf_counter()
    _, ii, si = op.solve(v, restart=args.restart, tol=args.tol, max_iter=args.max_iter, mode=q.SOLVE_MIXED_IR)
    ti = time.perf_counter() - t
    print(f"[bench] mixed-precision form: {ti:.2f} s, {ii[0]['iterations']} inner steps", file=sys.stderr,
          flush=True)
    block_sps = 64 / tb
    out = {
        "plain_fp64_single_solves_per_s": plain_solves_per_s,
        "block_64_waves": {"solves_per_s": round(block_sps, 3), "s_per_64": round(tb, 3),
                           "block_steps": ib[0]["iterations"], "converged": all(i["converged"] for i in ib),
                           "worst_true_residual": max(i["rel_res_true"] for i in ib),
                           "vs_plain": round(block_sps / plain_solves_per_s, 1), "tile_tuning": tiles["64"]},
        "mixed_precision_refinement": {"solves_per_s": round(1.0 / ti, 3), "inner_steps": ii[0]["iterations"],
                                       "refinements": ii[0]["n_refine"], "converged": bool(ii[0]["converged"]),
                                       "true_residual": ii[0]["rel_res_true"],
                                       "vs_plain": round((1.0 / ti) / plain_solves_per_s, 2)},
    }
    if args.gmres50_steps > 0:
        t = time.perf_counter()
        _, i50, _ = op.solve(v, restart=50, tol=args.tol, max_iter=args.gmres50_steps)
        t50 = time.perf_counter() - t
        print(f"[bench] GMRES(50): {i50[0]['iterations']} steps, true residual {i50[0]['rel_res_true']:.2e}",
              file=sys.stderr, flush=True)
        out["gmres50"] = {"steps": i50[0]["iterations"], "restarts": i50[0]["restarts"],
                          "converged": bool(i50[0]["converged"]), "true_residual": i50[0]["rel_res_true"],
                          "preconditioned_residual": i50[0]["rel_res_prec"], "s": round(t50, 2),
                          "note": "the configured restart length, for a bounded step budget; the timed solves run "
                                  "unrestarted GMRES because GMRES(50) stalls on this array"}
    return out


def batching64_leg(args) -> dict:
    """The batching workload as one timed form of the default line: the 64 x 64 graded metalens
    array (589,824 unknowns), complex64 far factors by cross approximation, 64 plane waves solved
    by block GMRES as two 32-wide blocks (12,288 basis vectors each, no restart) to the tolerance."""
    import torch
    import paper_2603_10586_amd as q
    import workloads as W
    ctx = q.Context(0)
    arr = W.batching()
    geom = q.Geometry(ctx, arr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = q.Operator(ctx, geom, eps=args.eps, far_prec=q.PREC_C64_ONLY)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    try:
        tune_tiles(op)
        sw = W.sweep(32)
        v = q.rhs_plane_waves(ctx, geom, sw.theta_deg, sw.phi_deg, sw.pol)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, info, st = op.solve(v, restart=12288, tol=args.tol, max_iter=1200, mode=q.SOLVE_BLOCK, block_width=32)
        ts = time.perf_counter() - t
        print(f"[bench] batching 64x64: {ts:.1f} s for 64 waves, {info[0]['iterations']} block steps", file=sys.stderr,
              flush=True)
        return {"workload": f"{arr.name}: {arr.n_particles} disks, {geom.ndof} unknowns, 64 plane waves as two 32-wide "
                            f"blocks, complex64 far factors, tol {args.tol:g}",
                "solves_per_s": round(64 / ts, 3), "s_per_64": round(ts, 2), "build_s": round(build_s, 2),
                "block_steps": info[0]["iterations"], "converged": all(i["converged"] for i in info),
                "worst_true_residual": max(i["rel_res_true"] for i in info),
                "operator_device_bytes": op.stats()["device_bytes"]}
    finally:
        op.close()
        geom.close()
        ctx.close()


def serving_leg(args) -> dict:
    """A bounded stream of the serving workload (the seeded request recipe with array sides in
    the given range, 1-16 plane waves each, tolerance 1e-6, Poisson arrivals) through the
    library's native server; latency is arrival (submission) to result."""
    import workloads as W
    from paper_2603_10586_amd.server import Server, ServerOpts, replay
    lo, hi = args.serving_leg_side
    reqs = W.serving_requests(n=args.serving_leg, seed=0, rate_per_s=args.serving_leg_rate, side_lo=lo, side_hi=hi)
    srv = Server(ServerOpts(slots=3, hbm_budget=120 << 30, eps=args.eps, restart=8192, max_iter=8000))
    t0 = time.perf_counter()
    res = replay(srv, reqs, report=lambda m: print(f"[bench] serving {m}", file=sys.stderr, flush=True))
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    print(f"[bench] serving leg: {len(res)} requests in {wall:.1f} s, p50 {st['latency_p50_s']:.2f} s, "
          f"p99 {st['latency_p99_s']:.2f} s", file=sys.stderr, flush=True)
    return {"requests": len(res), "arrival_rate_per_s": args.serving_leg_rate, "array_sides": [lo, hi],
            "latency_ms_p50": round(st["latency_p50_s"] * 1e3, 1), "latency_ms_p99": round(st["latency_p99_s"] * 1e3, 1),
            "queue_wait_ms_p50": round(st["queue_wait_p50_s"] * 1e3, 1),
            "requests_per_s": round(st["requests_per_s"], 4), "rhs_solves_per_s": round(st["rhs_solves_per_s"], 3),
            "all_converged": all(r.status == 0 for r in res),
            "worst_true_residual": max(i["rel_res_true"] for r in res for i in r.info),
            "operators_built": st["ops_built"], "wall_s": round(wall, 1)}


if __name__ == "__main__":
    sys.exit(main())
