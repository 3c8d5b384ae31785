"""Benchmark of the matrix-free SIPG apply on one MI355X.

Workload: 32^3 hexahedra on the unit cube deformed by the sine map
(amplitude 0.05), degree k = 4 (4,096,000 DoFs), Jacobians stored at every
quadrature point, seeded uniform [-1,1] source.  A step is one operator
evaluation y = A u over the whole mesh (the fused cell + face pass).  The
headline value is FP64 DoF/s; beside it: the FP32 apply, per-launch
median/min with warm and flushed caches, the 64^3 affine/curved comparison,
the mixed-precision and FP64 solve latencies of the manufactured-solution
Poisson problem, the continuous-batching serving trace, and the oracle on
the host cores.

Every record carries its error against the FP64 oracle (err_vs_oracle):
the GPU result is kept on a sample of cells outside the timed region, and
the CPU-baseline leg, which times the oracle on the host cores, evaluates
the oracle on the same cells of the same input and compares.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-variants] [--solve-reps R] [--serve-requests R]
                       [--only f64|f32] [--copy-calibration MB]
                       [--legs headline,merged,...] [--variant NAME]
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

METRIC = "SIPG apply DoF/s (FP64 vs FP32, k=4 curved); mixed-prec solve p50/p99 ms"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1711_03590_amd", "csrc", "kernels.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sipg_apply_f64_curved_k4_32cubed_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "sipg_apply_curved_k4_32cubed_valu_counters.md")
LEGS = ("headline", "merged", "positions", "hermite", "advection", "shard", "variants", "degrees", "solve", "serve")
# parity bars: relative l2 against the FP64 oracle, 1e-12 in FP64 and 1e-5 in FP32
TOL = {"f64": 1e-12, "f32": 1e-5}
# GPU results kept for the oracle comparison in the CPU leg (outside every timed region)
PARITY = []


GEOMETRY_VALUES = {"curved": (10, 4), "curved-merged": (6, 4), "curved-positions": (4, 4), "affine-variable": (1, 1), "affine": (0, 0),
                   "advection": (3, 1)}


def algorithmic_bytes_per_dof(ncell, k, real_bytes, geometry="curved"):
    """src read + dst write + every stored geometry value read once.  Curved
    (G3): 10 per cell quadrature point (J^{-T}, c det J w) and 4 per face
    quadrature point (n.J^{-1}, c ds); affine with a variable coefficient:
    c det J w per cell point and c ds per face point; affine with a constant
    coefficient: nothing.  Merged curved storage (G4): the 6 entries of the
    symmetric c det J w J^{-1} J^{-T} per cell point, faces as G3.  Positions
    storage (G2): the 3 position components and c per cell point, faces as
    G3.  The
    advection operator: J^{-1} c det J w per cell point and (c.n) ds per face
    point.  Neighbour re-reads and tables are not counted."""
    n = k + 1
    cells = ncell ** 3
    faces = 3 * ncell * ncell * (ncell + 1)
    cv, fv = GEOMETRY_VALUES[geometry]
    vals = 2 * cells * n ** 3 + cv * cells * n ** 3 + fv * faces * n * n
    return vals * real_bytes / (cells * n ** 3)


def kernel_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


def measured_traffic(dtype):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it
    was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m = re.search(r"kernel_source_sha1:\s*(\w+)", txt)
    if not m or m.group(1) != kernel_hash():
        return None
    m = re.search(rf"{dtype}_hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


FP64_VECTOR_PEAK_TFLOPS = 78.6


def measured_flop_per_dof():
    """FP64 operations per DoF of the headline kernel (SQ_INSTS_VALU_FLOPS_FP64
    x 64 lanes, FMA = 2) from the committed counter summary, if it was taken
    on the current kernel source."""
    if not os.path.exists(VALU_FILE):
        return None
    txt = open(VALU_FILE).read()
    m = re.search(r"kernel_source_sha1:\s*(\w+)", txt)
    if not m or m.group(1) != kernel_hash():
        return None
    m = re.search(r"f64_flop_per_dof:\s*([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None



def time_apply(op, x, y, steps, warmup, torch):
    for _ in range(warmup):
        op.apply(x, y)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        op.apply(x, y)
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def measure_hbm(torch, gib=2, reps=10):
    """Practical HBM rates on this GPU: a read-only pass (sum) and a copy over
    arrays of gib GiB, far beyond the 256 MB last-level cache."""
    n = gib * (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    out = {}
    for name, fn, nbytes in (("read", lambda: a.sum(), n * 8), ("copy", lambda: b.copy_(a), 2 * n * 8)):
        fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        out[f"{name}_gbs"] = nbytes / (s.elapsed_time(e) / reps * 1e-3) / 1e9
    del a, b
    return out


def time_apply_each(op, x, y, reps, torch, flush=None):
    """Per-launch times (ms) of reps individually bracketed applies; with
    flush, a write of that tensor precedes every launch so that nothing of
    the operands is left in the 256 MB last-level cache (cold state)."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        if flush is not None:
            flush.fill_(1.0)
        a.record()
        op.apply(x, y)
        b.record()
    torch.cuda.synchronize()
    return sorted(a.elapsed_time(b) for a, b in ev)


# ---------------------------------------------------------------------------
# Parity bookkeeping: the GPU legs keep their results on a sample of cells
# (outside the timed regions); the CPU leg evaluates the oracle there.
# ---------------------------------------------------------------------------

def parity_cells(ncell, seed, count=96, boundary=24):
    import synth
    return synth.sample_cells(ncell, count, seed, n_boundary=boundary)


def keep_rows(rec, prec, y, cells, problem, src, global_cells=None):
    """Keep the rows of y (a device vector in DoF order) of the sampled cells
    for the oracle check.  problem: (ncell, degree, keyword arguments of the
    oracle's problem); src = (length, seed) of the FP64 source draw (FP32
    runs are compared with the oracle of the FP64 draw they round);
    global_cells: the same cells numbered in the oracle's mesh, if it is
    larger than the GPU operator's (a partition)."""
    import torch
    n3 = (problem[1] + 1) ** 3
    idx = torch.from_numpy(cells).to(y.device)
    rows = y.view(-1, n3).index_select(0, idx).double().cpu().numpy()
    PARITY.append(dict(rec=rec, kind="apply", tol=TOL[prec], rows=rows,
                       cells=cells if global_cells is None else global_cells, problem=problem, src=src))


def keep_solution(rec, x, b, problem, cells=None):
    """Keep a solve's FP64 solution (host) and right-hand side for the
    oracle's residual; cells: rows to check (None: every row)."""
    PARITY.append(dict(rec=rec, kind="residual", x=x.cpu().numpy(), b=b.cpu().numpy(), cells=cells,
                       problem=problem))


def check_parity(oracle):
    """The oracle on every kept sample: relative l2 of the GPU rows against
    the oracle's rows (apply), or the oracle's relative residual
    ||b - A x|| / ||b|| of a solution (on sampled rows for the large solves)."""
    import numpy as np
    import synth
    last = [None, None]   # the last source drawn: (length, seed), vector
    t0 = time.perf_counter()
    for item in PARITY:
        ncell, k, kw = item["problem"]
        p = oracle.problem(ncell, k, **kw)
        if item["kind"] == "apply":
            if last[0] != item["src"]:
                last[:] = [item["src"], None]
                last[1] = synth.src_vector(*item["src"])
            ref = oracle.apply_cells(p, last[1], item["cells"])
            err = float(np.linalg.norm(item["rows"] - ref) / np.linalg.norm(ref))
            item["rec"]["err_vs_oracle"] = {"rel_l2": err, "tol": item["tol"], "ok": bool(err <= item["tol"]),
                                            "cells": int(len(item["cells"])),
                                            "of": "rows of the sampled cells (random, corners, boundary)"}
        else:
            x, b, cells = item["x"], item["b"], item["cells"]
            n3 = (k + 1) ** 3
            if cells is None:
                r = b - oracle.apply(p, x)
                nb = np.linalg.norm(b)
                what = "every row"
            else:
                bb = b.reshape(-1, n3)[cells]
                r = bb - oracle.apply_cells(p, x, cells)
                nb = np.linalg.norm(bb)
                what = f"rows of {len(cells)} sampled cells"
            item["rec"]["oracle_rel_residual"] = {"value": float(np.linalg.norm(r) / nb), "of": what}
    PARITY.clear()
    return time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(ncell, k, budget_s=8.0):
    """The CPU leg: the oracle timed on the host cores, and the oracle
    checks of every kept GPU result.
      on the fly  the oracle's matrix-free apply (plain point-by-point
                  quadrature, OpenMP over cells) on a sample of the headline
                  mesh, repeated for budget_s; DoF/s over the processed cells
                  (extrapolated to the whole mesh: the cost per cell is flat);
      matrix      the matrix-based comparator: block rows assembled by full
                  quadrature (7 dense n^3 x n^3 blocks per cell) and the
                  block-sparse product, config 1 whole and config 2 at k=2..4
                  on a contiguous run of block rows; assembly seconds and
                  SpMV DoF/s per row are extrapolated to the whole mesh (the
                  whole config-2 matrices, 1.3 to 28.7 GB, take minutes to
                  assemble)."""
    import numpy as np
    import oracle
    import synth
    p = oracle.problem(ncell, k, curved=True)
    nd = oracle.n_dofs(p)
    src = synth.src_vector(nd, synth.seed_for(2, k))
    cells = np.arange(min(4096, ncell ** 3), dtype=np.int64)
    n3 = (k + 1) ** 3
    oracle.apply_cells(p, src, cells[:64])  # warm up tables and threads
    done, t0 = 0, time.perf_counter()
    while True:
        oracle.apply_cells(p, src, cells)
        done += len(cells)
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    out = {"value": done * n3 / el, "unit": "DoF/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"{len(cells)} cells ({len(cells) * n3} DoFs) of the {ncell}^3 curved k={k} mesh, "
                     f"applied {done // len(cells)} times in {el:.1f} s (matrix-free, on the fly)",
           "extrapolated_from_sample": True, "sample_fraction": len(cells) / ncell ** 3,
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    out["matrix_based"] = matrix_baseline(oracle, np, synth)
    out["parity_check_s"] = check_parity(oracle)
    return out


# a sampled matrix below this size may be served partly from the host's
# last-level cache, so its SpMV rate can exceed what the whole matrix gets
CPU_LLC_BOUND_BYTES = 512 << 20
MATRIX_CASES = (("config1_8cubed_affine_k3", 8, 3, dict(), 512),
                ("config2_32cubed_curved_k2", 32, 2, dict(curved=True), 2048),
                ("config2_32cubed_curved_k3", 32, 3, dict(curved=True), 1024),
                ("config2_32cubed_curved_k4", 32, 4, dict(curved=True), 512))


def matrix_baseline(oracle, np, synth, cases=MATRIX_CASES, spmv_s=1.5):
    """Assembly seconds and block-sparse SpMV rate of the oracle's matrix per
    case (name, cells per edge, degree, problem keywords, block rows
    assembled), extrapolated from the assembled rows to the whole mesh."""
    out = {}
    for name, ncell, k, kw, rows in cases:
        p = oracle.problem(ncell, k, **kw)
        total = ncell ** 3
        cells = np.arange(min(rows, total), dtype=np.int64)
        n3 = (k + 1) ** 3
        src = synth.src_vector(oracle.n_dofs(p), synth.seed_for(1 if ncell == 8 else 2, k))
        t0 = time.perf_counter()
        blocks = oracle.block_rows(p, cells)
        t_asm = time.perf_counter() - t0
        y = oracle.spmv_blocks(p, cells, blocks, src)  # first touch
        reps, t0 = 0, time.perf_counter()
        while True:
            y = oracle.spmv_blocks(p, cells, blocks, src)
            reps += 1
            el = time.perf_counter() - t0
            if el >= spmv_s:
                break
        # the matrix-based product is the same operator (pinned), checked here on the sample
        ref = oracle.apply_cells(p, src, cells[:64])
        err = float(np.linalg.norm(y[:64] - ref) / np.linalg.norm(ref))
        frac = len(cells) / total
        out[name] = {"rows_assembled": int(len(cells)), "of_rows": total, "sample_fraction": frac,
                     "extrapolated_from_sample": frac < 1.0, "matrix_bytes": int(blocks.nbytes / frac),
                     "sample_matrix_bytes": int(blocks.nbytes),
                     "sample_may_be_cache_resident": bool(blocks.nbytes < CPU_LLC_BOUND_BYTES),
                     "assembly_s": t_asm / frac, "spmv_dofs_per_s": reps * len(cells) * n3 / el,
                     "spmv_gbs": reps * blocks.nbytes / el / 1e9, "spmv_vs_matrix_free_rel_l2": err}
        del blocks
    return out


PAPER_CONTEXT = {
    "note": "Intel CPU results of the paper (Hermite-like basis, Cartesian meshes); context, not comparable one to one",
    "broadwell_2x14_full_operator_dofs_per_s": {"p2": 1.243e9, "p3": 1.336e9, "p5": 1.527e9, "p8": 1.203e9},
    "broadwell_or_knl_operator_without_exchange_dofs_per_s": "1.8e9 to 2.1e9 for 3 <= p <= 8",
    "knl_64_cores_compute_only_dofs_per_s": "above 3e9 for 2 <= p <= 10",
    "haswell_e5_2697v3_node_p5_56.6M_dofs": {"fp64_dofs_per_s": 1.36e9, "fp32_dofs_per_s": 2.59e9},
    "hypershell_geometry_computed_on_the_fly_dofs_per_s": "at most 3.5e8 (28 Broadwell cores)",
}
VARIANTS = ("affine-variable", "curved", "curved-merged")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--ncell", type=int, default=32)
    ap.add_argument("--degree", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["f64", "f32"], default=None)
    ap.add_argument("--no-variants", dest="variants", action="store_false",
                    help="skip every leg but the headline, the solves and the serving trace")
    ap.add_argument("--legs", default=",".join(LEGS), help="comma-separated legs to run: " + ",".join(LEGS))
    ap.add_argument("--variant", choices=VARIANTS, default=None,
                    help="run only this geometry in the 64^3 comparison (variants leg)")
    ap.add_argument("--solve-reps", type=int, default=20,
                    help="repeated config-4 solves per mode for the latency percentiles (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests in the serving trace (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-budget-gib", type=float, default=128.0, help="HBM admission budget")
    ap.add_argument("--serve-low-rate", type=float, default=10.0,
                    help="arrival rate of a second, lighter trace (0: skip)")
    ap.add_argument("--serve-low-requests", type=int, default=100,
                    help="requests in the lighter trace")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one MI355X only; runs on more than one GPU are not supported "
              "(the one-GPU share of a sharded apply is the 'shard' entry of the output)", file=sys.stderr)
        sys.exit(2)
    legs = set(args.legs.split(","))
    unknown = legs - set(LEGS)
    if unknown:
        ap.error(f"unknown legs {sorted(unknown)}")
    if not args.variants:
        legs &= {"headline", "solve", "serve"}
    if args.solve_reps <= 0:
        legs.discard("solve")
    if args.serve_requests <= 0:
        legs.discard("serve")

    import numpy as np
    import torch

    import paper_1711_03590_amd as dg
    import synth

    torch.cuda.set_device(0)
    k, N = args.degree, args.ncell
    seed = synth.seed_for(2, k)
    res = {}
    if "headline" in legs:
        op = dg.Operator(N, k, curved=True, amplitude=synth.AMPLITUDE)
        nd = op.n_dofs
        src = synth.src_vector(nd, seed)
        cells = parity_cells(N, seed)
        flush = torch.empty(512 * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        for prec in ("f64", "f32"):
            if args.only and prec != args.only:
                continue
            dt = torch.float64 if prec == "f64" else torch.float32
            x = torch.from_numpy(src).to(dtype=dt, device="cuda")
            y = torch.empty_like(x)
            ms = time_apply(op, x, y, args.steps, args.warmup, torch)
            bpd = algorithmic_bytes_per_dof(N, k, 8 if prec == "f64" else 4)
            achieved = bpd * nd / (ms * 1e-3) / 1e9
            traffic = measured_traffic(prec)
            warm = time_apply_each(op, x, y, 50, torch)
            cold = time_apply_each(op, x, y, 20, torch, flush=flush)
            r = dict(ms=ms, dofs=nd / (ms * 1e-3), bytes_per_dof=bpd, achieved_gbs=achieved,
                     frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                     per_launch_us={"median": 1e3 * warm[len(warm) // 2], "min": 1e3 * warm[0],
                                    "cold_median": 1e3 * cold[len(cold) // 2], "cold_min": 1e3 * cold[0]})
            keep_rows(r, prec, y, cells, (N, k, dict(curved=True)), (nd, seed))
            res[prec] = r
            del x, y
        del flush
        op.close()
    hbm = measure_hbm(torch) if "headline" in legs else None

    out = {}
    if "merged" in legs:
        out["merged_geometry"] = bench_merged(dg, torch, synth, N, k, args.steps, args.warmup, res)
    if "positions" in legs:
        out["positions_geometry"] = bench_merged(dg, torch, synth, N, k, args.steps, args.warmup, res,
                                                 storage="positions")
    if "hermite" in legs:
        out["hermite_basis"] = bench_hermite(dg, torch, synth, N, k, args.steps, args.warmup, res)
    if "advection" in legs:
        out["advection"] = bench_advection(dg, torch, synth, N, k, args.steps, args.warmup)
    if "shard" in legs:
        out["shard"] = bench_shard(dg, torch, synth, k, args.steps, args.warmup)
    if "variants" in legs:
        out["geometry_variants"] = bench_variants(dg, torch, synth, k, only=args.variant)
    if "degrees" in legs:
        out["degree_sweep"] = bench_degrees(dg, torch, synth)

    if args.copy_calibration:
        nel = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(nel, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b

    if "solve" in legs:
        out["solve"] = bench_solve(dg, torch, np, synth, args.solve_reps)
    if "serve" in legs:
        serving = bench_serve(synth, args.serve_requests, args.serve_rate, args.serve_budget_gib)
        if args.serve_low_rate > 0:
            serving["below_capacity"] = bench_serve(synth, args.serve_low_requests, args.serve_low_rate,
                                                    args.serve_budget_gib, keep_smallest=0)
        out["serve"] = serving

    head = res.get("f64") or res.get("f32")
    headp = "f64" if "f64" in res else "f32"
    kname = f"sipg_apply_kernel<{k + 1}, {'double' if headp == 'f64' else 'float'}, CURVED>"
    line = {
        "metric": METRIC,
        "value": head["dofs"] if head else None,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"] if head else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": headp,
        "data": "synthetic: seeded uniform [-1,1] source on a generated mesh",
        "config": {"workload": f"SIPG Laplacian apply, {N}^3 sine-curved hex mesh (amplitude 0.05), "
                               f"degree k={k}, G3 geometry at every quadrature point, {N ** 3 * (k + 1) ** 3} DoFs",
                   "ncell": N, "degree": k, "n_dofs": N ** 3 * (k + 1) ** 3, "geometry": "curved-G3"},
    }
    if head:
        alg = head["bytes_per_dof"] * line["config"]["n_dofs"]
        cold_us = head["per_launch_us"]["cold_median"]
        line["roofline"] = {
            "bound": "hbm", "achieved": head["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": head["frac"], "traffic": head["traffic"],
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": alg, "algorithmic_bytes_per_dof": head["bytes_per_dof"],
            "kernel": kname,
            "state": ("warm: back-to-back launches, successive ones walking the cells in opposite orders, so part "
                      "of the operands comes from the 256 MB MALL (an effective rate, above what DRAM alone gives)"),
            "cold": {"us_per_launch": cold_us, "achieved": alg / (cold_us * 1e-6) / 1e9,
                     "frac": alg / (cold_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                     "state": "median launch after a 512 MiB write evicted the operands from the MALL"}}
        line["per_launch_us"] = head["per_launch_us"]
        line["err_vs_oracle"] = None
        fpd = measured_flop_per_dof() if (headp == "f64" and k == 4 and N == 32) else None
        line["flop_rate"] = None if fpd is None else {
            "flop_per_dof": fpd, "tflops": head["dofs"] * fpd / 1e12, "peak_tflops": FP64_VECTOR_PEAK_TFLOPS,
            "frac": head["dofs"] * fpd / 1e12 / FP64_VECTOR_PEAK_TFLOPS}
        line["hbm_measured"] = dict(hbm, frac_of_read=head["achieved_gbs"] / hbm["read_gbs"])
    if "f32" in res and headp == "f64":
        r = res["f32"]
        line["fp32"] = {"value": r["dofs"], "ms_per_step": r["ms"], "achieved_gbs": r["achieved_gbs"],
                        "frac": r["frac"], "traffic": r["traffic"], "algorithmic_bytes_per_dof": r["bytes_per_dof"],
                        "per_launch_us": r["per_launch_us"], "speedup_vs_fp64": r["dofs"] / head["dofs"],
                        "err_vs_oracle": None}
    line.update(out)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(N, k)
    # the parity numbers of the headline records land in res (kept before the line existed)
    if "f64" in res or "f32" in res:
        if headp in res:
            line["err_vs_oracle"] = res[headp].get("err_vs_oracle")
        if "fp32" in line:
            line["fp32"]["err_vs_oracle"] = res["f32"].get("err_vs_oracle")
    line["paper_context"] = PAPER_CONTEXT
    print(json.dumps(line), flush=True)


def bench_variants(dg, torch, synth, k, ncell=64, steps=30, only=None):
    """64^3 cells, degree k: affine mesh with the variable coefficient (one
    stored value per cell and face point) against the sine-curved mesh with
    stored Jacobians (G3) and with the merged coefficient (G4), FP64 and
    FP32, to compare the traffic of affine and general geometry."""
    out = {}
    seed = synth.seed_for(3, k)
    nd = ncell ** 3 * (k + 1) ** 3
    cells = parity_cells(ncell, seed)
    for name, curved, var in (("affine-variable", False, True), ("curved", True, False),
                              ("curved-merged", True, False)):
        if only and name != only:
            continue
        op = dg.Operator(ncell, k, curved=curved, variable_coef=var, amplitude=synth.AMPLITUDE,
                         merged=name == "curved-merged")
        src = synth.src_vector(nd, seed)
        rec = {"n_dofs": nd}
        for prec in ("f64", "f32"):
            dt = torch.float64 if prec == "f64" else torch.float32
            x = torch.from_numpy(src).to(dtype=dt, device="cuda")
            y = torch.empty_like(x)
            ms = time_apply(op, x, y, steps, 3, torch)
            bpd = algorithmic_bytes_per_dof(ncell, k, 8 if prec == "f64" else 4, name)
            gbs = bpd * nd / (ms * 1e-3) / 1e9
            rec[prec] = {"dofs_per_s": nd / (ms * 1e-3), "us": ms * 1e3, "algorithmic_bytes_per_dof": bpd,
                         "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}
            keep_rows(rec[prec], prec, y, cells, (ncell, k, dict(curved=curved, variable_coef=var)),
                      (nd, seed))
            del x, y
        op.close()
        del src
        out[name] = rec
    out["workload"] = (f"{ncell}^3 cells, k={k}, affine with c = 1 + 0.5 sin(pi x) cos(pi y) z vs sine-curved, "
                       "stored Jacobians (G3) and merged coefficient (G4)")
    return out


def bench_degrees(dg, torch, synth, ncell=32, degrees=range(2, 9), steps=50):
    """The headline mesh (32^3 sine-curved, G3) at every degree 2..8: DoF/s
    and the fraction of the HBM roofline, FP64 and FP32."""
    out = {}
    for k in degrees:
        op = dg.Operator(ncell, k, curved=True, amplitude=synth.AMPLITUDE)
        nd = op.n_dofs
        seed = synth.seed_for(2, k)
        src = synth.src_vector(nd, seed)
        cells = parity_cells(ncell, seed, count=64 if k >= 7 else 96)
        rec = {"n_dofs": nd}
        for prec in ("f64", "f32"):
            dt = torch.float64 if prec == "f64" else torch.float32
            x = torch.from_numpy(src).to(dtype=dt, device="cuda")
            y = torch.empty_like(x)
            ms = time_apply(op, x, y, steps, 5, torch)
            bpd = algorithmic_bytes_per_dof(ncell, k, 8 if prec == "f64" else 4)
            gbs = bpd * nd / (ms * 1e-3) / 1e9
            rec[prec] = {"dofs_per_s": nd / (ms * 1e-3), "us": ms * 1e3, "algorithmic_bytes_per_dof": bpd,
                         "frac": gbs / HBM_PEAK_GBS}
            keep_rows(rec[prec], prec, y, cells, (ncell, k, dict(curved=True)),
                      (nd, seed))
            del x, y
        op.close()
        out[f"k{k}"] = rec
    out["workload"] = f"{ncell}^3 sine-curved, stored Jacobians (G3), degrees {min(degrees)}..{max(degrees)}"
    return out


def bench_merged(dg, torch, synth, ncell, k, steps, warmup, g3, storage="merged"):
    """The headline workload with the merged cell geometry (G4): same
    operator up to rounding, 6 instead of 10 values per cell point; or
    (storage="positions") with the quadrature-point positions (G2): 4 values
    per point, Jacobians by collocation derivatives in the kernel (the
    oracle's positions reading)."""
    op = dg.Operator(ncell, k, curved=True, amplitude=synth.AMPLITUDE, storage=storage)
    nd = op.n_dofs
    seed = synth.seed_for(2, k)
    src = synth.src_vector(nd, seed)
    cells = parity_cells(ncell, seed)
    name = "curved-merged" if storage == "merged" else "curved-positions"
    label = "merged cell geometry (G4)" if storage == "merged" else "cell geometry from quadrature-point positions (G2)"
    okw = dict(curved=True, cell_geometry="positions" if storage == "positions" else "map")
    out = {"workload": f"{ncell}^3 sine-curved, k={k}, {label}"}
    for prec in ("f64", "f32"):
        dt = torch.float64 if prec == "f64" else torch.float32
        x = torch.from_numpy(src).to(dtype=dt, device="cuda")
        y = torch.empty_like(x)
        ms = time_apply(op, x, y, steps, warmup, torch)
        bpd = algorithmic_bytes_per_dof(ncell, k, 8 if prec == "f64" else 4, name)
        gbs = bpd * nd / (ms * 1e-3) / 1e9
        out[prec] = {"dofs_per_s": nd / (ms * 1e-3), "us": ms * 1e3, "algorithmic_bytes_per_dof": bpd,
                     "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}
        if prec in g3:
            out[prec]["speedup_vs_g3"] = out[prec]["dofs_per_s"] / g3[prec]["dofs"]
        keep_rows(out[prec], prec, y, cells, (ncell, k, okw), (nd, seed))
        del x, y
    op.close()
    return out


def bench_hermite(dg, torch, synth, ncell, k, steps, warmup, g3):
    """The headline workload in the Hermite-like basis (a neighbour's face
    data from two of its N coefficients per normal line), with the stored
    Jacobians (G3) and with the merged coefficient (G4).  Same bytes per DoF
    as the nodal runs; a different, equivalent operator (the oracle's
    Hermite-like basis)."""
    out = {"workload": f"{ncell}^3 sine-curved, k={k}, Hermite-like basis"}
    seed = synth.seed_for(2, k)
    cells = parity_cells(ncell, seed)
    for geo, merged in (("G3", False), ("G4", True)):
        op = dg.Operator(ncell, k, curved=True, amplitude=synth.AMPLITUDE, merged=merged, basis="hermite")
        nd = op.n_dofs
        src = synth.src_vector(nd, seed)
        out[geo] = {}
        for prec in ("f64", "f32"):
            dt = torch.float64 if prec == "f64" else torch.float32
            x = torch.from_numpy(src).to(dtype=dt, device="cuda")
            y = torch.empty_like(x)
            ms = time_apply(op, x, y, steps, warmup, torch)
            bpd = algorithmic_bytes_per_dof(ncell, k, 8 if prec == "f64" else 4,
                                            "curved-merged" if merged else "curved")
            gbs = bpd * nd / (ms * 1e-3) / 1e9
            r = {"dofs_per_s": nd / (ms * 1e-3), "us": ms * 1e3, "algorithmic_bytes_per_dof": bpd,
                 "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}
            if geo == "G3" and prec in g3:
                r["speedup_vs_nodal"] = r["dofs_per_s"] / g3[prec]["dofs"]
            keep_rows(r, prec, y, cells, (ncell, k, dict(curved=True, basis="hermite")),
                      (nd, seed))
            out[geo][prec] = r
            del x, y
        op.close()
    return out


def bench_shard(dg, torch, synth, k, steps, warmup, ncell=64, parts=8):
    """One GPU's share of the 64^3 sine-curved mesh (variable c, G3) cut into
    `parts` z-slabs: a 64 x 64 x 8 slab with both z sides ghost.  A step is
    what that GPU computes per apply: the face traces of its two z sides
    (sent to its neighbours) and the apply with the traces it received.  The
    transfer itself is not part of a one-GPU run.  The source is one draw
    over the whole 64^3 mesh: the slab's own part, and the traces of the
    slabs below and above computed from theirs (traces depend on the
    coefficients alone, so this op computes them), so that the slab's rows
    are the whole mesh's rows of A u and the oracle checks them there."""
    nz = ncell // parts
    z0 = nz * (parts // 2 - 1)
    op = dg.Operator((ncell, ncell, nz), k, curved=True, amplitude=synth.AMPLITUDE, variable_coef=True,
                     bc=(0, 0, 0, 0, dg.GHOST, dg.GHOST), lo=(0.0, 0.0, z0 / ncell), hi=(1.0, 1.0, (z0 + nz) / ncell))
    nd = op.n_dofs
    n = k + 1
    plane = ncell * ncell
    seed = synth.seed_for(3, k)
    ndg = ncell ** 3 * n ** 3
    full = synth.src_vector(ndg, seed)
    out = {"workload": f"{ncell}x{ncell}x{nz} slab (z in [{z0}/{ncell}, {z0 + nz}/{ncell})) of the {ncell}^3 "
                       f"sine-curved mesh, k={k}, variable c, G3, ghost z sides; step = 2 trace launches + ghost apply",
           "n_dofs": nd, "halo_values_per_side": plane * 2 * n * n}
    cells = parity_cells((ncell, ncell, nz), seed)
    cells_global = cells + z0 * plane
    cells_n = plane * nz
    faces = 2 * (ncell + 1) * ncell * nz + plane * (nz + 1)
    for prec in ("f64", "f32"):
        dt = torch.float64 if prec == "f64" else torch.float32
        rb = 8 if prec == "f64" else 4
        part = lambda z: torch.from_numpy(full[z * plane * n ** 3:(z + nz) * plane * n ** 3]).to(dtype=dt,
                                                                                                   device="cuda")
        own, below, above = part(z0), part(z0 - nz), part(z0 + nz)
        ghost = {4: op.face_traces(5, below), 5: op.face_traces(4, above)}
        sent = {4: torch.empty_like(ghost[4]), 5: torch.empty_like(ghost[5])}
        y = torch.empty_like(own)

        def step():
            op.face_traces(4, own, sent[4])
            op.face_traces(5, own, sent[5])
            op.apply_ghost(own, ghost, y)

        def timed(fn):
            for _ in range(warmup):
                fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(steps):
                fn()
            b.record()
            torch.cuda.synchronize()
            return a.elapsed_time(b) / steps

        ms_step = timed(step)
        ms_apply = timed(lambda: op.apply_ghost(own, ghost, y))
        halo = 2 * plane * 2 * n * n
        # src + dst + G3 cell and face geometry + traces received; the trace
        # launches add their layers' reads and the traces sent
        apply_bytes = (2 + 10) * cells_n * n ** 3 * rb + 4 * faces * n * n * rb + halo * rb
        trace_bytes = 2 * plane * n ** 3 * rb + halo * rb
        out[prec] = {"us_per_step": ms_step * 1e3, "us_apply": ms_apply * 1e3, "dofs_per_s": nd / (ms_step * 1e-3),
                     "apply_algorithmic_bytes": apply_bytes, "trace_algorithmic_bytes": trace_bytes,
                     "frac": (apply_bytes + trace_bytes) / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "apply_frac": apply_bytes / (ms_apply * 1e-3) / 1e9 / HBM_PEAK_GBS}
        keep_rows(out[prec], prec, y, cells, (ncell, k, dict(curved=True, variable_coef=True)),
                  (ndg, seed), global_cells=cells_global)
        del own, below, above, ghost, sent, y
    op.close()
    return out


def bench_advection(dg, torch, synth, ncell, k, steps, warmup):
    """The advection operator with the upwind flux (Sec. 2 Eq. (1)) on the
    headline mesh: rotating velocity, FP64 and FP32."""
    op = dg.AdvectionOperator(ncell, k, curved=True, amplitude=synth.AMPLITUDE, velocity="rotation")
    nd = op.n_dofs
    seed = synth.seed_for(6, k)
    src = synth.src_vector(nd, seed)
    cells = parity_cells(ncell, seed)
    out = {"workload": f"{ncell}^3 sine-curved, k={k}, upwind advection, c = (1/2 - y, x - 1/2, 1/4)"}
    for prec in ("f64", "f32"):
        dt = torch.float64 if prec == "f64" else torch.float32
        x = torch.from_numpy(src).to(dtype=dt, device="cuda")
        y = torch.empty_like(x)
        ms = time_apply(op, x, y, steps, warmup, torch)
        bpd = algorithmic_bytes_per_dof(ncell, k, 8 if prec == "f64" else 4, "advection")
        gbs = bpd * nd / (ms * 1e-3) / 1e9
        out[prec] = {"dofs_per_s": nd / (ms * 1e-3), "us": ms * 1e3, "algorithmic_bytes_per_dof": bpd,
                     "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}
        keep_rows(out[prec], prec, y, cells, (ncell, k, dict(curved=True, op="advection", velocity="rotation")),
                  (nd, seed))
        del x, y
    op.close()
    return out


def bench_solve(dg, torch, np, synth, reps):
    """Manufactured Poisson solve on the 32^3 curved mesh, k=5, variable c,
    to 1e-10: mixed precision (FP32 CG inside FP64 refinement) against pure
    FP64 CG.  The FP64 operator (residuals, convergence check) always stores
    the Jacobians (G3).  Config 4 as written is restarted iterative
    refinement (mode 1: every outer step restarts the FP32 CG with inner
    tolerance 1e-4) with the stored Jacobians in both precisions; the fastest
    mixed scheme here keeps the FP32 CG's search direction across FP64
    residual refreshes (mode 2, reliable updates at a 0.3 drop) and runs its
    FP32 inner solver on the merged coefficient (G4, the same operator up to
    rounding).  Every solution's FP64 residual is re-verified with the
    oracle on sampled rows."""
    runs = (("config4_ir_restarted_g3", 1, dict(), "restarted iterative refinement, FP32 CG to 1e-4 per outer "
                                                   "step, stored Jacobians in both precisions"),
            ("mixed", 2, dict(storage="mixed"), "reliable updates (FP32 CG direction kept, FP64 residual "
                                                "refreshed at a 0.3 drop), FP32 on the merged coefficient"),
            ("mixed_fp32_g3", 2, dict(), "reliable updates, stored Jacobians in both precisions"),
            ("mixed_ir_restarted", 1, dict(storage="mixed"), "restarted iterative refinement, FP32 on the merged "
                                                             "coefficient"),
            ("fp64", 0, dict(), "FP64 Jacobi-CG"),
            ("mixed_hermite", 2, dict(storage="mixed", basis="hermite"), "reliable updates, Hermite-like basis"))
    out = {}
    cells = parity_cells(32, synth.seed_for(4, 5), count=48, boundary=16)
    for name, mode, kw, scheme in runs:
        op = dg.Operator(32, 5, curved=True, variable_coef=True, **kw)
        b = op.rhs()
        times, last = [], None
        for r in range(reps + 1):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, st = op.cg_solve(b, x, mode=mode, rel_tol=1e-10)
            torch.cuda.synchronize()
            if r > 0:
                times.append((time.perf_counter() - t0) * 1e3)
            last = (x, st)
        x, st = last
        l2, h1 = op.error_manufactured(x)
        t = np.array(times)
        out[name] = {"p50_ms": float(np.percentile(t, 50)), "p99_ms": float(np.percentile(t, 99)), "mode": mode,
                     "scheme": scheme,
                     "operator": {"storage": kw.get("storage", "jacobian"), "basis": kw.get("basis", "nodal")},
                     "reps": reps, "converged": st["converged"], "iters_inner": st["iters_inner"],
                     "iters_outer": st["iters_outer"], "applies_f64": st["applies_f64"],
                     "applies_f32": st["applies_f32"], "final_rel_residual": st["final_rel_residual"],
                     "l2_error_vs_exact": l2}
        if kw.get("basis") == "hermite":
            # the coefficients are in the Hermite-like basis: the oracle's
            # operator in that basis
            keep_solution(out[name], x, b, (32, 5, dict(curved=True, variable_coef=True, basis="hermite")), cells)
        else:
            keep_solution(out[name], x, b, (32, 5, dict(curved=True, variable_coef=True)), cells)
        op.close()
    out["workload"] = "32^3 curved, k=5 (7,077,888 DoFs), c = 1 + 0.5 sin(pi x) cos(pi y) z, to 1e-10"
    for name, _, _, _ in runs:
        if name != "fp64":
            out[name]["speedup_vs_fp64_p50"] = out["fp64"]["p50_ms"] / out[name]["p50_ms"]
    out["speedup_mixed_vs_fp64_p50"] = out["config4_ir_restarted_g3"]["speedup_vs_fp64_p50"]
    out["speedup_mixed_vs_fp64_p50_scheme"] = "config 4 as written: " + runs[0][3]
    out["speedup_best_mixed_vs_fp64_p50"] = out["mixed"]["speedup_vs_fp64_p50"]
    out["speedup_best_mixed_vs_fp64_p50_scheme"] = runs[1][3]
    return out


def bench_serve(synth, n_requests, rate, budget_gib, keep_smallest=3):
    """Config 5: open-loop Poisson arrivals, edge cells log-uniform in [4,48],
    degree uniform in 2..7, half curved; mixed-precision solves to 1e-8
    admitted by HBM footprint into one continuously batched solver.  The
    keep_smallest smallest requests keep their solutions, whose residual the
    oracle re-verifies."""
    from paper_1711_03590_amd import serve
    trace = synth.request_trace(n_requests, rate=rate, seed=5005)
    small = sorted(trace, key=lambda r: serve.request_bytes(r)[1])[:keep_smallest]
    keep_ids = {r["id"] for r in small}
    kept = []
    rep = serve.serve(trace, budget_bytes=int(budget_gib * (1 << 30)), max_slots=48, rounds_per_step=20,
                      rel_tol=1e-8, keep=lambda r: r["id"] in keep_ids,
                      log=lambda d: kept.append(d) if "x" in d else None)
    rep["workload"] = (f"{n_requests} requests, Poisson arrivals at {rate:g}/s, edge cells log-uniform in [4,48], "
                       "degree uniform in 2..7, 50% curved, seeded uniform RHS, mixed CG to 1e-8")
    checks = []
    for d in kept:
        c = {"id": d["id"], "ncell": list(d["ncell"]), "degree": d["degree"], "curved": d["curved"],
             "final_rel_residual": d["final_rel_residual"]}
        PARITY.append(dict(rec=c, kind="residual", x=d["x"], b=d["b"], cells=None,
                           problem=(tuple(d["ncell"]), d["degree"], dict(curved=d["curved"]))))
        checks.append(c)
    if checks:
        rep["oracle_checked_requests"] = checks
    return rep


if __name__ == "__main__":
    main()
