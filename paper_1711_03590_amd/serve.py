"""Request loop for SIPG Poisson solves with continuous batching.

Requests arrive open-loop at their trace times.  Each is admitted, first
come first served, when a batch slot is free and its HBM footprint
(operator geometry and diagonal in both precisions, right-hand side,
solution and solver workspace) fits in the budget next to the requests
already resident; its operator is then built on the GPU and its solve joins
the batch.  The loop advances all resident solves together a few CG
iterations at a time and retires finished ones as they complete.  Latency is
completion time minus arrival time.  Curved operators keep the stored
Jacobians for their FP64 residuals and the merged coefficient for the FP32
inner solver (the mixed geometry storage), which is the cheaper resident
footprint and the faster inner apply.
"""
from __future__ import annotations

import collections
import time

import numpy as np

from . import Batch, Operator, footprint

# bytes per DoF of a resident request besides the operator: b, x, FP64
# residual (8 B each) and the FP32 correction, residual, direction and
# product vectors (4 B each)
WORKSPACE_BYTES_PER_DOF = 3 * 8 + 4 * 4
STORAGE = "mixed"


def request_bytes(req):
    n = req["ncell"][0] * req["ncell"][1] * req["ncell"][2] * (req["degree"] + 1) ** 3
    return (footprint(req["ncell"], req["degree"], curved=req["curved"], storage=STORAGE)
            + WORKSPACE_BYTES_PER_DOF * n, n)


def serve(trace, *, budget_bytes, max_slots=32, rounds_per_step=10, rel_tol=1e-8, time_limit=None, log=None,
          keep=None):
    """Serve `trace` (dicts with arrival, ncell, degree, curved, rhs_seed).
    log(record) is called for every finished request; for requests where
    keep(request) is true the record also holds host copies of the
    right-hand side "b" and the solution "x" (for checking them elsewhere)."""
    import torch
    t0 = time.perf_counter()
    pending = collections.deque(sorted(trace, key=lambda r: r["arrival"]))
    waiting = collections.deque()
    inflight = {}
    done = []
    used = peak = 0
    # device memory actually in use (hipMemGetInfo), relative to the start
    free0, total = torch.cuda.mem_get_info()
    dev_peak = 0
    torch.cuda.reset_peak_memory_stats()
    alloc0 = torch.cuda.memory_allocated()
    batch = Batch(max_slots)
    try:
        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            if time_limit is not None and now > time_limit:
                break
            while pending and pending[0]["arrival"] <= now:
                waiting.append(pending.popleft())
            while waiting and batch.active < max_slots:
                req = waiting[0]
                need, ndofs = request_bytes(req)
                if need > budget_bytes:
                    waiting.popleft()            # can never fit: rejected
                    done.append(dict(req, rejected=True))
                    continue
                if used + need > budget_bytes:
                    break                        # wait for memory (FIFO)
                waiting.popleft()
                op = Operator(req["ncell"], req["degree"], curved=req["curved"], storage=STORAGE)
                g = torch.Generator(device="cuda")
                g.manual_seed(req["rhs_seed"])
                b = torch.rand(op.n_dofs, dtype=torch.float64, device="cuda", generator=g) * 2.0 - 1.0
                x = torch.zeros_like(b)
                slot = batch.admit(op, b, x, rel_tol=rel_tol)
                used += need
                peak = max(peak, used)
                inflight[slot] = dict(req=req, op=op, b=b, x=x, need=need, ndofs=ndofs,
                                      admitted=time.perf_counter() - t0)
            if inflight:
                batch.run(rounds_per_step)
                dev_peak = max(dev_peak, free0 - torch.cuda.mem_get_info()[0])
            elif pending:
                time.sleep(max(0.0, min(0.002, pending[0]["arrival"] - (time.perf_counter() - t0))))
            for slot, st in batch.poll():
                rec = inflight.pop(slot)
                t = time.perf_counter() - t0
                extra = {}
                if keep is not None and keep(rec["req"]):
                    extra = dict(b=rec["b"].cpu().numpy(), x=rec["x"].cpu().numpy())
                used -= rec["need"]
                rec["op"].close()
                done.append(dict(rec["req"], ndofs=rec["ndofs"], admitted=rec["admitted"], completed=t,
                                 latency=t - rec["req"]["arrival"], converged=st["final_rel_residual"] <= rel_tol,
                                 iters=st["iters_inner"], refinements=st["iters_outer"],
                                 final_rel_residual=st["final_rel_residual"], **extra))
                if log:
                    log(done[-1])
    finally:
        batch.close()
    elapsed = time.perf_counter() - t0
    ok = [d for d in done if not d.get("rejected")]
    lat = np.array([d["latency"] for d in ok]) if ok else np.array([np.nan])
    span = (trace[-1]["arrival"] - trace[0]["arrival"]) if len(trace) > 1 else 1.0
    return {
        "requests": len(trace), "completed": len(ok), "rejected": len(done) - len(ok),
        "unfinished": len(trace) - len(done),
        "all_converged": all(d["converged"] for d in ok),
        "elapsed_s": elapsed, "solves_per_s": len(ok) / elapsed,
        "offered_per_s": (len(trace) - 1) / span if len(trace) > 1 else None,
        "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_dofs": float(np.mean([d["ndofs"] for d in ok])) if ok else 0.0,
        "dofs_solved_per_s": float(np.sum([d["ndofs"] for d in ok]) / elapsed) if ok else 0.0,
        "peak_hbm_bytes": peak, "peak_hbm_bytes_is": "admission ledger (footprints of the resident requests)",
        "peak_device_bytes_measured": int(dev_peak),
        "peak_device_bytes_measured_is": "device memory held beyond the start (hipMemGetInfo after each step; includes blocks torch's caching allocator keeps)",
        "peak_torch_allocated_bytes": int(torch.cuda.max_memory_allocated() - alloc0),
        "budget_bytes": budget_bytes, "max_slots": max_slots,
    }
