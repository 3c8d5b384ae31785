"""Request loop for SIPG Poisson solves with continuous batching.

Requests arrive open-loop at their trace times.  Each is admitted, first
come first served, when a batch slot is free and its HBM footprint
(operator geometry and diagonal in both precisions, right-hand side,
solution and solver workspace) fits in the budget next to the requests
already resident; its operator is then built on the GPU and its solve joins
a batch.  The resident solves are spread over a few lanes, each a batch on
its own HIP stream advanced a few CG iterations at a time by its own host
thread (lane 0 by the thread that also admits requests): the lanes' kernels
overlap on the GPU, so that one lane's bandwidth-bound vector updates run
beside another lane's applies, and one lane's host work (residual checks,
refinement steps, retiring finished requests) beside the others' GPU work.
A request is handed to the lane with the fewest DoFs assigned to it, whose
thread builds its operator and admits it between two of its steps.
Latency is completion time minus arrival time.
Curved operators keep the stored Jacobians for their FP64 residuals and the
merged coefficient for the FP32 inner solver (the mixed geometry storage),
which is the cheaper resident footprint and the faster inner apply.
"""
from __future__ import annotations

import collections
import threading
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


def _materialize(req, stream):
    """The request's operator (built on `stream`), its seeded right-hand side
    and a zero initial guess, on the GPU."""
    import torch
    op = Operator(req["ncell"], req["degree"], curved=req["curved"], storage=STORAGE, stream=stream)
    g = torch.Generator(device="cuda")
    g.manual_seed(req["rhs_seed"])
    b = torch.rand(op.n_dofs, dtype=torch.float64, device="cuda", generator=g) * 2.0 - 1.0
    x = torch.zeros_like(b)
    return op, b, x


class _Lane:
    """One batch on its own stream.  Only the lane's driving thread touches
    the batch: the admitting thread hands it requests through its inbox."""

    def __init__(self, max_slots, torch):
        self.batch = Batch(max_slots)
        self.stream = torch.cuda.Stream()
        self.recs = {}                    # slot -> record of a resident request
        self.inbox = collections.deque()  # requests assigned, not yet admitted
        self.dofs = 0                     # DoFs assigned and not retired (guarded by serve's lock)
        self.wake = threading.Event()     # set when a request is assigned


def serve(trace, *, budget_bytes, max_slots=48, rounds_per_step=20, rel_tol=1e-8, time_limit=None, log=None,
          keep=None, lanes=4):
    """Serve `trace` (dicts with arrival, ncell, degree, curved, rhs_seed)
    over `lanes` batches on their own streams, with at most max_slots
    requests resident in all.  log(record) is called for every finished
    request; for requests where keep(request) is true the record also holds
    host copies of the right-hand side "b" and the solution "x" (for checking
    them elsewhere)."""
    import torch
    t0 = time.perf_counter()
    pending = collections.deque(sorted(trace, key=lambda r: r["arrival"]))
    waiting = collections.deque()
    done = []
    state = {"used": 0, "peak": 0, "inflight": 0}
    guard = threading.Lock()          # state, lane DoF counts, done and log
    # device memory actually in use (hipMemGetInfo), relative to the start
    free0, total = torch.cuda.mem_get_info()
    dev_peak = 0
    torch.cuda.reset_peak_memory_stats()
    alloc0 = torch.cuda.memory_allocated()
    pool = [_Lane(max_slots, torch) for _ in range(max(1, lanes))]
    stop = threading.Event()
    errors = []

    def admit(lane, req, need, ndofs):
        op, b, x = _materialize(req, lane.stream)
        slot = lane.batch.admit(op, b, x, rel_tol=rel_tol, stream=lane.stream)
        lane.recs[slot] = dict(req=req, op=op, b=b, x=x, need=need, ndofs=ndofs,
                               admitted=time.perf_counter() - t0)

    def retire(lane, slot, st):
        rec = lane.recs.pop(slot)
        t = time.perf_counter() - t0
        extra = {}
        if keep is not None and keep(rec["req"]):
            extra = dict(b=rec["b"].cpu().numpy(), x=rec["x"].cpu().numpy())
        rec["op"].close()
        with guard:
            state["used"] -= rec["need"]
            state["inflight"] -= 1
            lane.dofs -= rec["ndofs"]
            done.append(dict(rec["req"], ndofs=rec["ndofs"], admitted=rec["admitted"], completed=t,
                             latency=t - rec["req"]["arrival"], converged=st["final_rel_residual"] <= rel_tol,
                             iters=st["iters_inner"], refinements=st["iters_outer"],
                             final_rel_residual=st["final_rel_residual"], **extra))
            if log:
                log(done[-1])

    def step(lane):
        """Admit what the lane was handed, advance it by rounds_per_step
        rounds and retire what finished; False if it had nothing to do."""
        with torch.cuda.stream(lane.stream):
            while lane.inbox:
                admit(lane, *lane.inbox.popleft())
            if not lane.recs:
                return False
            lane.batch.run(rounds_per_step, stream=lane.stream)
            for slot, st in lane.batch.poll():
                retire(lane, slot, st)
        return True

    def drive(lane):
        try:
            while not stop.is_set():
                if not step(lane):
                    lane.wake.wait(0.002)
                    lane.wake.clear()
        except BaseException as e:  # re-raised by the admitting thread
            errors.append(e)
            stop.set()

    threads = [threading.Thread(target=drive, args=(lane,), daemon=True) for lane in pool[1:]]
    for th in threads:
        th.start()
    try:
        while not errors:
            now = time.perf_counter() - t0
            if time_limit is not None and now > time_limit:
                break
            while pending and pending[0]["arrival"] <= now:
                waiting.append(pending.popleft())
            while waiting:
                req = waiting[0]
                need, ndofs = request_bytes(req)
                if need > budget_bytes:
                    waiting.popleft()            # can never fit: rejected
                    with guard:
                        done.append(dict(req, rejected=True))
                    continue
                with guard:
                    if state["inflight"] >= max_slots or state["used"] + need > budget_bytes:
                        break                    # wait for a slot or for memory (FIFO)
                    state["used"] += need
                    state["inflight"] += 1
                    state["peak"] = max(state["peak"], state["used"])
                    lane = min(pool, key=lambda ln: ln.dofs)   # the lane with the least work resident
                    lane.dofs += ndofs
                waiting.popleft()
                lane.inbox.append((req, need, ndofs))
                lane.wake.set()
            with guard:
                idle = not pending and not waiting and state["inflight"] == 0
            if idle:
                break
            if not step(pool[0]):
                time.sleep(0.0005 if (waiting or not pending) else
                           max(0.0, min(0.002, pending[0]["arrival"] - (time.perf_counter() - t0))))
            dev_peak = max(dev_peak, free0 - torch.cuda.mem_get_info()[0])
    finally:
        stop.set()
        for th in threads:
            th.join()
        torch.cuda.synchronize()
        for lane in pool:
            lane.batch.close()
    if errors:
        raise errors[0]
    elapsed = time.perf_counter() - t0
    ok = [d for d in done if not d.get("rejected")]
    peak = state["peak"]
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
        "budget_bytes": budget_bytes, "max_slots": max_slots, "lanes": len(pool),
    }
