"""Host logic of the request loop (paper_1711_03590_amd/serve.py) without a
GPU: the batches, the operators and the device calls are stand-ins, so that
admission by HBM budget and slot count, first-come-first-served order, the
spreading of requests over lanes (each driven by its own thread),
retirement and error propagation are checked on the CPU.  The numerics of
served requests are checked on the GPU (tests/test_gpu_batch.py)."""
import contextlib
import threading

import numpy as np
import pytest

import synth


class _Arr:
    def __init__(self, n):
        self.n = n

    def cpu(self):
        return self

    def numpy(self):
        return np.zeros(self.n)


class _Op:
    def __init__(self, n):
        self.n_dofs = n
        self.closed = False

    def close(self):
        self.closed = True


class _World:
    """Shared bookkeeping of the stand-in batches."""

    def __init__(self, fail_on_lane=None):
        self.lock = threading.Lock()
        self.batches = []
        self.resident = 0
        self.peak_resident = 0
        self.order = []
        self.fail_on_lane = fail_on_lane

    def batch_class(self):
        world = self

        class Batch:
            def __init__(self, max_slots):
                self.max_slots = max_slots
                self.slots = {}
                self.next = 0
                self.lane = len(world.batches)
                self.admitted = 0
                self.threads = set()
                world.batches.append(self)

            def admit(self, op, b, x, rel_tol, stream=None):
                self.threads.add(threading.get_ident())
                assert len(self.slots) < self.max_slots
                s = self.next
                self.next += 1
                self.slots[s] = [op, 2 + op.n_dofs % 5]   # rounds to finish
                self.admitted += 1
                with world.lock:
                    world.resident += 1
                    world.peak_resident = max(world.peak_resident, world.resident)
                return s

            def run(self, rounds, stream=None):
                self.threads.add(threading.get_ident())
                if world.fail_on_lane == self.lane:
                    raise RuntimeError("lane failure")
                for v in self.slots.values():
                    v[1] -= rounds

            def poll(self):
                fin = [(s, dict(final_rel_residual=1e-9, iters_inner=7, iters_outer=1))
                       for s, v in self.slots.items() if v[1] <= 0]
                for s, _ in fin:
                    del self.slots[s]
                with world.lock:
                    world.resident -= len(fin)
                return fin

            @property
            def active(self):
                return len(self.slots)

            def close(self):
                pass

        return Batch


@pytest.fixture
def fake(monkeypatch):
    import torch
    from paper_1711_03590_amd import serve

    def install(world):
        monkeypatch.setattr(serve, "Batch", world.batch_class())

        def materialize(req, stream):
            with world.lock:
                world.order.append((id(stream), req["id"]))
            n = serve.request_bytes(req)[1]
            return _Op(n), _Arr(n), _Arr(n)

        monkeypatch.setattr(serve, "_materialize", materialize)
        monkeypatch.setattr(torch.cuda, "Stream", lambda: object())
        monkeypatch.setattr(torch.cuda, "stream", lambda s: contextlib.nullcontext())
        monkeypatch.setattr(torch.cuda, "mem_get_info", lambda: (1 << 40, 1 << 40))
        monkeypatch.setattr(torch.cuda, "reset_peak_memory_stats", lambda: None)
        monkeypatch.setattr(torch.cuda, "memory_allocated", lambda: 0)
        monkeypatch.setattr(torch.cuda, "max_memory_allocated", lambda: 0)
        monkeypatch.setattr(torch.cuda, "synchronize", lambda: None)
        return serve

    return install


def test_admission_budget_slots_and_lanes(fake):
    world = _World()
    serve = fake(world)
    trace = synth.request_trace(40, rate=1e5, seed=3, edge_range=(3, 12))
    sizes = [serve.request_bytes(r)[0] for r in trace]
    budget = int(2.5 * max(sizes))
    seen = []
    rep = serve.serve(trace, budget_bytes=budget, max_slots=5, rounds_per_step=1, lanes=3, log=seen.append,
                      keep=lambda r: r["id"] % 7 == 0)
    assert rep["completed"] == 40 and rep["rejected"] == 0 and rep["unfinished"] == 0 and rep["all_converged"]
    assert rep["lanes"] == 3 and len(world.batches) == 3
    assert 0 < rep["peak_hbm_bytes"] <= budget
    assert world.peak_resident <= 5
    # first come, first served: each lane builds the requests it was handed
    # in arrival order (ids increase with arrival time), and every request
    # is built once
    assert sorted(i for _, i in world.order) == list(range(40))
    for lane_stream in {s for s, _ in world.order}:
        ids = [i for s, i in world.order if s == lane_stream]
        assert ids == sorted(ids)
    # every lane got work, and each lane's batch is only touched by one thread
    assert all(b.admitted > 0 for b in world.batches)
    assert all(len(b.threads) == 1 for b in world.batches)
    assert len({next(iter(b.threads)) for b in world.batches}) == 3
    assert sorted(d["id"] for d in seen) == list(range(40))
    assert all(("x" in d) == (d["id"] % 7 == 0) for d in seen)
    assert all(d["latency"] >= 0 for d in seen)


def test_one_lane_matches_the_single_thread_loop(fake):
    world = _World()
    serve = fake(world)
    trace = synth.request_trace(12, rate=1e5, seed=4, edge_range=(3, 8))
    budget = 3 * max(serve.request_bytes(r)[0] for r in trace)
    rep = serve.serve(trace, budget_bytes=budget, max_slots=4, rounds_per_step=2, lanes=1)
    assert rep["completed"] == 12 and rep["lanes"] == 1
    assert len(world.batches) == 1 and world.batches[0].threads == {threading.get_ident()}


def test_oversized_request_is_rejected(fake):
    world = _World()
    serve = fake(world)
    trace = synth.request_trace(10, rate=1e5, seed=5, edge_range=(3, 10))
    sizes = sorted(serve.request_bytes(r)[0] for r in trace)
    budget = sizes[-1] - 1          # the largest can never fit
    rep = serve.serve(trace, budget_bytes=budget, max_slots=3, rounds_per_step=1, lanes=2)
    assert rep["rejected"] == sum(1 for s in sizes if s > budget) == 1
    assert rep["completed"] == 9 and rep["peak_hbm_bytes"] <= budget


def test_error_in_a_lane_thread_is_raised(fake):
    world = _World(fail_on_lane=1)
    serve = fake(world)
    trace = synth.request_trace(20, rate=1e5, seed=6, edge_range=(3, 8))
    budget = 10 * max(serve.request_bytes(r)[0] for r in trace)
    with pytest.raises(RuntimeError, match="lane failure"):
        serve.serve(trace, budget_bytes=budget, max_slots=8, rounds_per_step=1, lanes=3)
    assert not any(t.name.startswith("Thread") and t.is_alive() and t.daemon for t in threading.enumerate()
                   if t is not threading.current_thread())
