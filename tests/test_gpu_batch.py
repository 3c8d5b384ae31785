"""Continuous batching (persistent multi-request kernel): every request's
result is bitwise the same alone and in a mix admitted at different times,
and agrees with dg_cg_solve's reliable-update mode to the solver
tolerance; admission limits hold."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

REQS = [((6, 5, 4), 2, dict(curved=True)),
        ((4, 4, 4), 5, dict(curved=False)),
        ((3, 4, 5), 3, dict(curved=True, variable_coef=True)),
        ((5, 3, 3), 7, dict(curved=True)),
        ((4, 5, 3), 4, dict(curved=True, merged=True))]


@pytest.fixture(scope="module")
def dg():
    import torch
    import paper_1711_03590_amd as dg
    assert torch.cuda.is_available()
    dg.lib()
    return dg


def _make(dg, i):
    import torch
    ncell, k, kw = REQS[i]
    op = dg.Operator(ncell, k, **kw)
    b = torch.from_numpy(synth.src_vector(op.n_dofs, 100 + i)).cuda()
    return op, b


def _run_alone(dg, i):
    import torch
    op, b = _make(dg, i)
    batch = dg.Batch(4)
    x = torch.zeros_like(b)
    batch.admit(op, b, x, rel_tol=1e-9)
    out = []
    while batch.active:
        batch.run(7)
        out += batch.poll()
    batch.close()
    assert len(out) == 1
    return op, b, x, out[0][1]


def test_alone_equals_mix_equals_single_solve(dg):
    import torch
    alone = [_run_alone(dg, i) for i in range(len(REQS))]
    for op, b, x, st in alone:
        assert st["final_rel_residual"] <= 1e-9
    # the same requests admitted at different rounds into one batch
    batch = dg.Batch(3)
    mix = {}
    pend = list(range(len(REQS)))
    stats = {}
    rounds = 0
    while pend or batch.active:
        if pend and batch.active < 3 and rounds % 5 == 0:
            i = pend.pop(0)
            op, b = _make(dg, i)
            x = torch.zeros_like(b)
            slot = batch.admit(op, b, x, rel_tol=1e-9)
            mix[slot] = (i, op, b, x)
        batch.run(3)
        rounds += 3
        for slot, st in batch.poll():
            i, op, b, x = mix.pop(slot)
            stats[i] = (x, st)
    batch.close()
    for i in range(len(REQS)):
        x_mix, st_mix = stats[i]
        assert torch.equal(x_mix, alone[i][2]), f"request {i} differs alone vs in the mix"
        assert st_mix["iters_inner"] == alone[i][3]["iters_inner"]
    # and the single-request solver in its reliable-update mode: the same
    # method, but its p.(A p) comes out of the apply (workgroup partials in
    # another grouping), so the two agree to the solver tolerance
    for i, (op, b, x, st) in enumerate(alone):
        xs, sts = op.cg_solve(b, mode=2, rel_tol=1e-9, rel_tol_inner=0.3, check_every=10)
        assert sts["converged"]
        assert float(torch.linalg.norm(xs - x) / torch.linalg.norm(x)) <= 1e-6, \
            f"request {i}: batch differs from dg_cg_solve"
        assert abs(sts["iters_inner"] - st["iters_inner"]) <= 0.05 * st["iters_inner"] + 10


def test_batch_limits(dg):
    import torch
    batch = dg.Batch(1)
    op, b = _make(dg, 0)
    x = torch.zeros_like(b)
    batch.admit(op, b, x)
    op2, b2 = _make(dg, 1)
    with pytest.raises(dg.DGError) as e:
        batch.admit(op2, b2, torch.zeros_like(b2))
    assert e.value.status == dg.DG_ERR_OOM
    batch.close()
    batch = dg.Batch(2)
    op8 = dg.Operator(2, 8)
    b8 = torch.ones(op8.n_dofs, dtype=torch.float64, device="cuda")
    with pytest.raises(dg.DGError) as e:
        batch.admit(op8, b8, torch.zeros_like(b8))
    assert e.value.status == dg.DG_ERR_UNSUPPORTED
    batch.close()


def test_serve_small_trace(dg):
    from paper_1711_03590_amd import serve
    trace = synth.request_trace(24, rate=400.0, seed=7, edge_range=(3, 10))
    budget = 2 * max(serve.request_bytes(r)[0] for r in trace)
    seen = []
    rep = serve.serve(trace, budget_bytes=budget, max_slots=6, rounds_per_step=5, rel_tol=1e-8,
                      log=seen.append)
    assert rep["completed"] == 24 and rep["all_converged"]
    assert rep["peak_hbm_bytes"] <= budget
    assert all(d["latency"] > 0 for d in seen)
    assert np.isfinite(rep["p99_ms"])
