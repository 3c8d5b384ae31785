"""The allocation-free solve (dg_cg_solve_noalloc) against dg_cg_solve.

Both run the same kernels in the same order with deterministic reductions,
so the solutions and the statistics must agree bitwise; the workspace of the
allocation-free entry point is the library's static device array, which the
second, smaller call reuses with what the first left in it.  No allocation
may reach the op's allocator (torch's caching allocator) during the call,
and a solve whose workspace exceeds the static array is refused before any
work.  Each solution is also re-verified with the oracle's operator."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

# (cells, degree, operator keywords, solver mode): the second call is smaller
CASES = [((6, 5, 4), 3, dict(curved=True, variable_coef=True), 2),
         ((3, 4, 3), 2, dict(curved=True), 2),
         ((5, 4, 4), 3, dict(variable_coef=True), 0),
         ((3, 3, 4), 2, dict(), 1)]


@pytest.fixture(scope="module")
def dg():
    import torch
    import paper_1711_03590_amd as dg
    assert torch.cuda.is_available()
    dg.lib()
    return dg


def _allocations(torch):
    return torch.cuda.memory_stats().get("allocation.all.allocated", 0)


def _solve_pair(dg, orc, ncell, k, kw, mode, seed):
    import torch
    op = dg.Operator(ncell, k, **kw)
    b = torch.from_numpy(synth.src_vector(op.n_dofs, seed)).cuda()
    assert op.noalloc_bytes(mode) <= dg.lib().dg_cg_solve_noalloc_capacity()
    x0 = torch.zeros_like(b)
    torch.cuda.synchronize()
    before = _allocations(torch)
    xn, sn = op.cg_solve(b, x0, mode=mode, rel_tol=1e-10, check_every=5, noalloc=True)
    torch.cuda.synchronize()
    assert _allocations(torch) == before, "the allocation-free solve allocated through the op's allocator"
    xa, sa = op.cg_solve(b, mode=mode, rel_tol=1e-10, check_every=5)
    assert sn["converged"] and sa["converged"]
    assert torch.equal(xn, xa)
    for key in ("iters_inner", "iters_outer", "applies_f64", "applies_f32", "final_rel_residual"):
        assert sn[key] == sa[key], key
    # the oracle's residual of the allocation-free solution
    p = orc.problem(ncell, k, curved=kw.get("curved", False), variable_coef=kw.get("variable_coef", False))
    bh, xh = b.cpu().numpy(), xn.cpu().numpy()
    assert np.linalg.norm(bh - orc.apply(p, xh)) <= 2e-10 * np.linalg.norm(bh)
    op.close()


def test_two_calls_in_a_row_second_smaller(dg, orc):
    """The mixed reliable-update solve on a curved mesh, then on a smaller
    one: the second call finds the first call's data in the scratch array."""
    for i in (0, 1):
        ncell, k, kw, mode = CASES[i]
        _solve_pair(dg, orc, ncell, k, kw, mode, 700 + i)


def test_fp64_and_restarted_modes(dg, orc):
    for i in (2, 3):
        ncell, k, kw, mode = CASES[i]
        _solve_pair(dg, orc, ncell, k, kw, mode, 700 + i)


def test_workspace_beyond_capacity_is_refused(dg):
    """36^3 cells at k = 4 (5.8M DoFs) needs about 190 MB in FP64 mode: refused
    with DG_ERR_ARG and a message naming the limit, x untouched."""
    import torch
    op = dg.Operator(36, 4)
    assert op.noalloc_bytes(0) > dg.lib().dg_cg_solve_noalloc_capacity()
    b = torch.ones(op.n_dofs, dtype=torch.float64, device="cuda")
    x = torch.full_like(b, 7.0)
    with pytest.raises(dg.DGError) as e:
        op.cg_solve(b, x, mode=0, noalloc=True)
    assert e.value.status == dg.DG_ERR_ARG and "static scratch" in str(e.value)
    assert bool((x == 7.0).all())
    op.close()
