"""GPU Jacobi-PCG solves (FP64, and FP32 CG inside FP64 iterative refinement)
against the oracle: the solution of a small manufactured Poisson problem is
compared with a direct solve of the oracle's assembled matrix and load
vector, and the residual is re-verified with the oracle's own apply."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch
    import paper_1711_03590_amd as dg
    assert torch.cuda.is_available()
    dg.lib()
    return dg


@pytest.mark.parametrize("ncell,k,kw", [((4, 4, 4), 2, dict(curved=True, variable_coef=True)),
                                        ((3, 4, 3), 4, dict(curved=True, variable_coef=True)),
                                        ((5, 3, 4), 3, dict(variable_coef=True))])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_solve_matches_direct_solve(dg, orc, ncell, k, kw, mode):
    import scipy.sparse.linalg as spla
    import torch
    op = dg.Operator(ncell, k, **kw)
    p = orc.problem(ncell, k, **kw)
    b = op.rhs()
    bh = b.cpu().numpy()
    assert np.linalg.norm(bh - orc.rhs(p)) <= 1e-12 * np.linalg.norm(bh)
    x, st = op.cg_solve(b, mode=mode, rel_tol=1e-10, check_every=5)
    assert st["converged"] and st["final_rel_residual"] <= 1e-10
    xh = x.cpu().numpy()
    # residual re-checked with the oracle's operator
    assert np.linalg.norm(bh - orc.apply(p, xh)) <= 2e-10 * np.linalg.norm(bh)
    A = orc.assemble_sparse(p)
    xref = spla.spsolve(A.tocsc(), bh)
    assert np.linalg.norm(xh - xref) <= 1e-7 * np.linalg.norm(xref)
    if mode:
        assert st["iters_outer"] >= 1 and st["applies_f32"] > 0
    else:
        assert st["iters_outer"] == 0 and st["applies_f32"] == 0
    op.close()


def test_solve_config4_mixed_vs_fp64(dg):
    """32^3 curved, k=5, variable c (7.1M DoFs): both solvers reach the 1e-10
    FP64 residual, agree with each other, and give the discretisation error."""
    import torch
    op = dg.Operator(32, 5, curved=True, variable_coef=True)
    b = op.rhs()
    x64, s64 = op.cg_solve(b, mixed=False, rel_tol=1e-10)
    e64 = op.error_manufactured(x64)
    assert s64["converged"] and s64["final_rel_residual"] <= 1e-10
    assert e64[0] < 1e-6                      # O(h^6) L2 error at k = 5, h = 1/32
    for mode in (1, 2):
        xmx, smx = op.cg_solve(b, mode=mode, rel_tol=1e-10)
        assert smx["converged"] and smx["final_rel_residual"] <= 1e-10
        d = float(torch.linalg.norm(x64 - xmx) / torch.linalg.norm(x64))
        assert d <= 1e-6
        emx = op.error_manufactured(xmx)
        assert e64[0] == pytest.approx(emx[0], rel=1e-4)
    op.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_solve_deterministic(dg, mode):
    import torch
    op = dg.Operator(8, 3, curved=True, variable_coef=True)
    b = op.rhs()
    x1, _ = op.cg_solve(b, mode=mode, rel_tol=1e-9)
    x2, _ = op.cg_solve(b, mode=mode, rel_tol=1e-9)
    assert torch.equal(x1, x2)
    op.close()


def test_solve_argument_errors(dg):
    import torch
    op = dg.Operator(4, 2)
    b = op.rhs()
    with pytest.raises(dg.DGError) as e:
        op.cg_solve(b.float())
    assert e.value.status == dg.DG_ERR_ARG
    _, st = op.cg_solve(b, mixed=True, rel_tol=1e-14, max_iter=3, max_outer=1)
    assert not st["converged"]
    op.close()
    op32 = dg.Operator(4, 2, precisions=dg.PREC_F64)
    with pytest.raises(dg.DGError):
        op32.cg_solve(b, mixed=True)
    op32.close()
