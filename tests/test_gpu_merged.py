"""Merged cell geometry (G4 of Sec. 5): the symmetric effective coefficient
c det J w J^{-1} J^{-T} stored per cell quadrature point instead of the
inverse Jacobian and c det J w.  It is the same operator up to rounding, so
the bar is the oracle's, as for the stored Jacobian (G3)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5


@pytest.fixture(scope="module")
def dg():
    import torch
    import paper_1711_03590_amd as dg
    assert torch.cuda.is_available()
    dg.lib()
    return dg


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = [
    ((3, 5, 7), 2, dict(curved=True)),                               # ragged tail of the last workgroup
    ((4, 4, 4), 3, dict(curved=True, variable_coef=True)),
    ((4, 4, 4), 4, dict(curved=True)),
    ((3, 3, 3), 5, dict(curved=True, variable_coef=True, bc=(0, 1, 1, 0, 0, 1))),
    ((2, 3, 2), 7, dict(curved=True)),
    ((2, 2, 3), 8, dict(curved=True)),
    ((1, 1, 1), 5, dict(curved=True)),
    ((3, 4, 2), 4, dict(bc=(1,) * 6, curved=True, variable_coef=True)),  # all Neumann
]


@pytest.mark.parametrize("ncell,k,kw", CASES)
def test_merged_small_full(dg, orc, ncell, k, kw):
    import torch
    op = dg.Operator(ncell, k, merged=True, **kw)
    src = synth.src_vector(op.n_dofs, synth.seed_for(9, k))
    ref = orc.apply(orc.problem(ncell, k, **kw), src)
    dst = torch.full((op.n_dofs,), float("nan"), dtype=torch.float64, device="cuda")
    op.apply(torch.from_numpy(src).cuda(), dst)
    y64 = dst.cpu().numpy()
    assert np.isfinite(y64).all()
    assert _rel(y64, ref) <= TOL64
    y32 = op.apply(torch.from_numpy(src.astype(np.float32)).cuda()).double().cpu().numpy()
    assert _rel(y32, ref) <= TOL32
    op.close()


@pytest.mark.parametrize("k", [4, 6])
def test_merged_config2_sampled(dg, orc, k):
    """32^3 sine-curved mesh at full size, sampled cells."""
    import torch
    op = dg.Operator(32, k, curved=True, merged=True)
    p = orc.problem(32, k, curved=True)
    src = synth.src_vector(op.n_dofs, synth.seed_for(2, k))
    cells = synth.sample_cells(32, 1000 if k <= 5 else 300, seed=50 + k, n_boundary=60)
    ref = orc.apply_cells(p, src, cells)
    n3 = (k + 1) ** 3
    y = op.apply(torch.from_numpy(src).cuda()).cpu().numpy().reshape(-1, n3)[cells]
    assert _rel(y, ref) <= TOL64
    y32 = op.apply(torch.from_numpy(src.astype(np.float32)).cuda()).double().cpu().numpy().reshape(-1, n3)[cells]
    assert _rel(y32, ref) <= TOL32
    op.close()


def test_merged_matches_jacobian_storage(dg):
    """The two storages give the same operator up to rounding, on the full
    mesh; the merged one is symmetric like the other."""
    import torch
    a = dg.Operator(32, 4, curved=True, variable_coef=True)
    b = dg.Operator(32, 4, curved=True, variable_coef=True, merged=True)
    u = torch.from_numpy(synth.src_vector(a.n_dofs, 21)).cuda()
    v = torch.from_numpy(synth.src_vector(a.n_dofs, 22)).cuda()
    ya, yb = a.apply(u), b.apply(u)
    assert float(torch.linalg.norm(ya - yb) / torch.linalg.norm(ya)) <= 1e-13
    Bv = b.apply(v)
    assert abs(float(v @ yb - u @ Bv)) <= 1e-12 * float(torch.linalg.norm(yb) * torch.linalg.norm(v))
    a.close()
    b.close()


def test_merged_diagonal(dg, orc):
    import torch
    ncell, k, kw = (4, 4, 4), 3, dict(curved=True, variable_coef=True)
    op = dg.Operator(ncell, k, merged=True, **kw)
    ref = orc.diag(orc.problem(ncell, k, **kw))
    d64 = op.diagonal(torch.float64).cpu().numpy()
    assert _rel(d64, ref) <= TOL64
    op.close()


def test_merged_mixed_solve(dg):
    """Mixed-precision CG on the merged storage reaches the FP64 tolerance and
    the same solution as with the stored Jacobians."""
    import torch
    a = dg.Operator(8, 4, curved=True, variable_coef=True)
    b = dg.Operator(8, 4, curved=True, variable_coef=True, merged=True)
    rhs = a.rhs()
    xa, sa = a.cg_solve(rhs, torch.zeros_like(rhs), mode=2, rel_tol=1e-10)
    xb, sb = b.cg_solve(rhs, torch.zeros_like(rhs), mode=2, rel_tol=1e-10)
    assert sa["converged"] and sb["converged"]
    assert sb["final_rel_residual"] <= 1e-10
    assert float(torch.linalg.norm(xa - xb) / torch.linalg.norm(xa)) <= 1e-8
    a.close()
    b.close()


def test_mixed_storage_is_g3_in_fp64_and_g4_in_fp32(dg):
    """DG_STORE_MIXED: FP64 applies bitwise those of the stored-Jacobian op,
    FP32 applies bitwise those of the merged op; the diagonal is the G3 one."""
    import torch
    kw = dict(curved=True, variable_coef=True)
    g3 = dg.Operator((6, 5, 7), 4, **kw)
    g4 = dg.Operator((6, 5, 7), 4, merged=True, **kw)
    mx = dg.Operator((6, 5, 7), 4, storage="mixed", **kw)
    u = torch.from_numpy(synth.src_vector(g3.n_dofs, 41)).cuda()
    assert torch.equal(mx.apply(u), g3.apply(u))
    u32 = u.float()
    assert torch.equal(mx.apply(u32), g4.apply(u32))
    assert torch.equal(mx.diagonal(torch.float64), g3.diagonal(torch.float64))
    assert torch.equal(mx.diagonal(torch.float32), g3.diagonal(torch.float32))
    for op in (g3, g4, mx):
        op.close()


def test_mixed_storage_solves(dg):
    """Mixed-precision refinement on the mixed storage (FP32 inner solver on
    the merged coefficient, FP64 residuals on the stored Jacobians) reaches
    the FP64 tolerance and the G3 solution; the batch serves it too."""
    import torch
    kw = dict(curved=True, variable_coef=True)
    a = dg.Operator(8, 5, **kw)
    b = dg.Operator(8, 5, storage="mixed", **kw)
    rhs = a.rhs()
    xa, sa = a.cg_solve(rhs, mode=0, rel_tol=1e-10)
    xb, sb = b.cg_solve(rhs, mode=2, rel_tol=1e-10)
    assert sa["converged"] and sb["converged"] and sb["final_rel_residual"] <= 1e-10
    assert float(torch.linalg.norm(xa - xb) / torch.linalg.norm(xa)) <= 1e-8
    batch = dg.Batch(2)
    x = torch.zeros_like(rhs)
    batch.admit(b, rhs, x, rel_tol=1e-10)
    out = []
    while batch.active:
        batch.run(20)
        out += batch.poll()
    batch.close()
    assert out[0][1]["final_rel_residual"] <= 1e-10
    assert float(torch.linalg.norm(x - xa) / torch.linalg.norm(xa)) <= 1e-8
    a.close()
    b.close()
