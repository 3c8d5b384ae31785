"""Cell geometry from quadrature-point positions (G2 of Sec. 5): the apply
takes each cell Jacobian as the collocation derivative of the stored
positions.  The bar is the oracle with the same reading (the Jacobian of the
map's interpolant through the Gauss points), FP64 and FP32, for every degree,
with the diagonal, a solve and the batch."""
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
    ((3, 5, 7), 1, dict(curved=True)),                               # ragged tail of the last workgroup
    ((4, 3, 4), 2, dict(curved=True, variable_coef=True)),
    ((4, 4, 4), 3, dict(curved=True, amplitude=0.08)),
    ((4, 4, 4), 4, dict(curved=True)),
    ((3, 3, 3), 5, dict(curved=True, variable_coef=True, bc=(0, 1, 1, 0, 0, 1))),
    ((2, 3, 2), 6, dict(curved=True, lo=(0.1, -0.3, 0.0), hi=(1.0, 0.9, 2.0))),
    ((2, 3, 2), 7, dict(curved=True)),
    ((2, 2, 3), 8, dict(curved=True, variable_coef=True)),
    ((1, 1, 1), 4, dict(curved=True)),
    ((3, 4, 2), 4, dict(bc=(1,) * 6, curved=True, variable_coef=True)),  # all Neumann
]


@pytest.mark.parametrize("ncell,k,kw", CASES)
def test_positions_small_full(dg, orc, ncell, k, kw):
    import torch
    print(f"positions apply ncell={ncell} k={k} {kw}", flush=True)
    op = dg.Operator(ncell, k, storage="positions", **kw)
    src = synth.src_vector(op.n_dofs, synth.seed_for(12, k))
    ref = orc.apply(orc.problem(ncell, k, cell_geometry="positions", **kw), src)
    dst = torch.full((op.n_dofs,), float("nan"), dtype=torch.float64, device="cuda")
    op.apply(torch.from_numpy(src).cuda(), dst)
    y64 = dst.cpu().numpy()
    assert np.isfinite(y64).all()
    assert _rel(y64, ref) <= TOL64
    y32 = op.apply(torch.from_numpy(src.astype(np.float32)).cuda()).double().cpu().numpy()
    assert _rel(y32, ref) <= TOL32
    op.close()


@pytest.mark.parametrize("k", [4, 7])
def test_positions_config2_sampled(dg, orc, k):
    """32^3 sine-curved mesh at full size, sampled cells."""
    import torch
    print(f"positions 32^3 k={k}", flush=True)
    op = dg.Operator(32, k, curved=True, storage="positions")
    p = orc.problem(32, k, curved=True, cell_geometry="positions")
    src = synth.src_vector(op.n_dofs, synth.seed_for(2, k))
    cells = synth.sample_cells(32, 600 if k <= 5 else 150, seed=80 + k, n_boundary=60)
    ref = orc.apply_cells(p, src, cells)
    n3 = (k + 1) ** 3
    y = op.apply(torch.from_numpy(src).cuda()).cpu().numpy().reshape(-1, n3)[cells]
    assert _rel(y, ref) <= TOL64
    y32 = op.apply(torch.from_numpy(src.astype(np.float32)).cuda()).double().cpu().numpy().reshape(-1, n3)[cells]
    assert _rel(y32, ref) <= TOL32
    op.close()


def test_positions_affine_limit_and_closeness(dg):
    """On the full 32^3 curved mesh the G2 operator is close to the stored
    Jacobian one (interpolation error of the map, O(h^k)), and symmetric."""
    import torch
    a = dg.Operator(32, 4, curved=True, variable_coef=True)
    b = dg.Operator(32, 4, curved=True, variable_coef=True, storage="positions")
    u = torch.from_numpy(synth.src_vector(a.n_dofs, 23)).cuda()
    v = torch.from_numpy(synth.src_vector(a.n_dofs, 24)).cuda()
    ya, yb = a.apply(u), b.apply(u)
    assert float(torch.linalg.norm(ya - yb) / torch.linalg.norm(ya)) <= 1e-3
    Bv = b.apply(v)
    assert abs(float(v @ yb - u @ Bv)) <= 1e-12 * float(torch.linalg.norm(yb) * torch.linalg.norm(v))
    a.close()
    b.close()


@pytest.mark.parametrize("ncell,k,kw", [((4, 4, 4), 3, dict(curved=True, variable_coef=True)),
                                        ((3, 3, 4), 6, dict(curved=True, bc=(1, 0, 0, 1, 0, 0)))])
def test_positions_diagonal(dg, orc, ncell, k, kw):
    import torch
    op = dg.Operator(ncell, k, storage="positions", **kw)
    ref = orc.diag(orc.problem(ncell, k, cell_geometry="positions", **kw))
    assert _rel(op.diagonal(torch.float64).cpu().numpy(), ref) <= TOL64
    op.close()


def test_positions_solve_and_batch(dg):
    """Mixed-precision CG and the batch on the G2 operator reach the
    tolerance and agree; the error against the manufactured solution stays
    at the level of the stored-Jacobian operator's."""
    import torch
    kw = dict(curved=True, variable_coef=True)
    a = dg.Operator(8, 4, **kw)
    b = dg.Operator(8, 4, storage="positions", **kw)
    xa, sa = a.cg_solve(a.rhs(), mode=2, rel_tol=1e-10)
    rhs = b.rhs()
    xb, sb = b.cg_solve(rhs, mode=2, rel_tol=1e-10)
    assert sa["converged"] and sb["converged"] and sb["final_rel_residual"] <= 1e-10
    ea, eb = a.error_manufactured(xa)[0], b.error_manufactured(xb)[0]
    assert eb <= 1.5 * ea
    batch = dg.Batch(2)
    x = torch.zeros_like(rhs)
    batch.admit(b, rhs, x, rel_tol=1e-10)
    out = []
    while batch.active:
        batch.run(20)
        out += batch.poll()
    batch.close()
    assert out[0][1]["final_rel_residual"] <= 1e-10
    assert float(torch.linalg.norm(x - xb) / torch.linalg.norm(xb)) <= 1e-6
    a.close()
    b.close()
