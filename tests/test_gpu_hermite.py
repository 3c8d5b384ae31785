"""The SIPG operator in the Hermite-like basis (Sec. 3, face interpolation;
Sec. 4.4): face values and derivatives of a neighbour need two of its N
coefficients per normal line.  The bar is the oracle's operator in the same
basis (plain quadrature with the Hermite functions evaluated point by point);
solutions must agree with the nodal basis after the cell-wise change of basis."""
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


def _T3(orc, n):
    x = orc.gll(n)
    T = np.array([[orc.basis1d(n, "hermite", j, xi)[0] for j in range(n)] for xi in x])
    return np.kron(np.kron(T, T), T)


CASES = [
    ((3, 5, 7), 3, dict()),                                          # ragged tail, affine, c = 1
    ((4, 3, 5), 4, dict(variable_coef=True)),                        # affine, variable c
    ((4, 4, 4), 3, dict(curved=True, variable_coef=True)),
    ((4, 4, 4), 4, dict(curved=True)),
    ((3, 3, 3), 5, dict(curved=True, variable_coef=True, bc=(0, 1, 1, 0, 0, 1))),
    ((2, 3, 2), 6, dict(curved=True)),
    ((2, 3, 2), 7, dict(curved=True)),
    ((2, 2, 3), 8, dict(curved=True, variable_coef=True)),
    ((1, 1, 1), 4, dict(curved=True)),
    ((3, 4, 2), 4, dict(bc=(1,) * 6, curved=True, variable_coef=True)),  # all Neumann
    ((4, 3, 3), 4, dict(curved=True, merged=True)),                  # G4 storage
    ((3, 3, 4), 6, dict(curved=True, variable_coef=True, merged=True)),
]


@pytest.mark.parametrize("ncell,k,kw", CASES)
def test_hermite_small_full(dg, orc, ncell, k, kw):
    import torch
    okw = {key: v for key, v in kw.items() if key != "merged"}
    print(f"hermite apply ncell={ncell} k={k} {kw}", flush=True)
    op = dg.Operator(ncell, k, basis="hermite", **kw)
    src = synth.src_vector(op.n_dofs, synth.seed_for(11, k))
    ref = orc.apply(orc.problem(ncell, k, basis="hermite", **okw), src)
    dst = torch.full((op.n_dofs,), float("nan"), dtype=torch.float64, device="cuda")
    op.apply(torch.from_numpy(src).cuda(), dst)
    y64 = dst.cpu().numpy()
    assert np.isfinite(y64).all()
    assert _rel(y64, ref) <= TOL64
    y32 = op.apply(torch.from_numpy(src.astype(np.float32)).cuda()).double().cpu().numpy()
    assert _rel(y32, ref) <= TOL32
    op.close()


@pytest.mark.parametrize("k", [4, 7])
def test_hermite_config2_sampled(dg, orc, k):
    """32^3 sine-curved mesh at full size, sampled cells (corners and boundary included)."""
    import torch
    print(f"hermite 32^3 k={k}", flush=True)
    op = dg.Operator(32, k, curved=True, basis="hermite")
    p = orc.problem(32, k, curved=True, basis="hermite")
    src = synth.src_vector(op.n_dofs, synth.seed_for(2, k))
    cells = synth.sample_cells(32, 800 if k <= 5 else 200, seed=70 + k, n_boundary=60)
    ref = orc.apply_cells(p, src, cells)
    n3 = (k + 1) ** 3
    y = op.apply(torch.from_numpy(src).cuda()).cpu().numpy().reshape(-1, n3)[cells]
    assert _rel(y, ref) <= TOL64
    y32 = op.apply(torch.from_numpy(src.astype(np.float32)).cuda()).double().cpu().numpy().reshape(-1, n3)[cells]
    assert _rel(y32, ref) <= TOL32
    op.close()


def test_hermite_is_the_change_of_basis_of_the_nodal_operator(dg, orc):
    """On the full 32^3 curved mesh: A_H u = T^T A_N (T u) cell by cell, with
    T the Hermite functions at the Gauss-Lobatto nodes."""
    import torch
    k = 4
    n3 = (k + 1) ** 3
    a = dg.Operator(32, k, curved=True, variable_coef=True)
    b = dg.Operator(32, k, curved=True, variable_coef=True, basis="hermite")
    T3 = torch.from_numpy(_T3(orc, k + 1)).cuda()
    u = torch.from_numpy(synth.src_vector(a.n_dofs, 31)).cuda()
    yh = b.apply(u)
    yn = (a.apply((u.view(-1, n3) @ T3.T).reshape(-1)).view(-1, n3) @ T3).reshape(-1)
    assert float(torch.linalg.norm(yh - yn) / torch.linalg.norm(yn)) <= 1e-12
    a.close()
    b.close()


@pytest.mark.parametrize("ncell,k,kw", [((4, 4, 4), 3, dict(curved=True, variable_coef=True)),
                                        ((3, 4, 3), 5, dict()),
                                        ((3, 3, 3), 4, dict(curved=True, merged=True, bc=(1, 0, 0, 1, 0, 0)))])
def test_hermite_diagonal(dg, orc, ncell, k, kw):
    import torch
    okw = {key: v for key, v in kw.items() if key != "merged"}
    op = dg.Operator(ncell, k, basis="hermite", **kw)
    ref = orc.diag(orc.problem(ncell, k, basis="hermite", **okw))
    assert _rel(op.diagonal(torch.float64).cpu().numpy(), ref) <= TOL64
    assert _rel(op.diagonal(torch.float32).double().cpu().numpy(), ref) <= 1e-6
    op.close()


def test_hermite_rhs(dg, orc):
    ncell, k, kw = (3, 4, 3), 4, dict(curved=True, variable_coef=True)
    op = dg.Operator(ncell, k, basis="hermite", **kw)
    ref = orc.rhs(orc.problem(ncell, k, basis="hermite", **kw))
    assert _rel(op.rhs().cpu().numpy(), ref) <= TOL64
    op.close()


@pytest.mark.parametrize("mode", [0, 2])
def test_hermite_solve_matches_nodal(dg, orc, mode):
    """CG in the Hermite-like basis converges to the nodal solution (after the
    change of basis) with the same error against the manufactured solution."""
    import torch
    k = 4
    n3 = (k + 1) ** 3
    a = dg.Operator(8, k, curved=True, variable_coef=True)
    b = dg.Operator(8, k, curved=True, variable_coef=True, basis="hermite")
    xa, sa = a.cg_solve(a.rhs(), mode=mode, rel_tol=1e-10)
    xb, sb = b.cg_solve(b.rhs(), mode=mode, rel_tol=1e-10)
    assert sa["converged"] and sb["converged"]
    assert sb["final_rel_residual"] <= 1e-10
    T3 = torch.from_numpy(_T3(orc, k + 1)).cuda()
    xb_nodal = (xb.view(-1, n3) @ T3.T).reshape(-1)
    assert float(torch.linalg.norm(xb_nodal - xa) / torch.linalg.norm(xa)) <= 1e-8
    ea, eb = a.error_manufactured(xa), b.error_manufactured(xb)
    assert eb[0] == pytest.approx(ea[0], rel=1e-5)
    assert eb[1] == pytest.approx(ea[1], rel=1e-5)
    a.close()
    b.close()


def test_hermite_batch_unsupported(dg):
    import torch
    op = dg.Operator(3, 3, basis="hermite")
    b = torch.ones(op.n_dofs, dtype=torch.float64, device="cuda")
    batch = dg.Batch(1)
    with pytest.raises(dg.DGError) as e:
        batch.admit(op, b, torch.zeros_like(b))
    assert e.value.status == dg.DG_ERR_UNSUPPORTED
    batch.close()
    op.close()
