"""Optimal-order convergence of the oracle's discretisation (no GPU).

Solving A x = b with the load vector of u* = sin(pi x) sin(pi y) sin(pi z)
must give L2 errors of order k+1 and broken-H1 errors of order k under mesh
refinement -- the standard SIPG estimates for a smooth solution (the method
of Sec. 2, Eq. (2)).  A wrong Jacobian, normal, penalty, face sign or
coefficient placement destroys these rates, so this pins the whole oracle on
curved meshes with the variable coefficient, where exact integration is not
available.  Solves use scipy's CG on the oracle's matrix-free apply with the
oracle's diagonal as Jacobi preconditioner.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla


def _solve(orc, p):
    nd = orc.n_dofs(p)
    b = orc.rhs(p)
    d = orc.diag(p)
    A = spla.LinearOperator((nd, nd), matvec=lambda v: orc.apply(p, v), dtype=np.float64)
    M = spla.LinearOperator((nd, nd), matvec=lambda v: v / d, dtype=np.float64)
    x, info = spla.cg(A, b, rtol=1e-11, atol=0.0, maxiter=5000, M=M)
    assert info == 0
    assert np.linalg.norm(b - orc.apply(p, x)) <= 1e-10 * np.linalg.norm(b)
    return x


@pytest.mark.parametrize("k,Ns", [(1, (4, 8, 16)), (2, (2, 4, 8)), (3, (4, 8, 16))])
def test_convergence_curved_variable_coefficient(orc, k, Ns):
    errs = []
    for N in Ns:
        p = orc.problem(N, k, curved=True, amplitude=0.05, variable_coef=True)
        x = _solve(orc, p)
        errs.append(orc.errors(p, x, extra=3))
    e = np.array(errs)
    rate_l2 = np.log2(e[:-1, 0] / e[1:, 0])
    rate_h1 = np.log2(e[:-1, 1] / e[1:, 1])
    assert rate_l2[-1] == pytest.approx(k + 1, abs=0.2)
    assert rate_h1[-1] == pytest.approx(k, abs=0.2)


def test_convergence_affine_constant(orc):
    k = 2
    errs = []
    for N in (2, 4, 8):
        p = orc.problem(N, k)
        errs.append(orc.errors(p, _solve(orc, p), extra=3))
    e = np.array(errs)
    assert np.log2(e[-2, 0] / e[-1, 0]) == pytest.approx(k + 1, abs=0.2)
    assert np.log2(e[-2, 1] / e[-1, 1]) == pytest.approx(k, abs=0.2)


def test_convergence_curved_anisotropic(orc):
    """Cells of aspect ratio 2 on the curved map: the Jacobian's column scaling
    by the cell size per reference direction only shows here."""
    k = 2
    errs = []
    for N in ((2, 4, 2), (4, 8, 4), (8, 16, 8)):
        p = orc.problem(N, k, curved=True, amplitude=0.05, variable_coef=True)
        errs.append(orc.errors(p, _solve(orc, p), extra=3))
    e = np.array(errs)
    assert np.log2(e[-2, 0] / e[-1, 0]) == pytest.approx(k + 1, abs=0.25)
    assert np.log2(e[-2, 1] / e[-1, 1]) == pytest.approx(k, abs=0.25)
