"""Absolute pins of the oracle's error norms (no GPU).

errors(p, x) returns the L2 norm and the broken H1 seminorm of u_h - u* with
u* = sin(pi x) sin(pi y) sin(pi z), evaluated by quadrature on the mapped
cells.  The convergence pins only constrain ratios of these norms, so a
constant-factor mistake (a dropped weight, det J, a squared root) would pass
them.  Here the discrete function is chosen so that the norms have closed
forms on the unit cube:
  u_h = 0:            (||u*||, |u*|_1) = (2^{-3/2}, pi sqrt(3/8));
  u_h = 1:            ||1 - u*||^2 = 1 - 16/pi^3 + 1/8, |u*|_1 as above;
  u_h = x + 2y - z    (nodal interpolant, exact on affine cells):
                      ||L - u*||^2 = 3/2 - 16/pi^3 + 1/8,
                      |L - u*|_1^2 = 6 + 3 pi^2/8 (the cross term vanishes
                      because u* is zero on the boundary).
The sine map takes the unit cube onto itself, so the same values hold on the
curved meshes, up to the quadrature error of the non-polynomial integrand.
"""
import math

import numpy as np
import pytest

L2_ZERO = 2.0 ** -1.5
H1_ZERO = math.pi * math.sqrt(3.0 / 8.0)
L2_ONE = math.sqrt(1.0 - 16.0 / math.pi ** 3 + 0.125)
L2_LIN = math.sqrt(1.5 - 16.0 / math.pi ** 3 + 0.125)
H1_LIN = math.sqrt(6.0 + 3.0 * math.pi ** 2 / 8.0)


@pytest.mark.parametrize("curved,ncell,k,tol", [(False, 4, 2, 1e-10), (False, (3, 5, 4), 3, 1e-10),
                                                (True, 6, 2, 1e-7), (True, (4, 6, 5), 3, 1e-7)])
def test_errors_of_zero_and_one(orc, curved, ncell, k, tol):
    p = orc.problem(ncell, k, curved=curved, variable_coef=curved)
    nd = orc.n_dofs(p)
    l2, h1 = orc.errors(p, np.zeros(nd), extra=4)
    assert l2 == pytest.approx(L2_ZERO, rel=tol)
    assert h1 == pytest.approx(H1_ZERO, rel=tol)
    # the nodal basis reproduces constants: u_h = 1 from all-ones coefficients
    l2, h1 = orc.errors(p, np.ones(nd), extra=4)
    assert l2 == pytest.approx(L2_ONE, rel=tol)
    assert h1 == pytest.approx(H1_ZERO, rel=tol)


@pytest.mark.parametrize("ncell,k", [(3, 1), ((2, 3, 4), 2), (4, 4)])
def test_errors_of_linear_function(orc, ncell, k):
    """Affine cells: the nodal interpolant of L = x + 2y - z is L itself."""
    p = orc.problem(ncell, k)
    N = [p.ncell[0], p.ncell[1], p.ncell[2]]
    n = k + 1
    xi = orc.gll(n)
    x = np.empty(orc.n_dofs(p))
    for cz in range(N[2]):
        for cy in range(N[1]):
            for cx in range(N[0]):
                cell = cx + N[0] * (cy + N[1] * cz)
                for i3 in range(n):
                    for i2 in range(n):
                        for i1 in range(n):
                            X = (cx + xi[i1]) / N[0]
                            Y = (cy + xi[i2]) / N[1]
                            Z = (cz + xi[i3]) / N[2]
                            x[cell * n ** 3 + i1 + n * i2 + n * n * i3] = X + 2 * Y - Z
    l2, h1 = orc.errors(p, x, extra=4)
    assert l2 == pytest.approx(L2_LIN, rel=1e-10)
    assert h1 == pytest.approx(H1_LIN, rel=1e-10)
