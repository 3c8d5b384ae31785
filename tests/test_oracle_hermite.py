"""Pins of the oracle's Hermite-like basis (no GPU).

The basis of degree k >= 3 is dual to the functionals u(0), x_1 u'(0),
u(x_2), ..., u(x_{k-2}), -x_1 u'(1), u(1) on the Gauss-Lobatto points x_m:
face values and face derivatives then need at most two coefficients per
normal line, the property the paper asks of a Hermite-type basis (Sec. 3,
face interpolation; Sec. 4.4).  Pinned here by

  * the cubic case, which is the classical cubic Hermite basis in closed form;
  * reproduction of every polynomial of degree <= k from its functionals,
    and the mirror symmetry phi_{k-j}(x) = phi_j(1 - x);
  * the operator: both bases span the same polynomials on every cell, so with
    T[i, j] = phi^H_j(x_i) (the Hermite functions at the Lobatto nodes) every
    block of the Hermite operator is (T x T x T)^T B (T x T x T) of the nodal
    block B, the load vector transforms the same way, and the discrete
    solutions agree after the change of basis (same L2 and H1 errors).
"""
import numpy as np
import pytest


def _T(orc, n):
    """T[i, j] = phi^H_j at the i-th Gauss-Lobatto point."""
    x = orc.gll(n)
    return np.array([[orc.basis1d(n, "hermite", j, xi)[0] for j in range(n)] for xi in x])


def _T3(T):
    return np.kron(np.kron(T, T), T)  # index i1 + n i2 + n^2 i3, the same T along each axis


def test_cubic_is_the_classical_hermite_basis(orc):
    s = 0.5 - 0.5 / np.sqrt(5.0)       # first interior Gauss-Lobatto point of 4
    ref = [lambda x: (2 * x ** 3 - 3 * x ** 2 + 1, 6 * x ** 2 - 6 * x),
           lambda x: ((x ** 3 - 2 * x ** 2 + x) / s, (3 * x ** 2 - 4 * x + 1) / s),
           lambda x: (-(x ** 3 - x ** 2) / s, -(3 * x ** 2 - 2 * x) / s),
           lambda x: (-2 * x ** 3 + 3 * x ** 2, -6 * x ** 2 + 6 * x)]
    for x in np.linspace(-0.25, 1.25, 13):
        for j in range(4):
            v, d = orc.basis1d(4, "hermite", j, x)
            rv, rd = ref[j](x)
            assert v == pytest.approx(rv, abs=1e-13)
            assert d == pytest.approx(rd, abs=1e-12)


@pytest.mark.parametrize("n", [4, 5, 6, 7, 8, 9])
def test_reproduces_polynomials_from_their_functionals(orc, n):
    k = n - 1
    x = orc.gll(n)
    s = x[1]
    pts = np.random.default_rng(n).uniform(-0.2, 1.2, 9)
    for m in range(k + 1):
        q = lambda t: t ** m
        dq = lambda t: m * t ** (m - 1) if m > 0 else 0.0
        L = [q(0.0), s * dq(0.0)] + [q(x[i]) for i in range(2, k - 1)] + [-s * dq(1.0), q(1.0)]
        for t in pts:
            vals = [orc.basis1d(n, "hermite", j, t) for j in range(n)]
            assert sum(L[j] * vals[j][0] for j in range(n)) == pytest.approx(q(t), abs=1e-11)
            assert sum(L[j] * vals[j][1] for j in range(n)) == pytest.approx(dq(t), abs=1e-9)


@pytest.mark.parametrize("n", [4, 5, 6, 8])
def test_face_locality_and_mirror_symmetry(orc, n):
    for j in range(n):
        v0, d0 = orc.basis1d(n, "hermite", j, 0.0)
        v1, d1 = orc.basis1d(n, "hermite", j, 1.0)
        # only phi_0 has a value and only phi_1 a slope at 0, mirrored at 1
        assert (abs(v0) > 0.5) == (j == 0) and (abs(d0) > 1.0) == (j == 1)
        assert (abs(v1) > 0.5) == (j == n - 1) and (abs(d1) > 1.0) == (j == n - 2)
        for t in (0.1, 0.37, 0.8):
            a = orc.basis1d(n, "hermite", j, t)
            b = orc.basis1d(n, "hermite", n - 1 - j, 1.0 - t)
            assert a[0] == pytest.approx(b[0], abs=1e-13)
            assert a[1] == pytest.approx(-b[1], abs=1e-11)


def test_rejects_degrees_below_three(orc):
    with pytest.raises(RuntimeError):
        orc.apply(orc.problem(2, 2, basis="hermite"), np.zeros(2 ** 3 * 27))


CASES = [((2, 2, 2), 3, dict()),
         ((3, 2, 2), 3, dict(curved=True, variable_coef=True)),
         ((2, 2, 3), 4, dict(curved=True, bc=(0, 1, 0, 0, 1, 0))),
         ((2, 2, 2), 5, dict(curved=True, amplitude=0.08))]


@pytest.mark.parametrize("N,k,kw", CASES)
def test_blocks_are_the_change_of_basis_of_the_nodal_ones(orc, N, k, kw):
    pl = orc.problem(N, k, **kw)
    ph = orc.problem(N, k, basis="hermite", **kw)
    T3 = _T3(_T(orc, k + 1))
    cells = np.arange(orc.n_cells(pl))
    BL = orc.block_rows(pl, cells)
    BH = orc.block_rows(ph, cells)
    scale = np.abs(BH).max()
    ref = T3.T @ BL @ T3
    assert np.abs(BH - ref).max() <= 1e-12 * scale
    dh = orc.diag_cells(ph, cells)
    assert np.abs(dh - np.einsum("eii->ei", BH[:, 0])).max() <= 1e-13 * scale


@pytest.mark.parametrize("k", [3, 4])
def test_same_discrete_solution_as_the_nodal_basis(orc, k):
    import scipy.sparse.linalg as spla
    kw = dict(curved=True, variable_coef=True)
    pl = orc.problem(3, k, **kw)
    ph = orc.problem(3, k, basis="hermite", **kw)
    T3 = _T3(_T(orc, k + 1))
    bl, bh = orc.rhs(pl), orc.rhs(ph)
    n3 = (k + 1) ** 3
    assert np.abs(bh.reshape(-1, n3) - bl.reshape(-1, n3) @ T3).max() <= 1e-12 * np.abs(bl).max()
    xl = spla.spsolve(orc.assemble_sparse(pl).tocsc(), bl)
    xh = spla.spsolve(orc.assemble_sparse(ph).tocsc(), bh)
    xh_nodal = (xh.reshape(-1, n3) @ T3.T).reshape(-1)
    assert np.linalg.norm(xh_nodal - xl) <= 1e-9 * np.linalg.norm(xl)
    el, eh = orc.errors(pl, xl), orc.errors(ph, xh)
    assert eh[0] == pytest.approx(el[0], rel=1e-7)
    assert eh[1] == pytest.approx(el[1], rel=1e-7)
