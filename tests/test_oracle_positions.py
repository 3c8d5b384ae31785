"""Pins of the oracle's cell geometry from quadrature-point positions (no GPU).

Sec. 5 lists, as variant G2, keeping only the physical positions of the
quadrature points and computing the cell Jacobian from them by a collocation
derivative.  The oracle's reading: the SIPG cell term uses the Jacobian of the
tensor-product interpolant of the map through the cell's n^3 Gauss points.
Pinned by

  * affine meshes, where the interpolant is the map itself: every block row
    equals the map-Jacobian operator's;
  * the interpolated Jacobian converging to the map's at order k (relative
    error, the same physical points on meshes N = 8, 16, 32);
  * symmetry and the Neumann null space, which hold for any cell geometry;
  * the manufactured solve converging at order k + 1 in L2.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla


def test_affine_equals_the_map_operator(orc):
    kw = dict(variable_coef=True, lo=(0.0, -1.0, 0.5), hi=(2.0, 0.5, 1.0), bc=(0, 1, 0, 0, 1, 0))
    for k in (1, 3):
        a = orc.problem((3, 2, 2), k, **kw)
        b = orc.problem((3, 2, 2), k, cell_geometry="positions", **kw)
        cells = np.arange(orc.n_cells(a))
        A, B = orc.block_rows(a, cells), orc.block_rows(b, cells)
        assert np.abs(A - B).max() <= 1e-13 * np.abs(A).max()


def _fixed_cells(N):
    pts = [(0.1, 0.2, 0.3), (0.55, 0.45, 0.6), (0.8, 0.15, 0.9), (0.3, 0.7, 0.05), (0.95, 0.95, 0.5)]
    return [int(x * N) + N * (int(y * N) + N * int(z * N)) for x, y, z in pts]


@pytest.mark.parametrize("k", [2, 3])
def test_interpolated_jacobian_converges_at_order_k(orc, k):
    n = k + 1
    errs = []
    for N in (8, 16, 32):
        p = orc.problem(N, k, curved=True, amplitude=0.05, cell_geometry="positions")
        e = 0.0
        for cell in _fixed_cells(N):
            for q in range(n ** 3):
                J, Jmap = orc.cell_jacobian(p, cell, q)
                e = max(e, np.abs(J - Jmap).max() / np.abs(Jmap).max())
        errs.append(e)
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < errs[0]
    assert rates[-1] >= k - 0.4, (errs, rates)


def test_symmetry_and_neumann_null_space(orc):
    kw = dict(curved=True, amplitude=0.08, variable_coef=True, cell_geometry="positions")
    p = orc.problem((3, 2, 3), 3, **kw)
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(orc.n_dofs(p)), rng.standard_normal(orc.n_dofs(p))
    Au, Av = orc.apply(p, u), orc.apply(p, v)
    assert abs(v @ Au - u @ Av) <= 1e-13 * np.linalg.norm(Au) * np.linalg.norm(v)
    pn = orc.problem((3, 2, 3), 3, bc=(1,) * 6, **kw)
    A1 = orc.apply(pn, np.ones(orc.n_dofs(pn)))
    assert np.abs(A1).max() <= 1e-12 * np.abs(orc.diag(pn)).max()


def test_manufactured_convergence(orc):
    k = 2
    errs = []
    for N in (2, 4, 8):
        p = orc.problem(N, k, curved=True, variable_coef=True, cell_geometry="positions")
        x = spla.spsolve(orc.assemble_sparse(p).tocsc(), orc.rhs(p))
        errs.append(orc.errors(p, x, extra=3)[0])
    rate = np.log2(errs[-2] / errs[-1])
    assert rate == pytest.approx(k + 1, abs=0.35)


def test_rejected_for_advection(orc):
    with pytest.raises(RuntimeError):
        orc.apply(orc.problem(2, 2, op="advection", cell_geometry="positions"), np.zeros(8 * 27))


def test_cell_term_uses_the_interpolated_jacobian(orc):
    """One curved cell with Neumann sides (no face terms): the stiffness block
    equals sum_q c det J w (J^{-T} grad phi_i).(J^{-T} grad phi_j) built here
    from the Jacobian cell_jacobian reports, and differs from the block with
    the map's own Jacobian."""
    k, n = 2, 3
    kw = dict(curved=True, amplitude=0.1, bc=(1,) * 6, coef_value=1.7, lo=(0.1, 0.2, 0.05), hi=(0.6, 0.7, 0.55))
    p = orc.problem(1, k, cell_geometry="positions", **kw)
    pm = orc.problem(1, k, **kw)
    gx, gw = orc.gauss(n)
    val = np.array([[orc.basis1d(n, "gll", j, x)[0] for j in range(n)] for x in gx])   # [q, j]
    der = np.array([[orc.basis1d(n, "gll", j, x)[1] for j in range(n)] for x in gx])
    K = np.zeros((n ** 3, n ** 3))
    for q in range(n ** 3):
        q1, q2, q3 = q % n, (q // n) % n, q // (n * n)
        J, _ = orc.cell_jacobian(p, 0, q)
        Jit = np.linalg.inv(J).T
        w = gw[q1] * gw[q2] * gw[q3] * np.linalg.det(J) * 1.7
        G = np.zeros((n ** 3, 3))
        for i in range(n ** 3):
            i1, i2, i3 = i % n, (i // n) % n, i // (n * n)
            g = [der[q1, i1] * val[q2, i2] * val[q3, i3], val[q1, i1] * der[q2, i2] * val[q3, i3],
                 val[q1, i1] * val[q2, i2] * der[q3, i3]]
            G[i] = Jit @ np.array(g)
        K += w * G @ G.T
    B = orc.block_rows(p, np.array([0]))[0, 0]
    Bm = orc.block_rows(pm, np.array([0]))[0, 0]
    assert np.abs(B - K).max() <= 1e-12 * np.abs(K).max()
    assert np.abs(Bm - K).max() >= 1e-6 * np.abs(K).max()
