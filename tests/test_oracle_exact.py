"""Exact-rational brute force of the SIPG matrix on affine meshes (no GPU).

For degrees 1 and 2 the Gauss-Lobatto nodes are rational (0,1 and 0,1/2,1),
so on an axis-aligned brick with a constant coefficient every entry of A is a
rational number.  Here each entry is integrated exactly with sympy, written
directly from the element form of Sec. 2 Eq. (2) (cell term, adjoint and
primal consistency terms, penalty; averages, jumps and the Dirichlet mirror as
defined at the start of Sec. 2), using the tensor-product structure of the
basis (Sec. 2, the 1D-product shape functions) to split every 3D integral into
exact 1D integrals.  The oracle instead sums point by point with floating
point Gauss quadrature over all basis functions, so the two share nothing but
the definition.  n-point Gauss integrates the degree-2k integrands exactly,
so the two must agree to rounding.

Also pinned here: polynomial exactness on any degree (closed-form integrals
of global polynomials, which have zero jumps) and the first two moments of
the load vector.
"""
import itertools

import numpy as np
import pytest
import sympy as sp

X = sp.Symbol("x")


def _tables(k):
    nodes = [sp.Rational(j, k) for j in range(k + 1)]  # GLL points for k = 1, 2
    ell = []
    for j in range(k + 1):
        e = sp.Integer(1)
        for m in range(k + 1):
            if m != j:
                e *= (X - nodes[m]) / (nodes[j] - nodes[m])
        ell.append(sp.expand(e))
    n = k + 1
    M = [[sp.integrate(ell[i] * ell[j], (X, 0, 1)) for j in range(n)] for i in range(n)]
    K = [[sp.integrate(sp.diff(ell[i], X) * sp.diff(ell[j], X), (X, 0, 1)) for j in range(n)]
         for i in range(n)]
    V = [[ell[i].subs(X, s) for i in range(n)] for s in (0, 1)]
    D = [[sp.diff(ell[i], X).subs(X, s) for i in range(n)] for s in (0, 1)]
    return M, K, V, D


def exact_matrix(N, k, h, c, bc):
    """A as a dense array of sympy Rationals, from the element-local form."""
    n = k + 1
    n3 = n ** 3
    M, K, V, D = _tables(k)
    ncell = N[0] * N[1] * N[2]
    A = [[sp.Integer(0)] * (ncell * n3) for _ in range(ncell * n3)]
    vol = h[0] * h[1] * h[2]
    idx = list(itertools.product(range(n), repeat=3))  # (i3, i2, i1) -> reversed below
    loc = [(t[2], t[1], t[0]) for t in idx]           # loc[i] = (i1, i2, i3), i = i1 + n i2 + n^2 i3
    tau = [sp.Integer((k + 1) ** 2) / h[a] for a in range(3)]

    def cell_of(cx, cy, cz):
        return cx + N[0] * (cy + N[1] * cz)

    for cz, cy, cx in itertools.product(range(N[2]), range(N[1]), range(N[0])):
        e = cell_of(cx, cy, cz)
        ci = (cx, cy, cz)
        # cell term: c * sum_d K_d/h_d^2 prod_{e != d} M  * vol
        for i, ii in enumerate(loc):
            for j, jj in enumerate(loc):
                s = 0
                for d in range(3):
                    t = K[ii[d]][jj[d]] / h[d] ** 2
                    for o in range(3):
                        if o != d:
                            t *= M[ii[o]][jj[o]]
                    s += t
                A[e * n3 + i][e * n3 + j] += c * s * vol
        for f in range(6):
            a, side = f // 2, f % 2
            tang = [o for o in range(3) if o != a]
            area = h[tang[0]] * h[tang[1]]
            sg = 1 if side else -1
            nb = list(ci)
            nb[a] += sg
            interior = 0 <= nb[a] < N[a]
            if not interior and bc[f] == 1:
                continue

            def mt(ii, jj):
                return M[ii[tang[0]]][jj[tang[0]]] * M[ii[tang[1]]][jj[tang[1]]]

            s_own = side          # own trace at xi_a = side
            s_nb = 1 - side       # neighbour trace at xi_a = 1 - side
            for i, ii in enumerate(loc):
                phi_i = V[s_own][ii[a]]
                dn_i = sg * D[s_own][ii[a]] / h[a]
                for j, jj in enumerate(loc):
                    tm = mt(ii, jj) * area * c
                    phi_j = V[s_own][jj[a]]
                    dn_j = sg * D[s_own][jj[a]] / h[a]
                    if interior:
                        # own column: jump = phi_j, avg = dn_j / 2
                        A[e * n3 + i][e * n3 + j] += tm * (-sp.Rational(1, 2) * phi_j * dn_i
                                                          - sp.Rational(1, 2) * phi_i * dn_j
                                                          + tau[a] * phi_i * phi_j)
                        e2 = cell_of(*nb)
                        phi_p = V[s_nb][jj[a]]
                        dn_p = sg * D[s_nb][jj[a]] / h[a]
                        # neighbour column: jump = -phi_p, avg = dn_p / 2
                        A[e * n3 + i][e2 * n3 + j] += tm * (sp.Rational(1, 2) * phi_p * dn_i
                                                           - sp.Rational(1, 2) * phi_i * dn_p
                                                           - tau[a] * phi_i * phi_p)
                    else:
                        # Dirichlet mirror: jump = 2 phi_j, avg = dn_j
                        A[e * n3 + i][e * n3 + j] += tm * (-phi_j * dn_i - phi_i * dn_j
                                                          + 2 * tau[a] * phi_i * phi_j)
    return np.array([[float(v) for v in row] for row in A])


CASES = [
    # (N, k, box hi, c, bc)
    ((1, 1, 1), 1, (1, 1, 1), 1, (0,) * 6),
    ((2, 2, 2), 1, (1, 1, 1), 1, (0,) * 6),
    ((2, 1, 1), 2, (1, 1, 1), 1, (0,) * 6),
    ((1, 2, 3), 1, (2, 1, 3), sp.Rational(5, 2), (0, 1, 0, 0, 1, 0)),
    ((2, 2, 1), 2, (1, 2, 1), sp.Rational(3, 4), (1, 0, 0, 1, 0, 0)),
    ((3, 1, 2), 1, (1, 1, 1), 1, (1,) * 6),
]


@pytest.mark.parametrize("N,k,hi,c,bc", CASES)
def test_exact_rational_matrix(orc, N, k, hi, c, bc):
    h = [sp.Rational(hi[d]) / N[d] for d in range(3)]
    Aex = exact_matrix(N, k, h, c, bc)
    p = orc.problem(N, k, coef_value=float(c), bc=bc, hi=tuple(float(v) for v in hi))
    A = orc.assemble_dense(p)
    scale = np.abs(Aex).max()
    assert np.abs(A - Aex).max() <= 1e-13 * scale
    # the matrix-free route gives the same product
    u = np.random.default_rng(7).uniform(-1, 1, A.shape[0])
    assert np.abs(orc.apply(p, u) - Aex @ u).max() <= 1e-13 * scale * np.abs(u).sum() / len(u) * 50
    # the diagonal routine reads the same diagonal
    assert np.abs(orc.diag(p) - np.diag(Aex)).max() <= 1e-13 * scale


def _interpolate(orc, p, fun):
    """Coefficients of a function at the Gauss-Lobatto nodes of every cell."""
    n = p.degree + 1
    nodes = orc.gll(n)
    N = list(p.ncell)
    h = [(p.hi[d] - p.lo[d]) / N[d] for d in range(3)]
    out = np.empty(orc.n_dofs(p))
    n3 = n ** 3
    for e in range(orc.n_cells(p)):
        ci = [e % N[0], (e // N[0]) % N[1], e // (N[0] * N[1])]
        for i in range(n3):
            li = [i % n, (i // n) % n, i // (n * n)]
            x = [p.lo[d] + (ci[d] + nodes[li[d]]) * h[d] for d in range(3)]
            out[e * n3 + i] = fun(*x)
    return out


@pytest.mark.parametrize("k,N", [(2, (2, 3, 2)), (3, (2, 2, 2)), (4, (1, 2, 1)), (6, (1, 1, 1))])
def test_polynomial_exactness(orc, k, N):
    """v^T A u for global polynomials u, v (no jumps) equals the closed form
    int c grad u . grad v - sum_Dirichlet int (u dn v + v dn u) + sum 2 tau int u v."""
    x, y, z = sp.symbols("x y z")
    U = x ** 2 * y + z
    Vf = y * z + x * x - 2 * x * y
    c = 2.0
    bc = (0, 0, 0, 1, 0, 1)
    tau = [(k + 1) ** 2 * N[a] for a in range(3)]
    grad = lambda f: [sp.diff(f, s) for s in (x, y, z)]
    GU, GV = grad(U), grad(Vf)
    vol = sp.integrate(sum(GU[d] * GV[d] for d in range(3)), (x, 0, 1), (y, 0, 1), (z, 0, 1))
    total = c * vol
    syms = (x, y, z)
    for f in range(6):
        if bc[f] == 1:
            continue
        a, side = f // 2, f % 2
        sg = 1 if side else -1
        t = [s for s in syms if s != syms[a]]
        integrand = (-U * sg * GV[a] - Vf * sg * GU[a] + 2 * tau[a] * U * Vf).subs(syms[a], side)
        total += c * sp.integrate(integrand, (t[0], 0, 1), (t[1], 0, 1))
    total = float(total)
    p = orc.problem(N, k, coef_value=c, bc=bc)
    fu = sp.lambdify((x, y, z), U)
    fv = sp.lambdify((x, y, z), Vf)
    u = _interpolate(orc, p, fu)
    v = _interpolate(orc, p, fv)
    assert float(v @ orc.apply(p, u)) == pytest.approx(total, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("k", [1, 3, 5])
def test_rhs_moments(orc, k):
    """b_i = sum_q f phi_i JxW.  The nodal basis reproduces 1 and x exactly
    (sum_i phi_i = 1, sum_i x_i phi_i = x), so sum_i b_i and sum_i x_i b_i are
    quadratures of int f and int x f.  For c = 1, f = 3 pi^2 u* and these
    integrals are 24/pi and 12/pi on the unit cube."""
    p = orc.problem(8, k)
    b = orc.rhs(p)
    tol = 2e-4 if k == 1 else 1e-7
    assert b.sum() == pytest.approx(24.0 / np.pi, rel=tol)
    xs = _interpolate(orc, p, lambda x, y, z: x)
    assert float(xs @ b) == pytest.approx(12.0 / np.pi, rel=tol)
