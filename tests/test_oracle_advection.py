"""Pins of the oracle's advection operator (no GPU).

The form is Sec. 2 Eq. (1) with the upwind flux, looped over as in
Algorithm 1: y_i = -(grad phi_i, c u)_e + <phi_i, 1/2 (c.n)(u- + u+)
+ 1/2 |c.n| (u- - u+)>_{de}.  For a divergence-free velocity the divergence
theorem gives two closed forms whenever Gauss quadrature integrates the
integrands exactly (affine cells, velocity at most linear, faces that do not
straddle a sign change of c.n):

  constants   (A 1)_i = sum over the boundary faces of the cell of
              int phi_i (|c.n| - c.n) ds: interior rows vanish and only
              inflow faces act (mirror u+ = -u-);
  energy      u^T A u = sum_interior int 1/2 |c.n| [[u]]^2
                      + sum_boundary int (|c.n| - 1/2 c.n) u^2.

The reference values are computed here from the pinned 1D rules (Gauss
points and weights, Lagrange values on the Gauss-Lobatto nodes) with their
own face loops.  On curved meshes, where no closed form holds, the solution
of A u = b for the manufactured u* = sin(pi x) sin(pi y) sin(pi z) (inflow
data zero) must converge at order k+1 in L2.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla


def _lagrange_table(orc, n, pts):
    """L[j, q] = phi_j^{1D}(pts[q]) on the n Gauss-Lobatto nodes."""
    nodes = orc.gll(n)
    return np.array([[orc.lagrange(nodes, j, x)[0] for x in pts] for j in range(n)])


def _velocity(vel, x):
    if isinstance(vel, str):
        return np.array([0.5 - x[1], x[0] - 0.5, 0.25])
    return np.asarray(vel, dtype=float)


def _faces(N):
    """(cell, local face, neighbour or -1) for every cell face of the brick."""
    out = []
    for cz in range(N[2]):
        for cy in range(N[1]):
            for cx in range(N[0]):
                c = [cx, cy, cz]
                e = cx + N[0] * (cy + N[1] * cz)
                for f in range(6):
                    a, s = f // 2, f % 2
                    cc = list(c)
                    cc[a] += 1 if s else -1
                    nb = -1 if (cc[a] < 0 or cc[a] >= N[a]) else cc[0] + N[0] * (cc[1] + N[1] * cc[2])
                    out.append((e, c, f, nb))
    return out


def _trace(u_cell, L, Lend, a, s, n):
    """Values of the cell polynomial with GLL coefficients u_cell (index
    i1 + n i2 + n^2 i3) on its face (a, s) at the tensor Gauss points
    (q1 along the first tangential axis, q2 along the second)."""
    U = u_cell.reshape(n, n, n)            # [i3, i2, i1]
    U = np.moveaxis(U, [2, 1, 0], [0, 1, 2])  # [i1, i2, i3]
    end = Lend[:, 1] if s else Lend[:, 0]  # phi_j at xi_a = 1 or 0
    face = np.tensordot(U, end, axes=([a], [0]))  # remaining axes in increasing order
    return L.T @ face @ L                   # [q1, q2]


def _face_geometry(p, c, a, s, gx, gw):
    """Physical points and ds of face (a, s) of cell c on an affine brick."""
    N = list(p.ncell)
    h = [(p.hi[d] - p.lo[d]) / N[d] for d in range(3)]
    t1, t2 = [d for d in range(3) if d != a]
    pts = np.zeros((len(gx), len(gx), 3))
    for q1, x1 in enumerate(gx):
        for q2, x2 in enumerate(gx):
            X = [0.0, 0.0, 0.0]
            X[a] = p.lo[a] + (c[a] + s) * h[a]
            X[t1] = p.lo[t1] + (c[t1] + x1) * h[t1]
            X[t2] = p.lo[t2] + (c[t2] + x2) * h[t2]
            pts[q1, q2] = X
    ds = np.outer(gw, gw) * h[t1] * h[t2]
    return pts, ds


AFFINE_CASES = [
    ((2, 2, 2), 1, (1.0, -0.5, 0.25), dict()),
    ((2, 4, 2), 2, "rotation", dict()),
    ((4, 2, 2), 3, "rotation", dict(hi=(2.0, 1.0, 0.5))),
    ((2, 2, 4), 2, (-0.3, 0.7, 1.1), dict(lo=(0.0, -1.0, 0.0), hi=(1.0, 1.0, 2.0))),
]


@pytest.mark.parametrize("N,k,vel,kw", AFFINE_CASES)
def test_constants_only_see_inflow(orc, N, k, vel, kw):
    if isinstance(vel, str):
        kw = dict(kw, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0))  # the rotation axis sits at x = y = 1/2
    p = orc.problem(N, k, op="advection", velocity=vel, **kw)
    n = k + 1
    y = orc.apply(p, np.ones(orc.n_dofs(p))).reshape(-1, n, n, n)  # [cell, i3, i2, i1]
    gx, gw = orc.gauss(n)
    L = _lagrange_table(orc, n, gx)
    ref = np.zeros_like(y)
    for e, c, f, nb in _faces(list(p.ncell)):
        if nb >= 0:
            continue
        a, s = f // 2, f % 2
        pts, ds = _face_geometry(p, c, a, s, gx, gw)
        nvec = np.zeros(3)
        nvec[a] = 1.0 if s else -1.0
        cn = np.array([[_velocity(vel, pts[i, j]) @ nvec for j in range(n)] for i in range(n)])
        w = (np.abs(cn) - cn) * ds                     # [q1, q2]
        face_int = L @ w @ L.T                         # [j1, j2] along the tangential axes
        idx = [slice(None)] * 3
        idx[a] = n - 1 if s else 0                      # only the face's node layer is non-zero there
        block = np.zeros((n, n, n))                     # [i1, i2, i3]
        block[tuple(idx)] = face_int
        ref[e] += np.moveaxis(block, [0, 1, 2], [2, 1, 0])
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(y - ref).max() <= 1e-12 * scale
    interior = [e for e in range(orc.n_cells(p)) if min(orc.neighbours(p, e)) >= 0]
    for e in interior:
        assert np.abs(y[e]).max() <= 1e-13 * scale


@pytest.mark.parametrize("N,k,vel,kw", AFFINE_CASES)
def test_energy_identity(orc, N, k, vel, kw):
    if isinstance(vel, str):
        kw = dict(kw, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0))
    p = orc.problem(N, k, op="advection", velocity=vel, **kw)
    n = k + 1
    u = np.random.default_rng(7).uniform(-1, 1, orc.n_dofs(p))
    lhs = u @ orc.apply(p, u)
    gx, gw = orc.gauss(n)
    L = _lagrange_table(orc, n, gx)
    ends = _lagrange_table(orc, n, [0.0, 1.0])
    U = u.reshape(-1, n ** 3)
    rhs = 0.0
    for e, c, f, nb in _faces(list(p.ncell)):
        a, s = f // 2, f % 2
        pts, ds = _face_geometry(p, c, a, s, gx, gw)
        nvec = np.zeros(3)
        nvec[a] = 1.0 if s else -1.0
        cn = np.array([[_velocity(vel, pts[i, j]) @ nvec for j in range(n)] for i in range(n)])
        um = _trace(U[e], L, ends, a, s, n)
        if nb >= 0:
            if s == 0:
                continue                                 # each interior face once, from its lower cell
            up = _trace(U[nb], L, ends, a, 0, n)
            rhs += np.sum(0.5 * np.abs(cn) * (um - up) ** 2 * ds)
        else:
            rhs += np.sum((np.abs(cn) - 0.5 * cn) * um ** 2 * ds)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    assert lhs > 0


@pytest.mark.parametrize("k,Ns", [(1, (4, 8, 16)), (2, (2, 4, 8))])
def test_convergence_curved_rotation(orc, k, Ns):
    errs = []
    for N in Ns:
        p = orc.problem(N, k, curved=True, amplitude=0.05, op="advection", velocity="rotation")
        A = orc.assemble_sparse(p).tocsc()
        b = orc.rhs(p)
        x = spla.spsolve(A, b)
        assert np.linalg.norm(b - orc.apply(p, x)) <= 1e-9 * np.linalg.norm(b)
        errs.append(orc.errors(p, x, extra=3)[0])
    e = np.array(errs)
    rate = np.log2(e[:-1] / e[1:])
    assert rate[-1] == pytest.approx(k + 1, abs=0.35)
