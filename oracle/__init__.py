"""FP64 CPU oracle for the SIPG Laplacian and the upwind advection operator
(test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (built from
``oracle.c`` with gcc, see ``buildlib.py``), which evaluates y = A u for the
symmetric interior penalty form of Sec. 2, Eq. (2) of Kronbichler & Kormann
(arXiv 1711.03590) by plain point-by-point quadrature: no sum factorisation,
no shared code with the GPU library.

Parity status per function (what pins it is in tests/test_oracle_*.py):
  gauss, gll, lagrange          pinned: closed forms, exactness, delta property
  apply / apply_cells           pinned: exact-rational brute force (affine, k=1,2),
                                polynomial exactness, symmetry, Neumann null
                                space, SPD, convergence order (curved, variable c)
  block_rows / assemble         pinned through apply (column identity) and the
                                exact-rational brute force
  spmv_blocks                   pinned: equals apply on every row, and the
                                scipy product of the assembled matrix
  diag_cells                    pinned: equals the diagonal of the brute-force matrix
  face_point / volume           pinned: boundary area element, mapped volume
  rhs / errors                  pinned: GLL-weight closed form, convergence order
  basis1d("hermite") and apply  pinned: the defining functionals, the cubic Hermite
  with basis="hermite"          closed form, reproduction of polynomials, mirror
                                symmetry; block rows equal the cell-wise change of
                                basis of the nodal operator's; convergence order
  apply with cell_geometry=     pinned: equals the map's operator on affine meshes; the
  "positions"                   interpolated Jacobian converges to the map's at
                                order k; symmetry, Neumann null space and the
                                convergence order of the manufactured solve
  apply with op="advection"     pinned: constants map to the inflow flux alone and
                                the energy identity u^T A u = upwind jump terms
                                (affine, exact quadrature), convergence order of
                                the manufactured solve (curved, rotating velocity)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DG_ORACLE_LIB selects another build of the same source (the sanitizer build)
_LIB_PATH = os.environ.get("DG_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

DIRICHLET, NEUMANN = 0, 1
MAP_AFFINE, MAP_SINE = 0, 1
COEF_CONST, COEF_SINCOS = 0, 1
OP_SIPG, OP_ADVECTION = 0, 1
VEL_CONST, VEL_ROTATION = 0, 1
BASIS_GLL, BASIS_HERMITE = 0, 1


class Problem(ctypes.Structure):
    _fields_ = [
        ("ncell", ctypes.c_int32 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("bc", ctypes.c_int32 * 6),
        ("degree", ctypes.c_int32),
        ("map", ctypes.c_int32),
        ("amplitude", ctypes.c_double),
        ("coef", ctypes.c_int32),
        ("coef_value", ctypes.c_double),
        ("op", ctypes.c_int32),
        ("vel", ctypes.c_int32),
        ("vel_value", ctypes.c_double * 3),
        ("basis", ctypes.c_int32),
        ("cellgeo", ctypes.c_int32),
    ]


def problem(ncell, degree, *, curved=False, amplitude=0.05, variable_coef=False,
            coef_value=1.0, bc=(DIRICHLET,) * 6, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
            op="sipg", velocity="rotation", basis="gll", cell_geometry="map"):
    """op="sipg" (Sec. 2 Eq. (2)) or "advection" (Eq. (1)); for advection the
    velocity is "rotation" (1/2 - y, x - 1/2, 1/4) or a constant 3-vector.
    basis="gll" (Lagrange on the Gauss-Lobatto points) or "hermite" (the
    Hermite-like basis, degree >= 3).  cell_geometry="map" (the map's
    Jacobian) or "positions" (the Jacobian of the interpolant through the
    cell's Gauss-point positions, SIPG only)."""
    if basis not in ("gll", "hermite"):
        raise ValueError("basis is 'gll' or 'hermite'")
    if cell_geometry not in ("map", "positions"):
        raise ValueError("cell_geometry is 'map' or 'positions'")
    if isinstance(ncell, int):
        ncell = (ncell, ncell, ncell)
    p = Problem()
    p.ncell[:] = list(ncell)
    p.lo[:] = list(lo)
    p.hi[:] = list(hi)
    p.bc[:] = list(bc)
    p.degree = degree
    p.map = MAP_SINE if curved else MAP_AFFINE
    p.amplitude = amplitude
    p.coef = COEF_SINCOS if variable_coef else COEF_CONST
    p.coef_value = coef_value
    p.op = OP_ADVECTION if op == "advection" else OP_SIPG
    p.basis = BASIS_HERMITE if basis == "hermite" else BASIS_GLL
    p.cellgeo = 1 if cell_geometry == "positions" else 0
    if isinstance(velocity, str):
        p.vel = VEL_ROTATION
        p.vel_value[:] = [0.0, 0.0, 0.0]
    else:
        p.vel = VEL_CONST
        p.vel_value[:] = [float(v) for v in velocity]
    return p


def build(force: bool = False) -> str:
    from . import buildlib
    return buildlib.build(force=force)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_int64)
        pp = ctypes.POINTER(Problem)
        L.orc_gauss.argtypes = [ctypes.c_int, dp, dp]
        L.orc_gll.argtypes = [ctypes.c_int, dp]
        L.orc_lagrange.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_basis1d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_n_dofs.argtypes = [pp]
        L.orc_n_dofs.restype = ctypes.c_int64
        L.orc_apply.argtypes = [pp, dp, dp]
        L.orc_apply_cells.argtypes = [pp, dp, lp, ctypes.c_int64, dp]
        L.orc_diag_cells.argtypes = [pp, lp, ctypes.c_int64, dp]
        L.orc_block_rows.argtypes = [pp, lp, ctypes.c_int64, dp]
        L.orc_spmv_blocks.argtypes = [pp, lp, ctypes.c_int64, dp, dp, dp]
        L.orc_cell_jacobian.argtypes = [pp, ctypes.c_int64, ctypes.c_int, dp, dp]
        L.orc_face_point.argtypes = [pp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.orc_volume.argtypes = [pp, dp]
        L.orc_forcing_at.argtypes = [pp, dp]
        L.orc_forcing_at.restype = ctypes.c_double
        L.orc_rhs.argtypes = [pp, dp]
        L.orc_errors.argtypes = [pp, dp, ctypes.c_int, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _lp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(lib().orc_num_threads())


def gauss(n):
    x = np.zeros(n)
    w = np.zeros(n)
    _check(lib().orc_gauss(n, _dp(x), _dp(w)), "gauss")
    return x, w


def gll(n):
    x = np.zeros(n)
    _check(lib().orc_gll(n, _dp(x)), "gll")
    return x


def lagrange(nodes, j, xi):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    v = ctypes.c_double()
    d = ctypes.c_double()
    _check(lib().orc_lagrange(len(nodes), _dp(nodes), j, float(xi), ctypes.byref(v), ctypes.byref(d)),
           "lagrange")
    return v.value, d.value


def basis1d(n, basis, j, xi):
    """Value and derivative at xi of 1D basis function j of n ("gll" or "hermite")."""
    v = ctypes.c_double()
    d = ctypes.c_double()
    _check(lib().orc_basis1d(n, BASIS_HERMITE if basis == "hermite" else BASIS_GLL, j, float(xi),
                             ctypes.byref(v), ctypes.byref(d)), "basis1d")
    return v.value, d.value


def n_dofs(p) -> int:
    return int(lib().orc_n_dofs(ctypes.byref(p)))


def n_cells(p) -> int:
    return int(p.ncell[0] * p.ncell[1] * p.ncell[2])


def apply(p, src):
    src = np.ascontiguousarray(src, dtype=np.float64)
    if src.size != n_dofs(p):
        raise ValueError("src length does not match the problem")
    dst = np.empty_like(src)
    _check(lib().orc_apply(ctypes.byref(p), _dp(src), _dp(dst)), "apply")
    return dst


def apply_cells(p, src, cells):
    src = np.ascontiguousarray(src, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    n3 = (p.degree + 1) ** 3
    out = np.empty(len(cells) * n3)
    _check(lib().orc_apply_cells(ctypes.byref(p), _dp(src), _lp(cells), len(cells), _dp(out)),
           "apply_cells")
    return out.reshape(len(cells), n3)


def diag_cells(p, cells):
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    n3 = (p.degree + 1) ** 3
    out = np.empty(len(cells) * n3)
    _check(lib().orc_diag_cells(ctypes.byref(p), _lp(cells), len(cells), _dp(out)), "diag_cells")
    return out.reshape(len(cells), n3)


def diag(p):
    return diag_cells(p, np.arange(n_cells(p))).reshape(-1)


def block_rows(p, cells):
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    n3 = (p.degree + 1) ** 3
    out = np.empty(len(cells) * 7 * n3 * n3)
    _check(lib().orc_block_rows(ctypes.byref(p), _lp(cells), len(cells), _dp(out)), "block_rows")
    return out.reshape(len(cells), 7, n3, n3)


def spmv_blocks(p, cells, blocks, src):
    """Rows of the given cells of A src from their assembled block rows
    (as block_rows returns them): the matrix-based apply."""
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    blocks = np.ascontiguousarray(blocks, dtype=np.float64)
    src = np.ascontiguousarray(src, dtype=np.float64)
    n3 = (p.degree + 1) ** 3
    if blocks.size != len(cells) * 7 * n3 * n3 or src.size != n_dofs(p):
        raise ValueError("blocks or src do not match the problem")
    out = np.empty(len(cells) * n3)
    _check(lib().orc_spmv_blocks(ctypes.byref(p), _lp(cells), len(cells), _dp(blocks), _dp(src), _dp(out)),
           "spmv_blocks")
    return out.reshape(len(cells), n3)


def neighbours(p, cell):
    """Neighbour cell across local faces 0..5 (x-,x+,y-,y+,z-,z+), -1 at the boundary."""
    N = list(p.ncell)
    c = [cell % N[0], (cell // N[0]) % N[1], cell // (N[0] * N[1])]
    out = []
    for f in range(6):
        a, s = f // 2, f % 2
        cc = list(c)
        cc[a] += 1 if s else -1
        out.append(-1 if (cc[a] < 0 or cc[a] >= N[a]) else cc[0] + N[0] * (cc[1] + N[1] * cc[2]))
    return out


def assemble_sparse(p):
    """The assembled DG matrix as scipy.sparse.csr_matrix (small problems)."""
    import scipy.sparse as sp
    nc = n_cells(p)
    n3 = (p.degree + 1) ** 3
    blocks = block_rows(p, np.arange(nc))
    rows, cols, vals = [], [], []
    ii, jj = np.meshgrid(np.arange(n3), np.arange(n3), indexing="ij")
    for e in range(nc):
        nbs = [e] + neighbours(p, e)
        for b, nb in enumerate(nbs):
            if nb < 0:
                continue
            rows.append((e * n3 + ii).ravel())
            cols.append((nb * n3 + jj).ravel())
            vals.append(blocks[e, b].ravel())
    N = nc * n3
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def assemble_dense(p):
    return assemble_sparse(p).toarray()


def cell_jacobian(p, cell, q):
    """(J the cell term uses, the map's J) at Gauss point q of cell, 3x3 each."""
    a = np.zeros(9)
    b = np.zeros(9)
    _check(lib().orc_cell_jacobian(ctypes.byref(p), cell, q, _dp(a), _dp(b)), "cell_jacobian")
    return a.reshape(3, 3), b.reshape(3, 3)


def face_point(p, cell, face, q1, q2):
    out = np.zeros(12)
    _check(lib().orc_face_point(ctypes.byref(p), cell, face, q1, q2, _dp(out)), "face_point")
    return {"x": out[0:3], "normal": out[3:6], "ds": out[6], "x_nb": out[7:10], "ds_nb": out[10],
            "interior": bool(out[11])}


def volume(p):
    v = ctypes.c_double()
    _check(lib().orc_volume(ctypes.byref(p), ctypes.byref(v)), "volume")
    return v.value


def forcing_at(p, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().orc_forcing_at(ctypes.byref(p), _dp(x)))


def rhs(p):
    b = np.empty(n_dofs(p))
    _check(lib().orc_rhs(ctypes.byref(p), _dp(b)), "rhs")
    return b


def errors(p, x, extra=2):
    x = np.ascontiguousarray(x, dtype=np.float64)
    l2 = ctypes.c_double()
    h1 = ctypes.c_double()
    _check(lib().orc_errors(ctypes.byref(p), _dp(x), extra, ctypes.byref(l2), ctypes.byref(h1)),
           "errors")
    return l2.value, h1.value
