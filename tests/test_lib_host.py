"""Host-side checks of libdg.so (no GPU): it loads, exports every symbol
include/dg.h declares, its compiled-in 1D tables match closed forms, and
argument validation rejects bad problems before touching the device."""
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dg():
    import paper_1711_03590_amd as dg
    dg.lib()
    return dg


def test_exports_every_declared_symbol(dg):
    hdr = open(os.path.join(ROOT, "include", "dg.h")).read()
    names = set(re.findall(r"^\s*(?:dg_status|int64_t|size_t|int|const char \*)\s*\**\s*(dg_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 15
    L = dg.lib()
    for n in sorted(names):
        assert hasattr(L, n), n
    assert "dg_cg_solve_noalloc" in names and "dg_cg_solve_noalloc_capacity" in names


def test_noalloc_capacity(dg):
    """The allocation-free solve's static workspace: 128 MiB (host-only call)."""
    assert dg.lib().dg_cg_solve_noalloc_capacity() == 128 << 20


@pytest.mark.parametrize("k", range(1, 9))
def test_tables_closed_forms(dg, k):
    t = dg.tables(k)
    n = k + 1
    x, w = t["gx"], t["gw"]
    for m in range(2 * n):
        assert np.dot(w, x ** m) == pytest.approx(1.0 / (m + 1), rel=1e-14, abs=1e-15)
    # Gauss-Lobatto: 0, 1 and the roots of P'_k, i.e. Legendre derivative zeros
    lx = t["lx"]
    assert lx[0] == 0.0 and lx[-1] == 1.0
    if k > 1:
        dP = np.polynomial.legendre.Legendre.basis(k).deriv()
        assert np.abs(dP(2 * lx[1:-1] - 1)).max() < 1e-12 * max(1.0, np.abs(dP.coef).max())
    # S: Lagrange basis on lx at x reproduces polynomials of degree <= k
    for deg in range(n):
        assert np.allclose(t["S"] @ lx ** deg, x ** deg, atol=1e-14)
    # Dco: exact derivative of polynomials of degree < n on the Gauss points
    for deg in range(n):
        ref = deg * x ** (deg - 1) if deg > 0 else 0 * x
        assert np.allclose(t["Dco"] @ x ** deg, ref, atol=1e-12)
    if n == 3:
        assert np.allclose(x, [0.5 - 0.5 * math.sqrt(0.6), 0.5, 0.5 + 0.5 * math.sqrt(0.6)], atol=1e-15)


def test_tables_symmetry(dg):
    for k in range(1, 9):
        t = dg.tables(k)
        S, D = t["S"], t["Dco"]
        assert np.abs(S[::-1, ::-1] - S).max() < 1e-14
        assert np.abs(D[::-1, ::-1] + D).max() < 1e-12 * np.abs(D).max()


def test_validation_without_device(dg):
    with pytest.raises(dg.DGError) as e:
        dg.footprint(0, 3)
    assert e.value.status == dg.DG_ERR_ARG
    with pytest.raises(dg.DGError) as e:
        dg.footprint(4, 9)
    assert e.value.status == dg.DG_ERR_UNSUPPORTED
    with pytest.raises(dg.DGError):
        dg.footprint(4, 0)
    with pytest.raises(dg.DGError):
        dg.footprint(4, 2, precisions=0)
    with pytest.raises(dg.DGError):
        dg.footprint(2000, 4)   # more than 2^31-1 DoFs


def _apply_threads(n):
    """Threads of an apply workgroup: two waves, or one where whole cells of
    n^2 lines fill one wave as well as two."""
    n2 = n * n
    base = 128 if n2 <= 128 else -(-n2 // 64) * 64
    if n2 <= 64 and (64 // n2) * n2 * base == (base // n2) * n2 * 64:
        return 64
    return base


def _geo_cells(cells, n):
    """Cells the stored cell-geometry arrays hold: padded to whole groups of
    one apply workgroup's cells (n^2 threads per cell)."""
    g = _apply_threads(n) // (n * n)
    return -(-cells // g) * g


def test_geometry_groups_per_degree(dg):
    # one-wave workgroups at 2, 3, 4, 7 and 8 points (16, 7, 4, 1, 1 cells),
    # two waves at 5 and 6 (5 and 3 cells), and 128 threads, one cell, at 9
    assert [_apply_threads(n) // (n * n) for n in range(2, 10)] == [16, 7, 4, 5, 3, 1, 1, 1]
    for k, N in ((2, 10), (1, 5), (6, 3), (5, 7)):
        n = k + 1
        cells = N ** 3
        faces = 3 * N * N * (N + 1)
        vals = 10 * _geo_cells(cells, n) * n ** 3 + 4 * faces * n ** 2
        assert dg.footprint(N, k, curved=True, precisions=dg.PREC_F64) == vals * 8 + cells * n ** 3 * 8


def test_footprint_counts(dg):
    # curved: 10 values per cell point, 4 per face point, plus the diagonal
    k, N = 4, 32
    n = k + 1
    cells = N ** 3
    gc = _geo_cells(cells, n)
    assert gc == 32770
    faces = 3 * N * N * (N + 1)
    vals = 10 * gc * n ** 3 + 4 * faces * n ** 2
    assert dg.footprint(N, k, curved=True, precisions=dg.PREC_F64) == vals * 8 + cells * n ** 3 * 8
    assert dg.footprint(N, k, precisions=dg.PREC_F64 | dg.PREC_F32) == cells * n ** 3 * 12
    assert dg.footprint(N, k, variable_coef=True, precisions=dg.PREC_F32) == \
        (gc * n ** 3 + faces * n ** 2) * 4 + cells * n ** 3 * 4


def test_footprint_merged_geometry(dg):
    # merged (G4): 6 values per cell point instead of 10; faces unchanged
    k, N = 4, 32
    n = k + 1
    gc = _geo_cells(N ** 3, n)
    full = dg.footprint(N, k, curved=True)
    merged = dg.footprint(N, k, curved=True, merged=True)
    assert full - merged == 4 * gc * n ** 3 * (8 + 4)
    # the storage choice does not apply to affine maps
    assert dg.footprint(N, k, merged=True) == dg.footprint(N, k)


def test_bad_storage_rejected(dg):
    import ctypes
    m = dg.make_mesh(4, (dg.DIRICHLET,) * 6)
    g = dg.Geometry(dg.MAP_SINE, 0.05, 7)
    c = dg.Coefficient(0, 1.0)
    out = ctypes.c_size_t()
    st = dg.lib().dg_footprint(ctypes.byref(m), 3, ctypes.byref(g), ctypes.byref(c), dg.PREC_F64, ctypes.byref(out))
    assert st == dg.DG_ERR_ARG


def test_footprint_advection(dg):
    # 3 values per cell point (J^{-1} c det J w), 1 per face point, no diagonal
    k, N = 4, 32
    n = k + 1
    cells = N ** 3
    faces = 3 * N * N * (N + 1)
    vals = 3 * _geo_cells(cells, n) * n ** 3 + faces * n ** 2
    assert dg.footprint_advection(N, k, curved=True) == vals * 12
    assert dg.footprint_advection(N, k, velocity=(1.0, 0.0, 0.0), precisions=dg.PREC_F32) == vals * 4
    with pytest.raises(ValueError):
        dg.footprint_advection(N, k, velocity="spin")


def test_bad_velocity_rejected(dg):
    import ctypes
    m = dg.make_mesh(4, (dg.DIRICHLET,) * 6)
    g = dg.Geometry(dg.MAP_SINE, 0.05, 0)
    v = dg.Velocity()
    v.kind = 5
    out = ctypes.c_size_t()
    st = dg.lib().dg_footprint_advection(ctypes.byref(m), 3, ctypes.byref(g), ctypes.byref(v), dg.PREC_F64,
                                         ctypes.byref(out))
    assert st == dg.DG_ERR_ARG


def test_build_entry_compiles_the_oracle():
    import os
    import oracle
    path = oracle.build(force=True)
    assert os.path.exists(path) and path.endswith("liboracle.so")


@pytest.mark.parametrize("k", range(3, 9))
def test_basis_tables_match_the_oracle(dg, orc, k):
    """The library's compiled-in Hermite-like and nodal tables against the
    oracle's own construction of the same bases."""
    n = k + 1
    gx, _ = orc.gauss(n)
    for basis, obasis in (("hermite", "hermite"), ("nodal", "gll")):
        t = dg.basis_tables(k, basis)
        S = np.array([[orc.basis1d(n, obasis, j, x)[0] for j in range(n)] for x in gx])
        D = np.array([[orc.basis1d(n, obasis, j, x)[1] for j in range(n)] for x in gx])
        assert np.abs(t["S"] - S).max() <= 1e-13
        assert np.abs(t["D"] - D).max() <= 1e-12 * np.abs(D).max()
        for key, x, der in (("V0", 0.0, 0), ("V1", 1.0, 0), ("F0", 0.0, 1), ("F1", 1.0, 1)):
            ref = np.array([orc.basis1d(n, obasis, j, x)[der] for j in range(n)])
            assert np.abs(t[key] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    h = dg.basis_tables(k, "hermite")
    # face locality: one coefficient for the value and one for the slope at each end
    assert np.count_nonzero(h["V0"]) == 1 and np.count_nonzero(h["F0"]) == 1
    assert np.count_nonzero(h["V1"]) == 1 and np.count_nonzero(h["F1"]) == 1


def test_bad_basis_rejected(dg):
    import ctypes
    m = dg.make_mesh(4, (dg.DIRICHLET,) * 6)
    g = dg.Geometry(dg.MAP_SINE, 0.05, 0)
    c = dg.Coefficient(0, 1.0)
    h = ctypes.c_void_p()
    for degree, basis in ((3, 7), (2, dg.BASIS_HERMITE)):
        st = dg.lib().dg_setup_basis(ctypes.byref(m), degree, basis, ctypes.byref(g), ctypes.byref(c), dg.PREC_F64,
                                     None, None, ctypes.byref(h))
        assert st == dg.DG_ERR_ARG
    with pytest.raises(dg.DGError):
        dg.basis_tables(2, "hermite")
    with pytest.raises(ValueError):
        dg.basis_tables(3, "legendre")


def test_footprint_mixed_storage(dg):
    # G3 (10 values) in FP64, G4 (6 values) in FP32; faces (4 values) and the diagonal in both
    k, N = 4, 32
    n = k + 1
    cells = N ** 3
    faces = 3 * N * N * (N + 1)
    gc = _geo_cells(cells, n)
    f64 = (10 * gc * n ** 3 + 4 * faces * n ** 2 + cells * n ** 3) * 8
    f32 = (6 * gc * n ** 3 + 4 * faces * n ** 2 + cells * n ** 3) * 4
    assert dg.footprint(N, k, curved=True, storage="mixed") == f64 + f32
    assert dg.footprint(N, k, curved=True, storage="mixed", precisions=dg.PREC_F32) == f32
    with pytest.raises(ValueError):
        dg.footprint(N, k, curved=True, storage="packed")


def test_footprint_positions_storage(dg):
    # 3 positions and c per cell point, faces as G3, the diagonal
    k, N = 4, 32
    n = k + 1
    cells = N ** 3
    faces = 3 * N * N * (N + 1)
    vals = 4 * _geo_cells(cells, n) * n ** 3 + 4 * faces * n ** 2 + cells * n ** 3
    assert dg.footprint(N, k, curved=True, storage="positions") == vals * 12


def test_ghost_sides_validation(dg):
    """DG_BC_GHOST is a valid side for the SIPG operator (same footprint as a
    Dirichlet side), rejected for advection; the partition calls reject a
    null op before touching the device."""
    import ctypes
    ghost = (dg.DIRICHLET,) * 4 + (dg.GHOST, dg.GHOST)
    assert dg.footprint(6, 3, curved=True, bc=ghost) == dg.footprint(6, 3, curved=True)
    with pytest.raises(dg.DGError) as e:
        dg.footprint(6, 3, bc=(dg.DIRICHLET,) * 5 + (3,))
    assert e.value.status == dg.DG_ERR_ARG
    with pytest.raises(dg.DGError) as e:
        dg.footprint_advection(6, 3, bc=ghost)
    assert e.value.status == dg.DG_ERR_UNSUPPORTED
    v = dg.Vec(None, dg.F64, 0)
    assert dg.lib().dg_face_traces(None, 0, v, v, None) == dg.DG_ERR_ARG
    assert dg.lib().dg_apply_ghost(None, v, (dg.Vec * 6)(), v, None) == dg.DG_ERR_ARG
