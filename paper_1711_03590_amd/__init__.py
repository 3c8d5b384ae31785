"""Matrix-free SIPG Laplacian on MI355X: Python binding of libdg.so.

Argument marshalling only -- every step of the operator runs in the HIP
kernels behind the C ABI declared in include/dg.h.  PyTorch provides device
memory (the op's arrays come from torch's caching allocator through the
allocator callbacks) and streams.  If libdg.so is missing this module raises;
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdg.so")

DG_OK, DG_ERR_ARG, DG_ERR_OOM, DG_ERR_HIP, DG_ERR_UNSUPPORTED, DG_ERR_NOT_CONVERGED = range(6)
F64, F32 = 0, 1
DIRICHLET, NEUMANN, GHOST = 0, 1, 2
MAP_AFFINE, MAP_SINE = 0, 1
STORE_JACOBIAN, STORE_MERGED, STORE_MIXED, STORE_POSITIONS = 0, 1, 2, 3


def _storage(merged, storage):
    """storage "jacobian" (G3), "merged" (G4), "mixed" (G3 in FP64, G4 in
    FP32) or "positions" (G2: quadrature-point positions, Jacobians taken in
    the kernel); merged=True is short for "merged"."""
    if storage is None:
        storage = "merged" if merged else "jacobian"
    table = {"jacobian": STORE_JACOBIAN, "merged": STORE_MERGED, "mixed": STORE_MIXED,
             "positions": STORE_POSITIONS}
    if storage not in table:
        raise ValueError("storage must be 'jacobian', 'merged', 'mixed' or 'positions'")
    return table[storage]
COEF_CONST, COEF_SINCOS = 0, 1
PREC_F64, PREC_F32 = 1, 2
BASIS_NODAL, BASIS_HERMITE = 0, 1


class DGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dg status {status}: {msg}")
        self.status = status


class Mesh(ctypes.Structure):
    _fields_ = [("ncell", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("bc", ctypes.c_int32 * 6)]


class Geometry(ctypes.Structure):
    _fields_ = [("map", ctypes.c_int), ("amplitude", ctypes.c_double), ("storage", ctypes.c_int)]


class Coefficient(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("value", ctypes.c_double)]


VEL_CONST, VEL_ROTATION = 0, 1


class Velocity(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("value", ctypes.c_double * 3)]


def _velocity(velocity):
    """"rotation" (c = (1/2 - y, x - 1/2, 1/4)) or a constant 3-vector."""
    v = Velocity()
    if isinstance(velocity, str):
        if velocity != "rotation":
            raise ValueError("velocity must be 'rotation' or a 3-vector")
        v.kind = VEL_ROTATION
    else:
        v.kind = VEL_CONST
        v.value[:] = [float(c) for c in velocity]
    return v


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class Vec(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int), ("n", ctypes.c_int64)]


class SolveParams(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("rel_tol", ctypes.c_double), ("rel_tol_inner", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("max_outer", ctypes.c_int), ("check_every", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters_inner", ctypes.c_int), ("iters_outer", ctypes.c_int),
                ("applies_f64", ctypes.c_int), ("applies_f32", ctypes.c_int),
                ("final_rel_residual", ctypes.c_double), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# (name, restype, argtypes) of every entry point in include/dg.h
_P = ctypes.c_void_p
_SIGS = [
    ("dg_footprint", ctypes.c_int, [ctypes.POINTER(Mesh), ctypes.c_int, ctypes.POINTER(Geometry),
                                    ctypes.POINTER(Coefficient), ctypes.c_uint, ctypes.POINTER(ctypes.c_size_t)]),
    ("dg_setup", ctypes.c_int, [ctypes.POINTER(Mesh), ctypes.c_int, ctypes.POINTER(Geometry),
                                ctypes.POINTER(Coefficient), ctypes.c_uint, ctypes.POINTER(Allocator), _P,
                                ctypes.POINTER(_P)]),
    ("dg_setup_basis", ctypes.c_int, [ctypes.POINTER(Mesh), ctypes.c_int, ctypes.c_int, ctypes.POINTER(Geometry),
                                      ctypes.POINTER(Coefficient), ctypes.c_uint, ctypes.POINTER(Allocator), _P,
                                      ctypes.POINTER(_P)]),
    ("dg_basis_tables", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                       ctypes.c_size_t]),
    ("dg_footprint_advection", ctypes.c_int, [ctypes.POINTER(Mesh), ctypes.c_int, ctypes.POINTER(Geometry),
                                              ctypes.POINTER(Velocity), ctypes.c_uint,
                                              ctypes.POINTER(ctypes.c_size_t)]),
    ("dg_setup_advection", ctypes.c_int, [ctypes.POINTER(Mesh), ctypes.c_int, ctypes.POINTER(Geometry),
                                          ctypes.POINTER(Velocity), ctypes.c_uint, ctypes.POINTER(Allocator), _P,
                                          ctypes.POINTER(_P)]),
    ("dg_n_dofs", ctypes.c_int64, [_P]),
    ("dg_apply", ctypes.c_int, [_P, Vec, Vec, _P]),
    ("dg_face_traces", ctypes.c_int, [_P, ctypes.c_int, Vec, Vec, _P]),
    ("dg_apply_ghost", ctypes.c_int, [_P, Vec, ctypes.POINTER(Vec), Vec, _P]),
    ("dg_diagonal", ctypes.c_int, [_P, Vec, _P]),
    ("dg_rhs", ctypes.c_int, [_P, Vec, _P]),
    ("dg_error_manufactured", ctypes.c_int, [_P, Vec, _P, ctypes.POINTER(ctypes.c_double)]),
    ("dg_cg_solve", ctypes.c_int, [_P, Vec, Vec, ctypes.POINTER(SolveParams), ctypes.POINTER(SolveStats), _P]),
    ("dg_cg_solve_noalloc", ctypes.c_int, [_P, Vec, Vec, ctypes.POINTER(SolveParams), ctypes.POINTER(SolveStats),
                                           _P]),
    ("dg_cg_solve_noalloc_bytes", ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    ("dg_cg_solve_noalloc_capacity", ctypes.c_size_t, []),
    ("dg_destroy", ctypes.c_int, [_P]),
    ("dg_last_error", ctypes.c_char_p, []),
    ("dg_tables", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t]),
    ("dg_batch_create", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Allocator), ctypes.POINTER(_P)]),
    ("dg_batch_admit", ctypes.c_int, [_P, _P, Vec, Vec, ctypes.POINTER(SolveParams),
                                      ctypes.POINTER(ctypes.c_int), _P]),
    ("dg_batch_run", ctypes.c_int, [_P, ctypes.c_int, _P]),
    ("dg_batch_poll", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(SolveStats), ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int)]),
    ("dg_batch_active", ctypes.c_int, [_P]),
    ("dg_batch_destroy", ctypes.c_int, [_P]),
]

_lib = None


def lib():
    """The loaded libdg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no non-HIP fallback)")
        # torch first: its HIP runtime is then the one the library binds to
        # (loaded the other way round, the process would hold two runtimes)
        _torch()
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != DG_OK:
        msg = lib().dg_last_error()
        raise DGError(rc, msg.decode() if msg else "")
    return rc


def tables(degree):
    """The compiled-in 1D tables (host only): dict of gauss x/w, gll x, S, Dco."""
    import numpy as np
    n = degree + 1
    out = np.zeros(3 * n + 2 * n * n)
    check(lib().dg_tables(degree, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size))
    return {"gx": out[:n], "gw": out[n:2 * n], "lx": out[2 * n:3 * n],
            "S": out[3 * n:3 * n + n * n].reshape(n, n), "Dco": out[3 * n + n * n:].reshape(n, n)}


def _basis(basis):
    if basis not in ("nodal", "hermite"):
        raise ValueError("basis must be 'nodal' or 'hermite'")
    return BASIS_HERMITE if basis == "hermite" else BASIS_NODAL


def basis_tables(degree, basis="nodal"):
    """The compiled-in 1D basis tables (host only): S and D at the Gauss
    points, and values and slopes at the ends (V0, V1, F0, F1)."""
    import numpy as np
    n = degree + 1
    out = np.zeros(2 * n * n + 4 * n)
    check(lib().dg_basis_tables(degree, _basis(basis), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                out.size))
    o = 2 * n * n
    return {"S": out[:n * n].reshape(n, n), "D": out[n * n:o].reshape(n, n), "V0": out[o:o + n],
            "V1": out[o + n:o + 2 * n], "F0": out[o + 2 * n:o + 3 * n], "F1": out[o + 3 * n:o + 4 * n]}


def make_mesh(ncell, bc=(DIRICHLET,) * 6, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    if isinstance(ncell, int):
        ncell = (ncell,) * 3
    m = Mesh()
    m.ncell[:] = list(ncell)
    m.lo[:] = list(lo)
    m.hi[:] = list(hi)
    m.bc[:] = list(bc)
    return m


def footprint(ncell, degree, *, curved=False, amplitude=0.05, variable_coef=False, coef_value=1.0,
              precisions=PREC_F64 | PREC_F32, bc=(DIRICHLET,) * 6, merged=False, storage=None):
    m = make_mesh(ncell, bc)
    g = Geometry(MAP_SINE if curved else MAP_AFFINE, amplitude, _storage(merged, storage))
    c = Coefficient(COEF_SINCOS if variable_coef else COEF_CONST, coef_value)
    out = ctypes.c_size_t()
    check(lib().dg_footprint(ctypes.byref(m), degree, ctypes.byref(g), ctypes.byref(c), precisions,
                             ctypes.byref(out)))
    return out.value


def footprint_advection(ncell, degree, *, curved=False, amplitude=0.05, velocity="rotation",
                        precisions=PREC_F64 | PREC_F32, bc=(DIRICHLET,) * 6):
    m = make_mesh(ncell, bc)
    g = Geometry(MAP_SINE if curved else MAP_AFFINE, amplitude, STORE_JACOBIAN)
    v = _velocity(velocity)
    out = ctypes.c_size_t()
    check(lib().dg_footprint_advection(ctypes.byref(m), degree, ctypes.byref(g), ctypes.byref(v), precisions,
                                       ctypes.byref(out)))
    return out.value


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def vec(t):
    torch = _torch()
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("vectors must be contiguous device tensors")
    if t.dtype == torch.float64:
        dt = F64
    elif t.dtype == torch.float32:
        dt = F32
    else:
        raise ValueError("vectors must be float64 or float32")
    return Vec(t.data_ptr(), dt, t.numel())


class TorchAllocator:
    """dg_allocator backed by torch's caching allocator."""

    def __init__(self):
        torch = _torch()
        self._dev = torch.cuda.current_device()

        def _alloc(nbytes, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self._dev)
            except Exception:
                return None

        def _free(ptr, ctx):
            if ptr:
                torch.cuda.caching_allocator_delete(ptr)

        self._a = ALLOC_FN(_alloc)
        self._f = FREE_FN(_free)
        self.struct = Allocator(self._a, self._f, None)


class Operator:
    """One SIPG operator (mesh, degree, geometry, coefficient, basis) resident on the GPU.
    basis: "nodal" (Lagrange on the Gauss-Lobatto points) or "hermite" (the
    Hermite-like basis, degree >= 3)."""

    def __init__(self, ncell, degree, *, curved=False, amplitude=0.05, variable_coef=False, coef_value=1.0,
                 bc=(DIRICHLET,) * 6, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                 precisions=PREC_F64 | PREC_F32, torch_alloc=True, stream=None, merged=False, basis="nodal",
                 storage=None):
        self._h = None
        self.degree = degree
        self.mesh = make_mesh(ncell, bc, lo, hi)
        self.ncell = tuple(self.mesh.ncell)
        self.curved = curved
        st = _storage(merged, storage)
        self.merged = curved and st == STORE_MERGED
        self.storage = st
        self.variable_coef = variable_coef
        self.precisions = precisions
        self.basis = basis
        b = _basis(basis)
        self._alloc = TorchAllocator() if torch_alloc else None
        g = Geometry(MAP_SINE if curved else MAP_AFFINE, amplitude, st)
        c = Coefficient(COEF_SINCOS if variable_coef else COEF_CONST, coef_value)
        h = ctypes.c_void_p()
        alloc = ctypes.byref(self._alloc.struct) if self._alloc else None
        if b == BASIS_NODAL:
            check(lib().dg_setup(ctypes.byref(self.mesh), degree, ctypes.byref(g), ctypes.byref(c), precisions,
                                 alloc, _stream(stream), ctypes.byref(h)))
        else:
            check(lib().dg_setup_basis(ctypes.byref(self.mesh), degree, b, ctypes.byref(g), ctypes.byref(c),
                                       precisions, alloc, _stream(stream), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    @property
    def n_dofs(self):
        return int(lib().dg_n_dofs(self._h))

    def apply(self, src, dst=None, stream=None):
        torch = _torch()
        if dst is None:
            dst = torch.empty_like(src)
        check(lib().dg_apply(self._h, vec(src), vec(dst), _stream(stream)))
        return dst

    def side_cells(self, side):
        """Cells in the plane of side 0..5 (x-, x+, y-, y+, z-, z+)."""
        a = side // 2
        return self.ncell[1 if a == 0 else 0] * self.ncell[1 if a == 2 else 2]

    def face_traces(self, side, src, out=None, stream=None):
        """Value and normal derivative of src on every face of side `side`,
        as the partition across that side reads them on its ghost side."""
        torch = _torch()
        if out is None:
            n = self.degree + 1
            out = torch.empty(self.side_cells(side) * 2 * n * n, dtype=src.dtype, device=src.device)
        check(lib().dg_face_traces(self._h, side, vec(src), vec(out), _stream(stream)))
        return out

    def apply_ghost(self, src, ghost, dst=None, stream=None):
        """dst = this partition's rows of A u; ghost maps each ghost side
        (0..5) to the neighbour's face traces of that face plane."""
        torch = _torch()
        if dst is None:
            dst = torch.empty_like(src)
        g = (Vec * 6)()
        for f, t in dict(ghost).items():
            g[f] = vec(t)
        check(lib().dg_apply_ghost(self._h, vec(src), g, vec(dst), _stream(stream)))
        return dst

    def diagonal(self, dtype=None, stream=None):
        torch = _torch()
        d = torch.empty(self.n_dofs, dtype=dtype or torch.float64, device="cuda")
        check(lib().dg_diagonal(self._h, vec(d), _stream(stream)))
        return d

    def rhs(self, stream=None):
        torch = _torch()
        b = torch.empty(self.n_dofs, dtype=torch.float64, device="cuda")
        check(lib().dg_rhs(self._h, vec(b), _stream(stream)))
        return b

    def error_manufactured(self, x, stream=None):
        err = (ctypes.c_double * 2)()
        check(lib().dg_error_manufactured(self._h, vec(x), _stream(stream), err))
        return err[0], err[1]

    def cg_solve(self, b, x=None, *, mixed=True, mode=None, rel_tol=1e-10, rel_tol_inner=None, max_iter=20000,
                 max_outer=50, check_every=10, stream=None, noalloc=False):
        """Jacobi-PCG for A x = b (FP64 vectors).  mode 0: FP64 CG; 1: FP32 CG
        inside FP64 iterative refinement (default when mixed); 2: the same with
        reliable updates.  noalloc: run dg_cg_solve_noalloc (workspace in the
        library's static device array, nothing allocated).  Returns (x, stats
        dict with 'converged')."""
        torch = _torch()
        if mode is None:
            mode = 1 if mixed else 0
        if rel_tol_inner is None:
            rel_tol_inner = 0.3 if mode == 2 else 1e-4
        if x is None:
            x = torch.zeros_like(b)
        p = SolveParams(mode, rel_tol, rel_tol_inner, max_iter, max_outer, check_every)
        st = SolveStats()
        fn = lib().dg_cg_solve_noalloc if noalloc else lib().dg_cg_solve
        rc = fn(self._h, vec(b), vec(x), ctypes.byref(p), ctypes.byref(st), _stream(stream))
        if rc not in (DG_OK, DG_ERR_NOT_CONVERGED):
            check(rc)
        out = st.as_dict()
        out["converged"] = rc == DG_OK
        out["mode"] = mode
        return x, out

    def noalloc_bytes(self, mode):
        """Workspace bytes dg_cg_solve_noalloc needs in this mode."""
        out = ctypes.c_size_t()
        check(lib().dg_cg_solve_noalloc_bytes(self._h, mode, ctypes.byref(out)))
        return out.value

    def close(self):
        if self._h is not None and self._h.value:
            lib().dg_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AdvectionOperator:
    """The DG advection operator with the upwind flux (Sec. 2, Eq. (1))
    resident on the GPU.  bc 0 faces take the mirror u+ = -u- (homogeneous
    inflow data), bc 1 faces u+ = u- (outflow)."""

    def __init__(self, ncell, degree, *, curved=False, amplitude=0.05, velocity="rotation",
                 bc=(DIRICHLET,) * 6, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                 precisions=PREC_F64 | PREC_F32, torch_alloc=True, stream=None):
        self._h = None
        self.degree = degree
        self.mesh = make_mesh(ncell, bc, lo, hi)
        self.ncell = tuple(self.mesh.ncell)
        self.curved = curved
        self.velocity = velocity
        self.precisions = precisions
        self._alloc = TorchAllocator() if torch_alloc else None
        g = Geometry(MAP_SINE if curved else MAP_AFFINE, amplitude, STORE_JACOBIAN)
        v = _velocity(velocity)
        h = ctypes.c_void_p()
        check(lib().dg_setup_advection(ctypes.byref(self.mesh), degree, ctypes.byref(g), ctypes.byref(v), precisions,
                                       ctypes.byref(self._alloc.struct) if self._alloc else None, _stream(stream),
                                       ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    @property
    def n_dofs(self):
        return int(lib().dg_n_dofs(self._h))

    def apply(self, src, dst=None, stream=None):
        torch = _torch()
        if dst is None:
            dst = torch.empty_like(src)
        check(lib().dg_apply(self._h, vec(src), vec(dst), _stream(stream)))
        return dst

    def close(self):
        if self._h is not None and self._h.value:
            lib().dg_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Continuous batching of mixed-precision solves (dg_batch_* of the C ABI).

    Requests are admitted into free slots at any time; run(rounds) advances
    every active request by that many CG iterations, each one persistent
    apply launch per degree and geometry storage present plus three batched
    vector launches; poll() returns the requests that finished."""

    def __init__(self, max_slots, torch_alloc=True):
        self._alloc = TorchAllocator() if torch_alloc else None
        h = ctypes.c_void_p()
        check(lib().dg_batch_create(max_slots, ctypes.byref(self._alloc.struct) if self._alloc else None,
                                    ctypes.byref(h)))
        self._h = h
        self.max_slots = max_slots
        self._keep = {}

    def admit(self, op, b, x, *, rel_tol=1e-8, refine_factor=0.3, max_iter=20000, check_every=10, stream=None):
        p = SolveParams(2, rel_tol, refine_factor, max_iter, 1, check_every)
        slot = ctypes.c_int(-1)
        check(lib().dg_batch_admit(self._h, op.handle, vec(b), vec(x), ctypes.byref(p), ctypes.byref(slot),
                                   _stream(stream)))
        self._keep[slot.value] = (op, b, x)
        return slot.value

    def run(self, rounds, stream=None):
        check(lib().dg_batch_run(self._h, rounds, _stream(stream)))

    def poll(self):
        cap = self.max_slots
        slots = (ctypes.c_int * cap)()
        stats = (SolveStats * cap)()
        n = ctypes.c_int()
        check(lib().dg_batch_poll(self._h, slots, stats, cap, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            d = stats[i].as_dict()
            out.append((slots[i], d))
            self._keep.pop(slots[i], None)
        return out

    @property
    def active(self):
        return int(lib().dg_batch_active(self._h))

    def close(self):
        if self._h is not None and self._h.value:
            lib().dg_batch_destroy(self._h)
        self._h = None
        self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
