"""GPU parity of the fused advection apply (upwind flux, Sec. 2 Eq. (1))
against the FP64 oracle (needs MI355X).

Bar as for the SIPG apply: relative l2 error <= 1e-12 in FP64 and <= 1e-5 in
FP32 (source rounded to FP32, geometry stored in FP32, FP32 accumulation).
Small meshes are compared in full, the full-size mesh on sampled cells.
"""
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


def _oracle_kw(kw):
    o = {k: v for k, v in kw.items() if k in ("curved", "amplitude", "bc", "lo", "hi")}
    o["velocity"] = kw.get("velocity", "rotation")
    return o


CASES = [
    ((3, 5, 7), 2, dict(curved=True)),                                  # ragged tail of the last workgroup
    ((4, 4, 4), 1, dict(curved=True)),
    ((4, 4, 4), 3, dict(curved=True, velocity=(1.0, -0.5, 0.25))),
    ((4, 4, 4), 4, dict(curved=True)),
    ((3, 3, 3), 5, dict(curved=True, bc=(0, 1, 1, 0, 0, 1))),
    ((3, 3, 3), 6, dict(velocity=(-0.3, 0.7, 1.1))),
    ((2, 3, 2), 7, dict(curved=True)),
    ((2, 2, 3), 8, dict(curved=True, bc=(1,) * 6)),
    ((1, 1, 1), 5, dict(curved=True)),                                  # one cell, all faces on the boundary
    ((2, 1, 1), 4, dict(velocity=(0.2, 0.0, -1.0), hi=(2.0, 1.0, 0.5))),  # anisotropic box
]


@pytest.mark.parametrize("ncell,k,kw", CASES)
def test_advection_small_full(dg, orc, ncell, k, kw):
    import torch
    op = dg.AdvectionOperator(ncell, k, **kw)
    src = synth.src_vector(op.n_dofs, synth.seed_for(9, k))
    ref = orc.apply(orc.problem(ncell, k, op="advection", **_oracle_kw(kw)), src)
    dst = torch.full((op.n_dofs,), float("nan"), dtype=torch.float64, device="cuda")
    op.apply(torch.from_numpy(src).cuda(), dst)
    y64 = dst.cpu().numpy()
    assert np.isfinite(y64).all()
    assert _rel(y64, ref) <= TOL64
    y32 = op.apply(torch.from_numpy(src.astype(np.float32)).cuda()).double().cpu().numpy()
    assert _rel(y32, ref) <= TOL32
    op.close()


@pytest.mark.parametrize("k", [3, 4, 6])
def test_advection_32cubed_sampled(dg, orc, k):
    """32^3 sine-curved mesh, rotating velocity, in the benchmark's launch
    configuration; sampled cells (random, corners, boundary)."""
    import torch
    op = dg.AdvectionOperator(32, k, curved=True)
    p = orc.problem(32, k, curved=True, op="advection", velocity="rotation")
    src = synth.src_vector(op.n_dofs, synth.seed_for(6, k))
    cells = synth.sample_cells(32, 1000 if k <= 5 else 300, seed=60 + k, n_boundary=60)
    ref = orc.apply_cells(p, src, cells)
    n3 = (k + 1) ** 3
    y = op.apply(torch.from_numpy(src).cuda()).cpu().numpy().reshape(-1, n3)[cells]
    assert _rel(y, ref) <= TOL64
    y32 = op.apply(torch.from_numpy(src.astype(np.float32)).cuda()).double().cpu().numpy().reshape(-1, n3)[cells]
    assert _rel(y32, ref) <= TOL32
    op.close()


def test_advection_constants_and_determinism(dg):
    """A property at full size: on an affine mesh with a constant velocity the
    constant field only feels the inflow faces, so every interior cell's rows
    vanish; and two applies agree bitwise."""
    import torch
    op = dg.AdvectionOperator(24, 4, velocity=(0.4, -0.3, 0.2))
    one = torch.ones(op.n_dofs, dtype=torch.float64, device="cuda")
    y = op.apply(one).cpu().numpy().reshape(24, 24, 24, -1)
    assert np.abs(y[1:-1, 1:-1, 1:-1]).max() <= 1e-13 * np.abs(y).max()
    x = torch.from_numpy(synth.src_vector(op.n_dofs, 5)).cuda()
    assert torch.equal(op.apply(x), op.apply(x))
    op.close()


def test_advection_rejects_symmetric_only_calls(dg):
    import torch
    op = dg.AdvectionOperator(4, 2, curved=True)
    v = dg.vec(torch.zeros(op.n_dofs, dtype=torch.float64, device="cuda"))
    L = dg.lib()
    assert L.dg_diagonal(op.handle, v, None) == dg.DG_ERR_UNSUPPORTED
    assert L.dg_rhs(op.handle, v, None) == dg.DG_ERR_UNSUPPORTED
    b = torch.ones(op.n_dofs, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    prm = dg.SolveParams(0, 1e-8, 0.1, 100, 1, 10)
    st = dg.SolveStats()
    import ctypes
    assert L.dg_cg_solve(op.handle, dg.vec(b), dg.vec(x), ctypes.byref(prm), ctypes.byref(st), None) == \
        dg.DG_ERR_UNSUPPORTED
    op.close()
