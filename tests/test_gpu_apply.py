"""GPU parity of the fused SIPG apply against the FP64 oracle (needs MI355X).

Bar: relative l2 error <= 1e-12 in FP64 and <= 1e-5 in FP32 (source rounded
to FP32, geometry stored in FP32, FP32 accumulation), compared with the FP64
oracle on the FP64 source.  Small meshes are compared in full; the full-size
workloads on sampled cells (random cells, all corners, boundary cells),
which the oracle evaluates row block by row block.
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


def _kw_oracle(kw):
    o = dict(kw)
    o.pop("precisions", None)
    return o


SMALL = [
    ((8, 8, 8), 3, {}),                                              # config 1
    ((3, 5, 7), 2, dict(curved=True)),                               # ragged tail of the last workgroup
    ((4, 4, 4), 1, dict(curved=True)),
    ((4, 4, 4), 2, dict(curved=True)),
    ((4, 4, 4), 3, dict(curved=True)),
    ((4, 4, 4), 4, dict(curved=True)),
    ((3, 3, 3), 5, dict(curved=True)),
    ((3, 3, 3), 6, dict(curved=True)),
    ((2, 3, 2), 7, dict(curved=True)),
    ((2, 2, 3), 8, dict(curved=True)),
    ((5, 3, 4), 4, dict(variable_coef=True)),                        # affine, variable c
    ((4, 3, 5), 3, dict(curved=True, variable_coef=True, bc=(0, 1, 1, 0, 0, 1))),
    ((1, 1, 1), 5, dict(curved=True)),                               # one cell, all faces on the boundary
    ((1, 1, 9), 2, {}),
    ((2, 1, 1), 6, dict(coef_value=2.5, hi=(2.0, 1.0, 0.5))),         # anisotropic box
    ((3, 4, 2), 4, dict(bc=(1,) * 6, curved=True, variable_coef=True)),  # all Neumann
]


@pytest.mark.parametrize("ncell,k,kw", SMALL)
def test_apply_small_full(dg, orc, ncell, k, kw):
    import torch
    op = dg.Operator(ncell, k, **kw)
    p = orc.problem(ncell, k, **_kw_oracle(kw))
    src = synth.src_vector(op.n_dofs, synth.seed_for(9, k))
    ref = orc.apply(p, src)
    x64 = torch.from_numpy(src).cuda()
    dst = torch.full_like(x64, float("nan"))      # every entry must be written
    op.apply(x64, dst)
    y64 = dst.cpu().numpy()
    assert np.isfinite(y64).all()
    assert _rel(y64, ref) <= TOL64
    x32 = torch.from_numpy(src.astype(np.float32)).cuda()
    y32 = op.apply(x32).double().cpu().numpy()
    assert _rel(y32, ref) <= TOL32
    op.close()


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6, 7, 8])
def test_apply_config2_sampled(dg, orc, k):
    """32^3 sine-curved mesh, the benchmark's launch configuration."""
    import torch
    op = dg.Operator(32, k, curved=True)
    p = orc.problem(32, k, curved=True)
    src = synth.src_vector(op.n_dofs, synth.seed_for(2, k))
    cells = synth.sample_cells(32, 1500 if k <= 5 else 300, seed=k, n_boundary=60)
    ref = orc.apply_cells(p, src, cells)
    n3 = (k + 1) ** 3
    y = op.apply(torch.from_numpy(src).cuda()).cpu().numpy().reshape(-1, n3)[cells]
    assert _rel(y, ref) <= TOL64
    y32 = op.apply(torch.from_numpy(src.astype(np.float32)).cuda()).double().cpu().numpy().reshape(-1, n3)[cells]
    assert _rel(y32, ref) <= TOL32
    op.close()


@pytest.mark.parametrize("curved", [False, True])
def test_apply_config3_sampled(dg, orc, curved):
    """64^3, k=4, variable coefficient, affine and curved (32.8M DoFs)."""
    import torch
    op = dg.Operator(64, 4, curved=curved, variable_coef=True)
    p = orc.problem(64, 4, curved=curved, variable_coef=True)
    src = synth.src_vector(op.n_dofs, synth.seed_for(3, 4))
    cells = synth.sample_cells(64, 1500, seed=33, n_boundary=100)
    ref = orc.apply_cells(p, src, cells)
    y = op.apply(torch.from_numpy(src).cuda()).cpu().numpy().reshape(-1, 125)[cells]
    assert _rel(y, ref) <= TOL64
    y32 = op.apply(torch.from_numpy(src.astype(np.float32)).cuda()).double().cpu().numpy().reshape(-1, 125)[cells]
    assert _rel(y32, ref) <= TOL32
    op.close()


def test_apply_deterministic(dg):
    import torch
    op = dg.Operator(16, 4, curved=True, variable_coef=True)
    x = torch.from_numpy(synth.src_vector(op.n_dofs, 4)).cuda()
    a = op.apply(x)
    b = op.apply(x)
    assert torch.equal(a, b)
    op.close()


def test_apply_symmetry_and_null_space(dg):
    """Properties that hold at any size: u^T A v = v^T A u, and A 1 = 0 for
    the all-Neumann operator, on the full 32^3 curved mesh."""
    import torch
    op = dg.Operator(32, 4, curved=True, variable_coef=True)
    u = torch.from_numpy(synth.src_vector(op.n_dofs, 11)).cuda()
    v = torch.from_numpy(synth.src_vector(op.n_dofs, 12)).cuda()
    Au, Av = op.apply(u), op.apply(v)
    assert abs(float(v @ Au - u @ Av)) <= 1e-12 * float(torch.linalg.norm(Au) * torch.linalg.norm(v))
    op.close()
    opn = dg.Operator(32, 4, curved=True, variable_coef=True, bc=(1,) * 6)
    one = torch.ones(opn.n_dofs, dtype=torch.float64, device="cuda")
    r = float(opn.apply(one).abs().max())
    assert r <= 1e-12 * float(opn.apply(u).abs().max())
    opn.close()


@pytest.mark.parametrize("ncell,k,kw", [((4, 4, 4), 3, dict(curved=True, variable_coef=True)),
                                        ((3, 2, 4), 5, dict(bc=(0, 1, 0, 0, 1, 0))),
                                        ((2, 2, 2), 8, dict(curved=True))])
def test_diagonal(dg, orc, ncell, k, kw):
    import torch
    op = dg.Operator(ncell, k, **kw)
    ref = orc.diag(orc.problem(ncell, k, **kw))
    d64 = op.diagonal(torch.float64).cpu().numpy()
    assert _rel(d64, ref) <= TOL64
    d32 = op.diagonal(torch.float32).cpu().numpy()
    assert np.array_equal(d32, d64.astype(np.float32))
    op.close()


def test_diagonal_config4_sampled(dg, orc):
    import torch
    op = dg.Operator(32, 5, curved=True, variable_coef=True)
    cells = synth.sample_cells(32, 150, seed=4, n_boundary=40)
    ref = orc.diag_cells(orc.problem(32, 5, curved=True, variable_coef=True), cells)
    d = op.diagonal().cpu().numpy().reshape(-1, 216)[cells]
    assert _rel(d, ref) <= TOL64
    op.close()


@pytest.mark.parametrize("ncell,k,kw", [((4, 4, 4), 2, dict(curved=True, variable_coef=True)),
                                        ((8, 8, 8), 5, dict(curved=True, variable_coef=True)),
                                        ((3, 5, 2), 4, {})])
def test_rhs_and_error_norms(dg, orc, ncell, k, kw):
    import torch
    op = dg.Operator(ncell, k, **kw)
    p = orc.problem(ncell, k, **kw)
    b = op.rhs().cpu().numpy()
    ref = orc.rhs(p)
    assert _rel(b, ref) <= TOL64
    x = synth.src_vector(op.n_dofs, 77) * 1e-3
    l2, h1 = op.error_manufactured(torch.from_numpy(x).cuda())
    rl2, rh1 = orc.errors(p, x, extra=2)
    assert l2 == pytest.approx(rl2, rel=1e-10)
    assert h1 == pytest.approx(rh1, rel=1e-10)
    op.close()


def test_apply_argument_errors(dg):
    import torch
    op = dg.Operator(4, 2, precisions=dg.PREC_F64)
    x = torch.zeros(op.n_dofs, dtype=torch.float64, device="cuda")
    with pytest.raises(dg.DGError) as e:
        op.apply(x, x)                                  # aliasing
    assert e.value.status == dg.DG_ERR_ARG
    with pytest.raises(dg.DGError):
        op.apply(x, torch.zeros(op.n_dofs - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(dg.DGError):
        op.apply(x.float(), torch.zeros(op.n_dofs, dtype=torch.float32, device="cuda"))  # F32 not enabled
    op.close()


def test_apply_largest_size(dg, orc):
    """The largest problem the library accepts: 256^3 affine cells at k=4,
    2,097,152,000 DoFs (just under 2^31).  Offsets of the last cells pass
    2^31 elements and 16 GB, so this checks the 64-bit address arithmetic;
    sampled cells (corners, the very last cells, random) against the oracle."""
    import torch
    N, k = 256, 4
    n3 = (k + 1) ** 3
    op = dg.Operator(N, k, precisions=dg.PREC_F64)
    nd = op.n_dofs
    assert nd == N ** 3 * n3 and nd < 2 ** 31
    g = torch.Generator(device="cuda")
    g.manual_seed(256)
    x = torch.rand(nd, dtype=torch.float64, device="cuda", generator=g) * 2.0 - 1.0
    y = torch.full_like(x, float("nan"))
    op.apply(x, y)
    cells = np.unique(np.concatenate([synth.sample_cells(N, 200, seed=256, n_boundary=40),
                                      np.arange(N ** 3 - 8, N ** 3)]))
    rows = torch.from_numpy(cells).cuda()
    got = y.view(-1, n3).index_select(0, rows).cpu().numpy()
    assert np.isfinite(got).all()
    src = x.cpu().numpy()
    del y
    ref = orc.apply_cells(orc.problem(N, k), src, cells)
    assert _rel(got, ref) <= TOL64
    del x, src
    op.close()
    torch.cuda.empty_cache()


def test_alternating_sweep_order_is_invisible(dg):
    """Successive applies walk the cells in opposite orders (MALL reuse);
    every apply still returns bitwise the same result."""
    import torch
    for kw in (dict(curved=True), dict(curved=True, merged=True), dict(variable_coef=True)):
        op = dg.Operator((9, 7, 6), 4, **kw)
        u = torch.from_numpy(synth.src_vector(op.n_dofs, 77)).cuda()
        ys = [op.apply(u) for _ in range(3)]
        assert torch.equal(ys[0], ys[1]) and torch.equal(ys[1], ys[2])
        op.close()
