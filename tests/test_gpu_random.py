"""Seeded random configurations against the oracle: mesh shape, degree,
boundary conditions, box, map, coefficient, geometry storage and basis are
drawn together, so that combinations no hand-written case lists are covered.
Each case checks the FP64 and FP32 apply and the diagonal to the usual bar."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5


def _case(seed):
    rng = np.random.default_rng(9000 + seed)
    k = int(rng.integers(1, 9))
    n = k + 1
    # keep the oracle's O(n^6) per cell work small
    max_cells = max(1, int(60 * (4 / n) ** 3))
    while True:
        ncell = tuple(int(v) for v in rng.integers(1, 6, size=3))
        if np.prod(ncell) <= max_cells:
            break
    lo = tuple(float(v) for v in rng.uniform(-1.0, 0.5, size=3))
    hi = tuple(lo[d] + float(rng.uniform(0.5, 2.0)) for d in range(3))
    kw = dict(curved=bool(rng.integers(0, 2)), variable_coef=bool(rng.integers(0, 2)),
              bc=tuple(int(v) for v in rng.integers(0, 2, size=6)), lo=lo, hi=hi)
    if not kw["variable_coef"]:
        kw["coef_value"] = float(rng.uniform(0.5, 3.0))
    storage = ["jacobian", "merged", "mixed", "positions"][int(rng.integers(0, 4))]
    basis = "hermite" if k >= 3 and rng.integers(0, 2) else "nodal"
    return ncell, k, kw, storage, basis


@pytest.fixture(scope="module")
def dg():
    import torch
    import paper_1711_03590_amd as dg
    assert torch.cuda.is_available()
    dg.lib()
    return dg


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("seed", range(24))
def test_random_configuration(dg, orc, seed):
    import torch
    ncell, k, kw, storage, basis = _case(seed)
    print(f"random case {seed}: ncell={ncell} k={k} {kw} storage={storage} basis={basis}", flush=True)
    op = dg.Operator(ncell, k, storage=storage, basis=basis, **kw)
    geo = "positions" if storage == "positions" and kw["curved"] else "map"
    p = orc.problem(ncell, k, basis="hermite" if basis == "hermite" else "gll", cell_geometry=geo, **kw)
    src = synth.src_vector(op.n_dofs, 500 + seed)
    ref = orc.apply(p, src)
    dst = torch.full((op.n_dofs,), float("nan"), dtype=torch.float64, device="cuda")
    op.apply(torch.from_numpy(src).cuda(), dst)
    assert _rel(dst.cpu().numpy(), ref) <= TOL64
    y32 = op.apply(torch.from_numpy(src.astype(np.float32)).cuda()).double().cpu().numpy()
    assert _rel(y32, ref) <= TOL32
    assert _rel(op.diagonal(torch.float64).cpu().numpy(), orc.diag(p)) <= TOL64
    op.close()
