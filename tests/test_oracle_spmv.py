"""The oracle's matrix-based apply (no GPU): the block-sparse product of the
assembled block rows equals the matrix-free apply on every row (curved,
variable coefficient, Neumann sides, sampled rows in any order), so timing
it measures the same operator."""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("ncell,k,kw", [((3, 4, 2), 2, dict(curved=True, variable_coef=True)),
                                        ((2, 3, 3), 3, dict(bc=(0, 1, 0, 0, 1, 0))),
                                        (4, 1, dict(curved=True))])
def test_spmv_equals_apply(orc, ncell, k, kw):
    p = orc.problem(ncell, k, **kw)
    nc = orc.n_cells(p)
    cells = np.arange(nc)
    src = synth.src_vector(orc.n_dofs(p), 11)
    y = orc.spmv_blocks(p, cells, orc.block_rows(p, cells), src).reshape(-1)
    ref = orc.apply(p, src)
    assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)
    # the same through scipy's product of the assembled matrix
    assert np.linalg.norm(orc.assemble_sparse(p) @ src - y) <= 1e-13 * np.linalg.norm(ref)
    # a permuted subset of rows
    sub = np.random.default_rng(2).permutation(nc)[: max(1, nc // 2)]
    ys = orc.spmv_blocks(p, sub, orc.block_rows(p, sub), src)
    n3 = (k + 1) ** 3
    assert np.allclose(ys, ref.reshape(nc, n3)[sub], rtol=0, atol=1e-13 * np.abs(ref).max())


def test_spmv_rejects_bad_sizes(orc):
    p = orc.problem(2, 1)
    with pytest.raises(ValueError):
        orc.spmv_blocks(p, np.arange(2), np.zeros(3), np.zeros(orc.n_dofs(p)))
