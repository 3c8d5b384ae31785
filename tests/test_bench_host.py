"""Host-side checks of bench.py (no GPU): the algorithmic byte model, the
committed traffic summary matching the kernel source, and the one-GPU
contract."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as b
    return b


def test_algorithmic_bytes(bench):
    # k=4, 32^3 curved: src + dst + 10 cell values + 4 face values per point
    assert bench.algorithmic_bytes_per_dof(32, 4, 8) == pytest.approx(115.8, abs=0.05)
    assert bench.algorithmic_bytes_per_dof(32, 4, 4) == pytest.approx(57.9, abs=0.05)
    assert bench.algorithmic_bytes_per_dof(32, 4, 8, "curved-merged") == pytest.approx(83.8, abs=0.05)
    assert bench.algorithmic_bytes_per_dof(32, 4, 8, "curved-positions") == pytest.approx(67.8, abs=0.05)
    assert bench.algorithmic_bytes_per_dof(32, 4, 8, "advection") == pytest.approx(44.95, abs=0.01)
    assert bench.algorithmic_bytes_per_dof(64, 4, 8, "affine-variable") == pytest.approx(28.875, abs=0.01)


def test_traffic_summary_is_for_the_current_kernel(bench):
    """The committed --pmc summary carries the kernel-source hash; bench.py
    reports traffic only when it matches (so a changed kernel reports null
    until it is profiled again)."""
    t64 = bench.measured_traffic("f64")
    t32 = bench.measured_traffic("f32")
    if t64 is None or t32 is None:
        pytest.skip("the committed --pmc summary was taken on another kernel source; profile again")
    alg = 115.8 * 4096000
    assert 1.0 <= t64 / alg <= 1.6


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one MI355X" in (r.stdout + r.stderr)


def test_parity_bookkeeping(bench, orc):
    """keep_rows / check_parity on the host: rows equal to the oracle's give
    a zero error, perturbed rows an error above the FP64 bar; a kept
    solution's oracle residual is its true residual."""
    import numpy as np
    import torch

    import synth
    ncell, k = (3, 2, 4), 2
    p = orc.problem(ncell, k, curved=True)
    nd = orc.n_dofs(p)
    seed = 77
    y = orc.apply(p, synth.src_vector(nd, seed))
    cells = np.array([0, 5, 23], dtype=np.int64)
    good, bad = {}, {}
    bench.keep_rows(good, "f64", torch.from_numpy(y.copy()), cells, (ncell, k, dict(curved=True)), (nd, seed))
    yb = y.copy()
    yb[5 * 27 + 3] += 1e-9 * np.abs(y).max()
    bench.keep_rows(bad, "f64", torch.from_numpy(yb), cells, (ncell, k, dict(curved=True)), (nd, seed))
    sol = {}
    x = synth.src_vector(nd, 3)
    b = orc.apply(p, x)
    b[0] += 1.0
    bench.keep_solution(sol, torch.from_numpy(x), torch.from_numpy(b), (ncell, k, dict(curved=True)))
    bench.check_parity(orc)
    assert good["err_vs_oracle"]["rel_l2"] == 0.0 and good["err_vs_oracle"]["ok"]
    assert not bad["err_vs_oracle"]["ok"]
    assert sol["oracle_rel_residual"]["value"] == pytest.approx(1.0 / np.linalg.norm(b), rel=1e-9)
    assert not bench.PARITY


def test_matrix_baseline_small(bench, orc):
    """The matrix-based CPU comparator's bookkeeping on a tiny case: the
    block-sparse product equals the matrix-free apply, and the
    extrapolation is by the sampled fraction of rows."""
    import numpy as np

    import synth
    r = bench.matrix_baseline(orc, np, synth, cases=(("t", 4, 2, dict(curved=True), 16),), spmv_s=0.05)
    t = r["t"]
    assert t["rows_assembled"] == 16 and t["of_rows"] == 64 and t["extrapolated_from_sample"]
    assert t["spmv_vs_matrix_free_rel_l2"] <= 1e-13
    assert t["matrix_bytes"] == 64 * 7 * 27 * 27 * 8
