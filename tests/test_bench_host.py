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
