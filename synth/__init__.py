"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds no arithmetic of the method: only the workload descriptions (mesh
size, degree, geometry, coefficient) and seeded random draws.  The oracle
and the GPU library never import each other; both are fed from here.

Workloads (all on the unit cube, all six sides Dirichlet):
  C1  8^3 affine, k=3, c=1                                   (32,768 DoFs)
  C2  32^3 sine-curved map (amplitude 0.05), k=2..8          (k=4: 4,096,000 DoFs)
  C3a 64^3 affine, k=4, c = 1 + 0.5 sin(pi x) cos(pi y) z    (32,768,000 DoFs)
  C3b 64^3 sine-curved, k=4, same c                          (32,768,000 DoFs)
  C4  32^3 sine-curved, k=5, same c, manufactured load       (7,077,888 DoFs)
  C5  request stream: Poisson arrivals, edge cells log-uniform in [4,48],
      degree uniform in 2..7, 50/50 affine or curved
Source vectors: numpy default_rng(seed).uniform(-1, 1, n_dofs) in FP64 with
seed = 1000 * config + degree; FP32 runs round the same draw to nearest.
"""
from __future__ import annotations

import math

import numpy as np

AMPLITUDE = 0.05

CONFIGS = {
    "C1": dict(ncell=8, degree=3, curved=False, variable_coef=False),
    "C2": dict(ncell=32, degree=4, curved=True, variable_coef=False),
    "C3a": dict(ncell=64, degree=4, curved=False, variable_coef=True),
    "C3b": dict(ncell=64, degree=4, curved=True, variable_coef=True),
    "C4": dict(ncell=32, degree=5, curved=True, variable_coef=True),
}
CONFIG_ID = {"C1": 1, "C2": 2, "C3a": 3, "C3b": 3, "C4": 4}


def seed_for(config: int, degree: int) -> int:
    return 1000 * config + degree


def n_dofs(ncell, degree) -> int:
    if isinstance(ncell, int):
        ncell = (ncell,) * 3
    return int(ncell[0] * ncell[1] * ncell[2] * (degree + 1) ** 3)


def src_vector(n: int, seed: int) -> np.ndarray:
    """FP64 uniform [-1, 1) draw of length n."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def sample_cells(ncell, count: int, seed: int, n_boundary: int = 100) -> np.ndarray:
    """Random cells plus all 8 corner cells and some boundary cells (sorted, unique)."""
    if isinstance(ncell, int):
        ncell = (ncell,) * 3
    nx, ny, nz = ncell
    total = nx * ny * nz
    rng = np.random.default_rng(seed)
    cells = set(rng.integers(0, total, size=min(count, total)).tolist())
    for cz in (0, nz - 1):
        for cy in (0, ny - 1):
            for cx in (0, nx - 1):
                cells.add(cx + nx * (cy + ny * cz))
    for _ in range(n_boundary):
        c = [int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz))]
        a = int(rng.integers(0, 3))
        c[a] = 0 if rng.random() < 0.5 else (ncell[a] - 1)
        cells.add(c[0] + nx * (c[1] + ny * c[2]))
    return np.array(sorted(cells), dtype=np.int64)


def request_trace(n_requests: int, rate: float, seed: int = 5005, edge_range=(4, 48), degrees=(2, 7)):
    """Open-loop request stream: Poisson arrivals at `rate` per second, edge
    cells drawn independently log-uniform in edge_range and rounded, degree
    uniform in [degrees], curved with probability 1/2, RHS seed per request."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    lo, hi = math.log(edge_range[0]), math.log(edge_range[1])
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        ncell = tuple(int(round(math.exp(rng.uniform(lo, hi)))) for _ in range(3))
        out.append(dict(id=i, arrival=t, ncell=ncell, degree=int(rng.integers(degrees[0], degrees[1] + 1)),
                        curved=bool(rng.random() < 0.5), rhs_seed=int(rng.integers(0, 2 ** 31))))
    return out
