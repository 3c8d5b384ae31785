"""Invariants and geometry pins of the oracle on curved meshes and with the
variable coefficient (no GPU).

  symmetry        u^T A v = v^T A u: the SIPG form of Sec. 2 Eq. (2) is symmetric
  null space      all-Neumann operator annihilates constants (no jumps, no gradient)
  SPD             Dirichlet operator positive definite with tau = (k+1)^2/h
  translation     affine uniform mesh: every interior block row is the same
  boundary faces  the sine map fixes the cube's faces, so Nanson's area element
                  on a boundary face equals the unmapped one and the normal is +-e_a
  interior faces  both sides see the same physical point and area element
  volume          the map takes the unit cube onto itself: sum of JxW = 1
  forcing         f = -div(c grad u*) checked by central differences
"""
import numpy as np
import pytest

CURVED = dict(curved=True, amplitude=0.05)


@pytest.mark.parametrize("k,N,kw", [
    (2, 3, dict(CURVED, variable_coef=True)),
    (3, (2, 3, 2), dict(CURVED)),
    (4, 2, dict(variable_coef=True)),
    (1, 4, dict(CURVED, variable_coef=True, bc=(0, 1, 1, 0, 0, 1))),
])
def test_symmetry(orc, k, N, kw):
    p = orc.problem(N, k, **kw)
    rng = np.random.default_rng(11)
    u = rng.uniform(-1, 1, orc.n_dofs(p))
    v = rng.uniform(-1, 1, orc.n_dofs(p))
    Au, Av = orc.apply(p, u), orc.apply(p, v)
    scale = np.linalg.norm(Au) * np.linalg.norm(v)
    assert abs(v @ Au - u @ Av) <= 1e-13 * scale


@pytest.mark.parametrize("k,N,kw", [
    (2, 3, dict(CURVED, variable_coef=True)),
    (4, 2, dict(CURVED)),
    (3, (3, 2, 2), dict(variable_coef=True)),
])
def test_neumann_null_space(orc, k, N, kw):
    p = orc.problem(N, k, bc=(1,) * 6, **kw)
    one = np.ones(orc.n_dofs(p))
    u = np.random.default_rng(3).uniform(-1, 1, orc.n_dofs(p))
    ref = np.abs(orc.apply(p, u)).max()
    assert np.abs(orc.apply(p, one)).max() <= 1e-12 * ref


@pytest.mark.parametrize("k,N,kw", [
    (1, 3, {}), (2, 2, {}), (3, 2, dict(CURVED)), (4, 1, dict(CURVED, variable_coef=True)),
    (5, 1, {}), (2, 2, dict(CURVED, variable_coef=True)), (8, 1, dict(CURVED)),
])
def test_spd(orc, k, N, kw):
    p = orc.problem(N, k, **kw)
    A = orc.assemble_dense(p)
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    lam = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert lam[0] > 1e-8 * lam[-1]


def test_translation_invariance(orc):
    p = orc.problem(4, 2)
    inner = [1 + 4 * (1 + 4 * 1), 2 + 4 * (1 + 4 * 2), 1 + 4 * (2 + 4 * 2)]
    B = orc.block_rows(p, inner)
    for b in B[1:]:
        assert np.abs(b - B[0]).max() <= 1e-13 * np.abs(B[0]).max()


@pytest.mark.parametrize("N", [(4, 4, 4), (3, 5, 2)])
def test_boundary_faces_unchanged_by_map(orc, N):
    k = 4
    p = orc.problem(N, k, **CURVED)
    x, w = orc.gauss(k + 1)
    h = [1.0 / N[d] for d in range(3)]
    rng = np.random.default_rng(5)
    for _ in range(60):
        f = int(rng.integers(6))
        a, side = f // 2, f % 2
        t = [d for d in range(3) if d != a]
        ci = [int(rng.integers(N[d])) for d in range(3)]
        ci[a] = N[a] - 1 if side else 0
        e = ci[0] + N[0] * (ci[1] + N[1] * ci[2])
        q1, q2 = int(rng.integers(k + 1)), int(rng.integers(k + 1))
        fp = orc.face_point(p, e, f, q1, q2)
        assert not fp["interior"]
        assert fp["ds"] == pytest.approx(h[t[0]] * h[t[1]] * w[q1] * w[q2], rel=1e-13)
        nref = np.zeros(3)
        nref[a] = 1.0 if side else -1.0
        assert np.abs(fp["normal"] - nref).max() <= 1e-13
        assert fp["x"][a] == pytest.approx(float(side), abs=1e-15)
        # tangential position of the face point: the unmapped one
        assert fp["x"][t[0]] == pytest.approx((ci[t[0]] + x[q1]) * h[t[0]], abs=1e-15)
        assert fp["x"][t[1]] == pytest.approx((ci[t[1]] + x[q2]) * h[t[1]], abs=1e-15)


def test_interior_faces_agree(orc):
    k, N = 3, 4
    p = orc.problem(N, k, **CURVED)
    rng = np.random.default_rng(9)
    for _ in range(40):
        f = int(rng.integers(6))
        a, side = f // 2, f % 2
        ci = [int(rng.integers(N)) for _ in range(3)]
        ci[a] = int(rng.integers(N - 1)) + (1 if not side else 0)
        e = ci[0] + N * (ci[1] + N * ci[2])
        fp = orc.face_point(p, e, f, int(rng.integers(k + 1)), int(rng.integers(k + 1)))
        assert fp["interior"]
        assert np.abs(fp["x"] - fp["x_nb"]).max() <= 1e-14
        assert fp["ds_nb"] == pytest.approx(fp["ds"], rel=1e-13)
        assert np.linalg.norm(fp["normal"]) == pytest.approx(1.0, abs=1e-15)


def test_mapped_volume(orc):
    assert orc.volume(orc.problem(8, 4, **CURVED)) == pytest.approx(1.0, abs=1e-10)
    assert orc.volume(orc.problem((2, 3, 4), 2, hi=(2.0, 1.5, 0.5))) == pytest.approx(1.5, abs=1e-14)
    # the sine map changes every interior cell's volume but not the total
    p = orc.problem(2, 4, **CURVED)
    assert orc.volume(p) == pytest.approx(1.0, abs=1e-4)


@pytest.mark.parametrize("variable", [False, True])
def test_forcing_by_finite_differences(orc, variable):
    p = orc.problem(1, 2, variable_coef=variable)
    pi = np.pi

    def c(x):
        return 1.0 + 0.5 * np.sin(pi * x[0]) * np.cos(pi * x[1]) * x[2] if variable else 1.0

    def u(x):
        return np.sin(pi * x[0]) * np.sin(pi * x[1]) * np.sin(pi * x[2])

    hh = 1e-4
    rng = np.random.default_rng(2)
    for _ in range(10):
        x = rng.uniform(0.05, 0.95, 3)
        div = 0.0
        for d in range(3):
            e = np.zeros(3)
            e[d] = hh / 2
            fp = c(x + e) * (u(x + 2 * e) - u(x)) / hh
            fm = c(x - e) * (u(x) - u(x - 2 * e)) / hh
            div += (fp - fm) / hh
        assert orc.forcing_at(p, x) == pytest.approx(-div, rel=1e-5, abs=1e-5)
