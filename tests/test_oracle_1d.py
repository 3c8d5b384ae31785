"""Pins of the oracle's 1D rules against closed forms (no GPU).

The SIPG operator uses a nodal Lagrange basis on the Gauss-Lobatto points and
Gauss-Legendre quadrature on the same number of points per direction
(Sec. 2, Eq. (4); Sec. 3.1, Table 2's "Gaussian quadrature on k^d points").
"""
import math

import numpy as np
import pytest


def test_gauss_closed_forms(orc):
    x, w = orc.gauss(1)
    assert x[0] == pytest.approx(0.5, abs=1e-15) and w[0] == pytest.approx(1.0, abs=1e-15)
    x, w = orc.gauss(2)
    r = 1.0 / (2.0 * math.sqrt(3.0))
    assert np.allclose(x, [0.5 - r, 0.5 + r], atol=1e-15, rtol=0)
    assert np.allclose(w, [0.5, 0.5], atol=1e-15, rtol=0)
    x, w = orc.gauss(3)
    r = 0.5 * math.sqrt(3.0 / 5.0)
    assert np.allclose(x, [0.5 - r, 0.5, 0.5 + r], atol=1e-15, rtol=0)
    assert np.allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=1e-15, rtol=0)
    # 4 points: t = +-sqrt(3/7 -+ 2/7 sqrt(6/5)), w = (18 +- sqrt 30)/36 on [-1,1]
    x, w = orc.gauss(4)
    t1 = math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5))
    t2 = math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5))
    assert np.allclose(x, [0.5 - t2 / 2, 0.5 - t1 / 2, 0.5 + t1 / 2, 0.5 + t2 / 2], atol=1e-15, rtol=0)
    w1, w2 = (18 + math.sqrt(30)) / 72, (18 - math.sqrt(30)) / 72
    assert np.allclose(w, [w2, w1, w1, w2], atol=1e-15, rtol=0)


@pytest.mark.parametrize("n", range(1, 13))
def test_gauss_exactness(orc, n):
    x, w = orc.gauss(n)
    assert np.all(np.diff(x) > 0)
    for m in range(2 * n):
        assert np.dot(w, x ** m) == pytest.approx(1.0 / (m + 1), rel=2e-14, abs=2e-15)
    # and not exact one degree higher: the nodes are the roots of the shifted
    # Legendre polynomial P_n(2x-1), so the rule gives 0 for int P_n^2 = 1/(2n+1)
    P = np.polynomial.legendre.Legendre.basis(n)(2 * x - 1)
    assert np.abs(P).max() < 1e-13
    assert np.dot(w, P ** 2) < 1e-20


def test_gll_closed_forms(orc):
    assert np.allclose(orc.gll(2), [0, 1], atol=0)
    assert np.allclose(orc.gll(3), [0, 0.5, 1], atol=1e-16)
    r = 1.0 / (2.0 * math.sqrt(5.0))
    assert np.allclose(orc.gll(4), [0, 0.5 - r, 0.5 + r, 1], atol=1e-15, rtol=0)
    r = 0.5 * math.sqrt(3.0 / 7.0)
    assert np.allclose(orc.gll(5), [0, 0.5 - r, 0.5, 0.5 + r, 1], atol=1e-15, rtol=0)


@pytest.mark.parametrize("n", range(2, 13))
def test_gll_is_lobatto_rule(orc, n):
    # Lobatto nodes carry an interpolatory rule exact to degree 2n-3; the
    # weights 1/(n(n-1) P_{n-1}(t)^2) on [0,1] come from numpy's Legendre.
    x = orc.gll(n)
    t = 2 * x - 1
    P = np.polynomial.legendre.Legendre.basis(n - 1)(t)
    w = 1.0 / (n * (n - 1) * P ** 2)
    assert np.all(np.diff(x) > 0)
    for m in range(2 * n - 2):
        assert np.dot(w, x ** m) == pytest.approx(1.0 / (m + 1), rel=1e-13)
    # symmetric about 1/2
    assert np.allclose(x + x[::-1], 1.0, atol=1e-15, rtol=0)


@pytest.mark.parametrize("n", [2, 3, 5, 9])
def test_lagrange_delta_partition(orc, n):
    nodes = orc.gll(n)
    for j in range(n):
        for m in range(n):
            v, _ = orc.lagrange(nodes, j, nodes[m])
            assert v == pytest.approx(1.0 if j == m else 0.0, abs=1e-13)
    for xi in np.linspace(-0.1, 1.1, 13):
        vals = [orc.lagrange(nodes, j, xi) for j in range(n)]
        assert sum(v for v, _ in vals) == pytest.approx(1.0, abs=1e-12)
        assert sum(d for _, d in vals) == pytest.approx(0.0, abs=1e-10)
        # first moment: sum_j x_j phi_j(xi) = xi, derivative 1
        assert sum(nodes[j] * vals[j][0] for j in range(n)) == pytest.approx(xi, abs=1e-12)
        assert sum(nodes[j] * vals[j][1] for j in range(n)) == pytest.approx(1.0, abs=1e-10)


def test_lagrange_quadratic_closed_form(orc):
    nodes = orc.gll(3)  # 0, 1/2, 1
    for xi in [0.0, 0.13, 0.5, 0.77, 1.0]:
        ref = [(2 * xi - 1) * (xi - 1), 4 * xi * (1 - xi), xi * (2 * xi - 1)]
        dref = [4 * xi - 3, 4 - 8 * xi, 4 * xi - 1]
        for j in range(3):
            v, d = orc.lagrange(nodes, j, xi)
            assert v == pytest.approx(ref[j], abs=1e-15)
            assert d == pytest.approx(dref[j], abs=1e-14)
