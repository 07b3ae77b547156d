"""Pins of the oracle's Leja points, phi functions and divided differences.

They tie ``oracle.leja`` to closed forms (the first Leja points, 1/(t - x),
polynomials), to numpy/scipy special functions, to brute-force maximisation on
a fine grid, and to the interpolation property of the Newton form.
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import leja


def test_first_leja_points_closed_form():
    """xi_0 = 2, then -2 (farthest point), then 0 (argmax of 4 - x^2), then
    the argmax of |x^3 - 4x| on [-2, 2], attained at +-2/sqrt(3); ties go
    to the larger point."""
    xi = leja.leja_points(4)
    assert xi[0] == 2.0 and xi[1] == -2.0
    assert abs(xi[2]) < 1e-15
    assert xi[3] == pytest.approx(2.0 / math.sqrt(3.0), abs=1e-14)


def test_leja_points_maximise_product_brute_force():
    xi = leja.leja_points(60)
    grid = np.linspace(-2.0, 2.0, 400001)
    for k in range(1, 60):
        logp = np.sum(np.log(np.abs(grid[:, None] - xi[None, :k]) + 1e-300), axis=1)
        best_grid = logp.max()
        at_xi = np.sum(np.log(np.abs(xi[k] - xi[:k])))
        # the exact maximiser beats every grid point and sits within a cell of the best
        assert at_xi >= best_grid - 1e-9
        assert abs(grid[np.argmax(logp)] - xi[k]) < 1e-3 or abs(logp.max() - at_xi) < 1e-6
    assert len(np.unique(xi)) == 60
    assert np.all(np.abs(xi) <= 2.0)


def test_leja_table_prefix_stable():
    assert np.array_equal(leja.leja_points(30), leja.leja_points(200)[:30])


@pytest.mark.parametrize("z", [-300.0, -40.0, -1.0, -0.3, -1e-3, -1e-9, 0.0, 1e-7, 0.4, 2.0])
def test_phi1_matches_expm1(z):
    want = 1.0 if z == 0 else math.expm1(z) / z
    assert leja.phi(1, z) == pytest.approx(want, rel=1e-15, abs=1e-300)


@pytest.mark.parametrize("z", [-50.0, -2.0, -0.49, -0.51, 0.0, 0.3, 3.0])
def test_phi0_phi2_phi3(z):
    assert leja.phi(0, z) == pytest.approx(math.exp(z), rel=1e-15)
    with mpmath.workdps(60):
        zz = mpmath.mpf(z)
        if z == 0:
            p2, p3 = mpmath.mpf(1) / 2, mpmath.mpf(1) / 6
        else:
            p2 = (mpmath.exp(zz) - 1 - zz) / zz ** 2
            p3 = (mpmath.exp(zz) - 1 - zz - zz ** 2 / 2) / zz ** 3
        assert leja.phi(2, z) == pytest.approx(float(p2), rel=1e-14)
        assert leja.phi(3, z) == pytest.approx(float(p3), rel=1e-13)


def test_dd_recurrence_reciprocal_closed_form():
    """For f(x) = 1/(t - x): f[x_0..x_j] = 1 / prod_{i<=j} (t - x_i)."""
    nodes = [mpmath.mpf(v) for v in leja.leja_points(25)]
    t = mpmath.mpf(3)
    with mpmath.workdps(50):
        d = leja.dd_recurrence([1 / (t - x) for x in nodes], nodes)
        for j in range(25):
            want = mpmath.mpf(1)
            for i in range(j + 1):
                want /= (t - nodes[i])
            assert abs(d[j] - want) <= mpmath.mpf(10) ** -40 * abs(want)


def test_dd_recurrence_polynomial():
    """A cubic 2x^3 - x + 5 has f[x0..x3] = 2 and all higher differences 0;
    f[x0] = f(x0), f[x0,x1] = (f(x1) - f(x0))/(x1 - x0)."""
    nodes = [mpmath.mpf(v) for v in leja.leja_points(8)]
    f = lambda x: 2 * x ** 3 - x + 5
    with mpmath.workdps(50):
        d = leja.dd_recurrence([f(x) for x in nodes], nodes)
        assert d[0] == f(nodes[0])
        assert abs(d[1] - (f(nodes[1]) - f(nodes[0])) / (nodes[1] - nodes[0])) < 1e-40
        assert abs(d[3] - 2) < 1e-40
        for j in range(4, 8):
            assert abs(d[j]) < 1e-40


@pytest.mark.parametrize("k", [0, 1, 2])
@pytest.mark.parametrize("length", [1.0, 13.3, 100.0])
def test_divided_differences_interpolate(k, length):
    """The Newton interpolant with these differences reproduces
    f(x) = phi_k(delta (c + gamma x)) at the nodes and approximates it on all of
    [-2, 2] (the interval [a, b] = [-length, 0] mapped, delta = 1)."""
    a, b = -length, 0.0
    c, gamma = 0.5 * (a + b), 0.25 * (b - a)
    xi = leja.leja_points(101)
    d = leja.divided_differences(k, 1.0, c, gamma, xi)
    f = np.array([leja.phi(k, c + gamma * x) for x in xi])
    assert np.allclose(leja.newton_eval(d, xi, xi[:40]), f[:40], rtol=1e-12, atol=1e-14)
    grid = np.linspace(-2, 2, 257)
    fg = np.array([leja.phi(k, c + gamma * x) for x in grid])
    err = np.max(np.abs(leja.newton_eval(d, xi, grid) - fg))
    assert err < 1e-13, err


def test_divided_differences_exponential_scaling():
    """For f(x) = exp(s x) the differences scale as s^j / j! on coincident
    nodes; on distinct nodes they are positive and bounded by s^j/j! times
    exp(2s) (mean-value form of divided differences)."""
    s = 0.7
    xi = leja.leja_points(20)
    d = leja.divided_differences(0, 1.0, 0.0, s, xi)  # phi_0(s x)
    for j in range(20):
        bound = s ** j / math.factorial(j)
        assert 0 < d[j] <= bound * math.exp(2 * s) * (1 + 1e-12)
        assert d[j] >= bound * math.exp(-2 * s) * (1 - 1e-12)
