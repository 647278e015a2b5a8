"""Pins for the oracle's spectral derivatives (Sec. 3, pseudo-spectral space).

Band-limited trigonometric polynomials are differentiated exactly by the
Fourier method; the Nyquist-free gradient is real and skew-symmetric.
"""
import numpy as np
import pytest
import sympy as sp

import synthetic
from oracle.spectral import Grid, dot

X, Y, Z = sp.symbols("x y z", real=True)


def _eval(expr, grid):
    f = sp.lambdify((X, Y, Z), expr, "numpy")
    x3, y3, z3 = grid.coords()
    return np.broadcast_to(np.asarray(f(x3, y3, z3), dtype=float), x3.shape).copy()


@pytest.mark.parametrize("n", [16, 32])
def test_derivative_of_trig_polynomial_is_exact(n):
    g = Grid(n)
    expr = sp.sin(3 * X + 2 * Y) + sp.cos(5 * Z - X) * sp.sin(Y) + 0.3 * sp.cos(7 * Y)
    c = _eval(expr, g)
    for a, s in enumerate((X, Y, Z)):
        ref = _eval(sp.diff(expr, s), g)
        assert np.max(np.abs(g.deriv(c, a) - ref)) < 1e-12 * n


def test_nyquist_mode_is_dropped():
    n = 16
    g = Grid(n)
    x3, y3, z3 = g.coords()
    c = np.cos(n // 2 * x3)            # the Nyquist mode along x
    assert np.max(np.abs(g.deriv(c, 0))) < 1e-13
    c = np.cos(n // 2 * z3) * np.sin(y3)
    assert np.max(np.abs(g.deriv(c, 2))) < 1e-13


@pytest.mark.parametrize("a", [0, 1, 2])
def test_gradient_is_skew_symmetric(a):
    n = 16
    g = Grid(n)
    u = synthetic.random_field(n, 1)
    v = synthetic.random_field(n, 2)
    lhs = dot(g.deriv(u, a), v)
    rhs = -dot(u, g.deriv(v, a))
    assert abs(lhs - rhs) < 1e-11 * (abs(lhs) + 1.0)
    assert abs(dot(g.deriv(u, a), u)) < 1e-10


def test_constants_have_zero_gradient_and_divergence():
    g = Grid(16)
    c = np.full((16, 16, 16), 3.7)
    for a in range(3):
        assert np.max(np.abs(g.deriv(c, a))) < 1e-13
    assert np.max(np.abs(g.div(np.stack([c, 2 * c, -c])))) < 1e-13
