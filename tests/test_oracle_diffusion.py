"""Pins for the oracle's diffusion operator and Crank-Nicolson solve
(Eqs. e:diffusion_op, e:diffusion_tensor; Sec. 3, CN scheme and CG).
"""
import numpy as np
import pytest
import sympy as sp

import synthetic
from oracle import solvers
from oracle.spectral import Grid, dot, norm

X, Y, Z = sp.symbols("x y z", real=True)


def _eval(expr, grid):
    f = sp.lambdify((X, Y, Z), expr, "numpy")
    x3, y3, z3 = grid.coords()
    return np.broadcast_to(np.asarray(f(x3, y3, z3), dtype=float), x3.shape).copy()


def test_diffusion_operator_matches_analytic_divergence():
    # deg K + deg c < N/2: the pseudo-spectral product is alias-free.
    n = 16
    g = Grid(n)
    K = 1 + sp.Rational(3, 10) * sp.cos(X) + sp.Rational(1, 5) * sp.sin(2 * Y + Z)
    c = sp.sin(X + 2 * Y) + sp.cos(3 * Z)
    ref = sum(sp.diff(K * sp.diff(c, s), s) for s in (X, Y, Z))
    out = solvers.diffusion_op(g, _eval(K, g), _eval(c, g))
    assert np.max(np.abs(out - _eval(ref, g))) < 1e-11


def test_diffusion_operator_is_symmetric_negative_semidefinite():
    n = 16
    g = Grid(n)
    K = 0.05 + 0.1 * np.abs(synthetic.random_field(n, 3, 2.0))
    a = synthetic.random_field(n, 4)
    b = synthetic.random_field(n, 5)
    Da, Db = solvers.diffusion_op(g, K, a), solvers.diffusion_op(g, K, b)
    assert abs(dot(Da, b) - dot(a, Db)) < 1e-10 * abs(dot(Da, b))
    assert dot(Da, a) < 0


@pytest.mark.parametrize("k", [(1, 1, 1), (2, 0, 1), (0, 3, 0)])
def test_cn_constant_coefficient_mode_decay_is_exact(k):
    n, dt, kw = 16, 0.01, 0.1
    g = Grid(n)
    x3, y3, z3 = g.coords()
    c0 = np.sin(k[0] * x3 + k[1] * y3 + k[2] * z3)
    K = np.full((n, n, n), kw)
    w2 = sum(kk * kk for kk in k)
    a = 0.5 * dt * kw * w2
    c = c0.copy()
    nsteps = 100
    for s in range(nsteps):
        c, it, rr, ok = solvers.cn_diffusion(g, K, kw, dt, c, 1e-8, 100)
        assert ok and it <= 1                     # exact preconditioner
    factor = ((1 - a) / (1 + a)) ** nsteps
    assert np.max(np.abs(c - factor * c0)) < 1e-13
    # Against the continuous decay exp(-K |w|^2 t): the per-step error is
    # (1-a)/(1+a) - exp(-2a) = -(2/3) a^3 + O(a^4).
    exact = np.exp(-kw * w2 * dt * nsteps)
    assert abs(factor - exact) <= nsteps * (2.0 / 3.0) * a ** 3 * 1.01 + 1e-15
    assert abs(factor - exact) > 0  # not identical: CN is only second order


def test_cn_variable_coefficient_residual_certificate_and_mean():
    n, dt = 16, 0.01
    g = Grid(n)
    wm, gm, csf = synthetic.tissue_maps(n, 2.0, 7)
    K = 0.1 * wm + 0.01 * gm
    c0 = np.abs(synthetic.random_field(n, 8, 1.5))
    rtol = 1e-10
    c1, it, rr, ok = solvers.cn_diffusion(g, K, K.mean(), dt, c0, rtol, 200)
    assert ok and it > 1
    rhs = c0 + 0.5 * dt * solvers.diffusion_op(g, K, c0)
    res = rhs - (c1 - 0.5 * dt * solvers.diffusion_op(g, K, c1))
    assert norm(res) <= 1.05 * rtol * norm(rhs) + 1e-14
    # The zero mode of D vanishes: CN preserves the mean.
    assert abs(c1.mean() - c0.mean()) < 1e-13


def test_pcg_zero_rhs_and_converged_start():
    g = Grid(8)
    K = np.full((8, 8, 8), 0.1)
    z = np.zeros((8, 8, 8))
    x, it, rr, ok = solvers.cn_diffusion(g, K, 0.1, 0.01, z, 1e-8, 10)
    assert it == 0 and ok and not x.any()
    c = np.full((8, 8, 8), 0.7)
    x, it, rr, ok = solvers.cn_diffusion(g, K, 0.1, 0.01, c, 1e-8, 10)
    assert it == 0 and np.allclose(x, c, rtol=0, atol=1e-15)


def test_pcg_solves_a_dense_spd_system():
    rng = np.random.default_rng(0)
    m = rng.standard_normal((30, 30))
    A = m @ m.T + 30 * np.eye(30)
    b = rng.standard_normal(30)
    x, it, rr, ok = solvers.pcg(lambda v: A @ v, lambda r: r / np.diag(A), b, np.zeros(30), 1e-12, 200)
    assert ok
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    # fixed-iteration mode runs exactly that many iterations
    x3, it3, _, _ = solvers.pcg(lambda v: A @ v, lambda r: r, b, np.zeros(30), 1e-12, 200, fixed_iters=3)
    assert it3 == 3
