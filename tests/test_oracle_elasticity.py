"""Pins for the oracle's screened elasticity operator and solve
(Eqs. e:hook, e:variable_elasticity, e:screening, e:lame; Sec. 3).
"""
import numpy as np
import pytest
import sympy as sp

import synthetic
from oracle import reaction, solvers
from oracle.spectral import Grid, dot, norm

X, Y, Z = sp.symbols("x y z", real=True)
S = (X, Y, Z)


def _eval(expr, grid):
    f = sp.lambdify((X, Y, Z), expr, "numpy")
    x3, y3, z3 = grid.coords()
    return np.broadcast_to(np.asarray(f(x3, y3, z3), dtype=float), x3.shape).copy()


def test_operator_matches_analytic_screened_elasticity():
    n = 16
    g = Grid(n)
    mu = 1 + sp.Rational(1, 5) * sp.cos(X + Y)
    lam = 2 + sp.Rational(3, 10) * sp.sin(Z)
    eta = sp.Rational(1, 2) + sp.Rational(1, 10) * sp.cos(Y)
    u = [sp.sin(Y), sp.cos(X + Z), sp.sin(2 * X) + sp.cos(Y - Z)]
    # L u = div(mu (grad u + grad u^T)) + grad(lambda div u), written by components
    divu = sum(sp.diff(u[a], S[a]) for a in range(3))
    ref = []
    for a in range(3):
        Lu = sum(sp.diff(mu * (sp.diff(u[a], S[b]) + sp.diff(u[b], S[a])), S[b]) for b in range(3))
        Lu += sp.diff(lam * divu, S[a])
        ref.append(_eval(eta * u[a] - Lu, g))
    U = np.stack([_eval(c, g) for c in u])
    out = solvers.elasticity_op(g, _eval(mu, g), _eval(lam, g), _eval(eta, g), U)
    for a in range(3):
        assert np.max(np.abs(out[a] - ref[a])) < 1e-11


def test_operator_is_symmetric_positive_definite():
    n = 12
    g = Grid(n)
    mu = 500 + 200 * np.abs(synthetic.random_field(n, 1, 2.0))
    lam = 2000 + 500 * np.abs(synthetic.random_field(n, 2, 2.0))
    eta = 1e3 * np.abs(synthetic.random_field(n, 3, 2.0))
    a = synthetic.random_field(n, 4, ncomp=3)
    b = synthetic.random_field(n, 5, ncomp=3)
    Aa = solvers.elasticity_op(g, mu, lam, eta, a)
    Ab = solvers.elasticity_op(g, mu, lam, eta, b)
    assert abs(dot(Aa, b) - dot(a, Ab)) < 1e-10 * abs(dot(Aa, b))
    assert dot(Aa, a) > 0


def test_rigid_translation_has_no_elastic_response():
    n = 12
    g = Grid(n)
    mu = 500 + 100 * synthetic.random_field(n, 1, 2.0)
    lam = 2000 + 300 * synthetic.random_field(n, 2, 2.0)
    U = np.stack([np.full((n, n, n), v) for v in (0.3, -1.2, 2.0)])
    out = solvers.elasticity_op(g, mu, lam, np.zeros((n, n, n)), U)
    assert np.max(np.abs(out)) < 1e-9


def test_nyquist_corner_modes_need_screening():
    """The spectral derivative drops the Nyquist mode, so on a field such as
    (-1)^(jx + jz) every derivative vanishes: without screening the operator
    maps it to zero (as it does a translation), and with screening it is eta u.
    The force has content on such modes, so the solve requires eta > 0
    somewhere and refuses eta = 0 everywhere."""
    n = 12
    g = Grid(n)
    mu = 500 + 100 * synthetic.random_field(n, 1, 2.0)
    lam = 2000 + 300 * synthetic.random_field(n, 2, 2.0)
    j = np.arange(n)
    corner = ((-1.0) ** (j[:, None, None] + j[None, None, :])) * np.ones((n, n, n))   # [z][y][x]: (-1)^(jz + jx)
    U = np.stack([corner, 0.5 * corner, -corner])
    zero = np.zeros((n, n, n))
    assert np.max(np.abs(solvers.elasticity_op(g, mu, lam, zero, U))) < 1e-9
    eta = np.full((n, n, n), 3.0)
    assert np.max(np.abs(solvers.elasticity_op(g, mu, lam, eta, U) - 3.0 * U)) < 1e-9
    with pytest.raises(ValueError):
        solvers.solve_elasticity(g, mu, lam, zero, (mu.mean(), lam.mean(), 0.0), U, zero[None] * U, 1e-8, 50)


@pytest.mark.parametrize("k", [(1, 0, 0), (1, 2, -1), (0, 3, 2)])
def test_constant_coefficient_single_mode_closed_form(k):
    n = 16
    g = Grid(n)
    mu, lam, eta = 750.0, 3000.0, 1e4
    x3, y3, z3 = g.coords()
    phase = k[0] * x3 + k[1] * y3 + k[2] * z3
    b0 = np.array([0.7, -1.1, 0.4])
    force = np.stack([b0[a] * np.cos(phase) for a in range(3)])
    w = np.array(k, float)
    # Fourier symbol of (eta - L) for constant coefficients, solved as a 3x3 system.
    M = (eta + mu * w @ w) * np.eye(3) + (lam + mu) * np.outer(w, w)
    amp = np.linalg.solve(M, -b0)
    full = lambda c: np.full((n, n, n), c)
    u, it, rr, ok = solvers.solve_elasticity(g, full(mu), full(lam), full(eta), (mu, lam, eta),
                                             force, np.zeros_like(force), 1e-10, 50)
    assert ok and it == 1                              # exact preconditioner
    for a in range(3):
        assert np.max(np.abs(u[a] - amp[a] * np.cos(phase))) < 1e-13 * max(1.0, np.abs(amp).max())


def test_precond_inverts_constant_operator_on_random_field():
    n = 12
    g = Grid(n)
    mu, lam, eta = 300.0, 900.0, 50.0
    full = lambda c: np.full((n, n, n), c)
    r = synthetic.random_field(n, 9, ncomp=3)
    z = solvers.elasticity_precond(g, mu, lam, eta, r)
    back = solvers.elasticity_op(g, full(mu), full(lam), full(eta), z)
    assert np.max(np.abs(back - r)) < 1e-9 * np.abs(r).max()


def test_variable_coefficient_solve_certificate_and_outward_push():
    n = 16
    g = Grid(n)
    P = synthetic.params()
    wm, gm, csf = synthetic.tissue_maps(n, 2.0, 3)
    x3, y3, z3 = g.coords()
    c = np.pi
    r2 = (x3 - c) ** 2 + (y3 - c) ** 2 + (z3 - c) ** 2
    p = 0.5 * np.exp(-r2 / (2 * 0.6 ** 2))
    zero = np.zeros_like(p)
    co = reaction.refresh(P, p, zero, zero, gm, wm, csf)
    force = reaction.elastic_force(g, P["zeta"], p, zero)
    rtol = 1e-10
    u, it, rr, ok = solvers.solve_elasticity(g, co["mu"], co["lam"], co["eta"],
                                             (co["mubar"], co["lambar"], co["etabar"]),
                                             force, np.zeros_like(force), rtol, 500)
    assert ok and it > 1
    res = -force - solvers.elasticity_op(g, co["mu"], co["lam"], co["eta"], u)
    assert norm(res) <= 1.05 * rtol * norm(force)
    # The tumour pushes tissue outward near its rim.
    radial = (u[0] * (x3 - c) + u[1] * (y3 - c) + u[2] * (z3 - c))
    rim = (r2 > 0.4 ** 2) & (r2 < 0.9 ** 2)
    assert np.mean(radial[rim] > 0) > 0.95


def test_mirror_symmetric_tissue_gives_mirror_symmetric_displacement():
    n = 16
    g = Grid(n)
    P = synthetic.params()
    wm, gm, csf = synthetic.tissue_maps(n, 2.0, 4)
    # Mirror the tissue in x about x = pi (index j -> -j mod n).
    mir = lambda a: np.roll(a[:, :, ::-1], 1, axis=2)
    wm, gm, csf = 0.5 * (wm + mir(wm)), 0.5 * (gm + mir(gm)), 0.5 * (csf + mir(csf))
    x3, y3, z3 = g.coords()
    r2 = (x3 - np.pi) ** 2 + (y3 - 2.0) ** 2 + (z3 - 4.0) ** 2
    p = 0.5 * np.exp(-r2 / (2 * 0.5 ** 2))
    zero = np.zeros_like(p)
    co = reaction.refresh(P, p, zero, zero, gm, wm, csf)
    force = reaction.elastic_force(g, P["zeta"], p, zero)
    u, it, rr, ok = solvers.solve_elasticity(g, co["mu"], co["lam"], co["eta"],
                                             (co["mubar"], co["lambar"], co["etabar"]),
                                             force, np.zeros_like(force), 1e-11, 500)
    assert ok
    scale = np.abs(u).max()
    assert np.max(np.abs(mir(u[0]) + u[0])) < 1e-8 * scale     # u_x is odd
    assert np.max(np.abs(mir(u[1]) - u[1])) < 1e-8 * scale     # u_y, u_z are even
    assert np.max(np.abs(mir(u[2]) - u[2])) < 1e-8 * scale


def test_lame_species_values():
    # Young's modulus / Poisson ratio pairs of the synthetic workload: white and
    # gray matter (2100 Pa, 0.4), CSF (100 Pa, 0.1), tumour (2100 Pa, 0.45).
    mu, lam = reaction.lame_species(2100.0, 0.4)
    assert mu == pytest.approx(750.0, rel=1e-14) and lam == pytest.approx(3000.0, rel=1e-14)
    mu, lam = reaction.lame_species(100.0, 0.1)
    assert mu == pytest.approx(45.4545454545, rel=1e-10) and lam == pytest.approx(11.3636363636, rel=1e-10)
    mu, lam = reaction.lame_species(2100.0, 0.45)
    assert mu == pytest.approx(724.137931034, rel=1e-10) and lam == pytest.approx(6517.24137931, rel=1e-10)
