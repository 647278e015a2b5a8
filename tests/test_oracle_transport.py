"""Pins for the oracle's semi-Lagrangian transport (Sec. 3)."""
import numpy as np
import pytest

import synthetic
from oracle import transport
from oracle.spectral import Grid


def _const_velocity(n, vec):
    return np.stack([np.full((n, n, n), c) for c in vec])


def test_zero_velocity_is_the_identity():
    n = 16
    g = Grid(n)
    fields = {k: synthetic.random_field(n, s) for s, k in enumerate("pingwf")}
    out = transport.advect(g, fields, np.zeros((3, n, n, n)), 0.01)
    for k in "pingwf":
        assert np.array_equal(out[k], fields[k])


@pytest.mark.parametrize("shift", [(1, 0, 0), (2, -3, 1), (-5, 4, 7)])
def test_integer_cell_shift_is_exact(shift):
    n, dt = 16, 0.01
    g = Grid(n)
    v = _const_velocity(n, [s * g.h / dt for s in shift])
    q = synthetic.random_field(n, 3)
    out = transport.advect(g, {k: q for k in "pingwf"}, v, dt)
    ref = np.roll(q, shift=(shift[2], shift[1], shift[0]), axis=(0, 1, 2))
    for k in "pingwf":
        assert np.max(np.abs(out[k] - ref)) < 1e-13


def test_rk2_is_exact_for_constant_velocity():
    n, dt = 16, 0.01
    g = Grid(n)
    vec = (0.37, -1.9, 2.6)
    X = transport.departure_points(g, _const_velocity(n, vec), dt)
    base = transport.grid_indices(n)
    for a in range(3):
        assert np.max(np.abs(X[a] - (base[a] - dt * vec[a] / g.h))) < 1e-12


def test_fractional_shift_error_bound_and_fourth_order():
    # Cubic Lagrange on nodes -1..2: |err| <= max|f''''| h^4 max|prod(t - t_j)| / 4!
    # with max over t in [0, 1] of |(t+1) t (t-1) (t-2)| = 9/16.
    errs = []
    for n in (16, 32, 64):
        g = Grid(n)
        dt = 0.01
        frac = 0.37
        v = _const_velocity(n, [frac * g.h / dt, 0.0, 0.0])
        x3, y3, z3 = g.coords()
        q = np.sin(x3)
        out = transport.advect(g, {k: q for k in "pingwf"}, v, dt)["f"]
        exact = np.sin(x3 - frac * g.h)
        err = np.max(np.abs(out - exact))
        bound = g.h ** 4 * (9.0 / 16.0) / 24.0
        assert err <= bound
        errs.append(err)
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.8)


def test_cubic_polynomials_are_reproduced_on_interior_stencils():
    n = 16
    q = np.zeros((n, n, n))
    jz, jy, jx = np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij")
    poly = lambda x, y, z: 0.3 * x ** 3 - x * y * z + 2 * y ** 2 - z ** 3 / 7 + 1.5
    q[...] = poly(jx, jy, jz)
    rng = np.random.default_rng(5)
    pts = rng.uniform(2.0, n - 4.0, size=(3, 200))      # stencils stay inside [1, n-2]
    out = transport.interp(q, pts[0], pts[1], pts[2])
    assert np.max(np.abs(out - poly(pts[0], pts[1], pts[2]))) < 1e-10


def test_interp_hits_nodes_exactly_and_wraps():
    n = 8
    q = synthetic.random_field(n, 6)
    idx = np.array([0.0, 3.0, 7.0, 8.0, -1.0, 15.0])
    out = transport.interp(q, idx, idx, idx)
    j = np.mod(idx.astype(int), n)
    assert np.array_equal(out, q[j, j, j])


def test_advection_is_linear_and_conservative_source_vanishes_for_solenoidal_flow():
    n, dt = 16, 0.02
    g = Grid(n)
    v = synthetic.random_field(n, 11, 2.0, ncomp=3) * 3.0
    a = synthetic.random_field(n, 12, 1.0)
    b = synthetic.random_field(n, 13, 1.0)
    oa = transport.advect(g, {k: a for k in "pingwf"}, v, dt)
    ob = transport.advect(g, {k: b for k in "pingwf"}, v, dt)
    oab = transport.advect(g, {k: a + 2 * b for k in "pingwf"}, v, dt)
    assert np.max(np.abs(oab["p"] - oa["p"] - 2 * ob["p"])) < 1e-12
    # Divergence-free velocity (a curl): conservative and plain transport agree
    # up to the (round-off) spectral divergence.
    x3, y3, z3 = g.coords()
    vs = np.stack([np.sin(y3), np.cos(z3), np.sin(x3)]) * 5.0
    o = transport.advect(g, {k: a for k in "pingwf"}, vs, dt)
    assert np.max(np.abs(o["p"] - o["f"])) < 1e-13


def test_sampled_nodes_equal_the_whole_grid_step():
    """advect(..., nodes=...) evaluates the same step at a subset of nodes."""
    n, dt = 16, 0.01
    g = Grid(n)
    rng = np.random.default_rng(3)
    v = [0.3 * g.ifft(g.fft(rng.standard_normal((n, n, n)))) / dt * g.h for _ in range(3)]
    fields = {k: rng.random((n, n, n)) for k in ("p", "i", "n", "g", "w", "f")}
    full = transport.advect(g, fields, v, dt)
    idx = rng.integers(0, n, size=(3, 50))
    nodes = tuple(a.astype(np.float64) for a in idx)
    part = transport.advect(g, fields, v, dt, nodes=nodes)
    for k in full:
        assert np.array_equal(part[k], full[k][idx[2], idx[1], idx[0]]), k


# --- variable velocity: the 1-D compressible flow v = c sin(x_a) along one axis ---
# Its characteristics are exact: d/dt tan(x/2) = c tan(x/2), so the point that
# arrives at x after a time dt left from X with tan(X/2) = tan(x/2) e^{-c dt}.
# With q0 = 1 the conservative transport q_t + (q v)_x = 0 has the exact density
# q(x, t) = dX/dx = e^{-ct} / (cos^2(x/2) + sin^2(x/2) e^{-2ct}).
# One RK2 characteristic step and one Heun step of the source are both exact to
# O(dt^3) locally (second order globally); a first-order slip in either (e.g.
# X = x - dt v(X*), or the corrector's source taken at X instead of x) leaves an
# O(dt^2) local error, which the convergence rates below reject.

def _sine_flow(n, c, axis):
    g = Grid(n)
    coords = g.coords()           # (x, y, z)
    v = np.zeros((3, n, n, n))
    v[axis] = c * np.sin(coords[axis])
    return g, v, coords[axis]


def _exact_departure(x, c, t):
    # X in [0, 2 pi) with tan(X/2) = tan(x/2) e^{-ct}; x/2 in [0, pi) keeps the branch
    return 2.0 * np.arctan2(np.sin(0.5 * x) * np.exp(-c * t), np.cos(0.5 * x))


def _exact_density(x, c, t):
    return np.exp(-c * t) / (np.cos(0.5 * x) ** 2 + np.sin(0.5 * x) ** 2 * np.exp(-2.0 * c * t))


def _pdiff(a, b):
    d = a - b
    return d - 2.0 * np.pi * np.round(d / (2.0 * np.pi))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_rk2_departure_points_of_a_compressible_flow_are_third_order_locally(axis):
    n, c = 32, 1.5
    g, v, xa = _sine_flow(n, c, axis)
    errs = []
    for dt in (0.2, 0.1, 0.05):
        X = transport.departure_points(g, v, dt)
        err = np.max(np.abs(_pdiff(X[axis] * g.h, _exact_departure(xa, c, dt))))
        # the other two coordinates do not move
        for b in range(3):
            if b != axis:
                base = transport.grid_indices(n)[b]
                assert np.array_equal(X[b], base)
        errs.append(err)
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.7), (errs, rates)
    assert errs[-1] < 1e-4


def test_rk2_departure_points_converge_at_second_order_over_a_fixed_time():
    # Compose k characteristic steps of dt = T / k backwards from the arrival
    # points (the velocity is steady): global error O(dt^2).
    n, c, T = 32, 1.5, 0.4
    g, v, x = _sine_flow(n, c, 0)
    jx = np.arange(n, dtype=np.float64)
    nodes = (jx, np.zeros(n), np.zeros(n))
    errs = []
    for k in (2, 4, 8):
        dt = T / k
        # track the foot of each arrival node by re-evaluating the same
        # two-stage scheme at the current foot (interpolated velocity)
        pos = jx.copy()
        for _ in range(k):
            s = dt / g.h
            v0 = transport.interp(v[0], pos, np.zeros(n), np.zeros(n))
            xs = pos - s * v0
            vs = transport.interp(v[0], xs, np.zeros(n), np.zeros(n))
            pos = pos - 0.5 * s * (v0 + vs)
        errs.append(np.max(np.abs(_pdiff(pos * g.h, _exact_departure(jx * g.h, c, T)))))
        if k == 2:
            # the first of the k steps is exactly departure_points at the nodes
            X = transport.departure_points(g, v, dt, nodes=nodes)
            s = dt / g.h
            v0 = c * np.sin(jx * g.h)
            vs = transport.interp(v[0], jx - s * v0, np.zeros(n), np.zeros(n))
            assert np.allclose(X[0], jx - 0.5 * s * (v0 + vs), rtol=0, atol=1e-12)
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), (errs, rates)


@pytest.mark.parametrize("axis", [0, 2])
def test_heun_source_of_a_compressible_flow_is_third_order_locally(axis):
    n, c = 32, 1.5
    g, v, xa = _sine_flow(n, c, axis)
    one = np.ones((n, n, n))
    errs = []
    for dt in (0.2, 0.1, 0.05):
        out = transport.advect(g, {k: one for k in "pingwf"}, v, dt)
        exact = _exact_density(xa, c, dt)
        err = np.max(np.abs(out["p"] - exact))
        errs.append(err)
        # plain transport of a constant stays constant (cubic Lagrange reproduces it)
        assert np.allclose(out["f"], 1.0, rtol=0, atol=1e-13)
        # all conservative species follow the same update
        for k in "ingw":
            assert np.array_equal(out[k], out["p"])
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 2.7), (errs, rates)
    assert errs[-1] < 1e-4


def test_conservative_transport_of_a_constant_density_over_a_fixed_time_is_second_order():
    # k full SL steps (departure points, interpolation of q and div v, Heun
    # source) to T: the density approaches e^{-cT}/(cos^2 + sin^2 e^{-2cT}) at O(dt^2).
    n, c, T = 32, 1.5, 0.4
    g, v, x = _sine_flow(n, c, 0)
    errs = []
    for k in (2, 4, 8):
        q = np.ones((n, n, n))
        for _ in range(k):
            q = transport.advect(g, {kk: q for kk in "pingwf"}, v, T / k)["p"]
        errs.append(np.max(np.abs(q - _exact_density(x, c, T))))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), (errs, rates)
