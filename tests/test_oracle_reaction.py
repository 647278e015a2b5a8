"""Pins for the oracle's pointwise sub-steps (Sec. 2.3, 2.4; Sec. 3 splitting)."""
import json
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import synthetic
from oracle import reaction as rx
from oracle.spectral import Grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _P(**kw):
    return synthetic.params(**kw)


def test_table_setup_values_match_the_paper():
    with open(os.path.join(GOLDEN, "table_setup.json")) as f:
        gold = json.load(f)
    for k, v in gold["values"].items():
        assert synthetic.TABLE_SETUP[k] == v, k


def test_logistic_step_matches_ode_integration():
    # alpha0 = beta0 = gamma = 0 and o > o_inv (kappa = 1): pure logistic growth.
    P = _P(alpha0=0.0, beta0=0.0, gamma=0.0)
    dt, rho = 0.01, 10.0
    p = np.array([1e-4, 0.1, 0.5, 0.9, 1.0, 1.2])
    z = np.zeros_like(p)
    one = np.ones_like(p)
    p1, i1, n1, g1, w1 = rx.species_reaction(P, dt, p, z, z, 0.5 * one, 0.5 * one, one,
                                             rho * one, 0.1 * rho * one, z)
    for k in range(p.size):
        sol = solve_ivp(lambda t, y: rho * y * (1 - y), (0, dt), [p[k]], rtol=1e-13, atol=1e-15)
        assert p1[k] == pytest.approx(sol.y[0, -1], rel=1e-10, abs=1e-14)
    # Over many steps the flow composes to the closed form at t = 50 dt.
    q = p.copy()
    for s in range(50):
        q = rx.species_reaction(P, dt, q, z, z, 0.5 * one, 0.5 * one, one, rho * one, z, z)[0]
    t = 50 * dt
    closed = p * np.exp(rho * t) / (1 - p + p * np.exp(rho * t))
    assert np.allclose(q, closed, rtol=1e-12)


def test_heaviside_is_the_smoothed_step_without_cancellation():
    eps = 0.01
    x = np.linspace(-0.05, 0.05, 101)
    assert np.allclose(rx.heaviside(x, eps), 0.5 * (1 + np.tanh(x / eps)), rtol=0, atol=1e-15)
    # deep in the tail the value keeps full relative accuracy: (1+tanh(y))/2 = e^{2y}/(1+e^{2y})
    y = -15.0
    assert rx.heaviside(y * eps, eps) == pytest.approx(np.exp(2 * y) / (1 + np.exp(2 * y)), rel=1e-14)
    assert rx.heaviside(-10.0, eps) == 0.0 and rx.heaviside(10.0, eps) == 1.0


def test_oxygen_factor_matches_the_piecewise_definition():
    P = _P()
    o_inv, o_mit = P["o_inv"], 0.5 * (P["o_hyp"] + P["o_inv"])
    o = np.linspace(0.0, 1.2, 1201)
    piecewise = np.where(o > o_inv, 1.0, np.where(o >= o_mit, (o - o_mit) / (o_inv - o_mit), 0.0))
    assert np.allclose(rx.oxygen_factor(P, o), piecewise, rtol=0, atol=1e-15)


def _random_state(n, seed):
    rng = np.random.default_rng(seed)
    p = rng.uniform(0, 1, n)
    i = rng.uniform(0, 0.5, n)
    nn = rng.uniform(0, 0.3, n)
    g = rng.uniform(0, 1, n)
    w = rng.uniform(0, 1, n)
    o = rng.uniform(0.3, 1.0, n)
    dD = rng.uniform(-0.01, 0.01, n)
    rho = rng.uniform(0, 10, n)
    return p, i, nn, g, w, o, dD, rho


def test_reaction_conserves_total_cell_density_pointwise():
    # p + i + n + g + w is unchanged by diffusion + reaction (e:pw_mass_consv_gog).
    P = _P()
    p, i, n, g, w, o, dD, rho = _random_state(1000, 1)
    p1, i1, n1, g1, w1 = rx.species_reaction(P, 0.01, p, i, n, g, w, o, rho, 0.1 * rho, dD)
    before = p + (i - dD) + n + g + w
    after = p1 + i1 + n1 + g1 + w1
    assert np.max(np.abs(after - before)) < 1e-14


def test_reaction_structure():
    P = _P()
    dt = 0.01
    p, i, n, g, w, o, dD, rho = _random_state(500, 2)
    p1, i1, n1, g1, w1 = rx.species_reaction(P, dt, p, i, n, g, w, o, rho, 0.1 * rho, dD)
    h = P["gamma"] * 0.5 * (1 + np.tanh((P["o_hyp"] - o) / P["heaviside_eps"]))
    # transfers p <-> i cancel in the tumour total
    dRp = rx.logistic_flow(p, rho * rx.oxygen_factor(P, o), dt) - p
    dRi = rx.logistic_flow(i, 0.1 * rho * rx.oxygen_factor(P, o), dt) - i
    assert np.allclose(p1 + i1, p + i + dRp + dRi - dt * h * (p + i), rtol=0, atol=1e-14)
    # healthy tissue loses mass in proportion to its share
    lg = (g - g1) / g
    lw = (w - w1) / w
    assert np.allclose(lg, lw, rtol=1e-10, atol=1e-12)
    # necrosis only grows
    assert np.all(n1 >= n - 1e-15)


def test_hypoxia_switches():
    P = _P()
    dt = 0.01
    one = np.ones(1)
    z = np.zeros(1)
    # well oxygenated: no p -> i switch, full growth, no death
    p1, i1, n1, g1, w1 = rx.species_reaction(P, dt, 0.5 * one, z, z, 0.3 * one, 0.2 * one, one,
                                             10 * one, one, z)
    assert i1[0] < 1e-12 and n1[0] < 1e-12
    # severely hypoxic (o < o_mit): no growth, death at rate gamma, switch at rate alpha0
    o = 0.1 * one
    p1, i1, n1, g1, w1 = rx.species_reaction(P, dt, 0.5 * one, z, z, 0.3 * one, 0.2 * one, o,
                                             10 * one, one, z)
    assert p1[0] == pytest.approx(0.5 * (1 - dt * (P["alpha0"] + P["gamma"])), rel=1e-12)
    assert i1[0] == pytest.approx(0.5 * dt * P["alpha0"], rel=1e-12)
    assert n1[0] == pytest.approx(dt * P["gamma"] * (0.5 + 0.3 + 0.2), rel=1e-12)


def test_guard_when_no_healthy_tissue():
    P = _P()
    z = np.zeros(2)
    p1, i1, n1, g1, w1 = rx.species_reaction(P, 0.01, np.array([0.5, 0.5]), z, z, z, z,
                                             np.ones(2), 10 * np.ones(2), np.ones(2), z)
    assert np.allclose(g1, w1) and np.all(np.isfinite(g1))


def test_oxygen_step_fixed_point_and_first_order_accuracy():
    P = _P()
    dt = 0.01
    one = np.ones(1)
    # o = o_heal with no proliferative cells is a fixed point
    o1 = rx.oxygen_reaction(P, dt, P["o_heal"] * one, 0 * one, 0.4 * one, 0.6 * one)
    assert o1[0] == P["o_heal"]
    # explicit step vs the exact linear ODE solution: error O(dt^2)
    p, gw, o0 = 0.3, 0.8, 0.7
    a = P["delta_s"] * gw
    b = -P["delta_p"] * p + a * P["o_heal"]
    o_exact = b / a + (o0 - b / a) * np.exp(-a * dt)
    o_num = rx.oxygen_reaction(P, dt, o0 * one, p * one, gw * one, 0 * one)[0]
    second = a * abs(-a * o0 + b)          # |o''| at t = 0, bounds the local error
    assert abs(o_num - o_exact) <= 0.5 * second * dt ** 2 * 1.1
    assert abs(o_num - o_exact) > 0


def test_edema_fixed_point_and_drainage():
    P = _P()
    dt = 0.01
    i = np.array([0.05, 0.3, 0.8])
    l_star = P["delta_e"] * i * (1 - i) / ((i + P["delta_half"]) * P["delta_l"])
    assert np.allclose(rx.edema_reaction(P, dt, l_star, i), l_star, rtol=1e-14)
    l0 = np.array([0.5, 0.5, 0.5])
    l1 = rx.edema_reaction(P, dt, l0, np.zeros(3))
    assert np.allclose(l1, l0 * (1 - dt * P["delta_l"]))


def test_refresh_pure_tissues():
    P = _P()
    one = np.ones(1)
    z = np.zeros(1)
    co = rx.refresh(P, z, z, z, z, one, z)              # pure white matter
    assert co["K"][0] == P["k_w"] and co["rho_p"][0] == P["rho_w"]
    assert co["mu"][0] == pytest.approx(750.0) and co["lam"][0] == pytest.approx(3000.0)
    assert co["eta"][0] == P["eta_healthy"]
    co = rx.refresh(P, one, z, z, z, z, z)              # pure tumour
    assert co["eta"][0] == P["eta_tumor"] and co["K"][0] == 0.0
    assert co["mu"][0] == pytest.approx(2100 / 2.9)


def test_force_matches_analytic_gradient():
    n = 16
    g = Grid(n)
    x3, y3, z3 = g.coords()
    tau = 0.3 * np.sin(x3) + 0.2 * np.cos(2 * y3 + z3)
    grad = [0.3 * np.cos(x3), -0.4 * np.sin(2 * y3 + z3), -0.2 * np.sin(2 * y3 + z3)]
    b = rx.elastic_force(g, 4e4, tau, np.zeros_like(tau))
    for a in range(3):
        assert np.max(np.abs(b[a] - 4e4 * np.tanh(tau) * grad[a])) < 1e-9


# --- the i -> p transfer beta = beta0 H(sigma_b - p - i) o (e:beta), isolated ---
# alpha0 = gamma = 0 removes the p -> i switch and the death term, and rho = 0
# the logistic flows, so the transfer is the only reaction left.  The expected
# values below are worked by hand from e:gog (p_t = ... + beta i, i_t = ... -
# beta i) with one forward Euler step of length dt.

def _beta_only(p, i, o, beta0=0.02, sigma_b=0.9, dt=0.01):
    P = _P(alpha0=0.0, gamma=0.0, beta0=beta0, sigma_b=sigma_b)
    one = np.ones_like(p)
    z = np.zeros_like(p)
    return rx.species_reaction(P, dt, p, i, z, 0.4 * one, 0.3 * one, o, z, z, z)


def test_beta_transfer_below_the_carrying_threshold():
    # p + i = 0.3 < sigma_b = 0.9: the smoothed Heaviside is 1 to 1e-52, so the
    # rate is beta0 o.  beta0 = 0.02, dt = 0.01:
    #   o = 0.8: dt beta i = 0.01 * 0.02 * 0.8 * 0.2 = 3.2e-5
    #   o = 0.4: dt beta i = 0.01 * 0.02 * 0.4 * 0.2 = 1.6e-5
    p = np.array([0.1, 0.1])
    i = np.array([0.2, 0.2])
    o = np.array([0.8, 0.4])
    p1, i1, n1, g1, w1 = _beta_only(p, i, o)
    assert np.allclose(i1, [0.2 - 3.2e-5, 0.2 - 1.6e-5], rtol=0, atol=1e-16)
    assert np.allclose(p1, [0.1 + 3.2e-5, 0.1 + 1.6e-5], rtol=0, atol=1e-16)
    assert np.array_equal(n1, [0.0, 0.0])
    assert np.allclose(g1, 0.4, rtol=0, atol=1e-16) and np.allclose(w1, 0.3, rtol=0, atol=1e-16)


def test_beta_transfer_switches_off_above_the_carrying_threshold():
    # p + i = 1.2 > sigma_b: H(-0.3 / 0.01) = 1 / (1 + e^60) ~ 8.8e-27, so the
    # invasive cells stay put (to ~1e-30 absolute).
    p = np.array([0.7, 0.95])
    i = np.array([0.5, 0.25])
    o = np.array([0.9, 0.9])
    p1, i1, _, _, _ = _beta_only(p, i, o)
    assert np.allclose(i1, i, rtol=0, atol=1e-25)
    assert np.allclose(p1, p, rtol=0, atol=1e-25)


def test_beta_transfer_at_the_threshold_is_half_rate():
    # p + i = sigma_b exactly: H(0) = 1/2, so dt beta i = 0.01 * 0.02 * 0.5 * 1.0 * 0.4 = 4e-5.
    p = np.array([0.5])
    i = np.array([0.4])
    o = np.array([1.0])
    p1, i1, _, _, _ = _beta_only(p, i, o)
    assert i1[0] == pytest.approx(0.4 - 4e-5, rel=0, abs=1e-16)
    assert p1[0] == pytest.approx(0.5 + 4e-5, rel=0, abs=1e-16)


def test_beta_transfer_with_growth_on_is_additive_to_the_logistic_flow():
    # With growth on and o above o_inv (kappa = 1), the invasive cells follow the
    # logistic flow of rate rho_i and lose dt beta0 o i on top (frozen state):
    #   i' = Lambda(i, rho_i, dt) - dt beta0 o i,  Lambda(y, r, t) = y e^{rt} / (1 + y (e^{rt} - 1)).
    P = _P(alpha0=0.0, gamma=0.0, beta0=0.05)
    dt, rho_i = 0.01, 1.0
    i = np.array([0.3])
    o = np.array([0.95])
    one = np.ones(1)
    z = np.zeros(1)
    _, i1, _, _, _ = rx.species_reaction(P, dt, 0.2 * one, i, z, 0.5 * one, 0.5 * one, o, z, rho_i * one, z)
    e = np.exp(0.01)
    lam = 0.3 * e / (1.0 + 0.3 * (e - 1.0))
    assert i1[0] == pytest.approx(lam - 0.01 * 0.05 * 0.95 * 0.3, rel=1e-14)
