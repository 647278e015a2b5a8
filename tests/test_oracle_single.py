"""Pins for the oracle's single-species model (Sec. 2.2, e:rd; Sec. 3)."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import synthetic
from oracle import model, model_single
from oracle import reaction as rx


def test_logistic_growth_matches_ode_integration():
    rng = np.random.default_rng(5)
    c = rng.uniform(0.0, 1.0, 50)
    rho = rng.uniform(0.5, 12.0, 50)
    g = rng.uniform(0.1, 0.6, 50)
    w = rng.uniform(0.1, 0.6, 50)
    dt = 0.01
    c1, g1, w1 = rx.single_species_reaction(synthetic.params(), dt, c, c, g, w, rho)
    for k in range(50):
        sol = solve_ivp(lambda t, y: rho[k] * y * (1 - y), (0, dt), [c[k]], rtol=1e-13, atol=1e-15)
        assert abs(c1[k] - sol.y[0, -1]) < 1e-12


def test_conservation_and_proportional_sink():
    rng = np.random.default_rng(6)
    c_dag = rng.uniform(0, 0.8, 200)
    c_dd = c_dag + rng.normal(0, 0.01, 200)          # a diffusion increment
    g = rng.uniform(0.05, 0.6, 200)
    w = rng.uniform(0.05, 0.6, 200)
    rho = rng.uniform(1, 10, 200)
    c1, g1, w1 = rx.single_species_reaction(synthetic.params(), 0.01, c_dag, c_dd, g, w, rho)
    assert np.abs((c1 + g1 + w1) - (c_dag + g + w)).max() < 1e-15
    assert np.allclose((g - g1) * w, (w - w1) * g, rtol=0, atol=1e-16)


def test_guard_without_healthy_tissue():
    c1, g1, w1 = rx.single_species_reaction(synthetic.params(), 0.01, np.array([0.5]), np.array([0.4]),
                                            np.array([0.0]), np.array([0.0]), np.array([5.0]))
    assert g1[0] == w1[0] and abs(c1[0] + g1[0] + w1[0] - 0.5) < 1e-15


def test_inactive_step_is_the_identity():
    P = synthetic.params(rho_w=0.0, rho_g=0.0, k_w=0.0, k_g=0.0)
    inp = synthetic.workload_inputs("seed1_n32", n=16)
    st = model.init_state(P, 16, inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"], inp["weights"])
    before = {k: v.copy() for k, v in st.f.items()}
    model_single.step(st, dict(advection=False, elasticity=False))
    for k in before:
        assert np.array_equal(st.f[k], before[k]), k


def test_total_density_is_conserved_without_transport():
    P = synthetic.params()
    inp = synthetic.workload_inputs("seed1_n32", n=16)
    st = model.init_state(P, 16, inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"], inp["weights"])
    m0 = (st.f["p"] + st.f["g"] + st.f["w"]).sum()
    for _ in range(3):
        model_single.step(st, dict(advection=False))
    assert abs((st.f["p"] + st.f["g"] + st.f["w"]).sum() - m0) < 1e-12 * m0
    assert np.abs(st.u).max() > 0.0


def test_equals_the_multispecies_model_reduced_to_one_invasive_species():
    # With alpha0 = beta0 = gamma = 0, rho_i = rho_p and o = o_heal, the
    # multispecies model carrying its tumour in the invasive species i (which
    # diffuses) is the single-species model without mass effect.
    P = synthetic.params(alpha0=0.0, beta0=0.0, gamma=0.0, rho_inv_frac=1.0)
    inp = synthetic.workload_inputs("seed1_n32", n=16)
    multi = model.init_state(P, 16, inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"], inp["weights"])
    single = multi.copy()
    multi.f["i"], multi.f["p"] = multi.f["p"], np.zeros_like(multi.f["p"])
    multi.coef = rx.refresh(P, *(multi.f[k] for k in ("p", "i", "n", "g", "w", "f")))
    cfg = dict(elasticity=False, advection=False, edema=False)
    for _ in range(3):
        model.step(multi, cfg)
        model_single.step(single, cfg)
    assert np.abs(multi.f["i"] - single.f["p"]).max() < 1e-14
    for k in ("g", "w", "f"):
        assert np.abs(multi.f[k] - single.f[k]).max() < 1e-14, k
