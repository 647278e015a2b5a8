"""Pins for the oracle's initial condition and whole split step."""
import numpy as np
import pytest

import synthetic
from oracle import model, reaction as rx, solvers, transport
from oracle.spectral import Grid


def test_gaussian_basis_peak_symmetry_and_periodic_wrap():
    g = Grid(16)
    c = np.array([[g.h * 3, g.h * 5, g.h * 7]])
    p = model.gaussian_basis(g, c, [0.4], [0.8])
    assert p[7, 5, 3] == 0.8
    # symmetric about the centre
    assert p[7, 5, 3 + 2] == pytest.approx(p[7, 5, 3 - 2], rel=1e-14)
    # a centre at the domain edge wraps to both sides
    q = model.gaussian_basis(g, np.array([[0.0, 0.0, 0.0]]), [0.3], [1.0])
    assert q[0, 0, 1] == pytest.approx(q[0, 0, 15], rel=1e-14)
    assert q[0, 0, 1] == pytest.approx(np.exp(-g.h ** 2 / (2 * 0.09)), rel=1e-14)


def test_diffusion_plus_reaction_conserve_total_cell_density_pointwise():
    P = synthetic.params()
    inp = synthetic.workload_inputs("seed1_n32", n=16)
    st = model.init_state(P, 16, inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"], inp["weights"])
    rng = np.random.default_rng(3)
    st.f["i"] = 0.2 * rng.uniform(size=st.f["i"].shape)
    st.f["o"] = rng.uniform(0.3, 1.0, size=st.f["o"].shape)
    before = sum(st.f[k] for k in "pingw")
    model.step(st, dict(advection=False, elasticity=False))
    after = sum(st.f[k] for k in "pingw")
    assert np.max(np.abs(after - before)) < 1e-13


def test_global_mass_is_constant_without_transport():
    P = synthetic.params()
    inp = synthetic.workload_inputs("seed1_n32", n=16)
    st = model.init_state(P, 16, inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"], inp["weights"])
    m0 = sum(st.f[k].sum() for k in "pingw")
    for s in range(3):
        model.step(st, dict(advection=False))
    m1 = sum(st.f[k].sum() for k in "pingw")
    assert abs(m1 - m0) < 1e-12 * m0


def test_step_order_and_elasticity_certificate():
    # One full step on a tiny grid: the displacement solves the elasticity
    # system built from the refreshed coefficients and the new species.
    P = synthetic.params()
    inp = synthetic.workload_inputs("seed1_n32", n=16)
    st = model.init_state(P, 16, inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"], inp["weights"])
    cfg = dict(rtol_elast=1e-11)
    s1 = model.step(st, cfg)
    co = rx.refresh(P, *(st.f[k] for k in ("p", "i", "n", "g", "w", "f")))
    for k in ("K", "mu", "lam", "eta"):
        assert np.array_equal(co[k], st.coef[k])
    b = rx.elastic_force(st.grid, P["zeta"], st.f["p"], st.f["n"])
    res = -b - solvers.elasticity_op(st.grid, co["mu"], co["lam"], co["eta"], st.u)
    assert np.linalg.norm(res) <= 1.05e-11 * np.linalg.norm(b)
    assert s1["it_elast"] > 0 and not st.u_prev.any()
    # second step advects with v = u^1 / dt
    s2 = model.step(st, cfg)
    assert s2["max_cfl"] > 0


def test_run_is_deterministic():
    P = synthetic.params()
    inp = synthetic.workload_inputs("seed1_n32", n=16)
    a, sa = model.run(P, inp, 2)
    b, sb = model.run(P, inp, 2)
    for k in model.FIELDS:
        assert np.array_equal(a.f[k], b.f[k])
    assert [s["it_elast"] for s in sa] == [s["it_elast"] for s in sb]
