"""Pins for the fictitious-domain background material (Sec. 3; Table t:setup:
eta_bg, E_bg, nu_bg): Lame and screening contributions, the displacement
penalty outside the brain, and the adjoint's Lame-scale gradient."""
import numpy as np

import synthetic
from oracle import adjoint as adj
from oracle import model
from oracle import reaction as rx
from oracle import solvers
from test_oracle_adjoint import TIGHT


def test_background_mixture_values():
    P = synthetic.params()
    z = np.zeros((2, 2, 2))
    co = rx.refresh(P, z, z, z, z, z, z, bg=np.ones((2, 2, 2)))
    # E = 15000 Pa, nu = 0.48: mu = E / 2.96, lambda = 0.48 E / (0.04 * 1.48)
    assert np.allclose(co["mu"], 15000.0 / 2.96, rtol=1e-14)
    assert np.allclose(co["lam"], 7200.0 / 0.0592, rtol=1e-14)
    assert np.allclose(co["eta"], 1.0e6, rtol=0)
    assert np.all(co["K"] == 0.0) and np.all(co["rho_p"] == 0.0)
    # without a background the refresh is unchanged
    g = np.full((2, 2, 2), 0.5)
    a, b = rx.refresh(P, z, z, z, g, g, z), rx.refresh(P, z, z, z, g, g, z, bg=np.zeros((2, 2, 2)))
    for k in ("mu", "lam", "eta", "K"):
        assert np.array_equal(a[k], b[k])


def test_background_penalises_displacement_outside_the_brain():
    P = synthetic.params()
    inp = synthetic.workload_inputs("seeds3_n128", n=32, masked=True)
    st = model.init_state(P, 32, inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"],
                          inp["weights"], inp["bg"])
    co = st.coef
    force = rx.elastic_force(st.grid, P["zeta"], st.f["p"], st.f["n"])
    u, it, rr, ok = solvers.solve_elasticity(st.grid, co["mu"], co["lam"], co["eta"],
                                             (co["mubar"], co["lambar"], co["etabar"]), force,
                                             np.zeros_like(force), 1e-8, 2000)
    assert ok
    umag = np.sqrt((u ** 2).sum(axis=0))
    outside = inp["bg"] > 0.999
    inside = inp["bg"] < 0.001
    assert outside.any() and inside.any()
    assert umag[outside].max() < 1e-2 * umag[inside].max()


def test_lame_scale_gradient_with_background():
    steps = 2
    P = synthetic.params(delta_p=60.0)
    inp = synthetic.workload_inputs("seeds3_n128", n=16, masked=True)
    Pt = dict(P, rho_w=P["rho_w"] * 1.1, rho_g=P["rho_g"] * 1.1)
    st, _ = model.run(Pt, inp, steps, TIGHT)
    target = st.f["p"] + st.f["i"] + st.f["n"]
    L, grad, gw, lam = adj.gradient(P, inp, steps, target, TIGHT)

    def loss(Pv):
        s, _ = model.run(Pv, inp, steps, TIGHT)
        return adj.loss(Pv, s.grid, s, target)

    e = 1e-5
    fd = (loss(dict(P, lame_scale=1.0 + e)) - loss(dict(P, lame_scale=1.0 - e))) / (2 * e)
    assert abs(fd - grad["lame_scale"]) <= 1e-5 * abs(fd) + 1e-12 * abs(L), (fd, grad["lame_scale"])
    # the background changes the answer (the pin is not vacuous)
    L0, grad0, _, _ = adj.gradient(P, dict(inp, bg=None), steps, target, TIGHT)
    assert abs(grad0["lame_scale"] - grad["lame_scale"]) > 1e-6 * abs(grad["lame_scale"])
