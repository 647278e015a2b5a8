"""Pins for the oracle's discrete adjoint.

Linear pieces are pinned by dot-product identities <J x, y> = <x, J^T y>;
nonlinear pieces by central finite differences of the oracle's own forward
functions; the whole multi-step gradient by central finite differences of
the loss (solves at rtol 1e-13 so that the difference quotient is not
swamped by solver noise).
"""
import numpy as np
import pytest

import synthetic
from oracle import adjoint as adj
from oracle import model, reaction as rx, solvers, transport
from oracle.spectral import Grid, dot

TIGHT = dict(rtol_diff=1e-13, rtol_elast=1e-13, rtol_adj=1e-13, max_it=2000)


def test_interp_transpose_dot_identity():
    n = 12
    rng = np.random.default_rng(0)
    q = rng.standard_normal((n, n, n))
    pts = rng.uniform(-n, 2 * n, size=(3, 500))
    y = rng.standard_normal(500)
    lhs = dot(transport.interp(q, *pts), y)
    rhs = dot(q, adj.interp_transpose(y, *pts, n))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_interp_gradient_matches_finite_differences():
    n = 12
    rng = np.random.default_rng(1)
    q = synthetic.random_field(n, 2, 1.0)
    pts = rng.uniform(0.1, n - 0.1, size=(3, 300))
    g = adj.interp_gradient(q, *pts)
    e = 1e-6
    for a in range(3):
        d = np.zeros((3, 1))
        d[a] = e
        fd = (transport.interp(q, *(pts + d)) - transport.interp(q, *(pts - d))) / (2 * e)
        # avoid points within e of a cell face, where the cubic pieces join
        frac = pts[a] - np.floor(pts[a])
        ok = (frac > 1e-4) & (frac < 1 - 1e-4)
        assert np.max(np.abs(fd[ok] - g[a][ok])) < 1e-6 * np.abs(q).max()


def test_lagrange_weight_derivatives():
    t = np.linspace(0.01, 0.99, 50)
    e = 1e-6
    w_p = transport.lagrange_weights(t + e)
    w_m = transport.lagrange_weights(t - e)
    d = adj.lagrange_dweights(t)
    for k in range(4):
        assert np.allclose((w_p[k] - w_m[k]) / (2 * e), d[k], atol=1e-8)


def _smooth_state(n, seed):
    return {k: np.abs(synthetic.random_field(n, seed + j, 1.5)) * 0.3 for j, k in enumerate("pingwf")}


def test_transport_adjoint_dot_product_with_fd_jvp():
    n, dt = 12, 0.01
    g = Grid(n)
    F0 = _smooth_state(n, 10)
    v = synthetic.random_field(n, 20, 2.0, ncomp=3) * 20.0      # about 0.2 cells per step
    dF = {k: synthetic.random_field(n, 30 + j, 1.0) for j, k in enumerate("pingwf")}
    dv = synthetic.random_field(n, 40, 2.0, ncomp=3) * 20.0
    ybar = {k: synthetic.random_field(n, 50 + j, 1.0) for j, k in enumerate("pingwf")}
    e = 1e-6
    plus = transport.advect(g, {k: F0[k] + e * dF[k] for k in F0}, v + e * dv, dt)
    minus = transport.advect(g, {k: F0[k] - e * dF[k] for k in F0}, v - e * dv, dt)
    lhs = sum(dot((plus[k] - minus[k]) / (2 * e), ybar[k]) for k in "pingwf")
    fb, vb = adj.transport_adjoint(g, F0, v, dt, ybar)
    rhs = sum(dot(dF[k], fb[k]) for k in "pingwf") + dot(dv, vb)
    assert abs(lhs - rhs) < 1e-7 * abs(lhs)


def test_cn_adjoint():
    n, dt = 12, 0.01
    g = Grid(n)
    wm, gm, csf = synthetic.tissue_maps(n, 2.0, 3)
    K = 0.1 * wm + 0.01 * gm
    c0 = np.abs(synthetic.random_field(n, 4, 1.0))
    ybar = synthetic.random_field(n, 5, 1.0)
    fwd = lambda c, KK: solvers.cn_diffusion(g, KK, K.mean(), dt, c, 1e-14, 500)[0]
    c1 = fwd(c0, K)
    cb, Kb = adj.cn_adjoint(g, K, K.mean(), dt, c0, c1, ybar, 1e-14, 500)
    dc = synthetic.random_field(n, 6, 1.0)
    assert abs(dot(fwd(dc, K), ybar) - dot(dc, cb)) < 1e-11 * abs(dot(dc, cb))
    dK = 0.01 * synthetic.random_field(n, 7, 1.5)
    e = 1e-4
    fd = dot((fwd(c0, K + e * dK) - fwd(c0, K - e * dK)) / (2 * e), ybar)
    assert abs(fd - dot(dK, Kb)) < 1e-7 * abs(fd)


def test_elasticity_and_force_adjoint():
    n = 12
    g = Grid(n)
    P = synthetic.params()
    wm, gm, csf = synthetic.tissue_maps(n, 2.0, 8)
    x3, y3, z3 = g.coords()
    p = 0.5 * np.exp(-((x3 - 3) ** 2 + (y3 - 3) ** 2 + (z3 - 3) ** 2) / (2 * 0.7 ** 2))
    z = np.zeros_like(p)

    def solve(pp, mu_d=0.0, lam_d=0.0, eta_d=0.0):
        co = rx.refresh(P, pp, z, z, gm, wm, csf)
        co = dict(co, mu=co["mu"] + mu_d, lam=co["lam"] + lam_d, eta=co["eta"] + eta_d)
        b = rx.elastic_force(g, P["zeta"], pp, z)
        return solvers.solve_elasticity(g, co["mu"], co["lam"], co["eta"], (co["mubar"], co["lambar"], co["etabar"]),
                                        b, np.zeros_like(b), 1e-14, 1000)[0], co, b

    u, co, b = solve(p)
    ubar = synthetic.random_field(n, 9, 1.0, ncomp=3)
    bb, mub, lamb, etab = adj.elasticity_adjoint(g, co, u, ubar, 1e-14, 1000)
    # b -> u is linear: u = A^-1(-b)
    db = synthetic.random_field(n, 10, 1.0, ncomp=3)
    ud = solvers.solve_elasticity(g, co["mu"], co["lam"], co["eta"], (co["mubar"], co["lambar"], co["etabar"]),
                                  db, np.zeros_like(db), 1e-14, 1000)[0]
    assert abs(dot(ud, ubar) - dot(db, bb)) < 1e-10 * abs(dot(db, bb))
    # coefficient sensitivities by finite differences
    e = 1e-3
    for name, field in (("mu", mub), ("lam", lamb), ("eta", etab)):
        d = 50.0 * np.abs(synthetic.random_field(n, 11, 1.5))
        kw = {f"{name}_d": e * d}
        up = solve(p, **kw)[0]
        kw = {f"{name}_d": -e * d}
        um = solve(p, **kw)[0]
        fd = dot((up - um) / (2 * e), ubar)
        assert abs(fd - dot(d, field)) < 1e-6 * abs(fd), name
    # force -> tau
    dtau = 0.1 * synthetic.random_field(n, 12, 1.5)
    e = 1e-6
    fd = dot((rx.elastic_force(g, P["zeta"], p + e * dtau, z) - rx.elastic_force(g, P["zeta"], p - e * dtau, z)) / (2 * e),
             bb)
    assert abs(fd - dot(dtau, adj.force_adjoint(g, P["zeta"], p, bb))) < 1e-7 * abs(fd)


@pytest.mark.parametrize("o_range", [(0.3, 1.0), (0.58, 0.72)])
def test_reaction_adjoint_matches_finite_differences(o_range):
    P = synthetic.params()
    rng = np.random.default_rng(3)
    m = 400
    x = dict(p=rng.uniform(0.05, 0.9, m), i=rng.uniform(0.0, 0.5, m), n=rng.uniform(0, 0.3, m),
             g=rng.uniform(0.05, 1, m), w=rng.uniform(0.05, 1, m), o=rng.uniform(*o_range, m),
             rp=rng.uniform(0, 10, m), ri=rng.uniform(0, 1, m), dD=rng.uniform(-0.01, 0.01, m))
    # keep away from the clamp kinks of the oxygen factor
    o_mit = 0.5 * (P["o_hyp"] + P["o_inv"])
    x["o"] = np.where(np.abs(x["o"] - o_mit) < 1e-3, x["o"] + 2e-3, x["o"])
    x["o"] = np.where(np.abs(x["o"] - P["o_inv"]) < 1e-3, x["o"] + 2e-3, x["o"])
    order = ("p", "i", "n", "g", "w", "o", "rp", "ri", "dD")
    f = lambda d: rx.species_reaction(P, 0.01, d["p"], d["i"], d["n"], d["g"], d["w"], d["o"], d["rp"], d["ri"],
                                      d["dD"])
    ob = [rng.standard_normal(m) for _ in range(5)]
    bars = adj.reaction_adjoint(P, 0.01, x["p"], x["i"], x["n"], x["g"], x["w"], x["o"], x["rp"], x["ri"],
                                x["dD"], *ob)
    e = 1e-7
    for k, name in enumerate(order):
        xp = dict(x)
        xm = dict(x)
        xp[name] = x[name] + e
        xm[name] = x[name] - e
        fp, fm = f(xp), f(xm)
        fd = sum(((a - b) / (2 * e)) * o for a, b, o in zip(fp, fm, ob))
        assert np.allclose(fd, bars[k], rtol=1e-5, atol=1e-6), name


def _grad_case(n=16, steps=3, seed_params=None):
    P = synthetic.params(**(seed_params or {}))
    inp = synthetic.workload_inputs("lattice_n128", n=n)
    # target from a run with perturbed parameters
    Pt = dict(P, rho_w=P["rho_w"] * 1.1, rho_g=P["rho_g"] * 1.1, k_w=P["k_w"] * 0.9)
    st, _ = model.run(Pt, inp, steps, TIGHT)
    target = st.f["p"] + st.f["i"] + st.f["n"]
    return P, inp, target


def _loss_of(P, inp, steps, target):
    st, _ = model.run(P, inp, steps, TIGHT)
    return adj.loss(P, st.grid, st, target)


@pytest.mark.slow
def test_whole_gradient_matches_central_differences():
    steps = 3
    P, inp, target = _grad_case(steps=steps, seed_params=dict(delta_p=60.0))
    L, grad, gw, lam = adj.gradient(P, inp, steps, target, TIGHT)
    assert L > 0
    checks = {
        "rho": lambda P, e: dict(P, rho_w=P["rho_w"] + e, rho_g=P["rho_g"] + e),
        "k_w": lambda P, e: dict(P, k_w=P["k_w"] + e),
        "k_g": lambda P, e: dict(P, k_g=P["k_g"] + e),
        "k_f": lambda P, e: dict(P, k_f=P["k_f"] + e),
        "lame_scale": lambda P, e: dict(P, lame_scale=P["lame_scale"] + e),
    }
    steps_fd = dict(rho=1e-4, k_w=1e-5, k_g=1e-5, k_f=1e-5, lame_scale=1e-5)
    for name, mk in checks.items():
        e = steps_fd[name]
        fd = (_loss_of(mk(P, e), inp, steps, target) - _loss_of(mk(P, -e), inp, steps, target)) / (2 * e)
        assert abs(fd - grad[name]) <= 1e-5 * abs(fd) + 1e-12 * abs(L), (name, fd, grad[name])
    for k in (0, 21, 63):
        e = 1e-5
        ip = dict(inp, weights=inp["weights"].copy())
        im = dict(inp, weights=inp["weights"].copy())
        ip["weights"][k] += e
        im["weights"][k] -= e
        fd = (_loss_of(P, ip, steps, target) - _loss_of(P, im, steps, target)) / (2 * e)
        assert abs(fd - gw[k]) <= 1e-5 * abs(fd) + 1e-12 * abs(L), (k, fd, gw[k])


def test_directional_gradient_on_all_species_slots():
    # Perturb the full initial state along a random direction: the adjoint
    # state at t=0 must predict the change of the loss (covers o, l, g, w, f, u
    # slots that the parameter gradient does not reach directly).
    steps = 2
    n = 12
    P = synthetic.params(delta_p=60.0)
    inp = synthetic.workload_inputs("seed1_n32", n=n)
    st0 = model.init_state(P, n, inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"], inp["weights"])
    target = 0.8 * (st0.f["p"])
    rng = np.random.default_rng(11)
    dirs = {k: 0.01 * np.abs(synthetic.random_field(n, 60 + j, 1.5)) for j, k in enumerate(model.FIELDS)}

    def run_from(eps, with_tape=False):
        st = st0.copy()
        for k in model.FIELDS:
            st.f[k] = st.f[k] + eps * dirs[k]
        st.coef = rx.refresh(P, *(st.f[k] for k in ("p", "i", "n", "g", "w", "f")))
        tapes = []
        for s in range(steps):
            tp = {}
            model.step(st, TIGHT, tape=tp)
            tapes.append(tp)
        return st, tapes

    st, tapes = run_from(0.0)
    g = st.grid
    seed = g.h ** 3 * (st.f["p"] + st.f["i"] + st.f["n"] - target)
    lam = {k: np.zeros_like(seed) for k in model.FIELDS}
    for k in "pin":
        lam[k] = seed.copy()
    lam["u"] = np.zeros((3,) + seed.shape)
    lam["u_prev"] = np.zeros((3,) + seed.shape)
    grad = {k: 0.0 for k in adj.GRAD_NAMES}
    for tp in reversed(tapes):
        lam = adj.adjoint_step(P, g, tp, lam, grad, TIGHT)
    pred = sum(dot(lam[k], dirs[k]) for k in model.FIELDS)
    e = 1e-5
    Lp = adj.loss(P, g, run_from(e)[0], target)
    Lm = adj.loss(P, g, run_from(-e)[0], target)
    fd = (Lp - Lm) / (2 * e)
    assert abs(fd - pred) < 1e-5 * abs(fd)
