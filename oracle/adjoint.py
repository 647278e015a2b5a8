"""Discrete adjoint of the split step (oracle; test infrastructure only).

The paper names adjoint-based inversion as future work (Sec. 5) and computes
sensitivities by finite differences (Sec. 4, sensitivity analysis).  This is
the exact transpose of the linearisation of one forward step as the oracle
computes it (``model.step``), with every PCG solve treated as an exact
inverse.  Sub-steps are reversed in the opposite order of S1..S7:

  S7  the u^{n+1} and u^n slots of the adjoint state;
  S6  adjoint elasticity solve y = A^-1 u_bar (A is symmetric), b_bar = -y,
      coefficient sensitivities mu_bar = -1/2 sum_ab E_ab(y) E_ab(u),
      lambda_bar = -div y div u, eta_bar = -y . u with E_ab(u) = G_b u_a + G_a u_b,
      and the force b = zeta tanh(tau) G tau transposed into tau = p + n;
  S5  the Lame/screening mixture transposed onto the species and the Lame scale;
  S4  oxygen and edema updates (pointwise Jacobians);
  S3  species reaction (pointwise Jacobian, including the Heaviside-gated rates,
      the clamped oxygen factor with one-sided derivative 1/(o_inv - o_mit) on
      the closed interval and 0 outside, and the exact logistic flows);
  S2  adjoint CN solves y = A^-1 c_bar+, c_bar- = B y, and
      K_bar = -dt/2 sum_a G_a y . G_a (c- + c+);
  S1  semi-Lagrangian transport: transposed interpolation (scatter-add), the
      Heun source factor, and the velocity sensitivity through both
      departure points (gradient of the interpolant at X and X*);
  S0  the coefficients of the step (K, rho from the species at step start)
      transposed onto w, g, f and the parameters.

Parameters: theta = (rho, k_w, k_g, k_f, lame_scale, w_1..w_K); "rho" moves
rho_w and rho_g together (the gradient is d/d rho_w + d/d rho_g).  The
loss of the adjoint workloads is 1/2 h^3 sum (tau_T - tau_target)^2 with
tau = p + i + n.
"""
from __future__ import annotations

import numpy as np

from . import model, reaction as rx, solvers, transport
from .spectral import dot

GRAD_NAMES = ("rho", "k_w", "k_g", "k_f", "lame_scale")


# ---------------------------------------------------------------- interpolation
def lagrange_dweights(t):
    """Derivatives d w_k / dt of the cubic Lagrange weights on nodes -1..2."""
    return (-(3 * t * t - 6 * t + 2) / 6.0,
            (3 * t * t - 4 * t - 1) / 2.0,
            -(3 * t * t - 2 * t - 2) / 2.0,
            (3 * t * t - 1) / 6.0)


def _stencil(j, n):
    base = np.floor(j)
    t = j - base
    b = base.astype(np.int64)
    return [np.mod(b + o, n) for o in (-1, 0, 1, 2)], t


def interp_transpose(vals, jx, jy, jz, n):
    """Transpose of transport.interp: scatter-add vals * weights onto the grid."""
    out = np.zeros((n, n, n))
    (ix, tx), (iy, ty), (iz, tz) = (_stencil(j, n) for j in (jx, jy, jz))
    wx, wy, wz = (transport.lagrange_weights(t) for t in (tx, ty, tz))
    for c in range(4):
        for b in range(4):
            for a in range(4):
                np.add.at(out, (iz[c], iy[b], ix[a]), (wz[c] * wy[b] * wx[a]) * vals)
    return out


def interp_gradient(q, jx, jy, jz):
    """d/d(jx, jy, jz) of the tricubic interpolant of q at the given points."""
    n = q.shape[0]
    (ix, tx), (iy, ty), (iz, tz) = (_stencil(j, n) for j in (jx, jy, jz))
    wx, wy, wz = (transport.lagrange_weights(t) for t in (tx, ty, tz))
    dx, dy, dz = (lagrange_dweights(t) for t in (tx, ty, tz))
    gx = np.zeros(np.shape(jx))
    gy = np.zeros(np.shape(jx))
    gz = np.zeros(np.shape(jx))
    for c in range(4):
        for b in range(4):
            for a in range(4):
                val = q[iz[c], iy[b], ix[a]]
                gx += wz[c] * wy[b] * dx[a] * val
                gy += wz[c] * dy[b] * wx[a] * val
                gz += dz[c] * wy[b] * wx[a] * val
    return gx, gy, gz


# -------------------------------------------------------------------- transport
def transport_adjoint(grid, F0, v, dt, bar):
    """Adjoint of transport.advect.

    F0: fields at step start; v: velocity; bar: adjoints of the outputs
    (p, i, n, g, w after the conservative transport, f after the plain one).
    Returns (adjoints of the input fields, adjoint of v).
    """
    n = grid.n
    s = dt / grid.h
    delta = grid.div(v)
    jx, jy, jz = transport.grid_indices(n)
    xs = (jx - s * v[0], jy - s * v[1], jz - s * v[2])
    vs = [transport.interp(v[a], *xs) for a in range(3)]
    X = (jx - 0.5 * s * (v[0] + vs[0]), jy - 0.5 * s * (v[1] + vs[1]), jz - 0.5 * s * (v[2] + vs[2]))
    dX = transport.interp(delta, *X)
    # q+ = q(X) * c with c = 1 - dt/2 (delta(X) + delta) + dt^2/2 delta(X) delta
    cfac = 1.0 - 0.5 * dt * (dX + delta) + 0.5 * dt * dt * dX * delta
    cbar = np.zeros_like(delta)
    out = {}
    Jbar = [np.zeros_like(delta) for _ in range(3)]
    for name in ("p", "i", "n", "g", "w"):
        qX = transport.interp(F0[name], *X)
        cbar += bar[name] * qX
        qbar_X = bar[name] * cfac
        out[name] = interp_transpose(qbar_X, *X, n)
        gr = interp_gradient(F0[name], *X)
        for a in range(3):
            Jbar[a] += gr[a] * qbar_X
    out["f"] = interp_transpose(bar["f"], *X, n)
    gr = interp_gradient(F0["f"], *X)
    for a in range(3):
        Jbar[a] += gr[a] * bar["f"]
    dXbar = cbar * (-0.5 * dt + 0.5 * dt * dt * delta)
    delta_bar = cbar * (-0.5 * dt + 0.5 * dt * dt * dX)
    delta_bar += interp_transpose(dXbar, *X, n)
    gr = interp_gradient(delta, *X)
    for a in range(3):
        Jbar[a] += gr[a] * dXbar
    # X = x - s/2 (v + v*),  v*_a = I[v_a](X*),  X* = x - s v
    vbar = np.stack([-0.5 * s * Jbar[a] for a in range(3)])
    vsbar = [-0.5 * s * Jbar[a] for a in range(3)]
    Jsbar = [np.zeros_like(delta) for _ in range(3)]
    for b in range(3):
        vbar[b] += interp_transpose(vsbar[b], *xs, n)
        gr = interp_gradient(v[b], *xs)
        for a in range(3):
            Jsbar[a] += gr[a] * vsbar[b]
    for a in range(3):
        vbar[a] += -s * Jsbar[a]
    # delta = div v = sum_a G_a v_a ; G_a^T = -G_a
    for a in range(3):
        vbar[a] -= grid.deriv(delta_bar, a)
    return out, vbar


# -------------------------------------------------------------------- solves
def _solve(apply_a, apply_m, rhs, rtol, max_it):
    x, it, rr, ok = solvers.pcg(apply_a, apply_m, rhs, np.zeros_like(rhs), rtol, max_it)
    return x


def cn_adjoint(grid, K, Kbar, dt, c_minus, c_plus, cbar_plus, rtol, max_it):
    """Adjoint of c+ = (1 - dt/2 D_K)^-1 (1 + dt/2 D_K) c-.  Returns (c-_bar, K_bar field)."""
    h = 0.5 * dt
    y = _solve(lambda x: solvers.cn_matrix(grid, K, dt, x), lambda r: solvers.cn_precond(grid, Kbar, dt, r),
               cbar_plus, rtol, max_it)
    cbar_minus = solvers.cn_rhs(grid, K, dt, y)
    s = c_minus + c_plus
    Kb = np.zeros_like(K)
    for a in range(3):
        Kb -= h * grid.deriv(y, a) * grid.deriv(s, a)
    return cbar_minus, Kb


def elasticity_adjoint(grid, coef, u, ubar, rtol, max_it):
    """Adjoint of u = A^-1 (-b): returns (b_bar, mu_bar, lambda_bar, eta_bar)."""
    rhs = np.array(ubar, dtype=np.float64)
    y = _solve(lambda x: solvers.elasticity_op(grid, coef["mu"], coef["lam"], coef["eta"], x),
               lambda r: solvers.elasticity_precond(grid, coef["mubar"], coef["lambar"], coef["etabar"], r),
               rhs, rtol, max_it)
    gy = solvers.strain_grads(grid, y)
    gu = solvers.strain_grads(grid, u)
    mub = np.zeros_like(u[0])
    for a in range(3):
        for b in range(3):
            mub -= 0.5 * (gy[a][b] + gy[b][a]) * (gu[a][b] + gu[b][a])
    divy = gy[0][0] + gy[1][1] + gy[2][2]
    divu = gu[0][0] + gu[1][1] + gu[2][2]
    lamb = -divy * divu
    etab = -(y * u).sum(axis=0)
    return -y, mub, lamb, etab


def force_adjoint(grid, zeta, tau, bbar):
    """Adjoint of b = zeta tanh(tau) G tau with respect to tau."""
    t = np.tanh(tau)
    g = grid.grad(tau)
    out = np.zeros_like(tau)
    for a in range(3):
        out += zeta * (1.0 - t * t) * g[a] * bbar[a]
        out -= grid.deriv(zeta * t * bbar[a], a)
    return out


# ------------------------------------------------------------------ pointwise
def dheaviside(x, eps):
    H = rx.heaviside(x, eps)
    return (2.0 / eps) * H * (1.0 - H)


def logistic_partials(y, r, t):
    """(d Lambda / dy, d Lambda / dr) of the exact logistic flow."""
    e = np.exp(r * t)
    D = 1.0 + y * (e - 1.0)
    return e / (D * D), t * e * y * (1.0 - y) / (D * D)


def reaction_adjoint(P, dt, p, i, n, g, w, o, rho_p, rho_i, dD, pb, ib, nb, gb, wb):
    """Transpose of species_reaction's Jacobian applied to the output adjoints.

    Returns adjoints of (p, i, n, g, w, o, rho_p, rho_i, dD).
    """
    eps = P["heaviside_eps"]
    Ha = rx.heaviside(P["o_inv"] - o, eps)
    alpha = P["alpha0"] * Ha
    alpha_o = -P["alpha0"] * dheaviside(P["o_inv"] - o, eps)
    Hb = rx.heaviside(P["sigma_b"] - p - i, eps)
    beta = P["beta0"] * Hb * o
    beta_pi = -P["beta0"] * dheaviside(P["sigma_b"] - p - i, eps) * o
    beta_o = P["beta0"] * Hb
    h = P["gamma"] * rx.heaviside(P["o_hyp"] - o, eps)
    h_o = -P["gamma"] * dheaviside(P["o_hyp"] - o, eps)
    o_mit = 0.5 * (P["o_hyp"] + P["o_inv"])
    kappa = rx.oxygen_factor(P, o)
    kappa_o = np.where((o >= o_mit) & (o <= P["o_inv"]), 1.0 / (P["o_inv"] - o_mit), 0.0)
    Lp_y, Lp_r = logistic_partials(p, rho_p * kappa, dt)
    Li_y, Li_r = logistic_partials(i, rho_i * kappa, dt)
    dRp = rx.logistic_flow(p, rho_p * kappa, dt) - p
    dRi = rx.logistic_flow(i, rho_i * kappa, dt) - i
    S = dD + dRp + dRi
    gw = g + w
    small = gw < 1e-12
    safe = np.where(small, 1.0, gw)
    phig = np.where(small, 0.5, g / safe)
    phiw = np.where(small, 0.5, w / safe)
    inv2 = np.where(small, 0.0, 1.0 / (safe * safe))
    dphig_g, dphig_w = w * inv2, -g * inv2
    dphiw_g, dphiw_w = -w * inv2, g * inv2
    Sb = -phig * gb - phiw * wb
    tot = p + i + g + w
    p_bar = pb * (Lp_y + dt * (-alpha + beta_pi * i - h)) + ib * dt * (alpha - beta_pi * i) \
        + nb * dt * h + Sb * (Lp_y - 1.0)
    i_bar = pb * dt * (beta + beta_pi * i) + ib * (Li_y + dt * (-beta - beta_pi * i - h)) \
        + nb * dt * h + Sb * (Li_y - 1.0)
    n_bar = nb
    g_bar = nb * dt * h + gb * (1.0 - dphig_g * S - dt * h) + wb * (-dphiw_g * S)
    w_bar = nb * dt * h + gb * (-dphig_w * S) + wb * (1.0 - dphiw_w * S - dt * h)
    o_bar = pb * (Lp_r * rho_p * kappa_o + dt * (-alpha_o * p + beta_o * i - h_o * p)) \
        + ib * (Li_r * rho_i * kappa_o + dt * (alpha_o * p - beta_o * i - h_o * i)) \
        + nb * dt * h_o * tot + Sb * (Lp_r * rho_p + Li_r * rho_i) * kappa_o \
        - gb * dt * h_o * g - wb * dt * h_o * w
    rho_p_bar = (pb + Sb) * Lp_r * kappa
    rho_i_bar = (ib + Sb) * Li_r * kappa
    return p_bar, i_bar, n_bar, g_bar, w_bar, o_bar, rho_p_bar, rho_i_bar, Sb


def lame_parts(P):
    parts = {}
    for sp, (E, nu) in dict(w=("E_wm", "nu_wm"), g=("E_gm", "nu_gm"), f=("E_csf", "nu_csf"),
                            t=("E_tumor", "nu_tumor")).items():
        parts[sp] = rx.lame_species(P[E], P[nu])
    return parts


# ------------------------------------------------------------------- one step
ADJ_FIELDS = model.FIELDS  # p, i, n, o, l, g, w, f


def adjoint_step(P, grid, tape, lam, grad, cfg=None):
    """Reverse one recorded step.

    tape: the intermediates recorded by model.step(..., tape=tape).
    lam: dict with the adjoints of the state after the step (species, "u", "u_prev").
    grad: dict accumulating d/d(rho, k_w, k_g, k_f, lame_scale).
    Returns the adjoint of the state before the step.
    """
    c = dict(model.DEFAULT_CFG)
    if cfg:
        c.update(cfg)
    dt = c["dt"]
    rt = c.get("rtol_adj", 1e-12)
    mi = c["max_it"]
    F0, adv, c0, c1 = tape["F0"], tape["adv"], tape["coef0"], tape["coef1"]
    p1, i1, n1, g1, w1, o1 = tape["p1"], tape["i1"], tape["n1"], tape["g1"], tape["w1"], tape["o1"]
    bar = {k: np.array(lam[k], dtype=np.float64, copy=True) for k in ADJ_FIELDS}
    u_bar_prev_slot = np.array(lam["u_prev"], dtype=np.float64, copy=True)   # -> u^n
    u_bar_new = np.array(lam["u"], dtype=np.float64, copy=True)              # -> u^{n+1}
    s = P["lame_scale"]
    parts = lame_parts(P)

    # S6 (elasticity) and the force
    if c["elasticity"]:
        bbar, mub, lamb, etab = elasticity_adjoint(grid, c1, tape["u_new"], u_bar_new, rt, mi)
        taub = force_adjoint(grid, P["zeta"], p1 + n1, bbar)
        bar["p"] += taub
        bar["n"] += taub
        # S5: mixture of the Lame fields and the screening
        tau = p1 + i1 + n1
        for name, field in (("w", w1), ("g", g1), ("f", adv["f"])):
            mu_s, la_s = parts[name]
            bar[name] += s * mu_s * mub + s * la_s * lamb + P["eta_healthy"] * etab
        mu_t, la_t = parts["t"]
        tb = s * mu_t * mub + s * la_t * lamb + P["eta_tumor"] * etab
        for k in ("p", "i", "n"):
            bar[k] += tb
        mu_base = sum(parts[k][0] * f for k, f in (("w", w1), ("g", g1), ("f", adv["f"]), ("t", tau)))
        la_base = sum(parts[k][1] * f for k, f in (("w", w1), ("g", g1), ("f", adv["f"]), ("t", tau)))
        if tape.get("bg") is not None:
            mu_b, la_b = rx.lame_species(P["E_bg"], P["nu_bg"])
            mu_base = mu_base + mu_b * tape["bg"]
            la_base = la_base + la_b * tape["bg"]
        grad["lame_scale"] += dot(mu_base, mub) + dot(la_base, lamb)
    else:
        u_bar_prev_slot = u_bar_prev_slot + u_bar_new      # u^{n+1} = u^n
    # S4b edema, S4 oxygen
    if c["edema"]:
        l_dag_bar = bar["l"] * (1.0 - dt * P["delta_l"])
        dh = P["delta_half"]
        bar["i"] += bar["l"] * dt * P["delta_e"] * (dh * (1.0 - i1) / (i1 + dh) ** 2 - i1 / (i1 + dh))
    else:
        l_dag_bar = bar["l"]
    o_dag = tape["o_dag"]
    o_dag_bar = bar["o"] * (1.0 - dt * P["delta_s"] * (g1 + w1))
    bar["p"] += bar["o"] * (-dt * P["delta_p"])
    gw_o = bar["o"] * dt * P["delta_s"] * (P["o_heal"] - o_dag)
    bar["g"] += gw_o
    bar["w"] += gw_o
    # S3 reaction
    i_dd = tape["i_dd"]
    dD = i_dd - adv["i"]
    pb, ib, nb, gb, wb, ob, rpb, rib, dDb = reaction_adjoint(
        P, dt, adv["p"], i_dd, adv["n"], adv["g"], adv["w"], o_dag, c0["rho_p"], c0["rho_i"], dD,
        bar["p"], bar["i"], bar["n"], bar["g"], bar["w"])
    o_dag_bar = o_dag_bar + ob
    i_dd_bar = ib + dDb
    # S2 diffusion
    K = c0["K"]
    i_dag_bar, Kb = cn_adjoint(grid, K, c0["Kbar"], dt, adv["i"], i_dd, i_dd_bar, rt, mi)
    i_dag_bar = i_dag_bar - dDb
    o_bar0, Kb2 = cn_adjoint(grid, K, c0["Kbar"], dt, F0["o"], o_dag, o_dag_bar, rt, mi)
    Kb += Kb2
    if c["edema"]:
        l_bar0, Kb3 = cn_adjoint(grid, K, c0["Kbar"], dt, F0["l"], tape["l_dag"], l_dag_bar, rt, mi)
        Kb += Kb3
    else:
        l_bar0 = l_dag_bar
    # S1 transport
    adv_bar = dict(p=pb, i=i_dag_bar, n=nb, g=gb, w=wb, f=bar["f"])
    v = tape["v"]
    if c["advection"]:
        fb, vbar = transport_adjoint(grid, F0, v, dt, adv_bar)
    else:
        fb, vbar = adv_bar, np.zeros_like(v)
    # S0 coefficients of the step
    rho_tot = rpb + P["rho_inv_frac"] * rib
    out = {k: fb[k] for k in ("p", "i", "n", "g", "w", "f")}
    out["o"] = o_bar0
    out["l"] = l_bar0
    out["w"] = out["w"] + P["k_w"] * Kb + P["rho_w"] * rho_tot
    out["g"] = out["g"] + P["k_g"] * Kb + P["rho_g"] * rho_tot
    out["f"] = out["f"] + P["k_f"] * Kb
    grad["k_w"] += dot(F0["w"], Kb)
    grad["k_g"] += dot(F0["g"], Kb)
    grad["k_f"] += dot(F0["f"], Kb)
    grad["rho"] += dot(F0["w"] + F0["g"], rho_tot)
    # u slots: v = (u^n - u^{n-1}) / dt
    out["u"] = u_bar_prev_slot + vbar / dt
    out["u_prev"] = -vbar / dt
    return out


def gaussian_basis_functions(grid, centers, sigmas):
    return [model.gaussian_basis(grid, [c], [s], [1.0]) for c, s in zip(centers, sigmas)]


def loss(P, grid, st, tau_target):
    tau = st.f["p"] + st.f["i"] + st.f["n"]
    return 0.5 * grid.h ** 3 * float(((tau - tau_target) ** 2).sum())


def gradient(P, inputs, steps, tau_target, cfg=None, u0=None, u_prev0=None):
    """Loss and its gradient with respect to (rho, k_w, k_g, k_f, lame_scale, ic weights).

    u0, u_prev0: optional initial displacements (default zero), held fixed;
    the returned adjoint state holds their adjoints in lam["u"], lam["u_prev"]."""
    c = dict(model.DEFAULT_CFG)
    if cfg:
        c.update(cfg)
    st = model.init_state(P, inputs["n"], inputs["wm"], inputs["gm"], inputs["csf"], inputs["centers"],
                          inputs["sigmas"], inputs["weights"], inputs.get("bg"))
    if u0 is not None:
        st.u = np.array(u0, dtype=np.float64)
    if u_prev0 is not None:
        st.u_prev = np.array(u_prev0, dtype=np.float64)
    grid = st.grid
    tapes = []
    for k in range(steps):
        tp = {}
        model.step(st, c, tape=tp)
        tapes.append(tp)
    L = loss(P, grid, st, tau_target)
    seed = grid.h ** 3 * (st.f["p"] + st.f["i"] + st.f["n"] - tau_target)
    z = np.zeros_like(seed)
    lam = {k: z.copy() for k in ADJ_FIELDS}
    lam["p"] = seed.copy()
    lam["i"] = seed.copy()
    lam["n"] = seed.copy()
    lam["u"] = np.zeros((3,) + seed.shape)
    lam["u_prev"] = np.zeros((3,) + seed.shape)
    grad = {k: 0.0 for k in GRAD_NAMES}
    for tp in reversed(tapes):
        lam = adjoint_step(P, grid, tp, lam, grad, c)
    phis = gaussian_basis_functions(grid, inputs["centers"], inputs["sigmas"])
    gw = np.array([dot(ph, lam["p"]) for ph in phis])
    return L, grad, gw, lam
