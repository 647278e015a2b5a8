"""Pointwise parts of the split step: reaction, necrosis, oxygen, edema, and the
coefficient refresh.  All FP64.

Model terms (Sec. 2.3, Eq. e:gog and the rate laws that follow it):
* death         h = gamma H(o_hyp - o)                              (e:death)
* p -> i rate   alpha = alpha0 H(o_inv - o)                         (e:alpha)
* i -> p rate   beta = beta0 H(sigma_b - p - i) o                   (e:beta)
* growth        R = kappa(o) rho p (1 - p), R~ = kappa(o) rho_i i (1 - i) with
  the piecewise oxygen factor of e:gog_reac_op rewritten exactly as
  kappa(o) = clamp((o - o_mit)/(o_inv - o_mit), 0, 1), o_mit = (o_hyp + o_inv)/2
* oxygen        d_t o = D o - delta_p p + delta_s (o_heal - o)(g + w)  (e:ox)
* edema         l_t = D l + delta_e i/(i + delta_half) (1 - i) - delta_l l (e:edema)

Readings (the paper says only that the reaction equations are solved
explicitly, Sec. 3):
* H(x) = (1 + tanh(x / eps)) / 2, the smoothed Heaviside, eps = 0.01,
  evaluated as 1 / (1 + exp(-2 x / eps)) (same function, no cancellation);
* all rates are frozen at the start of the sub-step; the logistic terms use
  their exact flow Lambda(y, r, dt) = y e^{r dt} / (1 + y (e^{r dt} - 1)),
  the linear transfer, death, supply and edema terms are forward Euler;
* the healthy-tissue sink g/(g+w) (D + R + R~) uses the increment actually
  produced by this step's invasive-cell diffusion and the two logistic flows,
  which keeps p + i + n + g + w unchanged by diffusion + reaction;
* where g + w < 1e-12 the split fractions are 1/2 each.

Coefficient refresh (Eqs. e:diffusion_tensor, e:reaction_op, e:lame,
e:screening): K = k_w w + k_g g + k_f f, rho_p = rho_w w + rho_g g,
rho_i = rho_inv_frac rho_p, and with the tumour species tau = p + i + n
mu = s sum_s E_s/(2(1+nu_s)) iota_s, lambda = s sum_s nu_s E_s/((1-2nu_s)(1+nu_s)) iota_s
over iota in {w, g, f, tau}, eta = eta_tumor tau + eta_healthy (g + w + f).
The preconditioners use the voxel means of K, mu, lambda and eta.
"""
from __future__ import annotations

import numpy as np


def heaviside(x, eps):
    """Smoothed Heaviside (1 + tanh(x/eps))/2, evaluated as 1/(1 + exp(-2x/eps)).

    The two forms are equal in exact arithmetic; the second avoids the
    cancellation of 1 + tanh(x/eps) for x/eps << 0, where the rates it gates
    (alpha, h) are tiny but still drive the invasive and necrotic fields.
    """
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-2.0 * np.asarray(x, dtype=np.float64) / eps))


def logistic_flow(y, r, t):
    """Exact solution at time t of y' = r y (1 - y) from y."""
    e = np.exp(r * t)
    return y * e / (1.0 + y * (e - 1.0))


def oxygen_factor(P, o):
    o_mit = 0.5 * (P["o_hyp"] + P["o_inv"])
    return np.clip((o - o_mit) / (P["o_inv"] - o_mit), 0.0, 1.0)


def species_reaction(P, dt, p, i, n, g, w, o, rho_p, rho_i, dD):
    """Reaction sub-step for (p, i, n, g, w) with oxygen o and frozen growth rates.

    ``dD`` is the invasive-cell increment of this step's diffusion sub-step.
    Returns (p', i', n', g', w').
    """
    eps = P["heaviside_eps"]
    alpha = P["alpha0"] * heaviside(P["o_inv"] - o, eps)
    beta = P["beta0"] * heaviside(P["sigma_b"] - p - i, eps) * o
    h = P["gamma"] * heaviside(P["o_hyp"] - o, eps)
    kappa = oxygen_factor(P, o)
    dRp = logistic_flow(p, rho_p * kappa, dt) - p
    dRi = logistic_flow(i, rho_i * kappa, dt) - i
    p1 = p + dRp + dt * (-alpha * p + beta * i - h * p)
    i1 = i + dRi + dt * (alpha * p - beta * i - h * i)
    n1 = n + dt * h * (p + i + g + w)
    s = dD + dRp + dRi
    gw = g + w
    small = gw < 1e-12
    safe = np.where(small, 1.0, gw)
    phi_g = np.where(small, 0.5, g / safe)
    phi_w = np.where(small, 0.5, w / safe)
    g1 = g - phi_g * s - dt * h * g
    w1 = w - phi_w * s - dt * h * w
    return p1, i1, n1, g1, w1


def oxygen_reaction(P, dt, o_dag, p1, g1, w1):
    """Explicit oxygen consumption and supply after the species reaction."""
    return o_dag + dt * (-P["delta_p"] * p1 + P["delta_s"] * (P["o_heal"] - o_dag) * (g1 + w1))


def edema_reaction(P, dt, l_dag, i1):
    """Explicit edema source and drainage (e:edema), driven by the new invasive cells."""
    src = P["delta_e"] * i1 / (i1 + P["delta_half"]) * (1.0 - i1)
    return l_dag + dt * (src - P["delta_l"] * l_dag)


def lame_species(E, nu):
    """(mu_s, lambda_s) of one species from Young's modulus and Poisson ratio (e:lame)."""
    return E / (2.0 * (1.0 + nu)), nu * E / ((1.0 - 2.0 * nu) * (1.0 + nu))


def refresh(P, p, i, n, g, w, f, bg=None):
    """Coefficient fields and their voxel means from the current species.

    bg: optional static background-material fraction (fictitious domain,
    Sec. 3): it enters the Lame mixture with (E_bg, nu_bg) (e:lame) and the
    screening with eta_bg (e:screening); it carries no diffusion or growth, so
    the tumour flux vanishes outside the brain."""
    tau = p + i + n
    K = P["k_w"] * w + P["k_g"] * g + P["k_f"] * f
    rho_p = P["rho_w"] * w + P["rho_g"] * g
    rho_i = P["rho_inv_frac"] * rho_p
    s = P["lame_scale"]
    mu_w, la_w = lame_species(P["E_wm"], P["nu_wm"])
    mu_g, la_g = lame_species(P["E_gm"], P["nu_gm"])
    mu_f, la_f = lame_species(P["E_csf"], P["nu_csf"])
    mu_t, la_t = lame_species(P["E_tumor"], P["nu_tumor"])
    mu = s * (mu_w * w + mu_g * g + mu_f * f + mu_t * tau)
    lam = s * (la_w * w + la_g * g + la_f * f + la_t * tau)
    eta = P["eta_tumor"] * tau + P["eta_healthy"] * (g + w + f)
    if bg is not None:
        mu_b, la_b = lame_species(P["E_bg"], P["nu_bg"])
        mu = mu + s * mu_b * bg
        lam = lam + s * la_b * bg
        eta = eta + P["eta_bg"] * bg
    return dict(K=K, rho_p=rho_p, rho_i=rho_i, mu=mu, lam=lam, eta=eta,
                Kbar=float(K.mean()), mubar=float(mu.mean()),
                lambar=float(lam.mean()), etabar=float(eta.mean()))


def elastic_force(grid, zeta, p, n):
    """Body force b = zeta tanh(p + n) grad(p + n)  (e:forcingfunction)."""
    tau = p + n
    t = np.tanh(tau)
    g = grid.grad(tau)
    return np.stack([zeta * t * g[a] for a in range(3)])


def single_species_reaction(P, dt, c_dag, c_dd, g, w, rho):
    """Reaction sub-step of the single-species model (Sec. 2.2, e:rd; Sec. 3,
    single-species splitting list).

    The tumour grows logistically, R = rho c (1 - c) (e:reac_op), with the
    growth rate rho = rho_w w + rho_g g frozen from the last refresh
    (e:reaction_op), integrated exactly over dt as in the multispecies step.
    Healthy tissue loses what the tumour gained in this step's diffusion and
    reaction sub-steps, split by g / (g + w) (e:gm, e:wm), so that c + g + w
    is conserved pointwise.

    c_dag: tumour after transport; c_dd: after diffusion.  Returns (c', g', w').
    """
    dD = c_dd - c_dag
    dR = logistic_flow(c_dd, rho, dt) - c_dd
    c1 = c_dd + dR
    s = dD + dR
    gw = g + w
    small = gw < 1e-12
    phig = np.where(small, 0.5, g / np.where(small, 1.0, gw))
    phiw = np.where(small, 0.5, w / np.where(small, 1.0, gw))
    return c1, g - phig * s, w - phiw * s
