"""One split step of the single-species reaction-diffusion model with mass
effect (Sec. 2.2, e:rd; Sec. 3, single-species splitting list), n -> n+1:

  S1  semi-Lagrangian transport of (c, g, w) (conservative) and f (plain)
      with the velocity u_t^n = (u^n - u^{n-1}) / dt;
  S2  Crank-Nicolson diffusion of c with the refreshed K;
  S3  reaction of (c, g, w) (reaction.single_species_reaction);
  S4  refresh of K, rho, the Lame fields and eta, the tumour species being c;
  S5  screened elasticity with the force b = zeta tanh(c) grad c (e:force);
  S6  u^{n-1} <- u^n, u^n <- u^{n+1}.

The state is the multispecies one (model.State) with c in the p slot and
i = n = l = 0, o = o_heal kept constant: the refresh and force formulas of the
multispecies model (tumour = p + i + n) then reduce exactly to the
single-species ones.  Readings as in the multispecies step (Lie splitting in
the listed order, u^0 = u^{-1} = 0, exact logistic flow, one refresh per
step after the reaction, K = k_w w + k_g g + k_f f with k_f = 0).
cfg["strang"] selects the symmetric form as in the multispecies step: S1
over dt/2 and a refresh before S2, S1 over dt/2 again after S3.
"""
from __future__ import annotations

import numpy as np

from . import reaction as rx
from . import solvers
from . import transport
from .model import DEFAULT_CFG, FIELDS, State, init_state, strang_halves, transport_half  # noqa: F401


def step(st: State, cfg=None, forced=None):
    c = dict(DEFAULT_CFG)
    if cfg:
        c.update(cfg)
    P, grid, dt = st.P, st.grid, c["dt"]
    F, coef = st.f, st.coef
    fx = forced if forced is not None else (None, None, None, None)

    v = (st.u - st.u_prev) / dt
    half = strang_halves(c)
    if half:
        adv, coef = transport_half(grid, P, F, v, dt, st.bg)
    elif c["advection"]:
        adv = transport.advect(grid, F, v, dt)
    else:
        adv = {k: F[k].copy() for k in ("p", "i", "n", "g", "w", "f")}

    c_dd, it_d, rr_d, ok = solvers.cn_diffusion(grid, coef["K"], coef["Kbar"], dt, adv["p"],
                                                c["rtol_diff"], c["max_it"], fx[0])
    conv = ok
    c1, g1, w1 = rx.single_species_reaction(P, dt, adv["p"], c_dd, adv["g"], adv["w"], coef["rho_p"])
    f1 = adv["f"]
    n1 = adv["n"]
    if half:
        back = transport.advect(grid, dict(p=c1, i=F["i"], n=n1, g=g1, w=w1, f=f1), v, 0.5 * dt)
        c1, n1, g1, w1, f1 = (back[k] for k in ("p", "n", "g", "w", "f"))
    z = np.zeros_like(c1)
    coef = rx.refresh(P, c1, z, z, g1, w1, f1, bg=st.bg)
    ie, re_ = 0, 0.0
    if c["elasticity"]:
        force = rx.elastic_force(grid, P["zeta"], c1, z)
        u_new, ie, re_, ok = solvers.solve_elasticity(
            grid, coef["mu"], coef["lam"], coef["eta"],
            (coef["mubar"], coef["lambar"], coef["etabar"]), force, st.u,
            c["rtol_elast"], c["max_it"], fx[3])
        conv &= ok
    else:
        u_new = st.u.copy()
    st.u_prev, st.u = st.u, u_new
    st.f = dict(p=c1, i=F["i"], n=n1, o=F["o"], l=F["l"], g=g1, w=w1, f=f1)
    st.coef = coef
    st.nstep += 1
    h3 = grid.h ** 3
    return dict(it_diff=[it_d, 0, 0], relres_diff=[rr_d, 0.0, 0.0], it_elast=ie, relres_elast=re_,
                converged=conv, mass={k: float(st.f[k].sum() * h3) for k in FIELDS})
