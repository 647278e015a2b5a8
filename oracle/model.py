"""Initial condition and one operator-split step of the multispecies model.

The step follows the multispecies splitting list of Sec. 3 in its listed
(sequential) order, n -> n+1:

  S1  semi-Lagrangian transport of (p, i, n, g, w) (conservative) and f
      (plain) with the current velocity u_t^n = (u^n - u^{n-1}) / dt;
  S2  Crank-Nicolson diffusion of i and o (and of the edema l, Sec. 2.4);
  S3  explicit reaction of (p, i, n, g, w) with the diffused oxygen;
  S4  explicit oxygen reaction, then the edema source/drainage;
  S5  refresh of the reaction, diffusion and elasticity coefficients;
  S6  screened elasticity with the force of e:forcingfunction;
  S7  u^{n-1} <- u^n, u^n <- u^{n+1} (backward-difference velocity).

Readings: the paper calls the splitting "Strang" but lists the sub-steps
sequentially and reports first-order convergence, so the listed order is
used once per step (Lie).  cfg["strang"] selects the symmetric variant: S1
over dt/2, a refresh of the half-transported state (its K, rho and means
drive S2 and S3), S2-S4 over dt, S1 again over dt/2 with the same velocity,
then S5-S7.  Oxygen and edema are not transported in either form.  Displacement starts undeformed, u^0 = u^{-1} = 0.
Coefficients used by S2, S3 (and the means used by the preconditioners)
come from the most recent refresh (from q^0 at initialisation).  The
initial tumour is p_0 = Phi w with unnormalised periodic Gaussians
phi_k = exp(-d(x, c_k)^2 / (2 sigma_k^2)), d the minimum-image distance;
i_0 = n_0 = l_0 = 0 and o_0 = o_heal.
"""
from __future__ import annotations

import numpy as np

from . import reaction as rx
from . import solvers
from . import transport
from .spectral import Grid

FIELDS = ("p", "i", "n", "o", "l", "g", "w", "f")


def periodic_delta(d):
    return d - 2.0 * np.pi * np.round(d / (2.0 * np.pi))


def gaussian_basis(grid, centers, sigmas, weights):
    """p_0 = sum_k w_k phi_k (the initial-condition parameterisation of e:gog)."""
    x = grid.axis()
    out = np.zeros((grid.n,) * 3)
    for c, s, wk in zip(np.asarray(centers, float), np.asarray(sigmas, float),
                        np.asarray(weights, float)):
        dx = periodic_delta(x - c[0])
        dy = periodic_delta(x - c[1])
        dz = periodic_delta(x - c[2])
        d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
        out += wk * np.exp(-d2 / (2.0 * s * s))
    return out


class State:
    """Species, displacement history and the coefficients of the last refresh."""

    def __init__(self, grid, P, fields, u, u_prev, bg=None):
        self.grid = grid
        self.P = P
        self.f = fields
        self.u = u
        self.u_prev = u_prev
        self.bg = bg          # static background-material fraction, or None
        self.coef = rx.refresh(P, *(fields[k] for k in ("p", "i", "n", "g", "w", "f")), bg=bg)
        self.nstep = 0

    def copy(self):
        s = State.__new__(State)
        s.grid, s.P = self.grid, self.P
        s.f = {k: v.copy() for k, v in self.f.items()}
        s.u, s.u_prev = self.u.copy(), self.u_prev.copy()
        s.bg = None if self.bg is None else self.bg.copy()
        s.coef = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in self.coef.items()}
        s.nstep = self.nstep
        return s


def init_state(P, n, wm, gm, csf, centers, sigmas, weights, bg=None):
    grid = Grid(n)
    p0 = gaussian_basis(grid, centers, sigmas, weights)
    z = np.zeros((n, n, n))
    fields = dict(p=p0, i=z.copy(), n=z.copy(), o=np.full((n, n, n), P["o_heal"]),
                  l=z.copy(), g=np.array(gm, float), w=np.array(wm, float),
                  f=np.array(csf, float))
    u = np.zeros((3, n, n, n))
    return State(grid, P, fields, u, u.copy(), None if bg is None else np.array(bg, float))


DEFAULT_CFG = dict(dt=0.01, rtol_diff=1e-8, rtol_elast=1e-8, max_it=1000,
                   edema=True, elasticity=True, advection=True, strang=False)


def strang_halves(c):
    """True when the step is the symmetric form: transport over dt/2 before and
    after the diffusion-reaction stage (only meaningful with advection on)."""
    return bool(c["strang"]) and bool(c["advection"])


def transport_half(grid, P, fields, v, dt, bg):
    """The dt/2 transport of the symmetric form and the refresh of its result."""
    adv = transport.advect(grid, fields, v, 0.5 * dt)
    return adv, rx.refresh(P, adv["p"], adv["i"], adv["n"], adv["g"], adv["w"], adv["f"], bg=bg)


def step(st: State, cfg=None, forced=None, tape=None):
    """Advance ``st`` by one split step in place.  Returns a stats dict.

    ``forced``: optional list of four iteration counts (i, o, l diffusion and
    elasticity) to run each solve for exactly that many iterations.
    ``tape``: optional dict that receives the step's intermediates (for the
    discrete adjoint).
    """
    c = dict(DEFAULT_CFG)
    if cfg:
        c.update(cfg)
    P, grid, dt = st.P, st.grid, c["dt"]
    F, coef = st.f, st.coef
    F_coef0 = coef
    fx = forced if forced is not None else (None, None, None, None)
    half = strang_halves(c)
    if half and tape is not None:
        raise ValueError("the discrete adjoint covers the sequential (Lie) step only")

    # S1: transport with the backward-difference velocity.
    v = (st.u - st.u_prev) / dt
    if half:
        adv, coef = transport_half(grid, P, F, v, dt, st.bg)
    elif c["advection"]:
        adv = transport.advect(grid, F, v, dt)
    else:
        adv = {k: F[k].copy() for k in ("p", "i", "n", "g", "w", "f")}

    # S2: Crank-Nicolson diffusion of i, o (and l) with the refreshed K.
    it = [0, 0, 0]
    rr = [0.0, 0.0, 0.0]
    conv = True
    i_dd, it[0], rr[0], ok = solvers.cn_diffusion(grid, coef["K"], coef["Kbar"], dt, adv["i"],
                                                  c["rtol_diff"], c["max_it"], fx[0])
    conv &= ok
    o_dag, it[1], rr[1], ok = solvers.cn_diffusion(grid, coef["K"], coef["Kbar"], dt, F["o"],
                                                   c["rtol_diff"], c["max_it"], fx[1])
    conv &= ok
    if c["edema"]:
        l_dag, it[2], rr[2], ok = solvers.cn_diffusion(grid, coef["K"], coef["Kbar"], dt, F["l"],
                                                       c["rtol_diff"], c["max_it"], fx[2])
        conv &= ok
    else:
        l_dag = F["l"].copy()
    dD = i_dd - adv["i"]

    # S3: species reaction with the diffused oxygen and frozen growth rates.
    p1, i1, n1, g1, w1 = rx.species_reaction(P, dt, adv["p"], i_dd, adv["n"], adv["g"], adv["w"],
                                             o_dag, coef["rho_p"], coef["rho_i"], dD)
    # S4: oxygen, then edema.
    o1 = rx.oxygen_reaction(P, dt, o_dag, p1, g1, w1)
    l1 = rx.edema_reaction(P, dt, l_dag, i1) if c["edema"] else l_dag
    f1 = adv["f"]
    if half:
        # second transport half-step, same velocity
        back = transport.advect(grid, dict(p=p1, i=i1, n=n1, g=g1, w=w1, f=f1), v, 0.5 * dt)
        p1, i1, n1, g1, w1, f1 = (back[k] for k in ("p", "i", "n", "g", "w", "f"))
    # S5: refresh.
    coef = rx.refresh(P, p1, i1, n1, g1, w1, f1, bg=st.bg)
    # S6: elasticity.
    ie, re_ = 0, 0.0
    if c["elasticity"]:
        force = rx.elastic_force(grid, P["zeta"], p1, n1)
        u_new, ie, re_, ok = solvers.solve_elasticity(
            grid, coef["mu"], coef["lam"], coef["eta"],
            (coef["mubar"], coef["lambar"], coef["etabar"]), force, st.u,
            c["rtol_elast"], c["max_it"], fx[3])
        conv &= ok
    else:
        u_new = st.u.copy()
    if tape is not None:
        tape.update(v=v, adv=adv, i_dd=i_dd, o_dag=o_dag, l_dag=l_dag, coef0=F_coef0,
                    p1=p1, i1=i1, n1=n1, g1=g1, w1=w1, o1=o1, l1=l1, coef1=coef,
                    u_new=u_new, u=st.u, u_prev=st.u_prev, F0={k: F[k] for k in F}, bg=st.bg)
    # S7: rotate.
    st.u_prev, st.u = st.u, u_new
    st.f = dict(p=p1, i=i1, n=n1, o=o1, l=l1, g=g1, w=w1, f=f1)
    st.coef = coef
    st.nstep += 1
    h3 = grid.h ** 3
    return dict(it_diff=it, relres_diff=rr, it_elast=ie, relres_elast=re_, converged=conv,
                mass={k: float(st.f[k].sum() * h3) for k in FIELDS},
                max_disp=float(np.sqrt((u_new ** 2).sum(axis=0)).max()),
                max_cfl=float(np.abs(v).max() * dt / grid.h))


def run(P, inputs, steps, cfg=None, forced=None):
    """Initialise from a ``synthetic.workload_inputs`` dict and take ``steps`` steps."""
    st = init_state(P, inputs["n"], inputs["wm"], inputs["gm"], inputs["csf"],
                    inputs["centers"], inputs["sigmas"], inputs["weights"], inputs.get("bg"))
    stats = []
    for k in range(steps):
        stats.append(step(st, cfg, None if forced is None else forced[k]))
    return st, stats
