"""Mass-effect diagnostics of a displacement field (Sec. 3, after e:jacobian;
Sec. 4, grid search over eta_healthy and zeta).

For a displacement u with displacement gradient F_ab = G_b u_a (spectral
first derivatives, Nyquist mode dropped, as everywhere in the oracle):

* stress (Hooke, e:hook): T = lambda tr(E) I + 2 mu E, E = (F + F^T) / 2;
  the paper visualises principal stresses by the stress trace tr T;
* maximum shear stress from Mohr's circle (e:princ_stress), in the x-y plane
  as the paper writes it: tau = sqrt(((T_xx - T_yy) / 2)^2 + T_xy^2);
* Jacobian of the deformation (e:jacobian): J = det(I + F);
* scalars of the grid search: the L2 norm of J - 1 over the domain,
  sqrt(h^3 sum (J - 1)^2), and d_max, the largest distance (in voxels) from
  the initial tumour seed of the points where |u| reaches `threshold` voxels.

Readings: with several seeds the distance is to the nearest seed (one seed
gives the paper's definition); distances are periodic minimum-image
distances on [0, 2 pi)^3; the L2 norm is taken of J - 1 (J = 1 without
deformation), the paper's "re-scaled" Jacobian being unspecified.
"""
from __future__ import annotations

import numpy as np


def displacement_gradient(grid, u):
    """F[a][b] = G_b u_a."""
    return [[grid.deriv(u[a], b) for b in range(3)] for a in range(3)]


def stress_tensor(mu, lam, F):
    """T_ab = mu (F_ab + F_ba) + lambda delta_ab tr F."""
    tr = F[0][0] + F[1][1] + F[2][2]
    return [[mu * (F[a][b] + F[b][a]) + (lam * tr if a == b else 0.0) for b in range(3)] for a in range(3)]


def jacobian(F):
    """det(I + F) by cofactor expansion along the first row."""
    a = [[F[i][j] + (1.0 if i == j else 0.0) for j in range(3)] for i in range(3)]
    return (a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1])
            - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0])
            + a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]))


def max_shear(T):
    """Mohr's circle in the x-y plane."""
    return np.sqrt((0.5 * (T[0][0] - T[1][1])) ** 2 + T[0][1] ** 2)


def seed_distance(grid, centers):
    """Periodic distance (length units) from every node to the nearest centre."""
    n = grid.n
    r = np.arange(n) * grid.h
    z, y, x = np.meshgrid(r, r, r, indexing="ij")
    best = np.full((n, n, n), np.inf)
    L = 2.0 * np.pi
    for c in np.atleast_2d(centers):
        d2 = 0.0
        for q, cq in ((x, c[0]), (y, c[1]), (z, c[2])):
            d = q - cq
            d = d - L * np.round(d / L)
            d2 = d2 + d * d
        best = np.minimum(best, np.sqrt(d2))
    return best


def diagnose(grid, mu, lam, u, centers, threshold=0.1):
    """Fields (trace, tau_max, J) and the scalar summary of a displacement."""
    F = displacement_gradient(grid, u)
    T = stress_tensor(mu, lam, F)
    trace = T[0][0] + T[1][1] + T[2][2]
    tau = max_shear(T)
    J = jacobian(F)
    h = grid.h
    umag = np.sqrt((u ** 2).sum(axis=0)) / h
    if len(np.atleast_2d(centers)) and np.atleast_2d(centers).shape[1] == 3:
        dist = seed_distance(grid, centers) / h
        mask = umag >= threshold
        d_max = float(dist[mask].max()) if mask.any() else 0.0
    else:
        d_max = 0.0
    scalars = dict(max_disp=float(umag.max()), trace_min=float(trace.min()), trace_max=float(trace.max()),
                   shear_max=float(tau.max()), jac_min=float(J.min()), jac_max=float(J.max()),
                   jac_l2=float(np.sqrt(h ** 3 * ((J - 1.0) ** 2).sum())), d_max=d_max)
    return dict(trace=trace, shear=tau, jac=J), scalars
