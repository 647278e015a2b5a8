"""Semi-Lagrangian transport (Sec. 3), written from its description.

Characteristics, second order in time:
    X* = x - dt v(x),      X = x - dt/2 (v(x) + v(X*)).
Field values at the off-grid points X* and X come from cubic interpolation.
Reading (the paper says "cubic" and "third order in space"): tensor-product
cubic Lagrange interpolation on the 4 nodes floor(X/h) - 1 .. floor(X/h) + 2
per axis, periodic wrap, no prefilter.  Positions are handled in grid-index
units X/h.

Source term (Heun, Sec. 3): with nu_X = nu(X) and g(nu, x) = -nu div v(x)
(the conservative form d_t q + div(q v) = 0 written along characteristics),
    nu*   = nu_X + dt g(nu_X, X),
    nu+   = nu_X + dt/2 (g(nu_X, X) + g(nu*, x)).
Cerebrospinal fluid obeys the non-conservative transport and is only
interpolated.
"""
from __future__ import annotations

import numpy as np


def lagrange_weights(t):
    """Cubic Lagrange weights for nodes at -1, 0, 1, 2 and offset t in [0, 1)."""
    return (-t * (t - 1.0) * (t - 2.0) / 6.0,
            (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0,
            -(t + 1.0) * t * (t - 2.0) / 2.0,
            (t + 1.0) * t * (t - 1.0) / 6.0)


def interp(q, jx, jy, jz):
    """Tricubic Lagrange interpolation of the periodic field q at grid-index points."""
    n = q.shape[0]
    out = np.zeros(np.shape(jx), dtype=np.float64)
    idx, wts = [], []
    for j in (jx, jy, jz):
        base = np.floor(j)
        t = j - base
        b = base.astype(np.int64)
        idx.append([np.mod(b + o, n) for o in (-1, 0, 1, 2)])
        wts.append(lagrange_weights(t))
    (ix, iy, iz), (wx, wy, wz) = idx, wts
    for c in range(4):
        for b in range(4):
            for a in range(4):
                out += (wz[c] * wy[b] * wx[a]) * q[iz[c], iy[b], ix[a]]
    return out


def grid_indices(n):
    r = np.arange(n, dtype=np.float64)
    jz, jy, jx = np.meshgrid(r, r, r, indexing="ij")
    return jx, jy, jz


def _at(field, nodes):
    """Values of a grid field at integer grid nodes (all nodes when nodes is None)."""
    if nodes is None:
        return field
    jx, jy, jz = nodes
    return field[jz.astype(np.int64), jy.astype(np.int64), jx.astype(np.int64)]


def departure_points(grid, v, dt, nodes=None):
    """RK2 departure points X (grid-index units) for velocity v = (vx, vy, vz).

    nodes: optional (jx, jy, jz) integer grid-index arrays; the points are
    then computed for those arrival nodes only (same arithmetic)."""
    jx, jy, jz = grid_indices(grid.n) if nodes is None else nodes
    s = dt / grid.h
    v0 = [_at(v[a], nodes) for a in range(3)]
    xs = (jx - s * v0[0], jy - s * v0[1], jz - s * v0[2])
    vs = [interp(v[a], *xs) for a in range(3)]
    return (jx - 0.5 * s * (v0[0] + vs[0]),
            jy - 0.5 * s * (v0[1] + vs[1]),
            jz - 0.5 * s * (v0[2] + vs[2]))


def advect(grid, fields, v, dt, nodes=None):
    """One SL step: conservative transport of p, i, n, g, w; plain transport of f.

    nodes: optional (jx, jy, jz) integer grid-index arrays; the step is then
    evaluated at those arrival nodes only (same arithmetic as the whole grid)."""
    delta = grid.div(v)
    X = departure_points(grid, v, dt, nodes)
    delta_X = interp(delta, *X)
    delta_here = _at(delta, nodes)
    out = {}
    for name in ("p", "i", "n", "g", "w"):
        q_X = interp(fields[name], *X)
        g0 = -q_X * delta_X
        q_star = q_X + dt * g0
        g_star = -q_star * delta_here
        out[name] = q_X + 0.5 * dt * (g0 + g_star)
    out["f"] = interp(fields["f"], *X)
    return out
