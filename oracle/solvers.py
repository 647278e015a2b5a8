"""Krylov solvers of the split step (Sec. 3), written from their definitions.

* ``pcg``: textbook preconditioned conjugate gradients.  Stops when the
  recursively updated, unpreconditioned residual satisfies
  ||r|| <= rtol * ||b||.  A zero right-hand side returns x = 0 after zero
  iterations.  ``fixed_iters`` runs exactly that many iterations (used only
  to put two implementations in iteration lockstep).
* Crank-Nicolson diffusion (Sec. 3, CN equation):
  (1 - dt/2 D) c+ = (1 + dt/2 D) c-, D c = div(K grad c), solved by CG and
  preconditioned by the constant-coefficient CN operator built from the voxel
  mean of K, inverted spectrally.
* Screened variable-coefficient elasticity (Eqs. e:variable_elasticity,
  e:screening): the system is solved as (eta - L) u = -b, the SPD form of
  -eta u + L u = b.  The preconditioner is the constant-coefficient operator
  with voxel-mean mu, lambda, eta, inverted per Fourier mode by the
  Sherman-Morrison formula of Sec. 3 with the screening term added to its
  diagonal.  The paper uses GMRES; the operator is SPD under the Nyquist-free
  gradient, so CG is used.
"""
from __future__ import annotations

import numpy as np

from .spectral import dot, norm


def pcg(apply_a, apply_minv, b, x0, rtol, max_it, fixed_iters=None):
    """Preconditioned CG.  Returns (x, iterations, relative residual, converged)."""
    bnorm = norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0, True
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - apply_a(x)
    rnorm = norm(r)
    limit = max_it if fixed_iters is None else int(fixed_iters)
    if fixed_iters is None and rnorm <= rtol * bnorm:
        return x, 0, rnorm / bnorm, True
    z = apply_minv(r)
    p = z.copy()
    rz = dot(r, z)
    it = 0
    while it < limit:
        it += 1
        q = apply_a(p)
        alpha = rz / dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        rnorm = norm(r)
        if fixed_iters is None and rnorm <= rtol * bnorm:
            return x, it, rnorm / bnorm, True
        if it == limit:
            break
        z = apply_minv(r)
        rz_new = dot(r, z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    converged = fixed_iters is not None or rnorm <= rtol * bnorm
    return x, it, rnorm / bnorm, converged


# ---------------------------------------------------------------------------
# Diffusion (Eqs. e:diffusion_op, e:diffusion_tensor; Sec. 3 CN scheme)
# ---------------------------------------------------------------------------
def diffusion_op(grid, K, c):
    """D c = sum_a G_a (K G_a c)."""
    out = grid.deriv(K * grid.deriv(c, 0), 0)
    out += grid.deriv(K * grid.deriv(c, 1), 1)
    out += grid.deriv(K * grid.deriv(c, 2), 2)
    return out


def cn_matrix(grid, K, dt, c):
    """(1 - dt/2 D) c."""
    return c - 0.5 * dt * diffusion_op(grid, K, c)


def cn_rhs(grid, K, dt, c):
    """(1 + dt/2 D) c."""
    return c + 0.5 * dt * diffusion_op(grid, K, c)


def cn_precond(grid, Kbar, dt, r):
    """Inverse of the constant-coefficient CN operator with K = mean(K)."""
    return grid.ifft(grid.fft(r) / (1.0 + 0.5 * dt * Kbar * grid.w2))


def cn_diffusion(grid, K, Kbar, dt, c_minus, rtol, max_it, fixed_iters=None):
    """One Crank-Nicolson step of dc/dt = D c.  Returns (c+, iters, relres, converged)."""
    rhs = cn_rhs(grid, K, dt, c_minus)
    return pcg(lambda x: cn_matrix(grid, K, dt, x),
               lambda r: cn_precond(grid, Kbar, dt, r),
               rhs, c_minus, rtol, max_it, fixed_iters)


# ---------------------------------------------------------------------------
# Elasticity (Eqs. e:hook, e:variable_elasticity, e:screening; Sec. 3)
# ---------------------------------------------------------------------------
def strain_grads(grid, u):
    """g[a][b] = G_b u_a."""
    return [grid.grad(u[a]) for a in range(3)]


def stress(mu, lam, g):
    """sigma_ab = mu (G_b u_a + G_a u_b) + lambda delta_ab div u  (Hooke, e:hook)."""
    divu = g[0][0] + g[1][1] + g[2][2]
    s = [[None] * 3 for _ in range(3)]
    for a in range(3):
        for b in range(3):
            v = mu * (g[a][b] + g[b][a])
            if a == b:
                v = v + lam * divu
            s[a][b] = v
    return s


def elasticity_op(grid, mu, lam, eta, u):
    """(eta - L) u with L u = div(mu (grad u + grad u^T)) + grad(lambda div u)."""
    s = stress(mu, lam, strain_grads(grid, u))
    out = np.empty_like(u)
    for a in range(3):
        acc = eta * u[a]
        for b in range(3):
            acc = acc - grid.deriv(s[a][b], b)
        out[a] = acc
    return out


def elasticity_precond(grid, mubar, lambar, etabar, r):
    """Constant-coefficient inverse per mode (Sherman-Morrison, Sec. 3).

    For the symbol a I + c w w^T with a = eta + mu |w|^2 and c = lambda + mu:
    z = (1/a) [r - c w (w . r) / (a + c |w|^2)].  Modes with a = 0 map to 0.
    """
    rh = [grid.fft(r[b]) for b in range(3)]
    a_ = etabar + mubar * grid.w2
    c = lambar + mubar
    wr = grid.w[0] * rh[0] + grid.w[1] * rh[1] + grid.w[2] * rh[2]
    pos = a_ > 0
    inv_a = np.where(pos, 1.0 / np.where(pos, a_, 1.0), 0.0)
    den = np.where(pos, a_ + c * grid.w2, 1.0)
    out = np.empty_like(r)
    for b in range(3):
        out[b] = grid.ifft(inv_a * (rh[b] - c * grid.w[b] * wr / den))
    return out


def solve_elasticity(grid, mu, lam, eta, means, force, u0, rtol, max_it, fixed_iters=None):
    """Solve (eta - L) u = -b by PCG from u0.  ``means`` = (mubar, lambar, etabar).

    The screening must be positive somewhere (e:screening).  Without it the
    operator vanishes on every mode whose derivative symbols are all zero (the
    mean and the Nyquist corner modes, where the dropped Nyquist derivative
    leaves no stiffness) while the force has content there: no solution.
    """
    if not np.any(np.asarray(eta) > 0.0):
        raise ValueError("the elasticity needs screening: eta > 0 somewhere")
    mubar, lambar, etabar = means
    rhs = -np.asarray(force, dtype=np.float64)
    return pcg(lambda x: elasticity_op(grid, mu, lam, eta, x),
               lambda r: elasticity_precond(grid, mubar, lambar, etabar, r),
               rhs, u0, rtol, max_it, fixed_iters)
