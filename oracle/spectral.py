"""Fourier pseudo-spectral operators on the 2*pi-periodic cube.

Sec. 3 places the brain in a cubic box (fictitious domain) discretised by a
uniform grid and uses pseudo-spectral derivatives.  The box is [0, 2*pi)^3,
so wave numbers are integers.  Arrays are indexed [z][y][x] (x fastest);
vector fields are stacked as (u_x, u_y, u_z).

Reading (the paper is silent): the first-derivative multiplier i*w drops the
Nyquist mode (w(-N/2) := 0).  This keeps every derivative real and exactly
skew-symmetric, so the diffusion and elasticity operators are symmetric and
CG applies.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft


def _workers() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


class Grid:
    """Uniform N^3 grid on [0, 2*pi)^3 with spectral derivatives."""

    def __init__(self, n: int):
        if n < 4 or n % 2:
            raise ValueError("grid size must be even and >= 4")
        self.n = n
        self.h = 2.0 * np.pi / n
        m = np.fft.fftfreq(n, d=1.0 / n)
        m[n // 2] = 0.0
        mr = np.arange(n // 2 + 1, dtype=np.float64)
        mr[n // 2] = 0.0
        self.wx = mr[None, None, :]
        self.wy = m[None, :, None]
        self.wz = m[:, None, None]
        self.w = (self.wx, self.wy, self.wz)
        self.w2 = self.wx ** 2 + self.wy ** 2 + self.wz ** 2
        self.workers = _workers()

    # -- transforms -------------------------------------------------------
    def fft(self, c):
        return sfft.rfftn(c, workers=self.workers)

    def ifft(self, ch):
        n = self.n
        return sfft.irfftn(ch, s=(n, n, n), workers=self.workers)

    # -- derivatives ------------------------------------------------------
    def deriv(self, c, a: int):
        """G_a c = F^-1 (i w_a F c), a = 0, 1, 2 for x, y, z."""
        return self.ifft(1j * self.w[a] * self.fft(c))

    def grad(self, c):
        ch = self.fft(c)
        return [self.ifft(1j * self.w[a] * ch) for a in range(3)]

    def div(self, v):
        return self.deriv(v[0], 0) + self.deriv(v[1], 1) + self.deriv(v[2], 2)

    # -- geometry ---------------------------------------------------------
    def axis(self):
        return self.h * np.arange(self.n, dtype=np.float64)

    def coords(self):
        """Node coordinates (X, Y, Z), each (n, n, n) indexed [z][y][x]."""
        x = self.axis()
        z3, y3, x3 = np.meshgrid(x, x, x, indexing="ij")
        return x3, y3, z3


def dot(a, b) -> float:
    """Euclidean inner product over all voxels (and components)."""
    return float(np.vdot(np.ravel(a), np.ravel(b)).real)


def norm(a) -> float:
    return float(np.sqrt(dot(a, a)))
