"""Pins for the oracle's mass-effect diagnostics (Sec. 3, e:princ_stress,
e:jacobian; Sec. 4 grid-search scalars) from closed forms."""
import numpy as np
import pytest

from oracle import diagnostics as dg
from oracle.spectral import Grid

N = 16
MU, LAM = 750.0, 3000.0


def _coords(g):
    r = np.arange(g.n) * g.h
    z, y, x = np.meshgrid(r, r, r, indexing="ij")
    return x, y, z


def _diag(u, centers=np.zeros((0, 3)), threshold=0.1):
    g = Grid(N)
    return g, dg.diagnose(g, np.full((N, N, N), MU), np.full((N, N, N), LAM), u, centers, threshold)


def test_rigid_translation_has_no_stress_and_unit_jacobian():
    u = np.stack([np.full((N, N, N), c) for c in (0.3, -0.2, 0.1)])
    g, (f, s) = _diag(u)
    assert np.abs(f["trace"]).max() < 1e-12 and np.abs(f["shear"]).max() < 1e-12
    assert np.abs(f["jac"] - 1.0).max() < 1e-14 and s["jac_l2"] < 1e-12


@pytest.mark.parametrize("k", [1, 3])
def test_uniaxial_mode(k):
    eps = 0.01
    g = Grid(N)
    x, y, z = _coords(g)
    u = np.stack([eps * np.sin(k * x), 0 * x, 0 * x])
    g, (f, s) = _diag(u)
    fxx = eps * k * np.cos(k * x)
    assert np.abs(f["jac"] - (1.0 + fxx)).max() < 1e-13
    assert np.abs(f["trace"] - (2 * MU + 3 * LAM) * fxx).max() < 1e-9
    assert np.abs(f["shear"] - MU * np.abs(fxx)).max() < 1e-10
    # sum over a full period of cos^2 is N/2 per line: ||J - 1|| = eps k sqrt(4 pi^3)
    assert abs(s["jac_l2"] - eps * k * np.sqrt(4 * np.pi ** 3)) < 1e-12


def test_pure_shear_keeps_volume():
    eps = 0.02
    g = Grid(N)
    x, y, z = _coords(g)
    u = np.stack([eps * np.sin(2 * y), 0 * x, 0 * x])
    g, (f, s) = _diag(u)
    fxy = 2 * eps * np.cos(2 * y)
    assert np.abs(f["jac"] - 1.0).max() < 1e-14
    assert np.abs(f["trace"]).max() < 1e-10
    assert np.abs(f["shear"] - MU * np.abs(fxy)).max() < 1e-10


def test_diagonal_deformation_jacobian_and_stresses():
    eps = 0.05
    g = Grid(N)
    x, y, z = _coords(g)
    u = np.stack([eps * np.sin(x), eps * np.sin(y), eps * np.sin(z)])
    g, (f, s) = _diag(u)
    c = [eps * np.cos(q) for q in (x, y, z)]
    assert np.abs(f["jac"] - (1 + c[0]) * (1 + c[1]) * (1 + c[2])).max() < 1e-13
    assert np.abs(f["trace"] - (2 * MU + 3 * LAM) * (c[0] + c[1] + c[2])).max() < 1e-9
    assert np.abs(f["shear"] - MU * np.abs(c[0] - c[1])).max() < 1e-10


def test_cyclic_shear_exercises_the_off_diagonal_cofactors():
    # F_xy = a, F_yz = b, F_zx = c and nothing else: det(I + F) = 1 + a b c
    eps = 0.3
    g = Grid(N)
    x, y, z = _coords(g)
    u = np.stack([eps * np.sin(y), eps * np.sin(z), eps * np.sin(x)])
    g, (f, s) = _diag(u)
    a, b, c = eps * np.cos(y), eps * np.cos(z), eps * np.cos(x)
    assert np.abs(f["jac"] - (1.0 + a * b * c)).max() < 1e-13
    # the transposed pattern gives the other triple product term
    u2 = np.stack([eps * np.sin(z), eps * np.sin(x), eps * np.sin(y)])
    g, (f2, s2) = _diag(u2)
    a2, b2, c2 = eps * np.cos(z), eps * np.cos(x), eps * np.cos(y)   # F_xz, F_yx, F_zy
    assert np.abs(f2["jac"] - (1.0 + a2 * b2 * c2)).max() < 1e-13


def test_d_max_of_a_gaussian_displacement():
    g = Grid(32)
    n, h = g.n, g.h
    r = np.arange(n) * h
    z, y, x = np.meshgrid(r, r, r, indexing="ij")
    c = np.array([10.0, 15.0, 20.0]) * h           # on a node: the peak |u| is exactly A
    d2 = 0.0
    for q, cq in ((x, c[0]), (y, c[1]), (z, c[2])):
        d = q - cq
        d = d - 2 * np.pi * np.round(d / (2 * np.pi))
        d2 = d2 + d * d
    A, s_w, thr = 3.0 * h, 0.6, 0.1
    u = np.stack([A * np.exp(-d2 / (2 * s_w ** 2)), 0 * x, 0 * x])
    f, s = dg.diagnose(g, np.full((n, n, n), MU), np.full((n, n, n), LAM), u, c[None, :], thr)
    R = s_w * np.sqrt(2 * np.log(A / (thr * h))) / h       # radius of the 0.1-voxel contour, in voxels
    assert R - np.sqrt(3) / 2 <= s["d_max"] <= R + 1e-9
    assert abs(s["max_disp"] - 3.0) < 1e-12
    # a second, far seed only shortens distances
    f2, s2 = dg.diagnose(g, np.full((n, n, n), MU), np.full((n, n, n), LAM), u,
                         np.stack([c, c + np.pi]), thr)
    assert s2["d_max"] <= s["d_max"] + 1e-12
