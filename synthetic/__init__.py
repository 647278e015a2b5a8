"""Seeded synthetic inputs for the multispecies glioblastoma split step.

This module is shared by the CPU oracle and the GPU path as a source of
*inputs only*: tissue probability maps, tumour-seed geometry and parameter
values.  It holds none of the method's arithmetic (no operator, no solver,
no reaction term, no Lame mixing); every derived quantity is computed by
each side on its own.

Recipe (stand-in for the BrainWeb atlas of Sec. 4, which is not available):

* three N(0,1) fields from ``numpy.random.default_rng(seed)``, each smoothed
  in Fourier space by exp(-sigma_c^2 |k_cell|^2 / 2) with sigma_c in cells,
  standardised to zero mean and unit standard deviation, then combined by a
  softmax into white matter, gray matter and CSF (they sum to 1 per voxel);
* tumour seeds drawn from ``default_rng(seed + 1000)``: one blob (width 0.3,
  weight 0.5) for the small case, three blobs (width ~ U(0.1, 0.3), weight
  0.5) for the large forward cases, and a 4x4x4 lattice of width-0.2 blobs
  spaced 0.4 apart with weights ~ U(0, 0.5) for the adjoint cases.

Parameter values follow Table t:setup (Sec. 2.5) with the overrides that the
workloads name (k_g = 0.01, rho = 10 in both tissues, alpha_0 = 1,
o_hypoxia = 0.5, Poisson ratio 0.4 for white and gray matter).
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi

# Table t:setup (Sec. 2.5) values, plus the few constants the model needs that
# the table leaves out (o_heal, the invasive-rate fraction, the Heaviside
# width, the Lame scale and a CSF diffusion coefficient).
TABLE_SETUP = dict(
    k_w=0.1, k_g=0.0, k_f=0.0,
    rho_w=8.0, rho_g=0.0, rho_inv_frac=0.1,          # rho_w^i = 0.8 = 0.1 * rho_w
    alpha0=0.15, beta0=0.02, gamma=1.0, sigma_b=0.9,
    o_hyp=0.65, o_inv=0.7, o_heal=1.0, delta_s=55.0, delta_p=8.0,
    delta_e=40.0, delta_half=0.01, delta_l=80.0,
    eta_tumor=0.0, eta_healthy=1.0e4,
    E_wm=2100.0, E_gm=2100.0, E_csf=100.0, E_tumor=2100.0,
    nu_wm=0.3, nu_gm=0.3, nu_csf=0.1, nu_tumor=0.45,
    lame_scale=1.0, zeta=4.0e4,
    heaviside_eps=0.01,
    E_bg=15000.0, nu_bg=0.48, eta_bg=1.0e6,          # background material (fictitious domain)
)

# Overrides shared by every synthetic workload.
WORKLOAD_OVERRIDES = dict(
    k_w=0.1, k_g=0.01, rho_w=10.0, rho_g=10.0, alpha0=1.0, o_hyp=0.5,
    nu_wm=0.4, nu_gm=0.4, nu_csf=0.1,
)

PARAM_ORDER = tuple(TABLE_SETUP.keys())

# The five workloads: grid size, precision, step count, tissue smoothing
# width (cells), tumour-seed recipe.
WORKLOADS = {
    "seed1_n32": dict(seed=0, n=32, precision="fp64", steps=10, sigma_cells=2.0, seeds="single"),
    "seeds3_n128": dict(seed=1, n=128, precision="fp64", steps=100, sigma_cells=4.0, seeds="three"),
    "seeds3_n256": dict(seed=2, n=256, precision="mixed", steps=100, sigma_cells=8.0, seeds="three"),
    "lattice_n128": dict(seed=3, n=128, precision="fp64", steps=50, sigma_cells=4.0, seeds="lattice"),
    "lattice_n256": dict(seed=4, n=256, precision="mixed", steps=200, sigma_cells=8.0, seeds="lattice"),
}


def params(**overrides) -> dict:
    """Parameter dictionary: Table t:setup, workload overrides, then ``overrides``."""
    p = dict(TABLE_SETUP)
    p.update(WORKLOAD_OVERRIDES)
    for k, v in overrides.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k!r}")
        p[k] = float(v)
    return p


def tissue_maps(n: int, sigma_cells: float, seed: int):
    """White matter, gray matter and CSF probability maps, shape (n, n, n), [z][y][x].

    Softmax of three standardised, Gaussian-smoothed N(0,1) fields.  Returns
    float64 C-contiguous arrays that sum to one in every voxel.
    """
    rng = np.random.default_rng(seed)
    raw = rng.standard_normal((3, n, n, n))
    m = np.fft.fftfreq(n, d=1.0 / n)                   # integer mode numbers
    mr = np.arange(n // 2 + 1, dtype=np.float64)
    kc2 = ((TWO_PI / n) ** 2) * (m[:, None, None] ** 2 + m[None, :, None] ** 2 + mr[None, None, :] ** 2)
    filt = np.exp(-0.5 * sigma_cells ** 2 * kc2)
    sm = np.empty_like(raw)
    for c in range(3):
        s = np.fft.irfftn(np.fft.rfftn(raw[c]) * filt, s=(n, n, n), axes=(0, 1, 2))
        s -= s.mean()
        s /= s.std()
        sm[c] = s
    sm -= sm.max(axis=0, keepdims=True)
    e = np.exp(sm)
    e /= e.sum(axis=0, keepdims=True)
    wm, gm, csf = (np.ascontiguousarray(e[c]) for c in range(3))
    return wm, gm, csf


def tumor_seeds(kind: str, seed: int):
    """Seed centres (k, 3) as (x, y, z) in [0, 2pi), widths (k,), weights (k,)."""
    rng = np.random.default_rng(seed + 1000)
    if kind == "single":
        c = rng.uniform(0.0, TWO_PI, size=(1, 3))
        return c, np.array([0.3]), np.array([0.5])
    if kind == "three":
        c = rng.uniform(0.0, TWO_PI, size=(3, 3))
        s = rng.uniform(0.1, 0.3, size=3)
        return c, s, np.full(3, 0.5)
    if kind == "lattice":
        centre = rng.uniform(0.0, TWO_PI, size=3)
        off = (np.arange(4) - 1.5) * 0.4
        gz, gy, gx = np.meshgrid(off, off, off, indexing="ij")
        c = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1) + centre[None, :]
        c = np.mod(c, TWO_PI)
        w = rng.uniform(0.0, 0.5, size=64)
        return c, np.full(64, 0.2), w
    raise ValueError(kind)


BRAIN_SEMI_AXES = (0.80 * math.pi, 0.92 * math.pi, 0.72 * math.pi)   # (x, y, z), centred at (pi, pi, pi)


def brain_mask(n: int, width_cells: float = 2.0):
    """Smooth ellipsoidal brain mask in (0, 1): 1/2 (1 - tanh(d / (width h))),
    d = (r - 1) min(semi-axes) with r the ellipsoidal radius about the centre."""
    h = TWO_PI / n
    c = np.arange(n) * h - math.pi
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    a, b, cz = BRAIN_SEMI_AXES
    r = np.sqrt((x / a) ** 2 + (y / b) ** 2 + (z / cz) ** 2)
    d = (r - 1.0) * min(BRAIN_SEMI_AXES)
    return 0.5 * (1.0 - np.tanh(d / (width_cells * h)))


def workload_inputs(name: str, n: int | None = None, masked: bool = False):
    """All inputs of a named workload (optionally at another grid size).

    masked: fictitious domain with a brain mask m (brain_mask): the tissue
    maps are multiplied by m, the background fraction bg = 1 - m is returned
    under "bg", and the tumour seeds are pulled towards the centre
    (c -> pi + 0.35 (c - pi)) so that they lie inside the brain."""
    wl = WORKLOADS[name]
    nn = wl["n"] if n is None else int(n)
    wm, gm, csf = tissue_maps(nn, wl["sigma_cells"], wl["seed"])
    centers, sigmas, weights = tumor_seeds(wl["seeds"], wl["seed"])
    out = dict(n=nn, wm=wm, gm=gm, csf=csf, centers=centers, sigmas=sigmas,
               weights=weights, steps=wl["steps"], precision=wl["precision"],
               dt=0.01, rtol=1e-8)
    if masked:
        m = brain_mask(nn)
        out.update(wm=wm * m, gm=gm * m, csf=csf * m, bg=1.0 - m,
                   centers=math.pi + 0.35 * (np.asarray(centers) - math.pi))
    return out


def random_field(n: int, seed: int, smooth_cells: float = 0.0, ncomp: int | None = None):
    """Generic seeded test field(s): N(0,1), optionally Gaussian-smoothed."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n) if ncomp is None else (ncomp, n, n, n)
    x = rng.standard_normal(shape)
    if smooth_cells > 0:
        m = np.fft.fftfreq(n, d=1.0 / n)
        mr = np.arange(n // 2 + 1, dtype=np.float64)
        kc2 = ((TWO_PI / n) ** 2) * (m[:, None, None] ** 2 + m[None, :, None] ** 2 + mr[None, None, :] ** 2)
        filt = np.exp(-0.5 * smooth_cells ** 2 * kc2)
        x = np.fft.irfftn(np.fft.rfftn(x, axes=(-3, -2, -1)) * filt, s=(n, n, n), axes=(-3, -2, -1))
    return np.ascontiguousarray(x)
