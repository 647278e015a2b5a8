"""Plain FP64 CPU oracle for the operator-split multispecies glioblastoma step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP path; the only
common module is ``synthetic`` (seeded inputs, no method arithmetic).

It follows Subramanian, Gholami & Biros, "Simulation of glioblastoma growth
using a 3D multispecies tumor model with mass effect" (arXiv 1810.05370):

* ``spectral``  -- Fourier pseudo-spectral derivatives on the periodic cube
  (Sec. 3, fictitious domain with a uniform grid);
* ``solvers``   -- preconditioned CG, Crank-Nicolson diffusion with the
  mean-coefficient spectral preconditioner, screened variable-coefficient
  elasticity with the constant-Lame Sherman-Morrison preconditioner (Sec. 3);
* ``transport`` -- semi-Lagrangian RK2 characteristics, tricubic Lagrange
  interpolation and the Heun source update (Sec. 3);
* ``reaction``  -- go-or-grow reaction, necrosis, oxygen, edema and the
  coefficient refresh (Sec. 2.3, 2.4, Eqs. e:gog, e:death, e:gog_reac_op,
  e:alpha, e:beta, e:edema, e:lame, e:diffusion_tensor, e:reaction_op);
* ``model``     -- initial condition and the split step in the order of the
  multispecies splitting list of Sec. 3;
* ``adjoint``   -- the discrete adjoint of the split step (the paper lists
  adjoint-based inversion as future work in Sec. 5);
* ``diagnostics`` -- stress trace, Mohr maximum shear, deformation Jacobian and
  the grid-search scalars (Sec. 3, e:princ_stress, e:jacobian; Sec. 4);
* ``model_single`` -- the split step of the single-species model with mass
  effect (Sec. 2.2, e:rd; Sec. 3).

Parity status: every building block is pinned by closed forms, invariants or
brute force in ``tests/test_oracle_*.py``.  The full coupled step has no
worked example in the paper; beyond the pinned blocks and the invariants
(mass balance, residual certificates) it is "parity unpinned".
"""
from . import spectral, solvers, transport, reaction, model, diagnostics, model_single  # noqa: F401
