"""Pins for the oracle's symmetric (Strang) form of the split step (Sec. 3).

The symmetric step transports over dt/2, refreshes the coefficients, runs the
diffusion-reaction stage over dt, transports over dt/2 again and then refreshes
and solves the elasticity.  The pins use facts that hold exactly:

* without advection the two forms are the same step;
* a uniform velocity whose half-step displacement is a whole number of cells
  makes each semi-Lagrangian half-step an exact shift (zero divergence, nodal
  departure points).  Every other stage commutes with shifts when the
  elasticity starts from a shift-invariant guess and the untransported oxygen
  and edema start uniform.  One symmetric step then equals the advection-free
  step followed by the total shift of the transported species, and by the
  second half-step's shift of oxygen and edema (created in the middle, moved
  only once).  The sequential step does not: its diffusion and reaction use
  coefficients of the unshifted tissue, and it misses this identity by far
  more than rounding.
"""
import numpy as np
import pytest

import synthetic
from oracle import model, model_single

N = 16
DT = 0.01
HALF_SHIFT = (1, -1, 2)   # cells per half-step along x, y, z


def _state(P, stepper=model.step, steps=2):
    inp = synthetic.workload_inputs("seed1_n32", n=N)
    st = model.init_state(P, N, inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"], inp["weights"])
    for _ in range(steps):                          # make i, n and u non-trivial
        stepper(st, dict(advection=False))
    return st


def _uniform_velocity(st, shift):
    """u = 0, u_prev = -dt v with v moving shift[a] cells per half-step along
    axis a; oxygen and edema set uniform (oxygen between o_hyp and o_inv, so
    growth, invasion and edema are all active)."""
    P = st.P
    st.f["o"] = np.full((N, N, N), P["o_hyp"] + 0.75 * (P["o_inv"] - P["o_hyp"]))
    st.f["l"] = np.full((N, N, N), 0.05)
    h = st.grid.h
    v = np.zeros((3, N, N, N))
    for a in range(3):
        v[a] = 2.0 * shift[a] * h / DT
    st.u = np.zeros((3, N, N, N))
    st.u_prev = -DT * v


def _roll(q, cells):
    # arrays are [z][y][x]; a positive velocity moves the pattern to larger indices
    return np.roll(q, (cells[2], cells[1], cells[0]), axis=(-3, -2, -1))


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _worst(st, ref, total, half):
    errs = {}
    for k in st.f:
        if np.linalg.norm(ref.f[k]) > 0:
            errs[k] = _rel(st.f[k], _roll(ref.f[k], half if k in ("o", "l") else total))
    errs["u"] = _rel(st.u, _roll(ref.u, total))
    return errs


@pytest.mark.parametrize("stepper", [model.step, model_single.step], ids=["multispecies", "single"])
def test_without_advection_the_symmetric_step_is_the_sequential_one(stepper):
    P = synthetic.params(delta_p=60.0)
    a = _state(P, stepper)
    b = a.copy()
    stepper(a, dict(advection=False))
    stepper(b, dict(advection=False, strang=True))
    for k in a.f:
        assert np.array_equal(a.f[k], b.f[k]), k
    assert np.array_equal(a.u, b.u)


@pytest.mark.parametrize("stepper", [model.step, model_single.step], ids=["multispecies", "single"])
def test_exact_shift_commutes_with_the_symmetric_step(stepper):
    P = synthetic.params(delta_p=60.0)
    base = _state(P, stepper)
    _uniform_velocity(base, HALF_SHIFT)
    total = tuple(2 * s for s in HALF_SHIFT)

    ref = base.copy()
    s_ref = stepper(ref, dict(advection=False))
    sym = base.copy()
    s_sym = stepper(sym, dict(strang=True))
    seq = base.copy()
    stepper(seq, dict(strang=False))

    assert s_sym["it_elast"] == s_ref["it_elast"] and s_sym["it_elast"] > 5
    e_sym = _worst(sym, ref, total, HALF_SHIFT)
    e_seq = _worst(seq, ref, total, HALF_SHIFT)
    assert max(e_sym.values()) < 1e-11, e_sym
    # the sequential step lags the coefficients by a whole step's shift
    assert max(e_seq.values()) > 1e-6, e_seq
    assert e_seq["p"] > 1e4 * max(e_sym["p"], 1e-16)


def test_symmetric_step_refuses_the_tape():
    P = synthetic.params()
    st = _state(P, steps=0)
    with pytest.raises(ValueError):
        model.step(st, dict(strang=True), tape={})
