"""Symmetric (Strang) form of the split step on the GPU, through the C ABI.

Against the FP64 oracle's symmetric step: iteration lockstep in FP64 (relL2
<= 1e-10 per species and displacement), free-running iteration counts within
one of the oracle's, and the mixed precision at relL2 <= 1e-5.  At 256^3 the
step is checked through a property that holds at any size: with a uniform
velocity that moves whole cells per half-step and uniform oxygen and edema,
one symmetric step equals the advection-free step followed by the shift (the
transported species and the displacement by the whole step's shift, oxygen and
edema by the second half-step's).
"""
import numpy as np
import pytest

import paper_1810_05370_amd as tm
import synthetic
from gpu_common import need_gpu, rel_l2, roll_cells, say, shift_case
from oracle import model, model_single

pytestmark = pytest.mark.gpu

SPECIES = ("p", "i", "n", "o", "l", "g", "w", "f")
STRANG = tm.F_DEFAULT | tm.F_STRANG


def _iters(s):
    return [s["it_diff"][0], s["it_diff"][1], s["it_diff"][2], s["it_elast"]]


def _oracle(P, inp, steps, stepper):
    st = model.init_state(P, inp["n"], inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"],
                          inp["weights"])
    stats = [stepper(st, dict(strang=True)) for _ in range(steps)]
    return st, stats


def _compare(sim, st, tol, label):
    worst = {}
    for k in SPECIES:
        got, ref = sim.get(k).cpu().numpy(), st.f[k]
        worst[k] = rel_l2(got, ref) if np.linalg.norm(ref) > 0 else float(np.abs(got).max())
    for k, ref in (("u", st.u), ("u_prev", st.u_prev)):
        got = sim.get(k).cpu().numpy()
        worst[k] = rel_l2(got, ref) if np.linalg.norm(ref) > 0 else float(np.abs(got).max())
    say(label, {k: f"{v:.2e}" for k, v in worst.items()})
    for k, v in worst.items():
        assert v <= tol, (label, k, v)


@pytest.mark.parametrize("model_name,n,steps,delta_p", [
    ("multispecies", 16, 2, None), ("multispecies", 32, 6, 60.0), ("single", 16, 3, None)])
def test_lockstep_parity(model_name, n, steps, delta_p):
    need_gpu()
    P = synthetic.params() if delta_p is None else synthetic.params(delta_p=delta_p)
    inp = synthetic.workload_inputs("seed1_n32", n=n)
    stepper = model.step if model_name == "multispecies" else model_single.step
    say(f"strang {model_name} n={n} steps={steps}")
    st, stats = _oracle(P, inp, steps, stepper)
    free = tm.from_inputs(inp, P, flags=STRANG, model=model_name)
    lock = tm.from_inputs(inp, P, flags=STRANG, model=model_name)
    for k in range(steps):
        sf = free.step(1)
        lock.force_iterations(_iters(stats[k]))
        lock.step(1)
        diff = np.abs(np.array(_iters(sf)) - np.array(_iters(stats[k])))
        assert diff.max() <= 1, (k, _iters(sf), _iters(stats[k]))
    _compare(lock, st, 1e-10, f"strang lockstep {model_name} n={n}")
    free.close()
    lock.close()


def test_mixed_precision_matches_fp64_oracle():
    need_gpu()
    P = synthetic.params()
    inp = synthetic.workload_inputs("seed1_n32")
    steps = 6
    st, _ = _oracle(P, inp, steps, model.step)
    sim = tm.from_inputs(inp, P, precision="mixed", flags=STRANG)
    for _ in range(steps):
        s = sim.step(1)
        assert s["relres_elast"] <= 1e-8 and max(s["relres_diff"]) <= 1e-8
    _compare(sim, st, 1e-5, "strang mixed n=32")
    sim.close()


def test_reported_cfl_is_the_full_step_one():
    # the transport entry point is the full-dt step of the same velocity
    need_gpu()
    P = synthetic.params()
    b = tm.from_inputs(synthetic.workload_inputs("seed1_n32", n=32), P, flags=STRANG)
    b.step(2)
    _, cfl_full = b.transport()
    sb = b.step(1)
    say(f"max CFL of the full step {cfl_full:.17g}, reported by the symmetric step {sb['max_cfl']:.17g}")
    assert sb["max_cfl"] > 0.0 and sb["max_cfl"] == cfl_full
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_exact_shift_commutes_with_the_symmetric_step_at_256(precision):
    torch = need_gpu()
    n, half = 256, (1, -1, 2)
    total = tuple(2 * s for s in half)
    P = synthetic.params(delta_p=60.0)
    say(f"generating the 256^3 three-seed inputs ({precision})")
    inp = synthetic.workload_inputs("seeds3_n256")
    ref = shift_case(torch, inp, P, precision, tm.F_ELASTICITY | tm.F_EDEMA, half)
    s_ref = ref.step(1)
    want = {k: ref.get(k) for k in SPECIES + ("u",)}
    ref.close()
    sym = shift_case(torch, inp, P, precision, STRANG, half)
    if precision == "fp64":
        sym.force_iterations(_iters(s_ref))      # same stopping point as the reference
    s_sym = sym.step(1)
    say(f"iterations: advection-free {_iters(s_ref)}, symmetric {_iters(s_sym)}")
    tol = 1e-10 if precision == "fp64" else 1e-5
    for k in SPECIES + ("u",):
        got = sym.get(k)
        exp = roll_cells(want[k], half if k in ("o", "l") else total)
        err = float((got - exp).norm() / exp.norm())
        say(f"  {k}: relL2 {err:.2e}")
        assert err < tol, k
    assert s_ref["it_elast"] > 5 and s_sym["relres_elast"] <= 1e-7
    sym.close()
