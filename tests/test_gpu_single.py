"""Single-species model (Sec. 2.2, e:rd) on the GPU against the FP64 oracle,
through the C ABI, in iteration lockstep (FP64, relL2 <= 1e-10) and in the
mixed precision (relL2 <= 1e-5)."""
import numpy as np
import pytest

import paper_1810_05370_amd as tm
import synthetic
from gpu_common import need_gpu, rel_l2, say
from oracle import model, model_single

pytestmark = pytest.mark.gpu

FIELDS = ("p", "i", "n", "o", "l", "g", "w", "f")


def _oracle(P, inp, steps, cfg=None):
    st = model.init_state(P, inp["n"], inp["wm"], inp["gm"], inp["csf"], inp["centers"], inp["sigmas"],
                          inp["weights"])
    stats = [model_single.step(st, cfg) for _ in range(steps)]
    return st, stats


def _compare(sim, st, tol, label):
    worst = {}
    for k in FIELDS:
        got, ref = sim.get(k).cpu().numpy(), st.f[k]
        worst[k] = rel_l2(got, ref) if np.linalg.norm(ref) > 0 else float(np.abs(got).max())
    for k, ref in (("u", st.u), ("u_prev", st.u_prev)):
        worst[k] = rel_l2(sim.get(k).cpu().numpy(), ref)
    say(label, {k: f"{v:.2e}" for k, v in worst.items()})
    for k, v in worst.items():
        assert v <= tol, (label, k, v)


@pytest.mark.parametrize("n,steps", [(16, 2), (32, 10)])
def test_lockstep_parity(n, steps):
    need_gpu()
    P = synthetic.params()
    inp = synthetic.workload_inputs("seed1_n32", n=n)
    st, stats = _oracle(P, inp, steps)
    free = tm.from_inputs(inp, P, model="single")
    lock = tm.from_inputs(inp, P, model="single")
    for k in range(steps):
        sf = free.step(1)
        its = [stats[k]["it_diff"][0], 0, 0, stats[k]["it_elast"]]
        assert abs(sf["it_diff"][0] - its[0]) <= 1 and abs(sf["it_elast"] - its[3]) <= 1, (k, sf, its)
        assert sf["it_diff"][1] == 0 and sf["it_diff"][2] == 0
        lock.force_iterations(its)
        lock.step(1)
    _compare(lock, st, 1e-10, f"single lockstep n={n}")
    free.close()
    lock.close()


def test_mixed_precision():
    need_gpu()
    P = synthetic.params()
    inp = synthetic.workload_inputs("seed1_n32")
    st, stats = _oracle(P, inp, 10)
    sim = tm.from_inputs(inp, P, precision="mixed", model="single")
    for _ in range(10):
        s = sim.step(1)
        assert s["relres_elast"] <= 1e-8 and s["relres_diff"][0] <= 1e-8
    _compare(sim, st, 1e-5, "single mixed n=32")
    sim.close()


def test_adjoint_is_rejected_for_the_single_species_model():
    need_gpu()
    P = synthetic.params()
    inp = synthetic.workload_inputs("seed1_n32", n=16)
    with pytest.raises(tm.TumorError) as e:
        tm.from_inputs(inp, P, model="single", flags=tm.F_DEFAULT | tm.F_ADJOINT)
    assert e.value.code == tm.EINVAL
