"""The 69-parameter gradient of the adjoint-with-parameters workload at its
own grid (128^3, FP64) against central finite differences, on the GPU.

Loss 1/2 h^3 ||tau_T - tau_target||^2 with tau = p + i + n; tau_target from a
forward run with the parameters perturbed by theta (1 + 0.1 xi), xi ~ N(0, 1)
seeded.  Parameters: rho (both tissues), k_w, k_g, k_f, the Lame scale and
the 64 initial-condition weights of the 4 x 4 x 4 seed lattice.

The trajectory is cut to 4 steps: the lattice inputs lose stability after
about 9 steps (the transport-elasticity loop gain exceeds 1), and the loop
amplifies every perturbation, finite-difference rounding included, several
times per step.  Every solve runs at rtol 1e-12; the +h and -h runs repeat the
base run's iteration counts (tumor_force_iterations), so each difference
quotient differentiates one fixed smooth map, and the adjoint (which takes
the solves as exact) differs from it by solve-tolerance terms only.
"""
import numpy as np
import pytest

import paper_1810_05370_amd as tm
import synthetic
from gpu_common import need_gpu, rel_l2, say

pytestmark = pytest.mark.gpu

N, STEPS, RTOL = 128, 4, 1e-12


def _theta_params(P0, theta, n_ic):
    P = dict(P0)
    P["rho_w"] = P["rho_g"] = float(theta[0])
    P["k_w"], P["k_g"], P["k_f"], P["lame_scale"] = (float(v) for v in theta[1:5])
    return P, np.asarray(theta[5:5 + n_ic], dtype=np.float64)


def _sim(inp, P, weights, flags=tm.F_DEFAULT):
    d = dict(inp)
    d["weights"] = weights
    return tm.from_inputs(d, P, precision="fp64", rtol_diff=RTOL, rtol_elast=RTOL, max_it=4000, flags=flags)


def _tau(inp, P0, theta, forced=None):
    P, w = _theta_params(P0, theta, len(inp["weights"]))
    sim = _sim(inp, P, w)
    counts = []
    for k in range(STEPS):
        if forced is not None:
            sim.force_iterations(forced[k])
        s = sim.step(1)
        counts.append([s["it_diff"][0], s["it_diff"][1], s["it_diff"][2], s["it_elast"]])
    t = (sim.get("p") + sim.get("i") + sim.get("n")).clone()
    sim.close()
    return t, counts


def test_all_69_parameter_gradients_match_central_differences_at_128():
    torch = need_gpu()
    say("generating the 128^3 lattice inputs")
    inp = synthetic.workload_inputs("lattice_n128")
    P0 = synthetic.params()
    n_ic = len(inp["weights"])
    theta0 = np.r_[P0["rho_w"], P0["k_w"], P0["k_g"], P0["k_f"], P0["lame_scale"], inp["weights"]]
    assert theta0.size == 69
    xi = np.random.default_rng(4).standard_normal(theta0.size)
    tgt, _ = _tau(inp, P0, theta0 * (1.0 + 0.1 * xi))
    h3 = (2 * np.pi / N) ** 3

    # gradient by the adjoint (every state and intermediate on the tape)
    base_counts = None
    P, w = _theta_params(P0, theta0, n_ic)
    sim = _sim(inp, P, w, tm.F_DEFAULT | tm.F_ADJOINT)
    sim.record(STEPS, 1)
    base_counts = []
    for k in range(STEPS):
        s = sim.step(1)
        base_counts.append([s["it_diff"][0], s["it_diff"][1], s["it_diff"][2], s["it_elast"]])
    tau0 = (sim.get("p") + sim.get("i") + sim.get("n")).clone()
    lam = torch.zeros((14, N, N, N), dtype=torch.float64, device="cuda")
    for k in range(3):
        lam[k].copy_(h3 * (tau0 - tgt))
    grad = np.zeros(5 + n_ic)
    for _ in range(STEPS):
        sim.adjoint_step(lam, grad)
    sim.close()
    say(f"base iteration counts per step (i, o, l, elasticity): {base_counts}")

    def loss(t):
        return 0.5 * h3 * float(torch.sum((t - tgt) ** 2))

    fd = np.zeros_like(grad)
    for j in range(theta0.size):
        hj = 1e-6 * max(1.0, abs(theta0[j]))
        vals = []
        for sgn in (1.0, -1.0):
            th = theta0.copy()
            th[j] += sgn * hj
            t, _ = _tau(inp, P0, th, forced=base_counts)
            vals.append(loss(t))
        fd[j] = (vals[0] - vals[1]) / (2 * hj)
    names = ["rho", "k_w", "k_g", "k_f", "lame_scale"] + [f"w{k}" for k in range(n_ic)]
    rel = np.abs(grad - fd) / np.maximum(np.abs(fd), 1e-300)
    for j in range(theta0.size):
        if j < 5 or j % 16 == 0:
            say(f"  {names[j]}: adjoint {grad[j]: .9e}  central difference {fd[j]: .9e}  rel {rel[j]:.1e}")
    whole = rel_l2(grad, fd)
    say(f"69-parameter gradient: relative L2 difference {whole:.2e}, worst component {rel.max():.2e} "
        f"({names[int(rel.argmax())]})")
    assert whole < 1e-6
    # every component that carries weight in the gradient agrees on its own
    big = np.abs(fd) > 1e-6 * np.abs(fd).max()
    assert np.all(rel[big] < 1e-4), [(names[j], rel[j]) for j in np.flatnonzero(big & (rel >= 1e-4))]
