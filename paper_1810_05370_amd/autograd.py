"""torch.autograd bridge for the split-step simulation.

``simulate(theta, spec)`` runs ``spec.steps`` split steps with the
parameters theta = (rho, k_w, k_g, k_f, lame_scale, w_1..w_K) and returns the
final tumour density tau = p + i + n (a float64 device tensor).  Its
backward pass runs the hand-written discrete adjoint of libtumor
(tumor_adjoint_step) with checkpointed recomputation, so
``loss.backward()`` yields d loss / d theta.  "rho" sets both tissue growth
rates rho_w and rho_g.  PyTorch only moves tensors; all work is in the HIP
library.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import F_ADJOINT, F_DEFAULT, Tumor


@dataclass
class SimSpec:
    inputs: dict                     # synthetic.workload_inputs(...) dictionary
    params: dict                     # full parameter dictionary (Table t:setup names)
    steps: int
    precision: str = "fp64"
    ckpt_every: int = 20
    rtol: float = 1e-8
    max_it: int = 1000
    flags: int = F_DEFAULT
    device: str = "cuda"
    last: dict = field(default_factory=dict)


def _params_from_theta(spec: SimSpec, theta: np.ndarray):
    P = dict(spec.params)
    P["rho_w"] = float(theta[0])
    P["rho_g"] = float(theta[0])
    P["k_w"], P["k_g"], P["k_f"], P["lame_scale"] = (float(v) for v in theta[1:5])
    return P, np.asarray(theta[5:], dtype=np.float64)


class _Simulate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, spec):
        th = theta.detach().cpu().double().numpy()
        P, weights = _params_from_theta(spec, th)
        inp = spec.inputs
        n = inp["n"]
        dev = torch.device(spec.device)
        t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(dev).contiguous()
        sim = Tumor(n, P, t(inp["wm"]), t(inp["gm"]), t(inp["csf"]), inp["centers"], inp["sigmas"], weights,
                    precision=spec.precision, rtol_diff=spec.rtol, rtol_elast=spec.rtol, max_it=spec.max_it,
                    flags=spec.flags | F_ADJOINT)
        try:
            sim.record(spec.steps, spec.ckpt_every)
            spec.last["stats"] = sim.step(spec.steps)
            tau = sim.get("p") + sim.get("i") + sim.get("n")
        except BaseException:
            sim.close()          # frees the context; the tape and workspace go with the tensors
            raise
        ctx.sim = sim
        ctx.spec = spec
        ctx.n_theta = th.size
        ctx.theta_device = theta.device
        ctx.theta_dtype = theta.dtype
        return tau

    @staticmethod
    def backward(ctx, tau_bar):
        sim, spec = ctx.sim, ctx.spec
        n = spec.inputs["n"]
        lam = torch.zeros((14, n, n, n), dtype=torch.float64, device=tau_bar.device)
        tb = tau_bar.to(torch.float64).contiguous()
        for k in range(3):
            lam[k].copy_(tb)
        grad = np.zeros(ctx.n_theta)
        try:
            for s in range(spec.steps):
                sim.adjoint_step(lam, grad)
        finally:
            sim.close()
            ctx.sim = None
        # the gradient lives where theta lives, in theta's dtype
        return torch.as_tensor(grad, dtype=torch.float64).to(device=ctx.theta_device, dtype=ctx.theta_dtype), None


def simulate(theta: torch.Tensor, spec: SimSpec) -> torch.Tensor:
    """Final tau = p + i + n after spec.steps steps; differentiable in theta."""
    return _Simulate.apply(theta, spec)


def theta_from(params: dict, weights) -> torch.Tensor:
    """Pack (rho, k_w, k_g, k_f, lame_scale, weights) from a parameter dictionary."""
    head = [params["rho_w"], params["k_w"], params["k_g"], params["k_f"], params["lame_scale"]]
    return torch.tensor(head + list(np.asarray(weights, dtype=np.float64)), dtype=torch.float64)
