"""Shared helpers of the GPU tests (not collected by pytest)."""
import sys

import numpy as np


def need_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(got - ref)
    if den == 0.0:
        return num
    return num / den


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to("cuda").contiguous()
