"""Helpers of the GPU parity tests: host <-> device copies of complex128 arrays."""
import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def zeros_dev(shape):
    import torch
    return torch.zeros(shape, dtype=torch.complex128, device="cuda")


def announce(*what):
    """Names the case on stdout before it touches the GPU."""
    print("[gpu case]", *what, flush=True)
