"""Training pipeline of the learned preconditioner: (source, FP64 solution) pairs produced by
the library's own FP64 CG on sub-lattices and on the full lattice, then Adam steps of the
library's GPU training kernels.  Argument marshalling and bookkeeping only."""
from __future__ import annotations

import time

import numpy as np

from . import F64, Gauge, Net, cg_solve, default_params


def block_origins(dims, bdims):
    """Origins of the non-overlapping blocks of extent bdims that tile dims."""
    out = []
    for t in range(0, dims[3] - bdims[3] + 1, bdims[3]):
        for z in range(0, dims[2] - bdims[2] + 1, bdims[2]):
            for y in range(0, dims[1] - bdims[1] + 1, bdims[1]):
                for x in range(0, dims[0] - bdims[0] + 1, bdims[0]):
                    out.append((x, y, z, t))
    return out


def solve_pairs(gauge: Gauge, mass: float, sources, tol: float = 1e-10):
    """x_j = A^-1 b_j by FP64 CG on the GPU for every source (complex128 [Vh][3] host arrays);
    returns the device (b, x) tensors."""
    import torch
    pairs = []
    for b in sources:
        bd = torch.from_numpy(np.ascontiguousarray(b)).cuda()
        xd = torch.zeros_like(bd)
        cg_solve(gauge, mass, bd, xd, default_params(tol=tol, inner=F64))
        pairs.append((gauge, bd, xd))
    torch.cuda.synchronize()
    return pairs


def train(net: Net, pairs, steps: int, batch: int, lr: float):
    """Adam steps over the pairs (cyclic minibatches); returns (loss history, seconds)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = net.train([p[0] for p in pairs], [p[1] for p in pairs], [p[2] for p in pairs],
                     steps, batch, lr)
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0
