"""Training pipeline of the learned preconditioner: (source, FP64 solution) pairs produced by
the library's own FP64 CG on sub-lattices and on the full lattice, then Adam steps of the
library's GPU training kernels on the A-norm loss.  Argument marshalling and bookkeeping
only."""
from __future__ import annotations

import time

import numpy as np

from . import F64, Batch, Gauge, Net, cg_solve, default_params


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
    returns the pairs (gauge, sigma = 4 m^2, device b, device x)."""
    import torch
    pairs = []
    for b in sources:
        bd = torch.from_numpy(np.ascontiguousarray(b)).cuda()
        xd = torch.zeros_like(bd)
        cg_solve(gauge, mass, bd, xd, default_params(tol=tol, inner=F64))
        pairs.append((gauge, 4.0 * mass * mass, bd, xd))
    torch.cuda.synchronize()
    return pairs


def solve_pairs_batched(fields, sources, mass: float, tol: float = 1e-10, check_every: int = 16):
    """x = A^-1 b for every source of every lattice at once, by the library's batched FP64 CG.
    fields: objects with .dims, .fat, .naik (one per lattice); sources[l]: list of nrhs
    complex128 [Vh][3] host arrays for lattice l (nrhs 1, 2 or 4, the same for every lattice).
    Returns (pairs, seconds of the batched solve, stats): pairs are (Gauge handle of the
    lattice, sigma = 4 m^2, device b, device x); the link upload and the handles are not
    timed."""
    import torch
    nrhs = len(sources[0])
    if any(len(s) != nrhs for s in sources):
        raise ValueError("every lattice needs the same number of sources")
    B = Batch([f.dims for f in fields], [f.fat for f in fields], [f.naik for f in fields],
              nrhs, F64)
    gauges = [Gauge(f.dims, f.fat, f.naik) for f in fields]
    bs = [torch.from_numpy(np.ascontiguousarray(b)).cuda() for srcs in sources for b in srcs]
    xs = [torch.zeros_like(b) for b in bs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stats = B.solve([mass] * len(fields), bs, xs,
                       default_params(tol=tol, inner=F64, check_every=check_every))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    B.free()
    pairs = [(gauges[k // nrhs], 4.0 * mass * mass, bs[k], xs[k]) for k in range(len(bs))]
    return pairs, dt, stats


def train(net: Net, pairs, steps: int, batch: int, lr: float):
    """Adam steps over the pairs (cyclic minibatches); returns (loss history, seconds)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = net.train([p[0] for p in pairs], [p[1] for p in pairs], [p[2] for p in pairs],
                     [p[3] for p in pairs], steps, batch, lr)
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0
