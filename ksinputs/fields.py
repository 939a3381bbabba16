"""Seeded sources and per-lattice parameters.

Colour-vector fields on one parity use the checkerboard layout complex128 [Vh][3]: the site
with lexicographic index i (parity (x+y+z+t) mod 2) sits at row i >> 1 of its parity's array.
"""
from __future__ import annotations

import numpy as np

# Seeds of the standard workloads: gauge 1000+k and source 2000+k for workload k; batch lattice
# j takes gauge 4000+j and right-hand side r takes 4200+4j+r, the batch masses come from 4100;
# the network's initial weights from 5000 and its training sources from 5100+i.
SEEDS = {
    "gauge": lambda k: 1000 + k,
    "source": lambda k: 2000 + k,
    "batch_gauge": lambda j: 4000 + j,
    "batch_rhs": lambda j, r: 4200 + 4 * j + r,
    "batch_mass": 4100,
    "net_init": 5000,
    "train_source": lambda i: 5100 + i,
}


def gaussian_source(vh: int, seed: int) -> np.ndarray:
    """Unit-variance complex Gaussian colour vectors, CN(0,1) per component, [vh][3]."""
    g = np.random.default_rng(seed).standard_normal((vh, 3, 2))
    return (g[..., 0] + 1j * g[..., 1]) * np.sqrt(0.5)


def gaussian_full(v: int, seed: int) -> np.ndarray:
    """CN(0,1) colour vectors on every site, lexicographic [v][3]."""
    return gaussian_source(v, seed)


def batch_masses(n: int, lo: float = 0.01, hi: float = 0.2, seed: int = 4100) -> np.ndarray:
    """Masses drawn uniformly from [lo, hi]."""
    return np.random.default_rng(seed).uniform(lo, hi, size=n)
