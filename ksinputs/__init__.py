"""Seeded synthetic inputs for the improved-staggered solver.

This package only draws random numbers and assembles the link fields and sources that the
operator takes as input.  It holds none of the solver's arithmetic (no Dslash, no Krylov
step), so both the FP64 CPU oracle's tests and the GPU path may take their inputs from it.
"""
from .gauge import (lattice_coords, lattice_volume, staggered_phase, time_bc_sign,
                    random_su3, thin_links, fat_and_naik, make_gauge, GaugeField, subblock)
from .fields import gaussian_source, gaussian_full, batch_masses, SEEDS
from .network import net_init_weights, flatten_weights, unflatten_weights

__all__ = ["lattice_coords", "lattice_volume", "staggered_phase", "time_bc_sign", "random_su3",
           "thin_links", "fat_and_naik", "make_gauge", "GaugeField", "gaussian_source",
           "gaussian_full", "batch_masses", "SEEDS", "net_init_weights", "flatten_weights",
           "unflatten_weights"]
