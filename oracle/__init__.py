"""FP64 CPU oracle for the even-odd preconditioned improved-staggered solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark import this package.  It shares no code with the GPU library (`paper_1611_00728_amd`)
and never imports it; the two meet only in the seeded inputs of `ksinputs`.

* `ks_oracle.c` (loaded through ctypes): the Dslash, the normal operator A_sigma, plain CG
  and multi-shift CG, each written out from its definition (Sec. 3 and Sec. 4 name these
  routines; the formulas are restated in that file's header).
* `network.py`: the gauge-covariant preconditioner network N = L^+ L, its A-norm loss,
  gradients and Adam.
* `solvers.py`: flexible CG with a preconditioner; M = 2m + D on the full lattice and its
  solve through the even-odd Schur complement with odd-site reconstruction; the link
  derivative (force) of the multi-shift pseudofermion action from the shifted solutions.
* `hisq.py`: two-level smeared fat links (fat7, U(3) projection, fat7 + Lepage) and the
  Naik link built from thin links.
* `quant.py`: the quantise-then-FP64 references of the reduced-precision storage formats
  (vectors, links, 12-real Naik storage), the Dslash with separately stored forward and
  backward links, and the per-component modulus sums that bound its rounding error.
"""
from .core import (lib, set_threads, max_threads, dslash_full, dslash_eo, apply_A, cg, multishift_cg, embed, restrict,
                   CGInfo, dense_A, lanczos_extremes, OracleError)
from . import hisq
from .quant import (quantise_f32, quantise_f16_sites, quantise_f16_links, f16_link_exponent,
                    rebuild_su3, naik_phase, naik12_scale, link_store_values, dslash_eo_fb,
                    dslash_eo_abs)
from .network import (Network, PATHS, transport, transport_adj, layer_forward,
                      network_forward, half_forward, adjoint_weights, tied_gradients,
                      loss_and_grad, adam_step, neighbour_tables)
from .solvers import (fcg, apply_M, full_solve, FullInfo, force_outer, rational_action,
                      parity_sign)

__all__ = ["hisq", "lib", "set_threads", "max_threads", "dslash_full", "dslash_eo", "apply_A", "cg", "multishift_cg", "embed",
           "restrict", "CGInfo", "dense_A", "lanczos_extremes", "OracleError", "quantise_f32",
           "quantise_f16_sites", "quantise_f16_links", "f16_link_exponent", "rebuild_su3",
           "naik_phase", "naik12_scale", "link_store_values", "dslash_eo_fb", "dslash_eo_abs", "Network", "PATHS",
           "transport", "transport_adj", "layer_forward", "network_forward", "half_forward",
           "adjoint_weights", "tied_gradients", "loss_and_grad",
           "adam_step", "neighbour_tables", "fcg", "apply_M", "full_solve", "FullInfo", "force_outer",
           "rational_action", "parity_sign"]
