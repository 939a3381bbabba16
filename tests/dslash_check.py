"""Element-wise parity of a Dslash output against the quantise-then-FP64 oracle reference.

The reference applies the FP64 oracle to the links and the input exactly as the device stores
them (`oracle.link_store_values`, the quantisers of `oracle.quant`), with the 12-real Naik
copies that the chosen link access reads.  What remains between the two is the device's own
arithmetic and the rounding of its output:

* every output component is a sum of 48 complex products; summed in a binary format with unit
  roundoff u, it differs from the exact sum by at most about 100 u times the sum of the
  products' moduli S (`oracle.dslash_eo_abs`), to which the FP32 rebuild of the third Naik row
  and the binary32 scale add a few u S: the bound is 2^-17 S for FP32 and FP16 arithmetic
  (u = 2^-24) and 2^-44 S for FP64;
* FP16 output is stored relative to its site maximum n: half a binary16 ulp there is 2^-12 n;
  the bound allows 2^-11 n.

A wrong link, neighbour, sign or conjugation changes a component by the size of one product,
about S / 16, far above these bounds, at any site.
"""
import numpy as np

import oracle

EPS = {"f64": 2.0 ** -44, "f32": 2.0 ** -17, "f16": 2.0 ** -17}


def reference(g, prec, recon, access, out_parity, psi):
    """(reference output, modulus sums S) for input psi (complex128 [Vh][3])."""
    fwd, bwd = oracle.link_store_values(g, prec, recon, access)
    q = {"f64": np.asarray(psi), "f32": oracle.quantise_f32(psi),
         "f16": oracle.quantise_f16_sites(psi)}[prec]
    ref = oracle.dslash_eo_fb(fwd, bwd, out_parity, q)
    S = oracle.dslash_eo_abs(fwd, out_parity, q)
    return ref, S


def bound(ref, S, prec):
    tol = EPS[prec] * S
    if prec == "f16":
        vh = ref.shape[0]
        n = np.max(np.abs(np.stack([ref.real, ref.imag], -1).reshape(vh, 6)), axis=1)
        tol = tol + 2.0 ** -11 * n[:, None]
    return tol


def worst(got, ref, S, prec):
    """Largest ratio |got - ref| / bound over all real components (<= 1 passes)."""
    tol = bound(ref, S, prec)
    tol = np.where(tol > 0, tol, np.finfo(float).tiny)
    r = np.maximum(np.abs(got.real - ref.real) / tol, np.abs(got.imag - ref.imag) / tol)
    return float(np.max(r))
