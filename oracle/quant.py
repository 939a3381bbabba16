"""Quantise-then-FP64 references for the reduced-precision storage formats (test
infrastructure).

The GPU solver stores colour vectors and links in FP32, or in IEEE binary16.  These functions
round FP64 data exactly as those formats are defined, so that the FP64 oracle applied to the
rounded data separates storage rounding from kernel mistakes:

* FP32: every real rounded to binary32 (round to nearest even).
* FP16 colour vectors: per site, n = binary32(max |real| over the site's 6 reals); each real v
  is stored as binary16(v / n) and read back as n * h; n = 0 stores zeros.
* FP16 links: each link class (fat, Naik) is scaled by 2^k, k = -e where max |real| of the
  class = f * 2^e with f in [0.5, 1); each real is stored as binary16(v * 2^k) and read back
  multiplied by 2^-k (the power-of-two scale adds no rounding of its own).
"""
from __future__ import annotations

import numpy as np


def quantise_f32(a: np.ndarray) -> np.ndarray:
    return np.asarray(a, dtype=np.complex128).astype(np.complex64).astype(np.complex128)


def quantise_f16_sites(v: np.ndarray) -> np.ndarray:
    """v complex128 [n][3] -> FP64 values of its FP16 + per-site norm encoding."""
    v = np.asarray(v, dtype=np.complex128)
    re = np.stack([v.real, v.imag], axis=-1).reshape(v.shape[0], 6)
    n = np.max(np.abs(re), axis=1).astype(np.float32).astype(np.float64)
    safe = np.where(n > 0, n, 1.0)
    h = (re / safe[:, None]).astype(np.float16).astype(np.float64)
    out = h * n[:, None]
    out = out.reshape(v.shape[0], 3, 2)
    return out[..., 0] + 1j * out[..., 1]


def f16_link_exponent(L: np.ndarray) -> int:
    m = max(float(np.max(np.abs(L.real))), float(np.max(np.abs(L.imag))))
    if m == 0:
        return 0
    return -int(np.frexp(m)[1])


def quantise_f16_links(L: np.ndarray) -> np.ndarray:
    k = f16_link_exponent(L)
    s = np.ldexp(1.0, k)
    re = (L.real * s).astype(np.float16).astype(np.float64) / s
    im = (L.imag * s).astype(np.float16).astype(np.float64) / s
    return re + 1j * im
