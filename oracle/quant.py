"""Quantise-then-FP64 references for the reduced-precision storage formats (test
infrastructure).

The GPU solver stores colour vectors and links in FP32, or in IEEE binary16.  These functions
round FP64 data exactly as those formats are defined, so that the FP64 oracle applied to the
rounded data separates storage rounding from kernel mistakes:

* FP32: every real rounded to binary32 (round to nearest even).
* FP16 colour vectors: the reals are first binary32 numbers v; per site n = max |v| over the
  site's 6 reals (a binary32 scale); each real is stored as binary16(binary32(v / n)) and read
  back as n * h; n = 0 stores zeros.
* FP16 links: each link class (fat, Naik) is scaled by 2^k, k = -e where max |real| of the
  class = f * 2^e with f in [0.5, 1); each real is stored as binary16(v * 2^k) and read back
  multiplied by 2^-k (the power-of-two scale adds no rounding of its own).
* 12-real Naik storage (links that are c * eta * bc * SU(3)): per stored matrix the first two
  rows of its SU(3) part, rounded to the storage format (binary16 at scale 1: SU(3) entries
  are at most 1 in modulus), the third row rebuilt as conj(row0 x row1), then multiplied by
  the real scale and the sign.

The link store keeps, per site, the forward matrices of the site and minus the adjoints of the
backward ones ("8-way" storage, Sec. 3).  With 12-real Naik storage the two copies of one link
are rounded separately (the backward copy stores rows of the SU(3) part's adjoint), so the
operator the device applies has different forward and backward Naik matrices; `dslash_eo_fb`
applies such an operator, built from the oracle's Dslash alone.
"""
from __future__ import annotations

import numpy as np


def quantise_f32(a: np.ndarray) -> np.ndarray:
    return np.asarray(a, dtype=np.complex128).astype(np.complex64).astype(np.complex128)


def quantise_f16_sites(v: np.ndarray) -> np.ndarray:
    """v complex128 [n][3] -> FP64 values of its FP16 + per-site norm encoding."""
    v = np.asarray(v, dtype=np.complex128)
    re = np.stack([v.real, v.imag], axis=-1).reshape(v.shape[0], 6).astype(np.float32)
    n = np.max(np.abs(re), axis=1)
    safe = np.where(n > 0, n, np.float32(1.0))
    h = (re / safe[:, None]).astype(np.float32).astype(np.float16).astype(np.float64)
    out = h * n.astype(np.float64)[:, None]
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


def _round_entries(a: np.ndarray, prec: str) -> np.ndarray:
    if prec == "f64":
        return np.asarray(a, dtype=np.complex128)
    if prec == "f32":
        return quantise_f32(a)
    re = a.real.astype(np.float16).astype(np.float64)
    im = a.imag.astype(np.float16).astype(np.float64)
    return re + 1j * im


def _dag(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


def rebuild_su3(rows01: np.ndarray) -> np.ndarray:
    """[..., 2, 3] first two rows -> [..., 3, 3] with row 2 = conj(row0 x row1) (FP64)."""
    a, b = rows01[..., 0, :], rows01[..., 1, :]
    r2 = np.conj(np.cross(a, b))
    return np.concatenate([rows01, r2[..., None, :]], axis=-2)


def naik_phase(dims) -> np.ndarray:
    """[4][V] real factors eta_mu(x) * bc3_mu(x) of the Naik links: the staggered phase times
    -1 on three-links that start at t >= Nt - 3 (they cross the antiperiodic boundary once)."""
    nx, ny, nz, nt = (int(d) for d in dims)
    i = np.arange(nx * ny * nz * nt, dtype=np.int64)
    x, y, z, t = i % nx, (i // nx) % ny, (i // (nx * ny)) % nz, i // (nx * ny * nz)
    out = np.empty((4, i.size))
    for mu, e in enumerate((np.zeros_like(x), x, x + y, x + y + z)):
        eta = np.where(e % 2 == 1, -1.0, 1.0)
        bc = np.where((t >= nt - 3), -1.0, 1.0) if mu == 3 else 1.0
        out[mu] = eta * bc
    return out


def naik12_scale(naik: np.ndarray) -> float:
    """The real scale c0 of 12-real storage: the real cube root of det W_0 at the origin (where
    the phase is +1)."""
    d = np.linalg.det(naik[0, 0])
    return float(np.cbrt(d.real))


def link_store_values(g, prec: str, recon: int, access: int = 8):
    """(fwd, bwd): two GaugeFields holding the FP64 values that the device's link store of
    precision `prec` ('f64', 'f32', 'f16') and Naik storage `recon` (18, 12) decodes to, for
    `dslash_eo_fb`: forward hops read fwd, backward hops read bwd (the hop from x - k mu
    applies -bwd(x - k mu)^+).  access = 8: a site reads its own backward slots, which hold a
    separately rounded copy; access = 4: the backward matrices are formed from the neighbours'
    forward slots, so bwd = fwd."""
    from ksinputs import GaugeField
    fat, naik = np.asarray(g.fat), np.asarray(g.naik)
    if prec == "f16":
        qfat = quantise_f16_links(fat)
    else:
        qfat = _round_entries(fat, prec)
    if recon == 18:
        qnaik = quantise_f16_links(naik) if prec == "f16" else _round_entries(naik, prec)
        f = GaugeField(g.dims, qfat, qnaik)
        return f, f
    c = naik12_scale(naik) * naik_phase(g.dims)[..., None, None]    # [4][V][1][1]
    su3 = naik / c
    fwd_naik = c * rebuild_su3(_round_entries(su3[..., :2, :], prec))
    fwd = GaugeField(g.dims, qfat, fwd_naik)
    if access == 4:
        return fwd, fwd
    adj = _dag(su3)
    bwd_naik = c * _dag(rebuild_su3(_round_entries(adj[..., :2, :], prec)))
    return fwd, GaugeField(g.dims, qfat, bwd_naik)


def dslash_eo_fb(fwd, bwd, out_parity: int, psi: np.ndarray) -> np.ndarray:
    """D_eo with forward hops from `fwd` and backward hops from `bwd`.

    Write D(L) = F(L) - B(L) with F the forward-hop sum (linear in the links) and B the
    backward-hop sum (antilinear: it applies L^+).  Multiplying every link by i gives
    D(iL) = i (F(L) + B(L)), hence F(L) = (D(L) - i D(iL)) / 2 and
    B(L) = (-i D(iL) - D(L)) / 2, and F(fwd) - B(bwd) is four calls of the oracle's Dslash."""
    from ksinputs import GaugeField
    from .core import dslash_eo

    def times_i(h):
        return GaugeField(h.dims, 1j * np.asarray(h.fat), 1j * np.asarray(h.naik))

    d_f = dslash_eo(fwd, out_parity, psi)
    d_if = dslash_eo(times_i(fwd), out_parity, psi)
    if bwd is fwd:
        return d_f
    d_b = dslash_eo(bwd, out_parity, psi)
    d_ib = dslash_eo(times_i(bwd), out_parity, psi)
    return 0.5 * (d_f - 1j * d_if + 1j * d_ib + d_b)


def dslash_eo_abs(g, out_parity: int, psi: np.ndarray) -> np.ndarray:
    """Per output component, sum over the 16 hops and 3 columns of |L_ab| |psi_b|: the sum of
    the moduli of every product the component is made of (the scale that bounds its rounding
    error).  With real non-negative links |L| and input |psi|, F + B = -i D(i|L|) adds the
    backward terms instead of subtracting them."""
    from ksinputs import GaugeField
    from .core import dslash_eo
    a = GaugeField(g.dims, 1j * np.abs(np.asarray(g.fat)), 1j * np.abs(np.asarray(g.naik)))
    out = -1j * dslash_eo(a, out_parity, np.abs(np.asarray(psi)).astype(np.complex128))
    return out.real
