"""Pins of the quantise-then-FP64 references against the binary16/binary32 formats' own
rounding bounds (unit roundoff 2^-11 for binary16, 2^-24 for binary32)."""
import numpy as np

import oracle
from ksinputs import gaussian_source, make_gauge


def test_f32_rounding_bound():
    v = gaussian_source(1000, 1) * 3.7
    q = oracle.quantise_f32(v)
    assert np.all(np.abs(q.real - v.real) <= np.abs(v.real) * 2.0 ** -24)
    assert np.all(np.abs(q.imag - v.imag) <= np.abs(v.imag) * 2.0 ** -24)


def test_f16_sites_bound_and_zero_site():
    v = gaussian_source(1000, 2) * np.geomspace(1e-6, 1e3, 1000)[:, None]
    v[17] = 0
    q = oracle.quantise_f16_sites(v)
    re = np.stack([v.real, v.imag], -1).reshape(1000, 6)
    n = np.max(np.abs(re), axis=1)
    err = np.abs(np.stack([(q - v).real, (q - v).imag], -1).reshape(1000, 6))
    # rounding of v/n to binary16 (<= 2^-11 relative to n) plus rounding of n to binary32
    assert np.all(err <= n[:, None] * (2.0 ** -11 + 2.0 ** -23))
    assert np.all(q[17] == 0)
    # the largest component of every site is representable exactly up to the norm rounding
    k = np.argmax(np.abs(re), axis=1)
    qre = np.stack([q.real, q.imag], -1).reshape(1000, 6)
    assert np.allclose(np.abs(qre[np.arange(1000), k]), n, rtol=2.0 ** -23)


def test_f16_links_power_of_two_scale():
    g = make_gauge((4, 4, 4, 4), 0.5, 3)
    for L in (g.fat, g.naik):
        k = oracle.f16_link_exponent(L)
        m = max(np.max(np.abs(L.real)), np.max(np.abs(L.imag))) * 2.0 ** k
        assert 0.5 <= m < 1.0
        q = oracle.quantise_f16_links(L)
        # binary16 spacing at scaled magnitude < 1 is at most 2^-11; subnormals 2^-24
        assert np.max(np.abs(q - L)) * 2.0 ** k <= 2.0 ** -11 * np.sqrt(2)
