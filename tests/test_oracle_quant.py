"""Pins of the quantise-then-FP64 references against the binary16/binary32 formats' own
rounding bounds (unit roundoff 2^-11 for binary16, 2^-24 for binary32)."""
import numpy as np

import oracle
from conftest import rel_l2
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


def test_f16_sites_is_a_binary32_encoding():
    """Every decoded real is n * h with n a binary32 number and h a binary16 number of modulus
    at most 1, and encoding twice changes nothing (the decoded values are representable)."""
    v = gaussian_source(500, 3) * np.geomspace(1e-5, 1e4, 500)[:, None]
    q = oracle.quantise_f16_sites(v)
    assert np.array_equal(oracle.quantise_f16_sites(q), q)
    re = np.stack([q.real, q.imag], -1).reshape(500, 6)
    n = np.max(np.abs(re), axis=1)
    assert np.array_equal(n.astype(np.float32).astype(np.float64), n)
    h = re / n[:, None]
    assert np.all(np.abs(h) <= 1.0)
    assert np.array_equal(h.astype(np.float16).astype(np.float64), h)


def test_rebuild_su3_reproduces_su3():
    from ksinputs import random_su3
    U = random_su3(np.random.default_rng(4), 200, 1.5)
    R = oracle.rebuild_su3(U[:, :2, :])
    assert np.max(np.abs(R - U)) <= 1e-14


def test_naik_is_scale_times_phase_times_su3():
    """The recipe's Naik links divided by c0 * eta * bc3 are SU(3): unitary, determinant 1
    (pins the sign pattern the 12-real storage divides out)."""
    g = make_gauge((6, 4, 4, 8), 0.5, 21)
    c0 = oracle.naik12_scale(g.naik)
    assert abs(c0 - (-1.0 / 24.0)) <= 1e-15
    U = g.naik / (c0 * oracle.naik_phase(g.dims)[..., None, None])
    eye = np.eye(3)
    assert np.max(np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - eye)) <= 1e-13
    assert np.max(np.abs(np.linalg.det(U) - 1.0)) <= 1e-13


def test_link_store_values():
    """12-real FP64 storage reproduces W; in FP32 / binary16 every entry of both copies is
    within the format's rounding of W (rows 0, 1) or of its rebuilt row; the 8-way backward
    copy is rounded separately (it differs from the forward copy), the 4-way one is the
    forward copy; 18-real storage is the plain rounding of both classes."""
    g = make_gauge((6, 4, 4, 8), 0.5, 22)
    for access in (8, 4):
        f, b = oracle.link_store_values(g, "f64", 12, access)
        assert np.max(np.abs(f.naik - g.naik)) <= 1e-16
        assert np.max(np.abs(b.naik - g.naik)) <= 1e-16
        assert np.array_equal(f.fat, g.fat)
    for prec, u in (("f32", 2.0 ** -24), ("f16", 2.0 ** -11)):
        f, b = oracle.link_store_values(g, prec, 12, 8)
        # entries of SU(3) have modulus <= 1; row 2 is a sum of two products of rounded entries
        for L in (f.naik, b.naik):
            err = np.abs(L - g.naik) * 24.0
            assert np.max(err[..., :2, :]) <= np.sqrt(2) * u
            assert np.max(err) <= 6 * u
        assert np.max(np.abs(f.naik - b.naik)) > 0
        f4, b4 = oracle.link_store_values(g, prec, 12, 4)
        assert f4 is b4 and np.array_equal(f4.naik, f.naik)
        f18, b18 = oracle.link_store_values(g, prec, 18, 8)
        assert f18 is b18
        ref = oracle.quantise_f32 if prec == "f32" else oracle.quantise_f16_links
        assert np.array_equal(f18.naik, ref(g.naik)) and np.array_equal(f18.fat, ref(g.fat))


def _point_columns(dims, y_site):
    """Checkerboard rows of y and of y -+ k mu for the even-odd layout."""
    nx, ny, nz, nt = dims
    c = [y_site % nx, (y_site // nx) % ny, (y_site // (nx * ny)) % nz, y_site // (nx * ny * nz)]

    def idx(cc):
        cc = [cc[k] % dims[k] for k in range(4)]
        return cc[0] + nx * (cc[1] + ny * (cc[2] + nz * cc[3]))
    return c, idx


def test_dslash_eo_fb_splits_forward_and_backward_hops():
    """A point source at odd site y: the even site y - k mu receives A_mu(y - k mu) psi(y)
    (forward hop, from fwd) and y + k mu receives -B_mu(y)^+ psi(y) (backward hop, from bwd);
    with fwd = bwd the operator is the oracle's D."""
    from ksinputs import GaugeField
    dims = (8, 8, 8, 10)
    A = make_gauge(dims, 0.5, 31)
    B = make_gauge(dims, 0.5, 32)
    vh = A.volume // 2
    y = 1 + 8 * (2 + 8 * (3 + 8 * 5))         # x=1, y=2, z=3, t=5: odd (extents >= 8: no two hops land on one site)
    c, idx = _point_columns(dims, y)
    psi = np.zeros((vh, 3), complex)
    chi = np.array([0.3 - 0.2j, 1.1, -0.4j])
    psi[y >> 1] = chi
    out = oracle.dslash_eo_fb(A, B, 0, psi)
    for mu in range(4):
        for k, W, Bw in ((1, A.fat, B.fat), (3, A.naik, B.naik)):
            cm = list(c)
            cm[mu] -= k
            xm = idx(cm)
            assert np.allclose(out[xm >> 1], W[mu, xm] @ chi, atol=1e-15)
            cp = list(c)
            cp[mu] += k
            xp = idx(cp)
            assert np.allclose(out[xp >> 1], -np.conj(Bw[mu, y]).T @ chi, atol=1e-15)
    assert np.count_nonzero(np.abs(out).sum(1)) == 16
    psi = gaussian_source(vh, 33)
    same = GaugeField(dims, A.fat.copy(), A.naik.copy())
    assert rel_l2(oracle.dslash_eo_fb(A, same, 1, psi), oracle.dslash_eo(A, 1, psi)) <= 1e-14


def test_dslash_eo_abs():
    """On a point source it is |L| |chi| at every receiving site (moduli, no signs); for any
    input it bounds |D psi| component by component."""
    dims = (8, 8, 8, 10)
    A = make_gauge(dims, 0.5, 34)
    vh = A.volume // 2
    y = 1 + 8 * (2 + 8 * (3 + 8 * 5))
    c, idx = _point_columns(dims, y)
    psi = np.zeros((vh, 3), complex)
    chi = np.array([0.3 - 0.2j, 1.1, -0.4j])
    psi[y >> 1] = chi
    S = oracle.dslash_eo_abs(A, 0, psi)
    for mu in range(4):
        for k, W in ((1, A.fat), (3, A.naik)):
            cm = list(c)
            cm[mu] -= k
            xm = idx(cm)
            assert np.allclose(S[xm >> 1], np.abs(W[mu, xm]) @ np.abs(chi), atol=1e-15)
            cp = list(c)
            cp[mu] += k
            assert np.allclose(S[idx(cp) >> 1], np.abs(W[mu, y]).T @ np.abs(chi), atol=1e-15)
    psi = gaussian_source(vh, 35)
    for par in (0, 1):
        D = oracle.dslash_eo(A, par, psi)
        S = oracle.dslash_eo_abs(A, par, psi)
        assert np.all(np.abs(D.real) <= S * (1 + 1e-14)) and np.all(np.abs(D.imag) <= S * (1 + 1e-14))


def test_elementwise_bound_discriminates():
    """The element-wise parity bound used on the GPU outputs accepts the reference rounded to
    each storage format and rejects an operator with one link of one site negated."""
    import dslash_check as dc
    from ksinputs import GaugeField
    dims = (8, 6, 10, 12)
    g = make_gauge(dims, 0.5, 36)
    vh = g.volume // 2
    psi = gaussian_source(vh, 37)
    for prec in ("f64", "f32", "f16"):
        for recon in (18, 12):
            ref, S = dc.reference(g, prec, recon, 8, 0, psi)
            out = {"f64": ref, "f32": oracle.quantise_f32(ref),
                   "f16": oracle.quantise_f16_sites(ref)}[prec]
            assert dc.worst(out, ref, S, prec) <= 1.0
            fwd, bwd = oracle.link_store_values(g, prec, recon, 8)
            bad = GaugeField(dims, fwd.fat, fwd.naik.copy())
            bad.naik[2, 1235] *= -1.0      # an even site: a forward hop of the even output
            q = {"f64": psi, "f32": oracle.quantise_f32(psi),
                 "f16": oracle.quantise_f16_sites(psi)}[prec]
            wrong = oracle.dslash_eo_fb(bad, bwd, 0, q)
            assert dc.worst(wrong, ref, S, prec) > 4.0
