"""Pins of the FP64 oracle's operator against facts fixed by the mathematics.

None of these re-derive the oracle's own loop: anti-Hermiticity, the closed-form free-field
action, gauge covariance, the explicit column structure for a point source, and the dense
4^4 spectrum would each fail for a dropped term, a wrong sign, a wrong link index or a
transposed matrix.
"""
import numpy as np
import pytest

import oracle
from ksinputs import (make_gauge, GaugeField, lattice_coords, staggered_phase, time_bc_sign,
                      random_su3, gaussian_source, gaussian_full)
from conftest import cvdot, rel_l2


def _rand_cb(vh, seed):
    return gaussian_source(vh, seed)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 8, 4), (8, 8, 4, 6)])
def test_anti_hermitian_eo(dims):
    g = make_gauge(dims, 0.5, 7)
    vh = int(np.prod(dims)) // 2
    xo = _rand_cb(vh, 1)
    ye = _rand_cb(vh, 2)
    lhs = cvdot(xo, oracle.dslash_eo(g, 1, ye))
    rhs = -cvdot(oracle.dslash_eo(g, 0, xo), ye)
    scale = np.linalg.norm(xo) * np.linalg.norm(ye) * 16
    assert abs(lhs - rhs) <= 1e-14 * scale


def test_anti_hermitian_full(gauge44):
    V = 256
    x = gaussian_full(V, 3)
    y = gaussian_full(V, 4)
    lhs = cvdot(x, oracle.dslash_full(gauge44, y))
    rhs = -cvdot(oracle.dslash_full(gauge44, x), y)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def free_field(dims, c1, c3):
    x, y, z, t = lattice_coords(dims)
    V = len(x)
    fat = np.zeros((4, V, 3, 3), dtype=np.complex128)
    naik = np.zeros_like(fat)
    for mu in range(4):
        eta = staggered_phase(mu, x, y, z, t)
        b1 = time_bc_sign(1, t, dims[3]) if mu == 3 else 1.0
        b3 = time_bc_sign(3, t, dims[3]) if mu == 3 else 1.0
        fat[mu] = (c1 * eta * b1)[:, None, None] * np.eye(3)
        naik[mu] = (c3 * eta * b3)[:, None, None] * np.eye(3)
    return GaugeField(tuple(dims), fat, naik)


def plane_wave(dims, n, chi):
    x, y, z, t = lattice_coords(dims)
    p = [2 * np.pi * n[0] / dims[0], 2 * np.pi * n[1] / dims[1], 2 * np.pi * n[2] / dims[2],
         2 * np.pi * (n[3] + 0.5) / dims[3]]
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return ph[:, None] * np.asarray(chi)[None, :], p


COEFFS = [(1.0, 0.0), (9.0 / 8.0, -1.0 / 24.0), (0.9, -1.0 / 24.0)]


@pytest.mark.parametrize("c1,c3", COEFFS)
@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 2, 0, 3), (3, 1, 2, 1)])
def test_free_field_pointwise(c1, c3, n):
    dims = (4, 8, 4, 6)
    g = free_field(dims, c1, c3)
    chi = np.array([0.3 + 0.1j, -0.7j, 1.1])
    psi, p = plane_wave(dims, n, chi)
    x, y, z, t = lattice_coords(dims)
    s = [c1 * np.sin(pm) + c3 * np.sin(3 * pm) for pm in p]
    fac = 2j * sum(staggered_phase(mu, x, y, z, t) * s[mu] for mu in range(4))
    expect = fac[:, None] * psi
    got = oracle.dslash_full(g, psi)
    assert np.max(np.abs(got - expect)) <= 1e-13 * max(np.max(np.abs(expect)), 1.0)


@pytest.mark.parametrize("c1,c3", COEFFS)
def test_free_field_A_eigen(c1, c3):
    dims = (4, 4, 8, 6)
    g = free_field(dims, c1, c3)
    sigma = 4 * 0.1 ** 2
    chi = np.array([1.0, 0.5j, -0.25])
    for n in [(0, 0, 0, 0), (1, 0, 3, 2), (2, 3, 5, 4)]:
        psi, p = plane_wave(dims, n, chi)
        psi_e = oracle.restrict(dims, 0, psi)
        s2 = sum((c1 * np.sin(pm) + c3 * np.sin(3 * pm)) ** 2 for pm in p)
        got = oracle.apply_A(g, sigma, psi_e)
        assert rel_l2(got, (sigma + 4 * s2) * psi_e) <= 1e-13


def _gauge_transform(g, G):
    """V'_mu(x) = G(x) V_mu(x) G(x+mu)^+ and W'_mu(x) = G(x) W_mu(x) G(x+3mu)^+."""
    nx, ny, nz, nt = g.dims
    V = g.volume
    i = np.arange(V)
    c = [i % nx, (i // nx) % ny, (i // (nx * ny)) % nz, i // (nx * ny * nz)]
    n = [nx, ny, nz, nt]

    def shifted(mu, k):
        cc = list(c)
        cc[mu] = (c[mu] + k) % n[mu]
        return cc[0] + nx * (cc[1] + ny * (cc[2] + nz * cc[3]))

    Gd = np.conj(np.swapaxes(G, -1, -2))
    fat = np.empty_like(g.fat)
    naik = np.empty_like(g.naik)
    for mu in range(4):
        fat[mu] = G @ g.fat[mu] @ Gd[shifted(mu, 1)]
        naik[mu] = G @ g.naik[mu] @ Gd[shifted(mu, 3)]
    return GaugeField(g.dims, fat, naik)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 6, 4, 8)])
def test_gauge_covariance(dims):
    g = make_gauge(dims, 0.5, 21)
    V = g.volume
    G = random_su3(np.random.default_rng(5), V, 1.7)
    gp = _gauge_transform(g, G)
    psi = gaussian_full(V, 8)
    lhs = oracle.dslash_full(gp, np.einsum("vab,vb->va", G, psi))
    rhs = np.einsum("vab,vb->va", G, oracle.dslash_full(g, psi))
    assert rel_l2(lhs, rhs) <= 1e-13


def test_point_source_columns(gauge8):
    """For psi = unit vector e_a at site y, (D psi)(x) is column a of the link that connects x
    to y: V_mu(y-mu) at x = y-mu, -V_mu(y)^+ at x = y+mu, W_mu(y-3mu) at x = y-3mu and
    -W_mu(y)^+ at x = y+3mu, and zero on every other site."""
    g = gauge8
    dims = g.dims
    n = list(dims)
    V = g.volume

    def idx(c):
        return c[0] + n[0] * (c[1] + n[1] * (c[2] + n[2] * c[3]))

    yc = [3, 5, 1, 6]
    y = idx(yc)
    for a in range(3):
        psi = np.zeros((V, 3), dtype=np.complex128)
        psi[y, a] = 1.0
        out = oracle.dslash_full(g, psi)
        expect = np.zeros_like(out)
        for mu in range(4):
            def at(k):
                c = list(yc)
                c[mu] = (c[mu] + k) % n[mu]
                return idx(c)
            expect[at(-1)] += g.fat[mu, at(-1)][:, a]
            expect[at(+1)] += -np.conj(g.fat[mu, y][a, :])
            expect[at(-3)] += g.naik[mu, at(-3)][:, a]
            expect[at(+3)] += -np.conj(g.naik[mu, y][a, :])
        assert np.max(np.abs(out - expect)) <= 1e-15


def test_embed_restrict_roundtrip():
    dims = (4, 6, 4, 8)
    vh = int(np.prod(dims)) // 2
    v = _rand_cb(vh, 9)
    for par in (0, 1):
        full = oracle.embed(dims, par, v)
        x, y, z, t = lattice_coords(dims)
        par_site = (x + y + z + t) & 1
        assert np.all(full[par_site != par] == 0)
        assert np.array_equal(oracle.restrict(dims, par, full), v)
        # each checkerboard row is the site of that parity with index i >> 1
        sites = np.nonzero(par_site == par)[0]
        assert np.array_equal(sites >> 1, np.arange(vh))


def test_dense_4444_spectrum_random(gauge44):
    m = 0.1
    sigma = 4 * m * m
    A = oracle.dense_A(gauge44, sigma)
    assert np.max(np.abs(A - A.conj().T)) <= 1e-13 * np.max(np.abs(A))
    w = np.linalg.eigvalsh(A)
    assert w[0] >= sigma * (1 - 1e-12)


@pytest.mark.parametrize("c1,c3", COEFFS)
def test_dense_4444_free_spectrum(c1, c3):
    dims = (4, 4, 4, 4)
    g = free_field(dims, c1, c3)
    sigma = 4 * 0.1 ** 2
    w = np.sort(np.linalg.eigvalsh(oracle.dense_A(g, sigma)))
    ex = []
    for n0 in range(4):
        for n1 in range(4):
            for n2 in range(4):
                for n3 in range(4):
                    p = [2 * np.pi * n0 / 4, 2 * np.pi * n1 / 4, 2 * np.pi * n2 / 4,
                         2 * np.pi * (n3 + 0.5) / 4]
                    s2 = sum((c1 * np.sin(q) + c3 * np.sin(3 * q)) ** 2 for q in p)
                    ex.append(sigma + 4 * s2)
    # p and p + (pi,pi,pi,pi) coincide on even sites: each class once, times three colours
    ex = np.sort(np.repeat(np.sort(ex)[::2], 3))
    assert np.max(np.abs(w - ex)) <= 1e-12 * max(ex)


def test_bad_dims_rejected():
    g = free_field((4, 4, 4, 4), 1.0, 0.0)
    g.dims = (5, 4, 4, 4)
    with pytest.raises(oracle.OracleError):
        oracle.dslash_full(g, np.zeros((320, 3), dtype=np.complex128))
