"""Pins of the oracle's two-level smeared links: the nested staple sums against an explicit
walk over every path at one site; unit links; gauge covariance; the U(3) projection against
the SVD polar factor; and the level-1 smearing's response to an abelian plane wave along mu,
which must be prod_{nu != mu} (1 + cos k_nu) / 2 (so a gluon with momentum pi in any
transverse direction does not couple: the taste-changing suppression the smearing is for)."""
import itertools

import numpy as np
import pytest

from oracle import hisq
from ksinputs import thin_links

DIMS = (4, 4, 4, 6)


def coords(dims, i):
    nx, ny, nz, nt = dims
    return [i % nx, (i // nx) % ny, (i // (nx * ny)) % nz, i // (nx * ny * nz)]


def index(dims, c):
    nx, ny, nz, nt = dims
    c = [c[k] % dims[k] for k in range(4)]
    return c[0] + nx * (c[1] + ny * (c[2] + nz * c[3]))


def walk(U, dims, site, steps):
    """Product of the links along a path of signed unit steps (axis, +-1) from `site`."""
    c = coords(dims, site)
    m = np.eye(3, dtype=complex)
    for ax, s in steps:
        if s > 0:
            m = m @ U[ax, index(dims, c)]
            c[ax] += 1
        else:
            c[ax] -= 1
            m = m @ np.conj(U[ax, index(dims, c)]).T
    return m


def paths_sum(U, dims, site, mu, coeffs):
    c1, c3, c5, c7, cL = coeffs
    dirs = [(nu, s) for nu in range(4) if nu != mu for s in (1, -1)]
    inv = lambda p: [(a, -s) for a, s in reversed(p)]
    total = c1 * U[mu, site]
    for a in dirs:
        total = total + c3 * walk(U, dims, site, [a, (mu, 1)] + inv([a]))
        total = total + cL * walk(U, dims, site, [a, a, (mu, 1)] + inv([a, a]))
    for a, b in itertools.permutations(dirs, 2):
        if a[0] == b[0]:
            continue
        total = total + c5 * walk(U, dims, site, [a, b, (mu, 1)] + inv([a, b]))
    for a, b, c in itertools.permutations(dirs, 3):
        if len({a[0], b[0], c[0]}) < 3:
            continue
        total = total + c7 * walk(U, dims, site, [a, b, c, (mu, 1)] + inv([a, b, c]))
    return total


@pytest.fixture(scope="module")
def U():
    return thin_links(DIMS, 0.5, 111)


@pytest.mark.parametrize("coeffs", [hisq.LEVEL1, hisq.LEVEL2, (0.3, -0.7, 1.1, 0.9, 0.4)])
def test_smear_equals_explicit_path_walk(U, coeffs):
    F = hisq.smear(U, DIMS, coeffs)
    for site, mu in ((0, 0), (77, 3), (200, 1), (383, 2)):
        ref = paths_sum(U, DIMS, site, mu, coeffs)
        assert np.max(np.abs(F[mu, site] - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_unit_links():
    V = np.zeros((4, int(np.prod(DIMS)), 3, 3), dtype=complex)
    V[..., [0, 1, 2], [0, 1, 2]] = 1.0
    X, N = hisq.hisq_links(V, DIMS, signs=False)
    assert np.allclose(X, 9.0 / 8.0 * V, atol=1e-14)
    assert np.allclose(N, -1.0 / 24.0 * V, atol=1e-15)
    assert np.allclose(hisq.smear(V, DIMS, hisq.LEVEL1), V, atol=1e-14)


def test_gauge_covariance(U):
    g = thin_links(DIMS, 0.9, 112)[0]      # a random SU(3) matrix per site
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[mu] = g @ U[mu] @ hisq.dagger(hisq.shift(g, DIMS, mu, 1))
    X, N = hisq.hisq_links(U, DIMS)
    Xg, Ng = hisq.hisq_links(Ug, DIMS)
    for mu in range(4):
        assert np.allclose(Xg[mu], g @ X[mu] @ hisq.dagger(hisq.shift(g, DIMS, mu, 1)),
                           atol=1e-12)
        assert np.allclose(Ng[mu], g @ N[mu] @ hisq.dagger(hisq.shift(g, DIMS, mu, 3)),
                           atol=1e-13)


def test_u3_projection_is_the_polar_factor(U):
    V = hisq.smear(U, DIMS, hisq.LEVEL1)
    W = hisq.u3_project(V)
    eye = np.eye(3)
    assert np.max(np.abs(hisq.dagger(W) @ W - eye)) <= 1e-13
    p, _, qh = np.linalg.svd(V)
    assert np.max(np.abs(W - p @ qh)) <= 1e-12
    assert np.max(np.abs(hisq.u3_project(U) - U)) <= 1e-13   # unitary input is fixed


@pytest.mark.parametrize("mu", [0, 3])
def test_level1_abelian_form_factor(mu):
    """U_mu(x) = exp(i e cos(k.x)) (others 1): V_mu(x) - 1 = i e f(k) cos(k.x) + O(e^2) with
    f(k) = prod_{nu != mu} (1 + cos k_nu) / 2."""
    vol = int(np.prod(DIMS))
    nx, ny, nz, nt = DIMS
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    xs = [a.reshape(-1) for a in (x, y, z, t)]
    eps = 1e-7
    for ks in itertools.product(*[np.arange(d) * 2 * np.pi / d for d in DIMS]):
        if sum(ks) > 7:      # a spread of momenta keeps the test short
            continue
        phase = sum(k * c for k, c in zip(ks, xs))
        U = np.zeros((4, vol, 3, 3), dtype=complex)
        U[..., [0, 1, 2], [0, 1, 2]] = 1.0
        U[mu] *= np.exp(1j * eps * np.cos(phase))[:, None, None]
        V = hisq.smear(U, DIMS, hisq.LEVEL1)
        resp = (V[mu, :, 0, 0] - 1.0) / (1j * eps)
        f = np.prod([(1 + np.cos(ks[nu])) / 2 for nu in range(4) if nu != mu])
        assert np.max(np.abs(resp - f * np.cos(phase))) <= 1e-6


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 0, 2, 1), (3, 1, 0, 4)])
def test_signs_of_unit_links_give_the_free_operator(n):
    """fold_signs, pinned through the closed-form free field: unit thin links give the
    unsigned X = 9/8 and N = -1/24; with the staggered phases and the antiperiodic time signs
    folded in, D on an antiperiodic plane wave psi = e^{ip.x} chi must be
    2i sum_mu eta_mu(x) s_mu(p) psi(x), s_mu = (9/8) sin p_mu - (1/24) sin 3p_mu (the free
    operator's closed form).  A wrong eta, a one-link boundary sign on the wrong slice or a
    three-link sign on the wrong slices breaks it."""
    import oracle
    from ksinputs import GaugeField, lattice_coords, staggered_phase
    dims = (4, 6, 4, 8)
    vol = int(np.prod(dims))
    U = np.zeros((4, vol, 3, 3), dtype=complex)
    U[..., [0, 1, 2], [0, 1, 2]] = 1.0
    X, N = hisq.hisq_links(U, dims, signs=True)
    g = GaugeField(dims, X, N)
    x, y, z, t = lattice_coords(dims)
    p = [2 * np.pi * n[0] / dims[0], 2 * np.pi * n[1] / dims[1], 2 * np.pi * n[2] / dims[2],
         2 * np.pi * (n[3] + 0.5) / dims[3]]
    chi = np.array([0.3 + 0.1j, -0.7j, 1.1])
    psi = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))[:, None] * chi[None, :]
    s = [9.0 / 8.0 * np.sin(pm) - np.sin(3 * pm) / 24.0 for pm in p]
    expect = (2j * sum(staggered_phase(mu, x, y, z, t) * s[mu] for mu in range(4)))[:, None] * psi
    got = oracle.dslash_full(g, psi)
    assert np.max(np.abs(got - expect)) <= 1e-13 * max(np.max(np.abs(expect)), 1.0)


def test_signs_count_boundary_crossings():
    """Every folded sign is eta_mu(x) times (-1)^(number of times the hop from x crosses the
    time boundary), with the crossings counted as floor((t + hops) / Nt)."""
    dims = (4, 4, 4, 6)
    vol = int(np.prod(dims))
    U = np.zeros((4, vol, 3, 3), dtype=complex)
    U[..., [0, 1, 2], [0, 1, 2]] = 1.0
    X, N = hisq.fold_signs(U, 2.0 * U, dims)
    for i in range(vol):
        c = coords(dims, i)
        for mu in range(4):
            eta = (-1.0) ** (sum(c[:mu]))
            for L, hops, f in ((X, 1, 1.0), (N, 3, 2.0)):
                cross = (c[3] + hops) // dims[3] if mu == 3 else 0
                assert L[mu, i, 1, 1] == f * eta * (-1.0) ** cross
