"""Pins of the oracle's CG and multi-shift CG: LAPACK dense solves at 4^4, independent
single-shift CG, true residuals, the Lanczos extremes against the dense spectrum, and the
recurrence's first step in closed form."""
import numpy as np
import pytest

import oracle
from ksinputs import make_gauge, gaussian_source
from conftest import rel_l2


def test_cg_matches_dense_solve(gauge44):
    m = 0.1
    sigma = 4 * m * m
    b = gaussian_source(128, 31)
    x, info = oracle.cg(gauge44, sigma, b, 1e-12)
    assert info.status == "ok" and info.true_rel_resid <= 1e-12
    A = oracle.dense_A(gauge44, sigma)
    xd = np.linalg.solve(A, b.ravel()).reshape(b.shape)
    w = np.linalg.eigvalsh(A)
    kappa = w[-1] / w[0]
    assert rel_l2(x, xd) <= 2 * 1e-12 * kappa


def test_cg_zero_source(gauge44):
    x, info = oracle.cg(gauge44, 0.04, np.zeros((128, 3), complex), 1e-10)
    assert info.status == "ok" and np.all(x == 0)


def test_cg_not_converged_flag(gauge44):
    b = gaussian_source(128, 5)
    x, info = oracle.cg(gauge44, 0.04, b, 1e-12, max_iter=3, max_restarts=0)
    assert info.status == "not converged" and info.iters == 3


def test_cg_restart_from_initial_guess(gauge8):
    sigma = 4 * 0.1 ** 2
    b = gaussian_source(2048, 2001)
    x1, i1 = oracle.cg(gauge8, sigma, b, 1e-6)
    x2, i2 = oracle.cg(gauge8, sigma, b, 1e-11, x0=x1)
    x3, i3 = oracle.cg(gauge8, sigma, b, 1e-11)
    assert i2.true_rel_resid <= 1e-11 and i2.iters < i3.iters
    assert rel_l2(x2, x3) <= 1e-8


def test_lanczos_extremes_inside_dense_spectrum(gauge44):
    sigma = 4 * 0.05 ** 2
    b = gaussian_source(128, 17)
    _, info = oracle.cg(gauge44, sigma, b, 1e-13)
    lo, hi = oracle.lanczos_extremes(info.alpha, info.beta)
    w = np.linalg.eigvalsh(oracle.dense_A(gauge44, sigma))
    # Ritz values lie inside the spectrum; after full convergence the extremes are found
    assert w[0] * (1 - 1e-8) <= lo and hi <= w[-1] * (1 + 1e-8)
    assert abs(lo - w[0]) <= 1e-6 * w[0] and abs(hi - w[-1]) <= 1e-6 * w[-1]


def test_multishift_matches_dense(gauge44):
    masses = np.geomspace(0.002, 0.5, 9)
    sig = 4 * masses ** 2
    b = gaussian_source(128, 41)
    xs, iters, res, st = oracle.multishift_cg(gauge44, sig, b, 1e-11)
    assert st == "ok"
    A0 = oracle.dense_A(gauge44, 0.0)
    for i, s in enumerate(sig):
        A = A0 + s * np.eye(A0.shape[0])
        xd = np.linalg.solve(A, b.ravel()).reshape(b.shape)
        w = np.linalg.eigvalsh(A)
        assert res[i] <= 1e-10
        assert rel_l2(xs[i], xd) <= 2 * 1e-10 * w[-1] / w[0]


def test_multishift_matches_single_shift_cg(gauge8):
    sig = [0.01, 0.09, 0.5]
    b = gaussian_source(2048, 43)
    xs, iters, res, st = oracle.multishift_cg(gauge8, sig, b, 1e-11)
    assert st == "ok" and np.all(res <= 2e-11)
    for i, s in enumerate(sig):
        x, info = oracle.cg(gauge8, s, b, 1e-11)
        assert rel_l2(xs[i], x) <= 1e-8
    # the smallest shift is the base system: its iteration count bounds the loop
    _, info0 = oracle.cg(gauge8, min(sig), b, 1e-11)
    assert abs(iters - info0.iters) <= 2


def test_multishift_first_step_closed_form(gauge44):
    """After one step, x_i = alpha_0 zeta_1 b with zeta_1 = 1 / (1 + delta_i alpha_0) and
    alpha_0 = |b|^2 / <b, A_0 b>: the residual b - (A_0 + delta) x_i is collinear with r_1."""
    sig = np.array([0.01, 0.3, 1.2])
    b = gaussian_source(128, 45)
    xs, iters, res, st = oracle.multishift_cg(gauge44, sig, b, 1e-30, max_iter=1)
    assert iters == 1
    Ab = oracle.apply_A(gauge44, sig[0], b)
    a0 = np.vdot(b, b).real / np.vdot(b, Ab).real
    r1 = b - a0 * Ab
    for i, s in enumerate(sig):
        z1 = 1.0 / (1.0 + (s - sig[0]) * a0)
        assert rel_l2(xs[i], a0 * z1 * b) <= 1e-14
        ri = b - oracle.apply_A(gauge44, s, xs[i])
        assert rel_l2(ri, z1 * r1) <= 1e-13


@pytest.mark.slow
def test_config1_cg(gauge8):
    """The 8^4, m = 0.1 workload solved to true relative residual 1e-10."""
    b = gaussian_source(2048, 2001)
    x, info = oracle.cg(gauge8, 4 * 0.1 ** 2, b, 1e-10)
    assert info.status == "ok" and info.true_rel_resid <= 1e-10
    lo, hi = oracle.lanczos_extremes(info.alpha, info.beta)
    assert 0.04 * (1 - 1e-9) <= lo < hi


def dense_M(g, mass):
    """M = 2m + D as a dense matrix over the full lattice, column by column from unit vectors."""
    n = g.volume * 3
    M = np.empty((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros((g.volume, 3), dtype=np.complex128)
        e.flat[j] = 1.0
        M[:, j] = (2 * mass * e + oracle.dslash_full(g, e)).ravel()
    return M


def test_full_solve_matches_dense_M(gauge44):
    """The even-odd Schur solve with odd reconstruction solves M x = b: it agrees with LAPACK
    on the dense M within tol * cond(M), and its M (assembled by parity) is the dense one."""
    g, m, tol = gauge44, 0.1, 1e-11
    rng = np.random.default_rng(5)
    b_e = gaussian_source(128, 41)
    b_o = gaussian_source(128, 42)
    x_e, x_o, info = oracle.full_solve(g, m, b_e, b_o, tol)
    assert info.true_rel_resid <= tol
    M = dense_M(g, m)
    b = oracle.embed(g.dims, 0, b_e) + oracle.embed(g.dims, 1, b_o)
    xd = np.linalg.solve(M, b.ravel()).reshape(b.shape)
    x = oracle.embed(g.dims, 0, x_e) + oracle.embed(g.dims, 1, x_o)
    assert rel_l2(x, xd) <= 2 * tol * np.linalg.cond(M)
    # apply_M against the dense matrix on a random vector
    v = rng.standard_normal((256, 3)) + 1j * rng.standard_normal((256, 3))
    me, mo = oracle.apply_M(g, m, oracle.restrict(g.dims, 0, v), oracle.restrict(g.dims, 1, v))
    mv = (M @ v.ravel()).reshape(v.shape)
    assert rel_l2(oracle.embed(g.dims, 0, me) + oracle.embed(g.dims, 1, mo), mv) <= 1e-14


def test_full_solve_even_block_is_the_normal_operator(gauge8):
    """M^+ M restricted to even sites is A = 4 m^2 - D_eo D_oe (D anti-Hermitian), checked
    against the C oracle's A; and with b_o = 0 the even solution is 2m A^-1 b_e."""
    g, m = gauge8, 0.1
    vh = g.volume // 2
    x = gaussian_source(vh, 43)
    me, mo = oracle.apply_M(g, m, x, np.zeros_like(x))
    # M^+ = 2m - D
    full = oracle.embed(g.dims, 0, me) + oracle.embed(g.dims, 1, mo)
    mtm = 2 * m * full - oracle.dslash_full(g, full)
    assert rel_l2(oracle.restrict(g.dims, 0, mtm), oracle.apply_A(g, 4 * m * m, x)) <= 1e-13
    assert np.abs(oracle.restrict(g.dims, 1, mtm)).max() <= 1e-12 * np.abs(mtm).max()
    b = gaussian_source(vh, 44)
    x_e, x_o, info = oracle.full_solve(g, m, b, np.zeros_like(b), 1e-12)
    xc, _ = oracle.cg(g, 4 * m * m, b, 1e-13)
    assert rel_l2(x_e, 2 * m * xc) <= 1e-10
    assert info.true_rel_resid <= 1e-12
