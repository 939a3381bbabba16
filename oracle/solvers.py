"""Flexible CG with a preconditioner, and the full-lattice solve of M = 2m + D by its
even-odd Schur complement; FP64 references (test infrastructure).

Flexible CG keeps only the last search direction (Notay's truncation to one):
    r = b - A x, z = N(r), p = z;
    repeat: q = A p, alpha = <p,r> / <p,q>, x += alpha p, r -= alpha q,
            z = N(r), beta = -<q,z> / <p,q>, p = z + beta p.
With N the identity this is CG step for step.  It falls back to plain CG from the current x
when z stops being finite, when Re<z,r> <= 0 (no descent), when |r| has not halved over the
last `stall` steps, or when the flexible budget runs out.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .core import apply_A, cg, dslash_eo, dslash_full, embed, restrict


@dataclass
class FCGInfo:
    iters: int
    fallback: bool
    fallback_iters: int
    true_rel_resid: float
    status: str


def fcg(g, sigma: float, b: np.ndarray, precond, tol: float, max_iter: int = 10000,
        stall: int = 50, x0: np.ndarray | None = None):
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0:
        return np.zeros_like(b), FCGInfo(0, False, 0, 0.0, "ok")
    r = b - apply_A(g, sigma, x)
    z = precond(r)
    p = z.copy()
    hist = [float(np.linalg.norm(r))]
    it = 0
    fallback = False
    while it < max_iter:
        zr = np.vdot(z, r)
        if not np.all(np.isfinite(z)) or zr.real <= 0:
            fallback = True
            break
        q = apply_A(g, sigma, p)
        pq = np.vdot(p, q).real
        alpha = np.vdot(p, r) / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        rn = float(np.linalg.norm(r))
        hist.append(rn)
        if rn <= tol * bnorm:
            rt = float(np.linalg.norm(b - apply_A(g, sigma, x)))
            if rt <= tol * bnorm:
                return x, FCGInfo(it, False, 0, rt / bnorm, "ok")
            r = b - apply_A(g, sigma, x)
        if len(hist) > stall and hist[-1] > 0.5 * hist[-1 - stall]:
            fallback = True
            break
        z = precond(r)
        beta = -np.vdot(q, z) / pq
        p = z + beta * p
    else:
        fallback = True
    x, info = cg(g, sigma, b, tol, max_iter=max(1, 10 * max_iter), x0=x)
    return x, FCGInfo(it + info.iters, fallback, info.iters, info.true_rel_resid, info.status)


@dataclass
class FullInfo:
    cg_iters: int
    cg_tol: float
    true_rel_resid: float


def apply_M(g, mass: float, x_e: np.ndarray, x_o: np.ndarray):
    """(M x) on both parities, M = 2m + D over the full lattice (no factor 1/2 in D)."""
    full = embed(g.dims, 0, x_e) + embed(g.dims, 1, x_o)
    y = 2.0 * mass * full + dslash_full(g, full)
    return restrict(g.dims, 0, y), restrict(g.dims, 1, y)


def full_solve(g, mass: float, b_e: np.ndarray, b_o: np.ndarray, tol: float):
    """Solves M x = b on the full lattice with |b - M x| <= tol |b|.

    Writing M in parity blocks [[2m, D_eo], [D_oe, 2m]] and eliminating the odd unknowns:
        (4 m^2 - D_eo D_oe) x_e = 2m b_e - D_eo b_o,      x_o = (b_o - D_oe x_e) / (2m).
    The even residual of M x = b is then r_e / (2m), r_e the residual of the even system, and
    the odd residual is zero, so the even system is solved to |r_e| <= 2m tol |b|.
    """
    bp = 2.0 * mass * b_e - dslash_eo(g, 0, b_o)
    nb = np.sqrt(np.linalg.norm(b_e) ** 2 + np.linalg.norm(b_o) ** 2)
    nbp = np.linalg.norm(bp)
    if nbp == 0.0:
        x_e = np.zeros_like(b_e)
        info_iters, cg_tol = 0, 0.0
    else:
        cg_tol = 2.0 * mass * tol * nb / nbp
        x_e, info = cg(g, 4.0 * mass * mass, bp, cg_tol)
        info_iters = info.iters
    x_o = (b_o - dslash_eo(g, 1, x_e)) / (2.0 * mass)
    me, mo = apply_M(g, mass, x_e, x_o)
    res = np.sqrt(np.linalg.norm(b_e - me) ** 2 + np.linalg.norm(b_o - mo) ** 2)
    return x_e, x_o, FullInfo(info_iters, cg_tol, float(res / nb) if nb > 0 else 0.0)


def _lattice_view(dims, full: np.ndarray) -> np.ndarray:
    """[V][3] (site index x + Nx (y + Ny (z + Nz t))) viewed as [t][z][y][x][3]."""
    nx, ny, nz, nt = dims
    return full.reshape(nt, nz, ny, nx, 3)


def _shift(dims, full: np.ndarray, mu: int, k: int) -> np.ndarray:
    """psi(x + k mu) at every site x (periodic; boundary signs live in the links)."""
    axis = 3 - mu      # x is the last lattice axis of the view
    v = _lattice_view(dims, full)
    return np.roll(v, -k, axis=axis).reshape(full.shape)


def parity_sign(dims) -> np.ndarray:
    """eps(x) = (-1)^(x+y+z+t) over the full lattice, [V]."""
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    return (1 - 2 * ((x + y + z + t) % 2)).reshape(-1).astype(np.float64)


def force_outer(g, residues, xs):
    """Link derivative of S = sum_i r_i phi^+ A_i^-1 phi given the solutions X_i = A_i^-1 phi.

    With Y_i = D_oe X_i and Psi_i = X_i on even sites, Y_i on odd sites, a variation of the
    links changes S by  sum_{x,mu} 2 Re Tr[dV_mu(x) FV_mu(x) + dW_mu(x) FW_mu(x)],
        FV_mu(x) = eps(x) sum_i r_i Psi_i(x+mu) Psi_i(x)^+,
        FW_mu(x) = eps(x) sum_i r_i Psi_i(x+3mu) Psi_i(x)^+,
    eps(x) = +1 on even and -1 on odd sites.  (dS_i = -X_i^+ dA_i X_i with
    dA_i = -(dD_eo D_oe + D_eo dD_oe), D anti-Hermitian for any links, so
    dS_i = X_i^+ dD_eo Y_i - Y_i^+ dD_oe X_i; each link enters D once forward and once as
    minus its adjoint backward.)  Returns FV, FW as [4][V][3][3] complex128.
    """
    dims = g.dims
    vol = int(np.prod(dims))
    eps = parity_sign(dims)
    fv = np.zeros((4, vol, 3, 3), dtype=np.complex128)
    fw = np.zeros((4, vol, 3, 3), dtype=np.complex128)
    for r, x in zip(residues, xs):
        y = dslash_eo(g, 1, x)
        psi = embed(dims, 0, x) + embed(dims, 1, y)
        for mu in range(4):
            p1 = _shift(dims, psi, mu, 1)
            p3 = _shift(dims, psi, mu, 3)
            fv[mu] += r * eps[:, None, None] * p1[:, :, None] * psi.conj()[:, None, :]
            fw[mu] += r * eps[:, None, None] * p3[:, :, None] * psi.conj()[:, None, :]
    return fv, fw


def rational_action(g, residues, sigmas, phi, tol: float = 1e-13):
    """S = sum_i r_i phi^+ (sigma_i - D_eo D_oe)^-1 phi by one CG solve per shift (real)."""
    s = 0.0
    for r, sg in zip(residues, sigmas):
        x, _ = cg(g, sg, phi, tol)
        s += r * float(np.vdot(phi, x).real)
    return s
