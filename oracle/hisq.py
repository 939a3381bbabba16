"""Two-level smeared (HISQ-type) fat and Naik links from thin links, FP64 reference (test
infrastructure).

Staple in the signed transverse direction (nu, s) of a field M living on mu-links:
    S_{nu,s}[M](x) = L(x) M(x + s nu) L(x + mu)^+,
with L(y) = U_nu(y) for s = +1 (the link from y to y + nu) and L(y) = U_nu(y - nu)^+ for
s = -1 (the link from y to y - nu).  A smearing with coefficients (c1, c3, c5, c7, cL) is the
path sum
    F_mu = c1 U_mu + c3 sum_a S_a[U_mu] + c5 sum_{a,b} S_a[S_b[U_mu]]
           + c7 sum_{a,b,c} S_a[S_b[S_c[U_mu]]] + cL sum_a S_a[S_a[U_mu]],
a, b, c signed directions on distinct axes, all transverse to mu (6, 24 and 48 terms; the
last sum is the 6 double-width staples).  It is evaluated here by the nesting
    F_mu = c1 U + cL sum_a S_a[S_a[U]] + sum_a S_a[ c3 U + sum_b S_b[ c5 U + c7 sum_c S_c[U] ] ],
which equals the path sum because each staple is linear in M.

Links: level 1 V = F(U; 1/8, 1/16, 1/64, 1/384, 0); projection W = V (V^+ V)^(-1/2) onto U(3);
level 2 X = F(W; 1, 1/16, 1/64, 1/384, -1/8); Naik N_mu(x) = -1/24 W_mu(x) W_mu(x+mu) W_mu(x+2mu).
For unit links V = W = 1, X = 9/8 and N = -1/24, so the free operator's derivative has
9/8 sin p - (1/24) sin 3p = p + O(p^3).  The staggered phases eta_mu(x) and the antiperiodic
time sign are folded into X and N afterwards (each path from x to x + mu crosses the time
boundary as often, mod 2, as the direct hop).
"""
from __future__ import annotations

import numpy as np

LEVEL1 = (1.0 / 8, 1.0 / 16, 1.0 / 64, 1.0 / 384, 0.0)
LEVEL2 = (1.0, 1.0 / 16, 1.0 / 64, 1.0 / 384, -1.0 / 8)
NAIK = -1.0 / 24


def dagger(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


def shift(a: np.ndarray, dims, mu: int, k: int) -> np.ndarray:
    """a(x + k mu) for a per-site array a[V, ...] (periodic wrap)."""
    nx, ny, nz, nt = dims
    v = a.reshape((nt, nz, ny, nx) + a.shape[1:])
    return np.roll(v, -k, axis=3 - mu).reshape(a.shape)


def hop(U: np.ndarray, dims, nu: int, s: int) -> np.ndarray:
    """The link from x to x + s nu, at every x."""
    return U[nu] if s > 0 else dagger(shift(U[nu], dims, nu, -1))


def staple(U: np.ndarray, dims, mu: int, nu: int, s: int, M: np.ndarray) -> np.ndarray:
    L = hop(U, dims, nu, s)
    return L @ shift(M, dims, nu, s) @ dagger(shift(L, dims, mu, 1))


def smear(U: np.ndarray, dims, coeffs) -> np.ndarray:
    """F(U; c1, c3, c5, c7, cL) over all four directions, [4][V][3][3]."""
    c1, c3, c5, c7, cL = coeffs
    dims = tuple(int(d) for d in dims)
    out = np.empty_like(U)
    for mu in range(4):
        dirs = [(nu, s) for nu in range(4) if nu != mu for s in (1, -1)]
        s1 = {d: staple(U, dims, mu, d[0], d[1], U[mu]) for d in dirs}
        f = c1 * U[mu]
        for a in dirs:
            inner = c3 * U[mu]
            for b in dirs:
                if b[0] == a[0]:
                    continue
                m = c5 * U[mu]
                if c7 != 0.0:
                    for c in dirs:
                        if c[0] not in (a[0], b[0]):
                            m = m + c7 * s1[c]
                inner = inner + staple(U, dims, mu, b[0], b[1], m)
            f = f + staple(U, dims, mu, a[0], a[1], inner)
            if cL != 0.0:
                f = f + cL * staple(U, dims, mu, a[0], a[1], s1[a])
        out[mu] = f
    return out


def u3_project(V: np.ndarray) -> np.ndarray:
    """W = V (V^+ V)^(-1/2), the unitary factor of V's polar decomposition."""
    h = dagger(V) @ V
    w, q = np.linalg.eigh(h)
    inv_sqrt = (q * (1.0 / np.sqrt(w))[..., None, :]) @ dagger(q)
    return V @ inv_sqrt


def naik(W: np.ndarray, dims, c: float = NAIK) -> np.ndarray:
    out = np.empty_like(W)
    for mu in range(4):
        out[mu] = c * (W[mu] @ shift(W[mu], dims, mu, 1) @ shift(W[mu], dims, mu, 2))
    return out


def fold_signs(X: np.ndarray, N: np.ndarray, dims):
    """eta_mu(x) times the antiperiodic-time sign of the 1- and 3-hop links, applied to copies."""
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    x, y, z, t = (a.reshape(-1) for a in (x, y, z, t))
    X, N = X.copy(), N.copy()
    for mu in range(4):
        e = (0, x, x + y, x + y + z)[mu]
        eta = 1.0 - 2.0 * (np.asarray(e) % 2) if mu else np.ones(x.shape)
        s1 = eta * np.where((mu == 3) & (t == nt - 1), -1.0, 1.0)
        s3 = eta * np.where((mu == 3) & (t >= nt - 3), -1.0, 1.0)
        X[mu] *= s1[:, None, None]
        N[mu] *= s3[:, None, None]
    return X, N


def hisq_links(U: np.ndarray, dims, level1=LEVEL1, level2=LEVEL2, c_naik=NAIK,
               signs: bool = True):
    """Fat and Naik links (phase-folded when `signs`) from unsigned thin links U[4][V][3][3]."""
    dims = tuple(int(d) for d in dims)
    V = smear(U, dims, level1)
    W = u3_project(V)
    X = smear(W, dims, level2)
    N = naik(W, dims, c_naik)
    return fold_signs(X, N, dims) if signs else (X, N)
