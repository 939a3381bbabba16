"""Synthetic improved-staggered gauge fields.

Recipe (one reading, since the paper prints no ensemble):

* thin link  U = exp(i s H), H = (G + G^H)/2 minus its trace/3, G with i.i.d. CN(0,1) entries
  (re and im ~ N(0, 1/2)); the exponential is taken through the Hermitian eigendecomposition
  and the result is reunitarised (Gram-Schmidt of rows 0 and 1, row 2 = conj(row0 x row1)),
  so det U = 1;
* fat link   V = 0.9 U + 0.05 N, N with i.i.d. CN(0,1) entries (not SU(3) times a scalar);
* Naik link  W_mu(x) = -(1/24) U_mu(x) U_mu(x+mu) U_mu(x+2mu) (unsigned U, periodic wrap);
* staggered phases eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z) and the
  antiperiodic time boundary are folded in: a one-link leaving t = Nt-1 and a three-link
  starting at t >= Nt-3 cross the boundary once and pick up -1.

Layout of every link array: complex128 [4][V][3][3], lexicographic site index
i = x + Nx (y + Ny (z + Nz t)), row index before column index.

Random streams: ``SeedSequence(seed).spawn(2)`` gives one stream for the G draws of U and one
for the N draws of V; each stream is consumed in site order, then mu, then matrix entry
(row-major), re before im.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

NAIK_COEFF = -1.0 / 24.0
FAT_DIAG = 0.9
FAT_NOISE = 0.05


def lattice_volume(dims) -> int:
    return int(np.prod([int(d) for d in dims]))


def lattice_coords(dims):
    """Coordinates (x, y, z, t) of every site, lexicographic order with x fastest."""
    nx, ny, nz, nt = (int(d) for d in dims)
    i = np.arange(nx * ny * nz * nt, dtype=np.int64)
    return i % nx, (i // nx) % ny, (i // (nx * ny)) % nz, i // (nx * ny * nz)


def staggered_phase(mu: int, x, y, z, t):
    """eta_mu(x) as +-1 floats."""
    if mu == 0:
        return np.ones_like(x, dtype=np.float64)
    s = (x, x + y, x + y + z)[mu - 1]
    return 1.0 - 2.0 * (s & 1)


def time_bc_sign(hops: int, t, nt: int):
    """-1 where a forward hop of `hops` links from time slice t wraps past Nt-1, else +1."""
    return np.where(t + hops >= nt, -1.0, 1.0)


def su3_from_gaussian(g: np.ndarray, scale: float) -> np.ndarray:
    """SU(3) matrices exp(i*scale*H) from Gaussian draws g[..., 3, 3, 2] (re, im)."""
    G = (g[..., 0] + 1j * g[..., 1]) * np.sqrt(0.5)
    H = 0.5 * (G + np.conj(np.swapaxes(G, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    H = H - tr[..., None, None] * np.eye(3)
    w, Q = np.linalg.eigh(H)
    U = (Q * np.exp(1j * scale * w)[..., None, :]) @ np.conj(np.swapaxes(Q, -1, -2))
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def random_su3(rng: np.random.Generator, n: int, scale: float) -> np.ndarray:
    """n random SU(3) matrices drawn with the thin-link recipe."""
    return su3_from_gaussian(rng.standard_normal((n, 3, 3, 2)), scale)


def _chunks(V: int, chunk: int = 1 << 17):
    for s in range(0, V, chunk):
        yield s, min(V, s + chunk)


_POOL_STATE = {}


def _shared_array(shape) -> np.ndarray:
    """A complex128 array in an anonymous shared mapping: forked worker processes write into
    the parent's memory (no named shared-memory files)."""
    import mmap
    buf = mmap.mmap(-1, int(np.prod(shape)) * 16)
    return np.ndarray(shape, dtype=np.complex128, buffer=buf)


def _pool_su3(args):
    s, e, g, scale = args
    _POOL_STATE["out"][:, s:e] = np.swapaxes(su3_from_gaussian(g, scale), 0, 1)
    return s


def thin_links(dims, scale: float, seed: int) -> np.ndarray:
    """Unsigned thin links U, complex128 [4][V][3][3].  The draws are taken chunk after chunk
    from one stream; on large lattices the matrices of the chunks are computed by a pool of
    worker processes writing into shared memory (the same operations on the same draws, so
    the result does not depend on the number of workers)."""
    V = lattice_volume(dims)
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(2)[0])
    chunks = list(_chunks(V))
    workers = _workers(len(chunks))
    if workers <= 1:
        U = np.empty((4, V, 3, 3), dtype=np.complex128)
        for s, e in chunks:
            g = rng.standard_normal((e - s, 4, 3, 3, 2))
            U[:, s:e] = np.swapaxes(su3_from_gaussian(g, scale), 0, 1)
        return U
    shape = (4, V, 3, 3)
    _POOL_STATE["out"] = _shared_array(shape)
    try:
        tasks = ((s, e, rng.standard_normal((e - s, 4, 3, 3, 2)), scale) for s, e in chunks)
        _run_pool(workers, _pool_su3, tasks)
        U = np.array(_POOL_STATE["out"])
    finally:
        _POOL_STATE.clear()
    return U


def _run_pool(workers: int, fn, tasks) -> None:
    """Run fn over tasks in forked workers.  The pool is closed and joined, so every worker
    returns from its loop and exits by itself (no worker is sent a signal)."""
    import multiprocessing as mp
    pool = mp.get_context("fork").Pool(workers)
    try:
        for _ in pool.imap_unordered(fn, tasks, chunksize=1):
            pass
        pool.close()
    except BaseException:
        pool.terminate()
        raise
    finally:
        pool.join()


def _workers(nchunks: int) -> int:
    """Worker processes for chunked generation: none for a few chunks, none once this process
    has initialised a GPU through torch, none under a ROCm profiler (its preloaded library
    has set up the GPU runtime before the program starts, and the workers are forked), else
    up to 16 (or the KS_INPUT_WORKERS environment variable)."""
    import os
    import sys
    if nchunks < 4:
        return 1
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_initialized():
        return 1
    if any(k.startswith("ROCPROF") for k in os.environ):
        return 1
    n = int(os.environ.get("KS_INPUT_WORKERS", min(16, os.cpu_count() or 1)))
    return max(1, min(n, nchunks))


def _shift_fwd(A: np.ndarray, dims, mu: int, hops: int) -> np.ndarray:
    """B[i] = A[i + hops*mu_hat] for a per-site array A[V, ...] (periodic wrap)."""
    nx, ny, nz, nt = (int(d) for d in dims)
    shaped = A.reshape((nt, nz, ny, nx) + A.shape[1:])
    axis = 3 - mu
    return np.roll(shaped, -hops, axis=axis).reshape(A.shape)


def naik_from_thin(U: np.ndarray, dims) -> np.ndarray:
    """Unsigned W_mu(x) = -(1/24) U_mu(x) U_mu(x+mu) U_mu(x+2mu)."""
    W = np.empty_like(U)
    for mu in range(4):
        W[mu] = NAIK_COEFF * (U[mu] @ _shift_fwd(U[mu], dims, mu, 1) @ _shift_fwd(U[mu], dims, mu, 2))
    return W


def _fat_chunk(U, s, e, g):
    N = (g[..., 0] + 1j * g[..., 1]) * np.sqrt(0.5)
    return FAT_DIAG * U[:, s:e] + FAT_NOISE * np.swapaxes(N, 0, 1)


def _site_shift(dims, s, e, mu, hops):
    """Index of site i + hops mu_hat for the sites i in [s, e) (periodic wrap)."""
    nx, ny, nz, nt = (int(d) for d in dims)
    i = np.arange(s, e, dtype=np.int64)
    c = [i % nx, (i // nx) % ny, (i // (nx * ny)) % nz, i // (nx * ny * nz)]
    n = (nx, ny, nz, nt)
    c[mu] = (c[mu] + hops) % n[mu]
    return c[0] + nx * (c[1] + ny * (c[2] + nz * c[3]))


def _pool_fat_naik(args):
    """Fat and Naik links of the sites [s, e), phases and boundary signs folded in: the same
    operations as the whole-lattice form, row by row."""
    s, e, g, dims = args
    U, fat, naik = _POOL_STATE["U"], _POOL_STATE["fat"], _POOL_STATE["naik"]
    fat[:, s:e] = _fat_chunk(U, s, e, g)
    for mu in range(4):
        U1 = U[mu][_site_shift(dims, s, e, mu, 1)]
        U2 = U[mu][_site_shift(dims, s, e, mu, 2)]
        naik[mu, s:e] = NAIK_COEFF * (U[mu, s:e] @ U1 @ U2)
    _fold_rows(fat, naik, dims, s, e)
    return s


def fat_and_naik(U: np.ndarray, dims, seed: int):
    """Phase-folded fat link V and Naik link W built from the unsigned thin links U.  On large
    lattices the chunks are computed by a pool of worker processes over shared memory (same
    draws, same operations per row, so the result does not depend on the number of
    workers)."""
    V = lattice_volume(dims)
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(2)[1])
    chunks = list(_chunks(V))
    workers = _workers(len(chunks))
    if workers <= 1:
        fat = np.empty_like(U)
        for s, e in chunks:
            fat[:, s:e] = _fat_chunk(U, s, e, rng.standard_normal((e - s, 4, 3, 3, 2)))
        naik = naik_from_thin(U, dims)
        fold_phases(fat, naik, dims)
        return fat, naik
    shape = U.shape
    _POOL_STATE["U"] = U                       # read by the forked workers, never written
    _POOL_STATE["fat"] = _shared_array(shape)
    _POOL_STATE["naik"] = _shared_array(shape)
    try:
        tasks = ((s, e, rng.standard_normal((e - s, 4, 3, 3, 2)), tuple(dims))
                 for s, e in chunks)
        _run_pool(workers, _pool_fat_naik, tasks)
        fat = np.array(_POOL_STATE["fat"])
        naik = np.array(_POOL_STATE["naik"])
    finally:
        _POOL_STATE.clear()
    return fat, naik


def _fold_rows(fat, naik, dims, s, e):
    nx, ny, nz, nt = (int(d) for d in dims)
    i = np.arange(s, e, dtype=np.int64)
    x, y, z, t = i % nx, (i // nx) % ny, (i // (nx * ny)) % nz, i // (nx * ny * nz)
    for mu in range(4):
        eta = staggered_phase(mu, x, y, z, t)
        s1 = eta * (time_bc_sign(1, t, nt) if mu == 3 else 1.0)
        s3 = eta * (time_bc_sign(3, t, nt) if mu == 3 else 1.0)
        fat[mu, s:e] *= s1[:, None, None]
        naik[mu, s:e] *= s3[:, None, None]


def fold_phases(fat: np.ndarray, naik: np.ndarray, dims) -> None:
    """Multiply eta_mu(x) and the antiperiodic-time sign into V and W in place."""
    x, y, z, t = lattice_coords(dims)
    nt = int(dims[3])
    for mu in range(4):
        eta = staggered_phase(mu, x, y, z, t)
        s1 = eta * (time_bc_sign(1, t, nt) if mu == 3 else 1.0)
        s3 = eta * (time_bc_sign(3, t, nt) if mu == 3 else 1.0)
        fat[mu] *= s1[:, None, None]
        naik[mu] *= s3[:, None, None]


@dataclass
class GaugeField:
    dims: tuple
    fat: np.ndarray            # complex128 [4][V][3][3], phases and BC folded in
    naik: np.ndarray           # complex128 [4][V][3][3], phases and BC folded in
    thin: np.ndarray | None = field(default=None, repr=False)   # unsigned U
    scale: float = 0.0
    seed: int = 0

    @property
    def volume(self) -> int:
        return lattice_volume(self.dims)


def make_gauge(dims, scale: float, seed: int, keep_thin: bool = False) -> GaugeField:
    """The full synthetic field (U, V, W) for one lattice."""
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or any(d < 4 or d % 2 for d in dims):
        raise ValueError("dims must be four even extents >= 4")
    U = thin_links(dims, scale, seed)
    fat, naik = fat_and_naik(U, dims, seed)
    return GaugeField(dims, fat, naik, U if keep_thin else None, scale, seed)


def _block_view(A: np.ndarray, dims, origin, bdims) -> np.ndarray:
    """The [4][V][3][3] links of the block [origin, origin + bdims) as a block lattice."""
    nx, ny, nz, nt = (int(d) for d in dims)
    ox, oy, oz, ot = origin
    bx, by, bz, bt = bdims
    shaped = A.reshape(4, nt, nz, ny, nx, 3, 3)
    sub = shaped[:, ot:ot + bt, oz:oz + bz, oy:oy + by, ox:ox + bx]
    return np.ascontiguousarray(sub).reshape(4, bx * by * bz * bt, 3, 3)


def subblock(field: GaugeField, origin, bdims) -> GaugeField:
    """A sub-lattice cut from a field generated with keep_thin=True: its thin and fat links
    are reused with block-periodic wrap, its Naik link rebuilt from the block's thin links,
    and the phases and the antiperiodic time boundary folded in for the block.  Block origins
    must be even so that the staggered phases do not change."""
    if field.thin is None:
        raise ValueError("the field must keep its thin links")
    if any(o % 2 for o in origin):
        raise ValueError("block origins must be even")
    dims = field.dims
    bdims = tuple(int(b) for b in bdims)
    U = _block_view(field.thin, dims, origin, bdims)
    fat = _block_view(field.fat, dims, origin, bdims)
    # undo the phases and the boundary signs of the big lattice on the block's fat links (the
    # signs at the block sites' coordinates in the big lattice)
    x, y, z, t = (c + o for c, o in zip(lattice_coords(bdims), origin))
    nt = int(dims[3])
    for mu in range(4):
        eta = staggered_phase(mu, x, y, z, t)
        s1 = eta * (time_bc_sign(1, t, nt) if mu == 3 else 1.0)
        fat[mu] *= s1[:, None, None]
    naik = naik_from_thin(U, bdims)
    fold_phases(fat, naik, bdims)
    return GaugeField(bdims, fat, naik, U, field.scale, field.seed)
