"""ctypes front of the C oracle (test infrastructure; see the package docstring)."""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_lib = None

ORC_STATUS = {0: "ok", 1: "not converged", 2: "breakdown", 3: "bad argument", 4: "out of memory"}


class OracleError(RuntimeError):
    pass


def lib():
    """The loaded oracle library (compiled with gcc on first use if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.orc_dslash_full.argtypes = [ip, dp, dp, dp, dp]
        L.orc_dslash_eo.argtypes = [ip, dp, dp, C.c_int, dp, dp]
        L.orc_apply_A.argtypes = [ip, dp, dp, C.c_double, dp, dp]
        L.orc_embed.argtypes = [ip, C.c_int, dp, dp]
        L.orc_restrict.argtypes = [ip, C.c_int, dp, dp]
        L.orc_cg.argtypes = [ip, dp, dp, C.c_double, dp, dp, C.c_double, C.c_int, C.c_int,
                             C.c_void_p, dp, dp]
        L.orc_multishift_cg.argtypes = [ip, dp, dp, C.c_int, dp, dp, dp, dp, C.c_int, ip, dp]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_max_threads.argtypes = []
        _lib = L
    return _lib


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    if d.shape != (4,):
        raise ValueError("dims must have four entries")
    return d


def _ptr(a: np.ndarray, dtype=np.complex128):
    if a.dtype != dtype or not a.flags.c_contiguous:
        raise ValueError("expected a C-contiguous %s array" % np.dtype(dtype).name)
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _check(rc, what):
    if rc not in (0,):
        raise OracleError("%s: %s" % (what, ORC_STATUS.get(rc, rc)))


def _links(g):
    fat = np.ascontiguousarray(g.fat, dtype=np.complex128)
    naik = np.ascontiguousarray(g.naik, dtype=np.complex128)
    return fat, naik


def set_threads(n: int) -> None:
    """Number of host threads the oracle's loops use (for timing it)."""
    _check(lib().orc_set_threads(int(n)), "set_threads")


def max_threads() -> int:
    return int(lib().orc_max_threads())


def dslash_full(g, psi: np.ndarray) -> np.ndarray:
    """D psi on the full lattice; psi complex128 [V][3]."""
    d = _dims(g.dims)
    fat, naik = _links(g)
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.empty_like(psi)
    _check(lib().orc_dslash_full(_ip(d), _ptr(fat), _ptr(naik), _ptr(psi), _ptr(out)), "dslash")
    return out


def dslash_eo(g, out_parity: int, psi_cb: np.ndarray) -> np.ndarray:
    """D restricted to output parity `out_parity`; psi_cb of the other parity, [Vh][3]."""
    d = _dims(g.dims)
    fat, naik = _links(g)
    psi = np.ascontiguousarray(psi_cb, dtype=np.complex128)
    out = np.empty_like(psi)
    _check(lib().orc_dslash_eo(_ip(d), _ptr(fat), _ptr(naik), int(out_parity), _ptr(psi),
                               _ptr(out)), "dslash_eo")
    return out


def apply_A(g, sigma: float, x: np.ndarray) -> np.ndarray:
    """A_sigma x = sigma x - D_eo D_oe x on even sites."""
    d = _dims(g.dims)
    fat, naik = _links(g)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty_like(x)
    _check(lib().orc_apply_A(_ip(d), _ptr(fat), _ptr(naik), float(sigma), _ptr(x), _ptr(out)),
           "apply_A")
    return out


def embed(dims, parity: int, cb: np.ndarray) -> np.ndarray:
    d = _dims(dims)
    cb = np.ascontiguousarray(cb, dtype=np.complex128)
    full = np.empty((2 * cb.shape[0], 3), dtype=np.complex128)
    lib().orc_embed(_ip(d), int(parity), _ptr(cb), _ptr(full))
    return full


def restrict(dims, parity: int, full: np.ndarray) -> np.ndarray:
    d = _dims(dims)
    full = np.ascontiguousarray(full, dtype=np.complex128)
    cb = np.empty((full.shape[0] // 2, 3), dtype=np.complex128)
    lib().orc_restrict(_ip(d), int(parity), _ptr(full), _ptr(cb))
    return cb


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("true_rel_resid", C.c_double)]


@dataclass
class CGInfo:
    status: str
    iters: int
    restarts: int
    true_rel_resid: float
    alpha: np.ndarray
    beta: np.ndarray


def cg(g, sigma: float, b: np.ndarray, tol: float, max_iter: int = 100000, max_restarts: int = 5,
       x0: np.ndarray | None = None):
    """Plain FP64 CG on A_sigma; returns (x, CGInfo)."""
    d = _dims(g.dims)
    fat, naik = _links(g)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128, order="C")
    info = _Info()
    al = np.zeros(max_iter)
    be = np.zeros(max_iter)
    rc = lib().orc_cg(_ip(d), _ptr(fat), _ptr(naik), float(sigma), _ptr(b), _ptr(x), float(tol),
                      int(max_iter), int(max_restarts), C.byref(info), _ptr(al, np.float64),
                      _ptr(be, np.float64))
    if rc not in (0, 1, 2):
        _check(rc, "cg")
    n = info.iters
    return x, CGInfo(ORC_STATUS[rc], n, info.restarts, info.true_rel_resid, al[:n], be[:n])


def multishift_cg(g, sigmas, b: np.ndarray, tols, max_iter: int = 100000):
    """Multi-shift CG for (sigma_i - D_eo D_oe) x_i = b; returns (x[nshift], iters, resid, status)."""
    d = _dims(g.dims)
    fat, naik = _links(g)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    s = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64))
    t = np.ascontiguousarray(np.broadcast_to(np.asarray(tols, dtype=np.float64), s.shape).copy())
    x = np.zeros((len(s),) + b.shape, dtype=np.complex128)
    it = np.zeros(1, dtype=np.int32)
    res = np.zeros(len(s))
    rc = lib().orc_multishift_cg(_ip(d), _ptr(fat), _ptr(naik), len(s), _ptr(s, np.float64),
                                 _ptr(b), _ptr(x), _ptr(t, np.float64), int(max_iter), _ip(it),
                                 _ptr(res, np.float64))
    if rc not in (0, 1, 2):
        _check(rc, "multishift_cg")
    return x, int(it[0]), res, ORC_STATUS[rc]


def dense_A(g, sigma: float) -> np.ndarray:
    """A_sigma as a dense (3Vh x 3Vh) matrix, one column per unit vector (small lattices)."""
    vh = int(np.prod(g.dims)) // 2
    n = 3 * vh
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((vh, 3), dtype=np.complex128)
    for j in range(n):
        e.flat[j] = 1.0
        M[:, j] = apply_A(g, sigma, e).ravel()
        e.flat[j] = 0.0
    return M


def lanczos_extremes(alpha: np.ndarray, beta: np.ndarray):
    """(lambda_min, lambda_max) of the Lanczos tridiagonal built from CG's alpha, beta."""
    k = len(alpha)
    if k == 0:
        return float("nan"), float("nan")
    diag = np.empty(k)
    off = np.empty(max(k - 1, 0))
    for j in range(k):
        diag[j] = 1.0 / alpha[j] + (beta[j - 1] / alpha[j - 1] if j > 0 else 0.0)
        if j < k - 1:
            off[j] = np.sqrt(beta[j]) / alpha[j]
    T = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    w = np.linalg.eigvalsh(T)
    return float(w[0]), float(w[-1])
