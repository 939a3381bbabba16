"""Flexible CG with a preconditioner, FP64 reference (test infrastructure).

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

from .core import apply_A, cg


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
