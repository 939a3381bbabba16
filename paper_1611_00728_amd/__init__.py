"""MI355X (gfx950) improved-staggered CG solver: Python binding of libks.so.

This module only marshals arguments for the C ABI of include/ks.h (ctypes); every step of the
computation runs in the library's HIP kernels.  Device arrays are torch CUDA tensors (their
data pointers are handed to the library); the default stream is torch's current stream.
There is no CPU path: if libks.so is missing, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libks.so")

F64, F32, F16 = 0, 1, 2
RECON_18, RECON_12 = 18, 12
EVEN, ODD = 0, 1
PREC = {"f64": F64, "f32": F32, "f16": F16}

STATUS = {0: "success", -1: "invalid argument", -2: "HIP error", -3: "out of device memory",
          -4: "links not c*SU(3)", -5: "not converged", -6: "breakdown", -7: "non-finite value"}


class KSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "error"), code, msg))
        self.code = code


class SolverParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("inner", C.c_int),
                ("recon", C.c_int), ("delta", C.c_double), ("check_every", C.c_int),
                ("max_restarts", C.c_int)]


class SolverStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("reliable_updates", C.c_int), ("restarts", C.c_int),
                ("fallback", C.c_int), ("true_rel_resid", C.c_double), ("seconds", C.c_double),
                ("model_bytes", C.c_double), ("model_flops", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DslashLaunch(C.Structure):
    _fields_ = [("threads", C.c_int), ("lds_bytes", C.c_int), ("links_per_pass", C.c_int),
                ("link_access", C.c_int), ("staged", C.c_int), ("tuned_us", C.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("reliable_updates", C.c_int), ("status", C.c_int),
                ("true_rel_resid", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp = C.c_void_p


def lib():
    """The loaded libks.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libks.so is not built (run __graft_entry__.build() or "
                               "python paper_1611_00728_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        L.ks_default_params.argtypes = [C.POINTER(SolverParams)]
        L.ks_default_params.restype = None
        L.ks_last_error.restype = C.c_char_p
        L.ks_gauge_load.argtypes = [C.POINTER(_vp), C.POINTER(C.c_int), _vp, _vp, C.c_int, _vp]
        L.ks_gauge_prepare.argtypes = [_vp, C.c_int, C.c_int, _vp]
        L.ks_gauge_free.argtypes = [_vp]
        L.ks_gauge_device_bytes.argtypes = [_vp]
        L.ks_gauge_device_bytes.restype = C.c_size_t
        L.ks_field_create.argtypes = [C.POINTER(_vp), _vp, C.c_int, C.c_int]
        L.ks_field_free.argtypes = [_vp]
        L.ks_field_import.argtypes = [_vp, _vp, _vp]
        L.ks_field_export.argtypes = [_vp, _vp, _vp]
        L.ks_dslash_eo.argtypes = [_vp, _vp, _vp, C.c_int, _vp]
        L.ks_apply_A.argtypes = [_vp, C.c_double, _vp, _vp, _vp]
        L.ks_apply_A_noalloc.argtypes = [_vp, C.c_double, _vp, _vp, _vp]
        L.ks_batch_create.argtypes = [C.POINTER(_vp), C.c_int, C.POINTER(C.c_int),
                                      C.POINTER(_vp), C.POINTER(_vp), C.c_int, C.c_int,
                                      C.c_int, _vp]
        L.ks_batch_solve.argtypes = [_vp, C.POINTER(C.c_double), C.POINTER(_vp),
                                     C.POINTER(_vp), C.POINTER(SolverParams),
                                     C.POINTER(BatchStats), _vp]
        L.ks_batch_tune.argtypes = [_vp, _vp]
        L.ks_batch_config.argtypes = [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                      C.POINTER(C.c_float), C.POINTER(C.c_double)]
        L.ks_batch_free.argtypes = [_vp]
        L.ks_tune_dslash.argtypes = [_vp, C.c_int, C.c_int, _vp]
        L.ks_dslash_config.argtypes = [_vp, C.c_int, C.c_int, C.POINTER(DslashLaunch)]
        L.ks_stream_copy.argtypes = [_vp, _vp, C.c_size_t, _vp]
        L.ks_stream_read.argtypes = [_vp, C.c_size_t, _vp]
        L.ks_cg_coefficients.argtypes = [_vp, C.c_int, _vp, _vp, C.POINTER(C.c_int)]
        L.ks_dslash_set_config.argtypes = [_vp, C.c_int, C.c_int, C.POINTER(DslashLaunch)]
        L.ks_cg_solve.argtypes = [_vp, C.c_double, _vp, _vp, C.POINTER(SolverParams),
                                  C.POINTER(SolverStats), _vp]
        L.ks_full_solve.argtypes = [_vp, C.c_double, _vp, _vp, _vp, _vp, C.POINTER(SolverParams),
                                    C.POINTER(SolverStats), _vp]
        L.ks_hisq_links.argtypes = [C.POINTER(C.c_int), _vp, _vp, _vp, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.c_double, _vp]
        L.ks_force.argtypes = [_vp, C.c_int, C.POINTER(C.c_double), C.POINTER(_vp), _vp, _vp, _vp]
        L.ks_hisq_release.argtypes = []
        L.ks_multishift_cg_solve.argtypes = [_vp, C.c_int, C.POINTER(C.c_double), _vp,
                                             C.POINTER(_vp), C.POINTER(C.c_double),
                                             C.POINTER(SolverParams), C.POINTER(SolverStats), _vp]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise KSError(rc, lib().ks_last_error().decode())


def _stream(stream):
    if stream is not None:
        return _vp(int(stream))
    import torch
    return _vp(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, what="tensor"):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128
            and t.is_contiguous()):
        raise ValueError("%s must be a contiguous complex128 CUDA tensor" % what)
    return _vp(t.data_ptr())


def _dev_vec(t, vh: int, what="vector"):
    """Device pointer of a one-parity field, checked to hold exactly [vh][3] complex128
    (the library cannot see array extents)."""
    p = _dev_ptr(t, what)
    if t.numel() != 3 * vh:
        raise ValueError("%s must hold %d complex numbers ([%d][3]), has %d"
                         % (what, 3 * vh, vh, t.numel()))
    return p


def default_params(**kw) -> SolverParams:
    p = SolverParams()
    lib().ks_default_params(C.byref(p))
    for k, v in kw.items():
        if k == "inner" and isinstance(v, str):
            v = PREC[v]
        setattr(p, k, v)
    return p


class Gauge:
    """A gauge field loaded into the library (ks_gauge_load)."""

    def __init__(self, dims, fat, naik, stream=None):
        import numpy as np
        import torch
        self.dims = tuple(int(d) for d in dims)
        self.volume = int(np.prod(self.dims))
        self.vh = self.volume // 2
        d = (C.c_int * 4)(*self.dims)
        h = _vp()
        for a, nm in ((fat, "fat"), (naik, "naik")):
            n = a.numel() if isinstance(a, torch.Tensor) else np.asarray(a).size
            if n != 36 * self.volume:
                raise ValueError("%s links must hold [4][V][3][3] complex numbers" % nm)
        if isinstance(fat, torch.Tensor):
            args = (_dev_ptr(fat, "fat"), _dev_ptr(naik, "naik"), 1)
        else:
            self._host = (np.ascontiguousarray(fat, dtype=np.complex128),
                          np.ascontiguousarray(naik, dtype=np.complex128))
            args = (_vp(self._host[0].ctypes.data), _vp(self._host[1].ctypes.data), 0)
        _check(lib().ks_gauge_load(C.byref(h), d, args[0], args[1], args[2], _stream(stream)))
        self._host = None
        self.handle = h

    def prepare(self, prec=F64, recon=RECON_18, stream=None):
        _check(lib().ks_gauge_prepare(self.handle, prec, recon, _stream(stream)))

    def tune(self, prec=F64, recon=RECON_18, stream=None) -> dict:
        """Autotunes the Dslash launch of one variant; returns its configuration."""
        _check(lib().ks_tune_dslash(self.handle, prec, recon, _stream(stream)))
        return self.config(prec, recon)

    def config(self, prec=F64, recon=RECON_18) -> dict:
        cfg = DslashLaunch()
        _check(lib().ks_dslash_config(self.handle, prec, recon, C.byref(cfg)))
        return cfg.as_dict()

    def set_config(self, prec=F64, recon=RECON_18, threads=256, lds_bytes=0,
                   links_per_pass=1, link_access=8, staged=0):
        """Sets one variant's Dslash launch configuration by hand."""
        cfg = DslashLaunch(threads, lds_bytes, links_per_pass, link_access, staged, 0.0)
        _check(lib().ks_dslash_set_config(self.handle, prec, recon, C.byref(cfg)))

    def device_bytes(self) -> int:
        return int(lib().ks_gauge_device_bytes(self.handle))

    def cg_coefficients(self, n_max: int = 1 << 20):
        """(alpha, beta) numpy arrays of the last CG run on this handle (ks_cg_coefficients)."""
        import numpy as np
        alpha = np.zeros(n_max)
        beta = np.zeros(n_max)
        n = C.c_int(0)
        _check(lib().ks_cg_coefficients(self.handle, n_max, alpha.ctypes.data, beta.ctypes.data,
                                        C.byref(n)))
        return alpha[:n.value].copy(), beta[:n.value].copy()

    def free(self):
        if self.handle:
            _check(lib().ks_gauge_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Field:
    """A one-parity colour-vector field in the library's layout (ks_field_create)."""

    def __init__(self, gauge: Gauge, parity: int, prec: int = F64):
        h = _vp()
        _check(lib().ks_field_create(C.byref(h), gauge.handle, parity, prec))
        self.handle = h
        self.gauge = gauge
        self.parity = parity
        self.prec = prec

    def load(self, t, stream=None):
        _check(lib().ks_field_import(self.handle, _dev_vec(t, self.gauge.vh), _stream(stream)))
        return self

    def store(self, t, stream=None):
        _check(lib().ks_field_export(self.handle, _dev_vec(t, self.gauge.vh), _stream(stream)))
        return t

    def free(self):
        if self.handle:
            _check(lib().ks_field_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def dslash_eo(gauge: Gauge, out: Field, inp: Field, recon: int = RECON_18, stream=None):
    _check(lib().ks_dslash_eo(gauge.handle, out.handle, inp.handle, recon, _stream(stream)))


def stream_copy(dst, src, stream=None):
    """dst = src (device tensors of equal byte size) by the library's streaming copy kernel."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n or not (src.is_cuda and dst.is_cuda):
        raise ValueError("stream_copy: two device tensors of equal byte size expected")
    if not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("stream_copy: contiguous tensors expected")
    _check(lib().ks_stream_copy(dst.data_ptr(), src.data_ptr(), n, _stream(stream)))
    return dst


def stream_read(src, stream=None):
    """Reads every byte of a contiguous device tensor by the library's streaming read kernel."""
    if not (src.is_cuda and src.is_contiguous()):
        raise ValueError("stream_read: a contiguous device tensor expected")
    _check(lib().ks_stream_read(src.data_ptr(), src.numel() * src.element_size(), _stream(stream)))


def apply_A(gauge: Gauge, sigma: float, x, out, stream=None):
    _check(lib().ks_apply_A(gauge.handle, float(sigma), _dev_vec(x, gauge.vh, "x"),
                            _dev_vec(out, gauge.vh, "out"),
                            _stream(stream)))
    return out


def apply_A_noalloc(gauge: Gauge, sigma: float, x, out, stream=None):
    """apply_A through the entry point that allocates no device memory (its temporaries sit in
    the library's fixed scratch array)."""
    _check(lib().ks_apply_A_noalloc(gauge.handle, float(sigma), _dev_vec(x, gauge.vh, "x"),
                                    _dev_vec(out, gauge.vh, "out"), _stream(stream)))
    return out


@dataclass
class SolveResult:
    status: int
    stats: dict

    @property
    def ok(self):
        return self.status == 0


def cg_solve(gauge: Gauge, mass: float, b, x, params: SolverParams | None = None,
             stream=None, raise_on_error: bool = True) -> SolveResult:
    """(4 m^2 - D_eo D_oe) x = b; x holds the initial guess and receives the solution."""
    p = params if params is not None else default_params()
    st = SolverStats()
    rc = lib().ks_cg_solve(gauge.handle, float(mass), _dev_vec(b, gauge.vh, "b"),
                           _dev_vec(x, gauge.vh, "x"),
                           C.byref(p), C.byref(st), _stream(stream))
    if rc != 0 and raise_on_error:
        _check(rc)
    return SolveResult(rc, st.as_dict())


def full_solve(gauge: Gauge, mass: float, b_even, b_odd, x_even, x_odd,
               params: SolverParams | None = None, stream=None,
               raise_on_error: bool = True) -> SolveResult:
    """(2m + D) x = b on both parities; x_even holds the initial guess of the even solve."""
    p = params if params is not None else default_params()
    st = SolverStats()
    rc = lib().ks_full_solve(gauge.handle, float(mass), _dev_vec(b_even, gauge.vh, "b_even"),
                             _dev_vec(b_odd, gauge.vh, "b_odd"),
                             _dev_vec(x_even, gauge.vh, "x_even"),
                             _dev_vec(x_odd, gauge.vh, "x_odd"), C.byref(p), C.byref(st),
                             _stream(stream))
    if rc != 0 and raise_on_error:
        _check(rc)
    return SolveResult(rc, st.as_dict())


def hisq_links(dims, thin, fat, naik, level1=None, level2=None, c_naik=-1.0 / 24.0,
               stream=None):
    """Fat and Naik links from thin links (ks_hisq_links); thin, fat, naik: complex128 CUDA
    tensors of 4 * V * 9 elements; level1, level2: five smearing coefficients or None."""
    dims = tuple(int(d) for d in dims)
    vol = dims[0] * dims[1] * dims[2] * dims[3]
    ptrs = []
    for t, name in ((thin, "thin"), (fat, "fat"), (naik, "naik")):
        ptrs.append(_dev_ptr(t, name))
        if t.numel() != 36 * vol:
            raise ValueError("%s must hold 4 * V * 9 complex numbers" % name)
    d = (C.c_int * 4)(*dims)
    l1 = None if level1 is None else (C.c_double * 5)(*[float(v) for v in level1])
    l2 = None if level2 is None else (C.c_double * 5)(*[float(v) for v in level2])
    _check(lib().ks_hisq_links(d, ptrs[0], ptrs[1], ptrs[2], l1, l2, float(c_naik),
                               _stream(stream)))



def hisq_release():
    """Frees the scratch the link construction keeps on the device between calls."""
    _check(lib().ks_hisq_release())

def force(gauge: Gauge, residues, xs, force_fat, force_naik, stream=None):
    """Link derivative of sum_i r_i phi^+ A_i^-1 phi from the solutions xs (ks_force);
    force_fat, force_naik: complex128 CUDA tensors of 4 * V * 9 elements."""
    n = len(residues)
    if len(xs) != n:
        raise ValueError("need one solution per residue")
    outs = []
    for f, name in ((force_fat, "force_fat"), (force_naik, "force_naik")):
        outs.append(_dev_ptr(f, name))
        if f.numel() != 36 * gauge.volume:
            raise ValueError("%s must hold 4 * V * 9 complex numbers" % name)
    r = (C.c_double * n)(*[float(v) for v in residues])
    ptrs = (_vp * n)(*[_dev_vec(x, gauge.vh, "x[%d]" % i).value for i, x in enumerate(xs)])
    _check(lib().ks_force(gauge.handle, n, r, ptrs, outs[0], outs[1], _stream(stream)))


def multishift_cg_solve(gauge: Gauge, sigmas, b, xs, tols, params: SolverParams | None = None,
                        stream=None, raise_on_error: bool = True):
    """(sigma_i - D_eo D_oe) x_i = b for every shift; returns (status, [stats])."""
    n = len(sigmas)
    p = params if params is not None else default_params()
    sig = (C.c_double * n)(*[float(s) for s in sigmas])
    tl = (C.c_double * n)(*([float(tols)] * n if isinstance(tols, (int, float)) else
                            [float(t) for t in tols]))
    if len(xs) != n:
        raise ValueError("need one solution vector per shift")
    ptrs = (_vp * n)(*[_dev_vec(x, gauge.vh, "x[%d]" % i).value for i, x in enumerate(xs)])
    st = (SolverStats * n)()
    rc = lib().ks_multishift_cg_solve(gauge.handle, n, sig, _dev_vec(b, gauge.vh, "b"), ptrs, tl,
                                      C.byref(p), st, _stream(stream))
    if rc != 0 and raise_on_error:
        _check(rc)
    return rc, [s.as_dict() for s in st]


class Batch:
    """Many lattices x nrhs right-hand sides solved together (ks_batch_create / _solve)."""

    def __init__(self, dims_list, fats, naiks, nrhs: int = 4, inner: int = F32, stream=None):
        import numpy as np
        n = len(dims_list)
        self.dims = [tuple(int(x) for x in d) for d in dims_list]
        self.nrhs = nrhs
        self.nlat = n
        d = (C.c_int * (4 * n))(*[x for dd in self.dims for x in dd])
        host = [np.ascontiguousarray(a, dtype=np.complex128) for a in fats] + \
               [np.ascontiguousarray(a, dtype=np.complex128) for a in naiks]
        for k, a in enumerate(host):
            if a.size != 36 * int(np.prod(self.dims[k % n])):
                raise ValueError("links of lattice %d must hold [4][V][3][3] complex numbers"
                                 % (k % n))
        fp = (_vp * n)(*[h.ctypes.data for h in host[:n]])
        np_ = (_vp * n)(*[h.ctypes.data for h in host[n:]])
        h = _vp()
        _check(lib().ks_batch_create(C.byref(h), n, d, fp, np_, 0, nrhs, inner, _stream(stream)))
        self.handle = h

    def tune(self, stream=None) -> dict:
        _check(lib().ks_batch_tune(self.handle, _stream(stream)))
        return self.config()

    def config(self) -> dict:
        t, p, us, sec = C.c_int(), C.c_int(), C.c_float(), C.c_double()
        _check(lib().ks_batch_config(self.handle, C.byref(t), C.byref(p), C.byref(us),
                                     C.byref(sec)))
        return {"tile_sites": t.value, "persistent_blocks": p.value, "tuned_us": us.value,
                "last_solve_seconds": sec.value}

    def solve(self, masses, bs, xs, params: SolverParams | None = None, stream=None,
              raise_on_error: bool = True):
        """bs, xs: nlat*nrhs complex128 CUDA tensors, pair p = lattice * nrhs + rhs."""
        npair = self.nlat * self.nrhs
        if len(bs) != npair or len(xs) != npair or len(masses) != self.nlat:
            raise ValueError("need %d masses and %d vectors" % (self.nlat, npair))
        p = params if params is not None else default_params()
        m = (C.c_double * self.nlat)(*[float(v) for v in masses])
        vhs = [int(d[0] * d[1] * d[2] * d[3]) // 2 for d in self.dims for _ in range(self.nrhs)]
        bp = (_vp * npair)(*[_dev_vec(b, vh, "b").value for b, vh in zip(bs, vhs)])
        xp = (_vp * npair)(*[_dev_vec(x, vh, "x").value for x, vh in zip(xs, vhs)])
        st = (BatchStats * npair)()
        rc = lib().ks_batch_solve(self.handle, m, bp, xp, C.byref(p), st, _stream(stream))
        if rc != 0 and raise_on_error:
            _check(rc)
        return rc, [s.as_dict() for s in st]

    def free(self):
        if self.handle:
            _check(lib().ks_batch_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


NET_WEIGHTS = 648
CHECKPOINT_MAGIC = b"KSNETCK1"


def write_checkpoint(path, weights, adam_m, adam_v, step: int):
    """Network checkpoint, little-endian: the 8-byte magic, uint32 number of complex weights,
    uint32 Adam step count, then float64 arrays: the weights as (re, im) pairs, Adam's first
    moments, Adam's second moments (2 * the number of weights each)."""
    import numpy as np
    w = np.asarray(weights, dtype=np.complex128).ravel()
    m = np.asarray(adam_m, dtype=np.float64).ravel()
    v = np.asarray(adam_v, dtype=np.float64).ravel()
    if m.size != 2 * w.size or v.size != 2 * w.size or step < 0:
        raise ValueError("inconsistent checkpoint state")
    head = CHECKPOINT_MAGIC + np.array([w.size, step], dtype="<u4").tobytes()
    body = b"".join(a.astype("<f8").tobytes() for a in (w.view(np.float64), m, v))
    tmp = str(path) + ".tmp"
    with open(tmp, "wb") as f:
        f.write(head + body)
    os.replace(tmp, path)


def read_checkpoint(path):
    """(weights, adam_m, adam_v, step) from a file written by write_checkpoint; ValueError for
    another format or a truncated file."""
    import numpy as np
    with open(path, "rb") as f:
        data = f.read()
    if len(data) < 16 or data[:8] != CHECKPOINT_MAGIC:
        raise ValueError("%s: not a network checkpoint" % path)
    n, step = (int(x) for x in np.frombuffer(data[8:16], dtype="<u4"))
    if len(data) != 16 + 3 * 2 * n * 8:
        raise ValueError("%s: %d bytes, expected %d" % (path, len(data), 16 + 48 * n))
    a = np.frombuffer(data[16:], dtype="<f8").astype(np.float64)
    w = a[:2 * n].copy().view(np.complex128)
    return w, a[2 * n:4 * n].copy(), a[4 * n:].copy(), step


class Net:
    """The preconditioner network N = L^+ L (ks_net_create); weights: complex128 [648], L's two
    free layers (1 -> 8, then 8 -> 8), each w[c_out][c_in][9]."""

    def __init__(self, weights):
        import numpy as np
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.complex128).ravel())
        if w.size != NET_WEIGHTS:
            raise ValueError("the network has %d complex weights" % NET_WEIGHTS)
        L = lib()
        L.ks_net_create.argtypes = [C.POINTER(_vp), _vp]
        L.ks_net_set_weights.argtypes = [_vp, _vp]
        L.ks_net_get_weights.argtypes = [_vp, _vp]
        L.ks_net_free.argtypes = [_vp]
        L.ks_net_get_state.argtypes = [_vp, _vp, _vp, _vp, C.POINTER(C.c_int)]
        L.ks_net_set_state.argtypes = [_vp, _vp, _vp, _vp, C.c_int]
        L.ks_net_apply.argtypes = [_vp, _vp, _vp, _vp, C.c_int, _vp]
        L.ks_net_apply_field.argtypes = [_vp, _vp, _vp, C.c_int, _vp]
        L.ks_net_loss_grad.argtypes = [_vp, C.c_int, C.POINTER(_vp), C.POINTER(C.c_double),
                                       C.POINTER(_vp), C.POINTER(_vp), C.POINTER(C.c_double),
                                       _vp, _vp]
        L.ks_net_train.argtypes = [_vp, C.c_int, C.POINTER(_vp), C.POINTER(C.c_double),
                                   C.POINTER(_vp), C.POINTER(_vp), C.c_int, C.c_int, C.c_double,
                                   _vp, _vp]
        L.ks_fcg_solve.argtypes = [_vp, _vp, C.c_double, _vp, _vp, C.POINTER(SolverParams),
                                   C.c_int, C.POINTER(SolverStats), _vp]
        h = _vp()
        _check(L.ks_net_create(C.byref(h), _vp(w.ctypes.data)))
        self.handle = h

    def set_weights(self, weights):
        import numpy as np
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.complex128).ravel())
        if w.size != NET_WEIGHTS:
            raise ValueError("the network has %d complex weights" % NET_WEIGHTS)
        _check(lib().ks_net_set_weights(self.handle, _vp(w.ctypes.data)))

    def get_weights(self):
        import numpy as np
        w = np.zeros(NET_WEIGHTS, dtype=np.complex128)
        _check(lib().ks_net_get_weights(self.handle, _vp(w.ctypes.data)))
        return w

    def get_state(self):
        """(weights complex128 [NET_WEIGHTS], Adam first and second moments float64
        [2 NET_WEIGHTS] each, Adam step count)."""
        import numpy as np
        w = np.zeros(NET_WEIGHTS, dtype=np.complex128)
        m = np.zeros(2 * NET_WEIGHTS)
        v = np.zeros(2 * NET_WEIGHTS)
        step = C.c_int()
        _check(lib().ks_net_get_state(self.handle, _vp(w.ctypes.data), _vp(m.ctypes.data),
                                      _vp(v.ctypes.data), C.byref(step)))
        return w, m, v, step.value

    def set_state(self, weights, adam_m, adam_v, step: int):
        import numpy as np
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.complex128).ravel())
        m = np.ascontiguousarray(np.asarray(adam_m, dtype=np.float64).ravel())
        v = np.ascontiguousarray(np.asarray(adam_v, dtype=np.float64).ravel())
        if w.size != NET_WEIGHTS or m.size != 2 * NET_WEIGHTS or v.size != 2 * NET_WEIGHTS:
            raise ValueError("state sizes: %d complex weights, %d reals per moment"
                             % (NET_WEIGHTS, 2 * NET_WEIGHTS))
        _check(lib().ks_net_set_state(self.handle, _vp(w.ctypes.data), _vp(m.ctypes.data),
                                      _vp(v.ctypes.data), int(step)))

    def save(self, path):
        """Checkpoint of the weights and the Adam state (format of write_checkpoint)."""
        write_checkpoint(path, *self.get_state())

    def load(self, path):
        """Restores a checkpoint written by save; training continues where it stopped."""
        self.set_state(*read_checkpoint(path))
        return self

    def apply(self, gauge: Gauge, x, out, mfma: bool = False, stream=None):
        _check(lib().ks_net_apply(self.handle, gauge.handle, _dev_vec(x, gauge.vh, "x"),
                                  _dev_vec(out, gauge.vh, "out"), int(bool(mfma)),
                                  _stream(stream)))
        return out

    def apply_field(self, inp: Field, out: Field, mfma: bool = False, stream=None):
        """out = N(inp) on even-parity fields in the solver's storage (FP64 or FP32)."""
        _check(lib().ks_net_apply_field(self.handle, out.handle, inp.handle, int(bool(mfma)),
                                        _stream(stream)))
        return out

    @staticmethod
    def _pairs(gauges, sigmas, bs, xs):
        n = len(gauges)
        if len(bs) != n or len(xs) != n or len(sigmas) != n:
            raise ValueError("one gauge, shift, source and solution per pair")
        gp = (_vp * n)(*[g.handle.value for g in gauges])
        sp = (C.c_double * n)(*[float(v) for v in sigmas])
        bp = (_vp * n)(*[_dev_vec(b, g.vh, "b").value for b, g in zip(bs, gauges)])
        xp = (_vp * n)(*[_dev_vec(x, g.vh, "x").value for x, g in zip(xs, gauges)])
        return n, gp, sp, bp, xp

    def loss_grad(self, gauges, sigmas, bs, xs, stream=None):
        """A-norm loss of the pairs (A_j = sigmas[j] - D_eo D_oe on gauges[j]) and its
        gradient with respect to the free weights."""
        import numpy as np
        n, gp, sp, bp, xp = self._pairs(gauges, sigmas, bs, xs)
        loss = C.c_double()
        grad = np.zeros(NET_WEIGHTS, dtype=np.complex128)
        _check(lib().ks_net_loss_grad(self.handle, n, gp, sp, bp, xp, C.byref(loss),
                                      _vp(grad.ctypes.data), _stream(stream)))
        return loss.value, grad

    def train(self, gauges, sigmas, bs, xs, steps: int, batch: int, lr: float = 1e-3,
              stream=None):
        import numpy as np
        n, gp, sp, bp, xp = self._pairs(gauges, sigmas, bs, xs)
        hist = np.zeros(max(steps, 1))
        _check(lib().ks_net_train(self.handle, n, gp, sp, bp, xp, int(steps), int(batch),
                                  float(lr), _vp(hist.ctypes.data), _stream(stream)))
        return hist[:steps]

    def free(self):
        if self.handle:
            _check(lib().ks_net_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def fcg_solve(gauge: Gauge, net: Net, mass: float, b, x, params: SolverParams | None = None,
              mfma: bool = False, stream=None, raise_on_error: bool = True) -> SolveResult:
    """Flexible CG for (4 m^2 - D_eo D_oe) x = b preconditioned by `net`."""
    p = params if params is not None else default_params()
    st = SolverStats()
    rc = lib().ks_fcg_solve(gauge.handle, net.handle, float(mass), _dev_vec(b, gauge.vh, "b"),
                            _dev_vec(x, gauge.vh, "x"), C.byref(p), int(bool(mfma)),
                            C.byref(st), _stream(stream))
    if rc != 0 and raise_on_error:
        _check(rc)
    return SolveResult(rc, st.as_dict())
