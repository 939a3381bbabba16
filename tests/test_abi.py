"""The C-ABI library loads on the host and exports every symbol that include/ks.h declares;
argument checks that run before any device work return their codes."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"\b(ks_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def libks():
    import paper_1611_00728_amd as ks
    if not os.path.exists(ks.LIB_PATH):
        from paper_1611_00728_amd import build
        build.build()
    return ks.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ks_gauge_load", "ks_dslash_eo", "ks_cg_solve", "ks_multishift_cg_solve"):
        assert required in names


def test_every_declared_symbol_is_exported(libks):
    missing = [n for n in declared_functions() if not hasattr(libks, n)]
    assert not missing, missing


def test_default_params(libks):
    import paper_1611_00728_amd as ks
    p = ks.default_params()
    assert p.tol == 1e-10 and p.inner == ks.F64 and p.recon == 18 and p.delta == 0.1
    assert p.check_every > 0 and p.max_iter > 0


def test_bad_dims_rejected_before_device_work(libks):
    import paper_1611_00728_amd as ks
    h = C.c_void_p()
    dummy = (C.c_double * 2)()
    for dims in ((5, 4, 4, 4), (4, 4, 4, 2), (4, 4, 0, 4)):
        d = (C.c_int * 4)(*dims)
        rc = libks.ks_gauge_load(C.byref(h), d, C.cast(dummy, C.c_void_p),
                                 C.cast(dummy, C.c_void_p), 0, None)
        assert rc == -1
        assert b"even" in libks.ks_last_error()
    rc = libks.ks_gauge_load(None, (C.c_int * 4)(4, 4, 4, 4), None, None, 0, None)
    assert rc == -1


def test_null_handles_rejected(libks):
    assert libks.ks_dslash_eo(None, None, None, 18, None) == -1
    assert libks.ks_gauge_prepare(None, 0, 18, None) == -1
    assert libks.ks_gauge_free(None) == 0
    assert libks.ks_field_free(None) == 0


def test_stream_copy_argument_checks(libks):
    """Sizes and addresses that are not multiples of 16, and overlapping buffers, are refused
    before any device work."""
    for dst, src, n in ((4096, 8192, 20), (4100, 8192, 32), (4096, 8200, 32), (4096, 4112, 64)):
        assert libks.ks_stream_copy(dst, src, n, None) == -1
    assert libks.ks_stream_copy(None, None, 0, None) == 0
    for src, n in ((4096, 20), (4100, 32)):
        assert libks.ks_stream_read(src, n, None) == -1
    assert libks.ks_stream_read(None, 16, None) == -1
    assert libks.ks_stream_read(None, 0, None) == 0


def test_cg_coefficients_argument_checks(libks):
    import ctypes
    n = ctypes.c_int(7)
    assert libks.ks_cg_coefficients(None, 0, None, None, ctypes.byref(n)) == -1
    assert libks.ks_cg_coefficients(ctypes.c_void_p(16), -1, None, None, ctypes.byref(n)) == -1
    assert libks.ks_cg_coefficients(ctypes.c_void_p(16), 4, None, None, ctypes.byref(n)) == -1


def _run_with_log(level):
    import subprocess
    import sys
    code = ("import ctypes as C, sys; sys.path.insert(0, %r)\n"
            "import paper_1611_00728_amd as ks\n"
            "L = ks.lib()\n"
            "p = ks.default_params()\n"
            "rc = L.ks_cg_solve(None, C.c_double(0.1), None, None, C.byref(p), None, None)\n"
            "print('rc', rc)\n") % ROOT
    env = dict(os.environ)
    env.pop("KS_LOG", None)
    if level is not None:
        env["KS_LOG"] = str(level)
    return subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                          timeout=120)


def test_ks_log_reports_errors(libks):
    """KS_LOG = 1: a failing call prints its entry point, code and message on stderr, prefixed
    "[ks]"; without KS_LOG (or at 0) the library prints nothing."""
    on = _run_with_log(1)
    assert on.returncode == 0 and "rc -1" in on.stdout
    assert "[ks] ks_cg_solve: error -1: ks_cg_solve: null argument" in on.stderr
    for level in (None, 0):
        off = _run_with_log(level)
        assert off.returncode == 0 and "rc -1" in off.stdout and "[ks]" not in off.stderr


def test_net_state_argument_checks(libks):
    """The training-state entry points refuse null handles and buffers before any device work."""
    w = (C.c_double * 4)()
    step = C.c_int()
    assert libks.ks_net_get_state(None, w, w, w, C.byref(step)) == -1
    assert libks.ks_net_set_state(None, w, w, w, 0) == -1
    assert b"null" in libks.ks_last_error()
