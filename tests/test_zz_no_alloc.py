"""The allocation-free normal operator (ks_apply_A_noalloc) against ks_apply_A and the FP64
oracle, through the C ABI: two calls in a row on one GPU, the second on a smaller lattice (its
scratch array keeps the first call's contents), and a lattice above the scratch limit refused
before any device work."""
import numpy as np
import pytest

import oracle
from ksinputs import make_gauge, gaussian_source
from conftest import rel_l2
from gpu_util import dev, host, zeros_dev, announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ks():
    import torch
    import paper_1611_00728_amd as ks
    assert torch.cuda.is_available()
    return ks


def test_apply_A_noalloc_matches_apply_A(ks):
    import torch
    for dims, sigma, seed in (((32, 32, 32, 32), 4e-4, 1002), ((8, 6, 10, 12), 0.37, 61)):
        announce("apply_A_noalloc", dims)
        g = make_gauge(dims, 0.5, seed)
        G = ks.Gauge(dims, g.fat, g.naik)
        vh = g.volume // 2
        x = gaussian_source(vh, seed + 1)
        xd = dev(x)
        want = zeros_dev((vh, 3))
        ks.apply_A(G, sigma, xd, want)
        got = zeros_dev((vh, 3)).fill_(float("nan"))
        ks.apply_A_noalloc(G, sigma, xd, got)
        torch.cuda.synchronize()
        # the same kernels in the same launch forms: bit for bit
        assert torch.equal(got, want)
        assert rel_l2(host(got), oracle.apply_A(g, sigma, x)) <= 1e-12
        assert torch.equal(xd, dev(x))          # the input is not touched
        G.free()


def test_apply_A_noalloc_limits(ks):
    """A lattice of 557056 even sites (above the 524288 of the scratch array) is refused with
    KS_ERR_ARG and a message naming the limit; aliasing and null pointers are refused too."""
    import torch
    announce("apply_A_noalloc limits")
    dims = (32, 32, 32, 34)
    V = int(np.prod(dims))
    eye = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3))
    G = ks.Gauge(dims, np.ascontiguousarray(eye), np.ascontiguousarray(eye))
    x = zeros_dev((V // 2, 3))
    out = zeros_dev((V // 2, 3))
    with pytest.raises(ks.KSError) as e:
        ks.apply_A_noalloc(G, 0.1, x, out)
    assert e.value.code == -1 and "524288" in str(e.value)
    G.free()
    g = make_gauge((4, 4, 4, 4), 0.5, 62)
    G = ks.Gauge(g.dims, g.fat, g.naik)
    x = zeros_dev((128, 3))
    with pytest.raises(ks.KSError) as e:
        ks.apply_A_noalloc(G, 0.1, x, x)
    assert e.value.code == -1
    G.free()
    torch.cuda.synchronize()
