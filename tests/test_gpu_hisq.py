"""GPU link construction (ks_hisq_links) against the FP64 oracle's two-level smearing,
element by element: FP64 on both sides, differing in summation order and in the method of the
U(3) projection (Newton polar iteration on the GPU, eigendecomposition in the oracle), each
accurate to a few units of roundoff, so 1e-11 of the largest entry."""
import numpy as np
import pytest

import oracle
from oracle import hisq
from ksinputs import thin_links, gaussian_source
from gpu_util import dev, host, announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ks():
    import torch
    import paper_1611_00728_amd as ks
    assert torch.cuda.is_available()
    return ks


def build(ks, dims, U, level1=None, level2=None, c_naik=-1.0 / 24):
    import torch
    t = dev(U.reshape(-1))
    fat = torch.empty_like(t)
    naik = torch.empty_like(t)
    ks.hisq_links(dims, t, fat, naik, level1, level2, c_naik)
    torch.cuda.synchronize()
    return host(fat).reshape(U.shape), host(naik).reshape(U.shape)


@pytest.mark.parametrize("dims", [(4, 4, 4, 6), (8, 6, 4, 8)])
def test_hisq_links_match_oracle(ks, dims):
    announce("hisq links", dims)
    U = thin_links(dims, 0.5, 121)
    fat, naik = build(ks, dims, U)
    ofat, onaik = hisq.hisq_links(U, dims)
    assert np.max(np.abs(fat - ofat)) <= 1e-11 * np.max(np.abs(ofat))
    assert np.max(np.abs(naik - onaik)) <= 1e-11 * np.max(np.abs(onaik))


def test_hisq_custom_coefficients(ks):
    announce("hisq custom coefficients")
    dims = (4, 4, 4, 4)
    U = thin_links(dims, 0.4, 122)
    l1, l2 = (0.3, 0.07, 0.01, 0.002, -0.02), (0.8, 0.05, 0.02, 0.001, -0.1)
    fat, naik = build(ks, dims, U, l1, l2, -0.05)
    ofat, onaik = hisq.hisq_links(U, dims, l1, l2, -0.05)
    assert np.max(np.abs(fat - ofat)) <= 1e-11 * np.max(np.abs(ofat))
    assert np.max(np.abs(naik - onaik)) <= 1e-11 * np.max(np.abs(onaik))


def test_hisq_links_drive_the_solver(ks):
    """Links built on the GPU load into the solver; its CG solution has the oracle's FP64
    residual on the oracle-built links."""
    announce("hisq links into CG")
    import torch
    dims = (8, 6, 4, 8)
    U = thin_links(dims, 0.5, 123)
    fat, naik = build(ks, dims, U)
    G = ks.Gauge(dims, fat, naik)
    ofat, onaik = hisq.hisq_links(U, dims)
    from ksinputs import GaugeField
    og = GaugeField(dims, ofat, onaik)
    vh = int(np.prod(dims)) // 2
    b = gaussian_source(vh, 124)
    x = torch.zeros(vh, 3, dtype=torch.complex128, device="cuda")
    res = ks.cg_solve(G, 0.05, dev(b), x, ks.default_params(tol=1e-10, inner=ks.F32))
    torch.cuda.synchronize()
    assert res.ok
    r = np.linalg.norm(b - oracle.apply_A(og, 0.01, host(x))) / np.linalg.norm(b)
    assert r <= 1e-10


def test_hisq_singular_links_rejected(ks):
    announce("hisq singular")
    import torch
    dims = (4, 4, 4, 4)
    z = torch.zeros(36 * 256, dtype=torch.complex128, device="cuda")
    with pytest.raises(ks.KSError) as e:
        ks.hisq_links(dims, z, torch.empty_like(z), torch.empty_like(z))
    assert e.value.code == -7
    z5 = torch.zeros(36 * 320, dtype=torch.complex128, device="cuda")
    with pytest.raises(ks.KSError) as e:
        ks.hisq_links((4, 4, 5, 4), z5, torch.empty_like(z5), torch.empty_like(z5))
    assert e.value.code == -1


def test_scratch_kept_between_calls(ks):
    """The scratch kept between calls gives the same links on a later call, on a smaller
    lattice after a larger one, and after it has been released."""
    import torch
    announce("hisq scratch reuse")
    outs = {}
    for dims in ((8, 8, 8, 8), (4, 6, 4, 8), (8, 8, 8, 8)):
        U = thin_links(dims, 0.5, 123)
        thin = dev(U.reshape(-1))
        fat, naik = torch.empty_like(thin), torch.empty_like(thin)
        ks.hisq_links(dims, thin, fat, naik)
        torch.cuda.synchronize()
        got = (host(fat), host(naik))
        if dims in outs:
            assert all(np.array_equal(a, b) for a, b in zip(got, outs[dims]))
        outs[dims] = got
    ks.hisq_release()
    dims = (4, 6, 4, 8)
    thin = dev(thin_links(dims, 0.5, 123).reshape(-1))
    fat, naik = torch.empty_like(thin), torch.empty_like(thin)
    ks.hisq_links(dims, thin, fat, naik)
    torch.cuda.synchronize()
    assert np.array_equal(host(fat), outs[dims][0]) and np.array_equal(host(naik), outs[dims][1])
