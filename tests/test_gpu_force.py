"""GPU link derivative of the multi-shift pseudofermion action (ks_force) against the FP64
oracle's outer-product sums, element by element, on the same solutions: FP64 on both sides,
the only difference the order of a few dozen products and sums (bound 1e-12 relative to the
largest entry); and along a random direction it reproduces the finite-difference derivative
of the action (the oracle's pin) to the same 1e-6."""
import numpy as np
import pytest

import oracle
from ksinputs import make_gauge, gaussian_source
from gpu_util import dev, host, announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ks():
    import torch
    import paper_1611_00728_amd as ks
    assert torch.cuda.is_available()
    return ks


# 6x6x6x4 has 864 sites: its last block of 64 sites is ragged (the other lattices fill theirs)
@pytest.mark.parametrize("dims,nterm", [((4, 4, 4, 6), 3), ((8, 6, 10, 12), 9), ((4, 4, 4, 4), 1),
                                        ((6, 6, 6, 4), 2)])
def test_force_matches_oracle(ks, dims, nterm):
    announce("force", dims, nterm)
    import torch
    g = make_gauge(dims, 0.5, 81)
    G = ks.Gauge(dims, g.fat, g.naik)
    vh = g.volume // 2
    rng = np.random.default_rng(82)
    xs = [gaussian_source(vh, 83 + i) for i in range(nterm)]
    res = rng.uniform(0.1, 2.0, nterm)
    fv = torch.zeros(4 * g.volume * 9, dtype=torch.complex128, device="cuda")
    fw = torch.zeros_like(fv)
    ks.force(G, res, [dev(x) for x in xs], fv, fw)
    torch.cuda.synchronize()
    ov, ow = oracle.force_outer(g, res, xs)
    for got, ref in ((host(fv).reshape(ov.shape), ov), (host(fw).reshape(ow.shape), ow)):
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_force_finite_difference(ks):
    """On the solutions of the GPU multi-shift solver, the GPU force gives the derivative of
    the oracle's action along a random fat-link direction."""
    announce("force finite difference")
    import torch
    from ksinputs import GaugeField
    g = make_gauge((4, 4, 4, 6), 0.5, 91)
    G = ks.Gauge(g.dims, g.fat, g.naik)
    phi = gaussian_source(g.volume // 2, 92)
    sig = np.array([0.05, 0.3])
    r = np.array([0.6, 1.4])
    xs = [torch.zeros(g.volume // 2, 3, dtype=torch.complex128, device="cuda") for _ in sig]
    rc, _ = ks.multishift_cg_solve(G, sig, dev(phi), xs, 1e-12)
    assert rc == 0
    fv = torch.zeros(4 * g.volume * 9, dtype=torch.complex128, device="cuda")
    fw = torch.zeros_like(fv)
    ks.force(G, r, xs, fv, fw)
    torch.cuda.synchronize()
    f = host(fv).reshape(4, g.volume, 3, 3)
    d = np.random.default_rng(93).standard_normal(f.shape) * (1 + 1j)
    an = 2.0 * float(np.einsum("mxab,mxba->", d, f).real)
    eps = 1e-5
    sp = oracle.rational_action(GaugeField(g.dims, g.fat + eps * d, g.naik), r, sig, phi)
    sm = oracle.rational_action(GaugeField(g.dims, g.fat - eps * d, g.naik), r, sig, phi)
    assert abs((sp - sm) / (2 * eps) - an) <= 1e-6 * abs(an)


def test_force_argument_errors(ks):
    announce("force args")
    import torch
    g = make_gauge((4, 4, 4, 4), 0.5, 94)
    G = ks.Gauge(g.dims, g.fat, g.naik)
    x = dev(gaussian_source(g.volume // 2, 95))
    fv = torch.zeros(4 * g.volume * 9, dtype=torch.complex128, device="cuda")
    with pytest.raises(ks.KSError):
        ks.force(G, [1.0] * 33, [x] * 33, fv, torch.zeros_like(fv))
    with pytest.raises(ks.KSError):
        ks.force(G, [1.0], [x], fv, fv)
    with pytest.raises(ValueError):
        ks.force(G, [1.0], [x], fv[:10], torch.zeros_like(fv))
