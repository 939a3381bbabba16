"""The benchmark's own configurations at full size, in the launch forms the benchmark times
(every variant autotuned on its lattice first, as bench.py does):

* every Dslash_eo output component of the six variants at 32^4, in the tuned launch form,
  against the oracle applied to the links and input as the device stores them (the 12-real
  Naik copies of the tuned link access), within the device's rounding bound
  (`dslash_check`), and the relative L2 distance to the plain FP64 oracle (FP64 1e-12, FP32
  5e-6, FP16 5e-3);
* the benchmark's CG solves at 32^4, m = 0.01 (FP64, FP32 with 18- and 12-real Naik, FP16 with
  12-real Naik), each x judged by the oracle's FP64 residual |b - A x| / |b| <= 1e-10;
* the benchmark's multi-shift solves at 32^3 x 48 (nine shifts, FP64, FP32 and FP16 inner with
  18-real Naik, FP64 and FP32 with 12-real Naik, per-shift target 1e-9), each x_i judged by the
  oracle's residual of its own shifted system;
* the benchmark's batches (64 lattices x 4 right-hand sides, tuned; FP32 inner with reliable
  updates at a 100-fold drop, binary16 inner at a 33-fold drop), every pair judged likewise.
"""
import numpy as np
import pytest

import oracle
from ksinputs import make_gauge, gaussian_source, SEEDS
from conftest import rel_l2
from gpu_util import dev, host, zeros_dev, announce
import dslash_check as dc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ks():
    import torch
    import paper_1611_00728_amd as ks
    assert torch.cuda.is_available()
    return ks


@pytest.fixture(scope="module")
def lat32(ks):
    dims = (32, 32, 32, 32)
    g = make_gauge(dims, 0.5, 1002)
    return g, ks.Gauge(dims, g.fat, g.naik), gaussian_source(g.volume // 2, 2002)


def true_rel(g, sigma, b, x):
    return float(np.linalg.norm(b - oracle.apply_A(g, sigma, x)) / np.linalg.norm(b))


@pytest.mark.parametrize("prec,recon", [("f64", 18), ("f64", 12), ("f32", 18), ("f32", 12),
                                         ("f16", 18), ("f16", 12)])
def test_tuned_dslash_32(ks, lat32, prec, recon):
    import torch
    g, G, psi = lat32
    vh = g.volume // 2
    P = ks.PREC[prec]
    tol = {"f64": 1e-12, "f32": 5e-6, "f16": 5e-3}[prec]
    G.prepare(P, recon)
    cfg = G.tune(P, recon)
    announce("tuned dslash 32^4", prec, recon, cfg)
    for out_par in (0, 1):
        inp = ks.Field(G, 1 - out_par, P).load(dev(psi))
        out = ks.Field(G, out_par, P)
        ks.dslash_eo(G, out, inp, recon)
        res = zeros_dev((vh, 3))
        out.store(res)
        torch.cuda.synchronize()
        got = host(res)
        assert rel_l2(got, oracle.dslash_eo(g, out_par, psi)) <= tol, (prec, recon, cfg)
        r, S = dc.reference(g, prec, recon, cfg["link_access"], out_par, psi)
        assert dc.worst(got, r, S, prec) <= 1.0, (prec, recon, cfg)
        del r, S


@pytest.mark.parametrize("inner,recon", [("f64", 18), ("f32", 18), ("f32", 12), ("f16", 12)])
def test_bench_cg_32(ks, lat32, inner, recon):
    import torch
    g, G, b = lat32
    announce("bench cg 32^4", inner, recon)
    G.prepare(ks.PREC[inner], recon)
    G.tune(ks.PREC[inner], recon)
    x = zeros_dev(b.shape)
    res = ks.cg_solve(G, 0.01, dev(b), x, ks.default_params(tol=1e-10, inner=inner, recon=recon),
                      raise_on_error=False)
    torch.cuda.synchronize()
    assert res.ok, res
    tr = true_rel(g, 4 * 0.01 ** 2, b, host(x))
    assert tr <= 1e-10
    assert abs(res.stats["true_rel_resid"] - tr) <= 1e-3 * tr


@pytest.fixture(scope="module")
def lat48(ks):
    dims = (32, 32, 32, 48)
    g = make_gauge(dims, 0.5, SEEDS["gauge"](3))
    G = ks.Gauge(dims, g.fat, g.naik)
    yield g, G, gaussian_source(g.volume // 2, SEEDS["source"](3))
    G.free()


@pytest.mark.parametrize("inner,recon", [("f32", 18), ("f64", 18), ("f16", 18), ("f32", 12),
                                         ("f64", 12)])
def test_bench_multishift_32x48(ks, lat48, inner, recon):
    import torch
    announce("bench multishift 32^3x48", inner, recon)
    g, G, b = lat48
    G.prepare(ks.PREC[inner], recon)
    G.tune(ks.PREC[inner], recon)
    sig = 4 * np.geomspace(0.002, 0.5, 9) ** 2
    xs = [zeros_dev(b.shape) for _ in sig]
    rc, stats = ks.multishift_cg_solve(G, sig, dev(b), xs, 1e-9,
                                       ks.default_params(inner=ks.PREC[inner], recon=recon,
                                                         check_every=16),
                                       raise_on_error=False)
    torch.cuda.synchronize()
    assert rc == 0
    for i, s in enumerate(sig):
        tr = true_rel(g, s, b, host(xs[i]))
        assert tr <= 1e-9, (i, tr)
        assert abs(stats[i]["true_rel_resid"] - tr) <= 1e-3 * tr


@pytest.mark.parametrize("inner,delta", [("f32", 0.01), ("f16", 0.03)])
def test_bench_batch(ks, inner, delta):
    """The benchmark's batch: 24 x 8^4 + 24 x 12^4 + 16 x 16^4 lattices x 4 right-hand sides,
    FP32 inner iterations with per-lattice reliable updates at a 100-fold drop, or binary16
    ones at a 33-fold drop, tuned schedule; every pair's x judged by the oracle's residual
    (<= 1e-10)."""
    import torch
    from ksinputs import batch_masses
    announce("bench batch 64 lattices x 4", inner)
    bdims = [(8, 8, 8, 8)] * 24 + [(12, 12, 12, 12)] * 24 + [(16, 16, 16, 16)] * 16
    gs = [make_gauge(d, 0.4, SEEDS["batch_gauge"](j)) for j, d in enumerate(bdims)]
    masses = batch_masses(len(bdims), 0.01, 0.2, SEEDS["batch_mass"])
    B = ks.Batch(bdims, [x.fat for x in gs], [x.naik for x in gs], 4, ks.PREC[inner])
    B.tune()
    bh = [gaussian_source(x.volume // 2, SEEDS["batch_rhs"](j, r)) for j, x in enumerate(gs)
          for r in range(4)]
    bs = [dev(b) for b in bh]
    xs = [zeros_dev(b.shape) for b in bh]
    rc, st = B.solve(masses, bs, xs, ks.default_params(tol=1e-10, check_every=8, delta=delta),
                     raise_on_error=False)
    torch.cuda.synchronize()
    assert rc == 0
    for p, b in enumerate(bh):
        j = p // 4
        tr = true_rel(gs[j], 4 * masses[j] ** 2, b, host(xs[p]))
        assert tr <= 1e-10, (p, tr)
    B.free()
