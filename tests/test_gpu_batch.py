"""GPU batched solver (many lattices of uneven sizes x several right-hand sides in one set of
launches) through the C ABI: every (lattice, RHS) pair is judged by the oracle's FP64
residual of its returned x, and must agree with the oracle's own CG solution on that lattice
within the R19 bound."""
import numpy as np
import pytest

import oracle
from ksinputs import make_gauge, gaussian_source, batch_masses
from conftest import rel_l2
from gpu_util import dev, host, zeros_dev, announce

pytestmark = pytest.mark.gpu

DIMS = [(4, 4, 4, 4), (8, 8, 8, 8), (6, 4, 8, 4), (8, 6, 4, 4), (12, 12, 12, 12)]


@pytest.fixture(scope="module")
def ks():
    import torch
    import paper_1611_00728_amd as ks
    assert torch.cuda.is_available()
    return ks


@pytest.fixture(scope="module")
def fields():
    gs = [make_gauge(d, 0.4, 4000 + j) for j, d in enumerate(DIMS)]
    masses = batch_masses(len(DIMS), seed=4100)
    return gs, masses


def true_rel(g, sigma, b, x):
    return float(np.linalg.norm(b - oracle.apply_A(g, sigma, x)) / np.linalg.norm(b))


def run_batch(ks, B, gs, masses, nrhs, tol=1e-10, **kw):
    import torch
    bs, xs, bh = [], [], []
    for j, g in enumerate(gs):
        for r in range(nrhs):
            b = gaussian_source(g.volume // 2, 4200 + 4 * j + r)
            bh.append(b)
            bs.append(dev(b))
            xs.append(zeros_dev(b.shape))
    rc, st = B.solve(masses, bs, xs, ks.default_params(tol=tol, **kw), raise_on_error=False)
    torch.cuda.synchronize()
    return rc, st, bh, [host(x) for x in xs]


@pytest.mark.parametrize("nrhs,inner", [(4, "f32"), (2, "f32"), (1, "f32"), (1, "f64"), (4, "f64"),
                                        (4, "f16"), (2, "f16"), (1, "f16")])
def test_batch_pairs_converge(ks, fields, nrhs, inner):
    announce("batch", nrhs, inner)
    gs, masses = fields
    B = ks.Batch([g.dims for g in gs], [g.fat for g in gs], [g.naik for g in gs], nrhs,
                 ks.PREC[inner])
    rc, st, bh, xh = run_batch(ks, B, gs, masses, nrhs, check_every=4)
    assert rc == 0, st
    for p, (b, x) in enumerate(zip(bh, xh)):
        j = p // nrhs
        sigma = 4 * masses[j] ** 2
        tr = true_rel(gs[j], sigma, b, x)
        assert tr <= 1e-10, (p, tr)
        assert st[p]["status"] == 0 and st[p]["seconds"] > 0
        assert abs(st[p]["true_rel_resid"] - tr) <= 1e-3 * tr + 1e-15
        if inner in ("f32", "f16"):
            assert st[p]["reliable_updates"] >= 1
    # each pair agrees with an independent oracle solve
    for p in (0, len(bh) - 1):
        j = p // nrhs
        sigma = 4 * masses[j] ** 2
        xo, info = oracle.cg(gs[j], sigma, bh[p], 1e-12)
        kappa = 16.5 / sigma
        assert rel_l2(xh[p], xo) <= 2e-10 * kappa
    B.free()


def test_batch_tuned_and_replayed(ks, fields):
    """After the autotuner picks a tile size / schedule, and on a second solve with other
    masses (the captured graph is replayed), every pair still converges."""
    announce("batch tuned replay")
    gs, masses = fields
    B = ks.Batch([g.dims for g in gs], [g.fat for g in gs], [g.naik for g in gs], 4, ks.F32)
    cfg = B.tune()
    assert cfg["tile_sites"] in (64, 128, 256) and cfg["tuned_us"] > 0
    for ms in (masses, masses[::-1] * 1.3):
        rc, st, bh, xh = run_batch(ks, B, gs, ms, 4, check_every=8)
        assert rc == 0
        for p, (b, x) in enumerate(zip(bh, xh)):
            j = p // 4
            assert true_rel(gs[j], 4 * ms[j] ** 2, b, x) <= 1e-10
    B.free()


def test_batch_matches_single_solves(ks, fields):
    announce("batch vs single")
    gs, masses = fields
    B = ks.Batch([g.dims for g in gs[:2]], [g.fat for g in gs[:2]], [g.naik for g in gs[:2]], 2,
                 ks.F64)
    rc, st, bh, xh = run_batch(ks, B, gs[:2], masses[:2], 2, check_every=1)
    assert rc == 0
    import torch
    for p in range(4):
        j = p // 2
        G = ks.Gauge(gs[j].dims, gs[j].fat, gs[j].naik)
        xd = zeros_dev(bh[p].shape)
        res = ks.cg_solve(G, masses[j], dev(bh[p]), xd, ks.default_params(tol=1e-10))
        torch.cuda.synchronize()
        # FP64 inner, same recurrences: the same number of steps
        assert abs(res.stats["iters"] - st[p]["iters"]) <= 1
        assert rel_l2(host(xd), xh[p]) <= 1e-7
    B.free()


@pytest.mark.parametrize("inner", ["f32", "f16"])
def test_batch_runs_are_bit_identical(ks, fields, inner):
    """Two solves of the same batch (reduced-precision inner, per-lattice reliable updates)
    return the same x bit for bit and the same step counts: the reductions have a fixed order
    and the reliable-update kernel's spread of work over the grid does not change any sum."""
    announce("batch repeatability", inner)
    gs, masses = fields
    B = ks.Batch([g.dims for g in gs], [g.fat for g in gs], [g.naik for g in gs], 4,
                 ks.PREC[inner])
    rc1, st1, _, x1 = run_batch(ks, B, gs, masses, 4, check_every=4)
    rc2, st2, _, x2 = run_batch(ks, B, gs, masses, 4, check_every=4)
    assert rc1 == 0 and rc2 == 0
    assert [s["iters"] for s in st1] == [s["iters"] for s in st2]
    assert [s["reliable_updates"] for s in st1] == [s["reliable_updates"] for s in st2]
    for a, c in zip(x1, x2):
        assert np.array_equal(a, c)
    B.free()


@pytest.mark.parametrize("inner", ["f32", "f16"])
def test_batch_zero_rhs_and_max_iter(ks, fields, inner):
    """A zero right-hand side finishes at once with x = 0 (binary16: all-zero records); a pair
    started from its own solution finishes in its first (FP64) check; a step cap returns
    KS_ERR_NOT_CONVERGED with the residual of the returned x."""
    announce("batch edge cases", inner)
    gs, masses = fields
    B = ks.Batch([gs[0].dims], [gs[0].fat], [gs[0].naik], 2, ks.PREC[inner])
    import torch
    b = gaussian_source(gs[0].volume // 2, 7)
    bs = [dev(np.zeros_like(b)), dev(b)]
    xs = [zeros_dev(b.shape), zeros_dev(b.shape)]
    rc, st = B.solve(masses[:1], bs, xs, ks.default_params(tol=1e-10), raise_on_error=False)
    torch.cuda.synchronize()
    assert rc == 0 and np.all(host(xs[0]) == 0) and st[0]["iters"] == 0
    assert true_rel(gs[0], 4 * masses[0] ** 2, b, host(xs[1])) <= 1e-10
    # restarted from its solution: no step, and x unchanged up to the FP64 check
    x1 = host(xs[1])
    rc, st = B.solve(masses[:1], bs, xs, ks.default_params(tol=1e-10), raise_on_error=False)
    torch.cuda.synchronize()
    assert rc == 0 and st[1]["iters"] == 0 and np.array_equal(host(xs[1]), x1)
    xs = [zeros_dev(b.shape), zeros_dev(b.shape)]
    rc, st = B.solve(masses[:1], [dev(b), dev(b)], xs, ks.default_params(tol=1e-10, max_iter=3),
                     raise_on_error=False)
    torch.cuda.synchronize()
    assert rc == -5 and all(s["status"] == -5 for s in st)
    # the step cap forces a reliable update: the reported residual is that of the returned x
    # (its FP32 increments added in before the update and again at the end)
    for k in range(2):
        tr = true_rel(gs[0], 4 * masses[0] ** 2, b, host(xs[k]))
        assert 1e-6 < tr < 1.0 and abs(st[k]["true_rel_resid"] - tr) <= 1e-6 * tr
    B.free()
