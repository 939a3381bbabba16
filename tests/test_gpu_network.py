"""GPU preconditioner network and flexible CG through the C ABI, against the FP64 oracle.

Tolerances: the FP32 path (transports and mixing in FP32, four layers) 1e-5 relative L2 on
outputs and 1e-4 on the gradient; the matrix-core path rounds the mixing operands (weights
and transported values) of the 8 -> 8, 8 -> 8 and 8 -> 1 layers to binary16 (unit roundoff
2^-11 ~ 4.9e-4 per operand, errors of 72 terms per output adding in quadrature: a few 1e-4
per layer), 3e-3.  One Adam
step moves each real by lr * g / (|g| + eps) ~ lr sign(g): weights after one step agree
with the oracle's to 1e-6 wherever |g| is not tiny.
"""
import numpy as np
import pytest

import oracle
from oracle import network as N
from ksinputs import make_gauge, gaussian_source, net_init_weights, flatten_weights
from conftest import rel_l2
from gpu_util import dev, host, zeros_dev, announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ks():
    import torch
    import paper_1611_00728_amd as ks
    assert torch.cuda.is_available()
    return ks


@pytest.fixture(scope="module")
def lat():
    g = make_gauge((4, 6, 4, 8), 0.5, 77)
    return g


def random_net(seed):
    ws = net_init_weights(seed)
    rng = np.random.default_rng(seed + 1)
    # perturb so that every path and channel matters
    return [w + 0.2 * (rng.standard_normal(w.shape) + 1j * rng.standard_normal(w.shape)) for w in ws]


@pytest.mark.parametrize("dims", [(4, 6, 4, 8), (8, 8, 8, 8), (6, 4, 4, 4)])
def test_forward_f32_and_mfma(ks, dims):
    announce("net forward", dims)
    import torch
    g = make_gauge(dims, 0.5, 78)
    G = ks.Gauge(dims, g.fat, g.naik)
    ws = random_net(5000)
    net = ks.Net(flatten_weights(ws))
    b = gaussian_source(g.volume // 2, 3)
    ref, _ = N.network_forward(N.Network(ws), g, b)
    out = zeros_dev(b.shape)
    net.apply(G, dev(b), out, mfma=False)
    torch.cuda.synchronize()
    assert rel_l2(host(out), ref) <= 1e-5
    net.apply(G, dev(b), out, mfma=True)
    torch.cuda.synchronize()
    assert rel_l2(host(out), ref) <= 3e-3
    net.free()


def test_identity_network(ks, lat):
    announce("net identity")
    import torch
    G = ks.Gauge(lat.dims, lat.fat, lat.naik)
    net = ks.Net(flatten_weights(N.Network.identity().weights))
    b = gaussian_source(lat.volume // 2, 4)
    out = zeros_dev(b.shape)
    net.apply(G, dev(b), out)
    torch.cuda.synchronize()
    assert rel_l2(host(out), b) <= 1e-7
    net.apply(G, dev(b), out, mfma=True)
    torch.cuda.synchronize()
    assert rel_l2(host(out), b) <= 1e-3


def test_loss_and_gradient(ks):
    announce("net loss grad")
    dims_list = [(4, 6, 4, 8), (4, 4, 4, 4)]
    gs = [make_gauge(d, 0.5, 80 + k) for k, d in enumerate(dims_list)]
    Gs = [ks.Gauge(g.dims, g.fat, g.naik) for g in gs]
    ws = random_net(5001)
    net = ks.Net(flatten_weights(ws))
    bs = [gaussian_source(g.volume // 2, 10 + k) for k, g in enumerate(gs)]
    xs = [gaussian_source(g.volume // 2, 20 + k) for k, g in enumerate(gs)]
    loss, grad = net.loss_grad(Gs, [dev(b) for b in bs], [dev(x) for x in xs])
    # oracle: the loss averages over all pairs; pairs on different lattices add their terms
    ref_loss = 0.0
    ref_grad = [np.zeros_like(w) for w in ws]
    for g, b, x in zip(gs, bs, xs):
        l, gr = N.loss_and_grad(N.Network([w.copy() for w in ws]), g, [b], [x])
        ref_loss += l / len(gs)
        for k in range(4):
            ref_grad[k] += gr[k] / len(gs)
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    assert rel_l2(grad, flatten_weights(ref_grad)) <= 1e-4
    # one Adam step
    net.set_weights(flatten_weights(ws))
    net.train(Gs, [dev(b) for b in bs], [dev(x) for x in xs], steps=1, batch=2, lr=1e-3)
    wn = net.get_weights()
    on = N.Network([w.copy() for w in ws])
    N.adam_step(on, ref_grad, lr=1e-3)
    rg = flatten_weights(ref_grad)
    big = (np.abs(rg.real) > 1e-4 * np.max(np.abs(rg))) & (np.abs(rg.imag) > 1e-4 * np.max(np.abs(rg)))
    assert np.max(np.abs((wn - flatten_weights(on.weights))[big])) <= 1e-6
    net.free()


def test_training_reduces_loss(ks, lat):
    announce("net training")
    G = ks.Gauge(lat.dims, lat.fat, lat.naik)
    sigma = 4 * 0.05 ** 2
    bs, xs = [], []
    for j in range(6):
        b = gaussian_source(lat.volume // 2, 100 + j)
        x, info = oracle.cg(lat, sigma, b, 1e-12)
        bs.append(dev(b))
        xs.append(dev(x))
    net = ks.Net(flatten_weights(net_init_weights(5000)))
    hist = net.train([G] * 6, bs, xs, steps=60, batch=3, lr=3e-3)
    assert hist[-1] < 0.8 * hist[0]
    net.free()


def test_batched_training_pairs(ks):
    """Training pairs from blocks cut out of a larger lattice, solved together by the batched
    FP64 CG: every x solves its own block's system to the oracle's FP64 residual, and the pair
    carries that block's gauge handle."""
    announce("batched training pairs")
    import torch
    from ksinputs import subblock
    from paper_1611_00728_amd import learn
    big = make_gauge((8, 8, 8, 8), 0.5, 91, keep_thin=True)
    origins = learn.block_origins(big.dims, (4, 4, 8, 8))
    assert len(origins) == 4
    blocks = [subblock(big, o, (4, 4, 8, 8)) for o in origins]
    srcs = [[gaussian_source(bk.volume // 2, 300 + 2 * j + r) for r in range(2)]
            for j, bk in enumerate(blocks)]
    pairs, secs, stats = learn.solve_pairs_batched(blocks, srcs, 0.05, tol=1e-10)
    assert len(pairs) == 8 and secs > 0 and all(s["status"] == 0 for s in stats)
    sigma = 4 * 0.05 ** 2
    for k, (G, b, x) in enumerate(pairs):
        bk = blocks[k // 2]
        assert G.dims == tuple(bk.dims)
        assert np.array_equal(host(b), srcs[k // 2][k % 2])
        xh = host(x)
        r = np.linalg.norm(host(b) - oracle.apply_A(bk, sigma, xh)) / np.linalg.norm(host(b))
        assert r <= 1e-10


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_fcg_identity_matches_cg(ks, lat, inner):
    announce("fcg identity", inner)
    import torch
    G = ks.Gauge(lat.dims, lat.fat, lat.naik)
    net = ks.Net(flatten_weights(N.Network.identity().weights))
    b = gaussian_source(lat.volume // 2, 55)
    x = zeros_dev(b.shape)
    res = ks.fcg_solve(G, net, 0.05, dev(b), x, ks.default_params(tol=1e-10, inner=ks.PREC[inner]))
    torch.cuda.synchronize()
    xh = host(x)
    tr = float(np.linalg.norm(b - oracle.apply_A(lat, 0.01, xh)) / np.linalg.norm(b))
    assert res.ok and tr <= 1e-10 and res.stats["fallback"] == 0
    _, info = oracle.cg(lat, 0.01, b, 1e-10)
    assert abs(res.stats["iters"] - info.iters) <= 3


@pytest.mark.parametrize("mfma", [False, True])
def test_fcg_network_preconditioner(ks, lat, mfma):
    announce("fcg network", mfma)
    import torch
    G = ks.Gauge(lat.dims, lat.fat, lat.naik)
    net = ks.Net(flatten_weights(net_init_weights(5000)))
    b = gaussian_source(lat.volume // 2, 56)
    x = zeros_dev(b.shape)
    res = ks.fcg_solve(G, net, 0.05, dev(b), x, ks.default_params(tol=1e-10, inner=ks.F32),
                       mfma=mfma, raise_on_error=False)
    torch.cuda.synchronize()
    tr = float(np.linalg.norm(b - oracle.apply_A(lat, 0.01, host(x))) / np.linalg.norm(b))
    assert res.status == 0 and tr <= 1e-10


def test_fcg_fallback(ks, lat):
    announce("fcg fallback")
    import torch
    G = ks.Gauge(lat.dims, lat.fat, lat.naik)
    bad = N.Network.identity()
    bad.weights[0] = -bad.weights[0]       # N = -1: Re<z, r> < 0
    net = ks.Net(flatten_weights(bad.weights))
    b = gaussian_source(lat.volume // 2, 57)
    x = zeros_dev(b.shape)
    res = ks.fcg_solve(G, net, 0.05, dev(b), x, ks.default_params(tol=1e-10, inner=ks.F32),
                       raise_on_error=False)
    torch.cuda.synchronize()
    tr = float(np.linalg.norm(b - oracle.apply_A(lat, 0.01, host(x))) / np.linalg.norm(b))
    # reason 2: Re<N(r), r> <= 0 before the first flexible step
    assert res.status == 0 and res.stats["fallback"] == 2 and tr <= 1e-10
    assert res.stats["restarts"] == res.stats["iters"]
