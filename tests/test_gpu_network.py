"""GPU preconditioner network N = L^+ L and flexible CG through the C ABI, against the FP64
oracle.

Tolerances:
* forward, FP32 path (transports and mixing in FP32, four layers): 1e-5 relative L2, and every
  output component within 2^-13 S of the oracle's, S the component's sum of product moduli
  (the oracle network run on |w|, |V| and |b|): four layers of FP32 sums of a few hundred
  terms each stay far inside it;
* forward, matrix-core path (every layer's input activations, stored links, transported
  values and weights rounded to binary16, unit roundoff 2^-11 per operand, some 200 terms
  per output adding in quadrature: about 5e-4 per layer): 3e-3 relative L2 and 2^-6 S per
  component;
* loss 1e-5 relative (the GPU takes x^+ A x as Re<x, b> and A (y - x) as A y - b, exact up to
  the pairs' FP64 solve tolerance); gradient 1e-4 relative L2 and every component within
  1e-4 of the largest (FP32 forward and backward passes, FP64 sums);
* one Adam step moves each real by lr * g / (|g| + eps) ~ lr sign(g): weights after one step
  agree with the oracle's to 1e-6 wherever |g| is not tiny.
Solves are judged by the oracle's FP64 residual of the returned x.
"""
import numpy as np
import pytest

import oracle
from oracle import network as N
from ksinputs import make_gauge, gaussian_source, net_init_weights, flatten_weights, GaugeField
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


def modulus_sums(g, ws, b):
    """Per output component, the sum of the moduli of every product the network adds."""
    ga = GaugeField(g.dims, np.abs(g.fat).astype(np.complex128), g.naik)
    out, _ = N.network_forward(N.Network([np.abs(w).astype(np.complex128) for w in ws]), ga,
                               np.abs(b).astype(np.complex128), keep_cache=False)
    return out.real


# (6, 6, 6, 6): Vh = 648 is not a multiple of the 16 sites of a wave, so one wave holds sites
# of both parities and the last block has lanes past the end
@pytest.mark.parametrize("dims", [(4, 6, 4, 8), (8, 8, 8, 8), (6, 4, 4, 4), (6, 6, 6, 6),
                                  (16, 16, 16, 16)])
def test_forward_f32_and_mfma(ks, dims):
    announce("net forward", dims)
    import torch
    g = make_gauge(dims, 0.5, 78)
    G = ks.Gauge(dims, g.fat, g.naik)
    ws = random_net(5000)
    net = ks.Net(flatten_weights(ws))
    b = gaussian_source(g.volume // 2, 3)
    ref, _ = N.network_forward(N.Network(ws), g, b, keep_cache=False)
    S = modulus_sums(g, ws, b)
    out = zeros_dev(b.shape)
    for mfma, l2, rel in ((False, 1e-5, 2.0 ** -13), (True, 3e-3, 2.0 ** -6)):
        net.apply(G, dev(b), out, mfma=mfma)
        torch.cuda.synchronize()
        got = host(out)
        assert rel_l2(got, ref) <= l2, mfma
        assert np.all(np.abs(got.real - ref.real) <= rel * S), mfma
        assert np.all(np.abs(got.imag - ref.imag) <= rel * S), mfma
    net.free()
    G.free()


@pytest.mark.parametrize("dims,prec", [((6, 6, 6, 6), "f64"), ((6, 6, 6, 6), "f32"),
                                       ((16, 16, 16, 16), "f32")])
def test_apply_field(ks, dims, prec):
    """N applied to the solver's own FP64 / FP32 even-site fields (what the flexible CG calls
    each step), both paths, every component against the oracle."""
    announce("net apply field", dims, prec)
    import torch
    g = make_gauge(dims, 0.5, 79)
    G = ks.Gauge(dims, g.fat, g.naik)
    ws = random_net(5004)
    net = ks.Net(flatten_weights(ws))
    b = gaussian_source(g.volume // 2, 7)
    if prec == "f32":
        b = b.astype(np.complex64).astype(np.complex128)   # the field stores FP32
    ref, _ = N.network_forward(N.Network(ws), g, b, keep_cache=False)
    S = modulus_sums(g, ws, b)
    fin = ks.Field(G, 0, ks.PREC[prec]).load(dev(b))
    fout = ks.Field(G, 0, ks.PREC[prec])
    out = zeros_dev(b.shape)
    for mfma, rel in ((False, 2.0 ** -13), (True, 2.0 ** -6)):
        net.apply_field(fin, fout, mfma=mfma)
        fout.store(out)
        torch.cuda.synchronize()
        got = host(out)
        assert np.all(np.abs(got.real - ref.real) <= rel * S), mfma
        assert np.all(np.abs(got.imag - ref.imag) <= rel * S), mfma
    with pytest.raises(ks.KSError):
        net.apply_field(fin, fin)
    odd = ks.Field(G, 1, ks.PREC[prec])
    with pytest.raises(ks.KSError):
        net.apply_field(fin, odd)
    f16 = ks.Field(G, 0, ks.F16)
    with pytest.raises(ks.KSError):
        net.apply_field(f16, fout)
    for f in (fin, fout, odd, f16):
        f.free()
    net.free()
    G.free()


def test_forward_32(ks):
    """One forward pass on the 32^4 benchmark lattice, both paths, every site."""
    announce("net forward 32^4")
    import torch
    dims = (32, 32, 32, 32)
    g = make_gauge(dims, 0.5, 1002)
    G = ks.Gauge(dims, g.fat, g.naik)
    ws = random_net(5002)
    net = ks.Net(flatten_weights(ws))
    b = gaussian_source(g.volume // 2, 2002)
    ref, _ = N.network_forward(N.Network(ws), g, b, keep_cache=False)
    out = zeros_dev(b.shape)
    for mfma, l2 in ((False, 1e-5), (True, 3e-3)):
        net.apply(G, dev(b), out, mfma=mfma)
        torch.cuda.synchronize()
        assert rel_l2(host(out), ref) <= l2, mfma
    net.free()
    G.free()


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


def test_hermitian_positive(ks, lat):
    """The GPU's N is Hermitian and positive: <u, N v> = conj<v, N u> and <v, N v> > 0."""
    announce("net hermitian")
    import torch
    G = ks.Gauge(lat.dims, lat.fat, lat.naik)
    net = ks.Net(flatten_weights(random_net(5003)))
    vh = lat.volume // 2
    u, v = gaussian_source(vh, 5), gaussian_source(vh, 6)
    Nu, Nv = zeros_dev(u.shape), zeros_dev(v.shape)
    net.apply(G, dev(u), Nu)
    net.apply(G, dev(v), Nv)
    torch.cuda.synchronize()
    a = np.vdot(u.ravel(), host(Nv).ravel())
    b = np.vdot(v.ravel(), host(Nu).ravel())
    assert abs(a - np.conj(b)) <= 1e-5 * abs(a)
    vNv = np.vdot(v.ravel(), host(Nv).ravel())
    assert vNv.real > 0 and abs(vNv.imag) <= 1e-5 * vNv.real


def _pairs(dims_list, masses, seeds):
    gs = [make_gauge(d, 0.5, s) for d, s in zip(dims_list, seeds)]
    sig = [4 * m * m for m in masses]
    bs = [gaussian_source(g.volume // 2, 10 + k) for k, g in enumerate(gs)]
    xs = [oracle.cg(g, s, b, 1e-12)[0] for g, s, b in zip(gs, sig, bs)]
    return gs, sig, bs, xs


@pytest.mark.parametrize("dims_list", [[(4, 6, 4, 8), (4, 4, 4, 4)], [(16, 16, 16, 16)]])
def test_loss_and_gradient(ks, dims_list):
    """Loss and gradient against the oracle (pairs on two lattices of different sizes, and one
    pair on a 16^4 block, the training block size), element by element, and one Adam step."""
    announce("net loss grad", dims_list)
    masses = [0.05, 0.2][:len(dims_list)]
    gs, sig, bs, xs = _pairs(dims_list, masses, [80 + k for k in range(len(dims_list))])
    Gs = [ks.Gauge(g.dims, g.fat, g.naik) for g in gs]
    ws = random_net(5001)
    net = ks.Net(flatten_weights(ws))
    loss, grad = net.loss_grad(Gs, sig, [dev(b) for b in bs], [dev(x) for x in xs])
    # oracle: the loss averages over all pairs; pairs on different lattices add their terms
    ref_loss = 0.0
    ref_grad = [np.zeros_like(w) for w in ws]
    for g, s, b, x in zip(gs, sig, bs, xs):
        l, gr = N.loss_and_grad(N.Network([w.copy() for w in ws]), g, [s], [b], [x])
        ref_loss += l / len(gs)
        for k in range(2):
            ref_grad[k] += gr[k] / len(gs)
    rg = flatten_weights(ref_grad)
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    assert rel_l2(grad, rg) <= 1e-4
    big = np.max(np.abs(rg))
    assert np.max(np.abs(grad.real - rg.real)) <= 1e-4 * big
    assert np.max(np.abs(grad.imag - rg.imag)) <= 1e-4 * big
    if len(dims_list) > 1:
        # one Adam step
        net.set_weights(flatten_weights(ws))
        net.train(Gs, sig, [dev(b) for b in bs], [dev(x) for x in xs], steps=1, batch=2, lr=1e-3)
        wn = net.get_weights()
        on = N.Network([w.copy() for w in ws])
        N.adam_step(on, ref_grad, lr=1e-3)
        sel = (np.abs(rg.real) > 1e-4 * big) & (np.abs(rg.imag) > 1e-4 * big)
        assert np.max(np.abs((wn - flatten_weights(on.weights))[sel])) <= 1e-6
    net.free()
    for G in Gs:
        G.free()


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
    hist = net.train([G] * 6, [sigma] * 6, bs, xs, steps=60, batch=3, lr=3e-3)
    assert hist[-1] < 0.8 * hist[0]
    net.free()


def test_checkpoint_resumes_training(ks, lat, tmp_path):
    """A checkpoint (weights, Adam moments, step count) taken after 10 Adam steps and restored
    into a fresh network continues training exactly as the original does: 10 more steps give
    the same loss history and the same weights bit for bit; a malformed state is refused."""
    announce("net checkpoint")
    G = ks.Gauge(lat.dims, lat.fat, lat.naik)
    sigma = 4 * 0.05 ** 2
    bs, xs = [], []
    for j in range(4):
        b = gaussian_source(lat.volume // 2, 700 + j)
        x, _ = oracle.cg(lat, sigma, b, 1e-12)
        bs.append(dev(b))
        xs.append(dev(x))
    args = ([G] * 4, [sigma] * 4, bs, xs)
    a = ks.Net(flatten_weights(net_init_weights(5000)))
    a.train(*args, steps=10, batch=2, lr=3e-3)
    path = tmp_path / "net.ckpt"
    a.save(path)
    w, m, v, step = ks.read_checkpoint(path)
    assert step == 10 and np.any(m != 0) and np.all(v >= 0)
    ha = a.train(*args, steps=10, batch=2, lr=3e-3)
    b2 = ks.Net(flatten_weights(net_init_weights(6000))).load(path)
    hb = b2.train(*args, steps=10, batch=2, lr=3e-3)
    assert np.array_equal(ha, hb)
    assert np.array_equal(a.get_weights(), b2.get_weights())
    assert a.get_state()[3] == b2.get_state()[3] == 20
    with pytest.raises(ks.KSError):
        b2.set_state(w, m, -np.abs(v) - 1.0, 3)
    with pytest.raises(ks.KSError):
        b2.set_state(w, m, v, -1)
    a.free()
    b2.free()
    G.free()


def test_batched_training_pairs(ks):
    """Training pairs from blocks cut out of a larger lattice, solved together by the batched
    FP64 CG: every x solves its own block's system to the oracle's FP64 residual, and the pair
    carries that block's gauge handle and shift."""
    announce("batched training pairs")
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
    for k, (G, s, b, x) in enumerate(pairs):
        bk = blocks[k // 2]
        assert G.dims == tuple(bk.dims) and s == sigma
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


@pytest.mark.parametrize("mfma,inner", [(False, "f32"), (True, "f32"), (True, "f64")])
def test_fcg_network_preconditioner(ks, lat, mfma, inner):
    """An untrained N = L^+ L is still positive: flexible CG never falls back (the network
    reads and writes the solver's FP32 or FP64 vectors)."""
    announce("fcg network", mfma, inner)
    import torch
    G = ks.Gauge(lat.dims, lat.fat, lat.naik)
    net = ks.Net(flatten_weights(random_net(5000)))
    b = gaussian_source(lat.volume // 2, 56)
    x = zeros_dev(b.shape)
    res = ks.fcg_solve(G, net, 0.05, dev(b), x,
                       ks.default_params(tol=1e-10, inner=ks.PREC[inner]),
                       mfma=mfma, raise_on_error=False)
    torch.cuda.synchronize()
    tr = float(np.linalg.norm(b - oracle.apply_A(lat, 0.01, host(x))) / np.linalg.norm(b))
    assert res.status == 0 and tr <= 1e-10 and res.stats["fallback"] == 0


def test_fcg_fallback(ks, lat):
    """N = 0 gives <z, r> = 0 (reason 2) and a non-finite weight a non-finite z (reason 1):
    both fall back to CG from the current x and still solve."""
    announce("fcg fallback")
    import torch
    G = ks.Gauge(lat.dims, lat.fat, lat.naik)
    b = gaussian_source(lat.volume // 2, 57)
    for w, reason in ((np.zeros(648, complex), 2),
                      (np.where(np.arange(648) == 3, np.nan, 0.1).astype(complex), 1)):
        net = ks.Net(w)
        x = zeros_dev(b.shape)
        res = ks.fcg_solve(G, net, 0.05, dev(b), x, ks.default_params(tol=1e-10, inner=ks.F32),
                           raise_on_error=False)
        torch.cuda.synchronize()
        tr = float(np.linalg.norm(b - oracle.apply_A(lat, 0.01, host(x))) / np.linalg.norm(b))
        assert res.status == 0 and res.stats["fallback"] == reason and tr <= 1e-10
        assert res.stats["restarts"] == res.stats["iters"]
        net.free()


def test_trained_network_cuts_iterations(ks):
    """The learned preconditioner's gain: on a 16^4 lattice of the large workload's recipe
    (thin-link scale 0.5) at m = 0.002, N trained by the library's kernels on FP64-CG pairs that
    the library generated cuts the flexible CG's steps well below plain CG's (both with FP32
    inner iterations and FP64 reliable updates), on a source it was not trained on, without
    falling back; both solutions judged by the oracle's FP64 residual."""
    announce("trained network gain 16^4 m=0.002")
    import torch
    from paper_1611_00728_amd import learn
    dims, mass = (16, 16, 16, 16), 0.002
    g = make_gauge(dims, 0.5, 1105)
    G = ks.Gauge(dims, g.fat, g.naik)
    vh = g.volume // 2
    pairs = learn.solve_pairs(G, mass, [gaussian_source(vh, 5100 + j) for j in range(32)])
    net = ks.Net(flatten_weights(net_init_weights(5000)))
    hist, _ = learn.train(net, pairs, steps=1000, batch=4, lr=1e-2)
    assert hist[-1] < 0.5 * hist[0]
    b = gaussian_source(vh, 5999)
    iters = {}
    for name in ("cg", "fcg"):
        x = zeros_dev(b.shape)
        p = ks.default_params(tol=1e-10, inner=ks.F32)
        if name == "cg":
            res = ks.cg_solve(G, mass, dev(b), x, p)
        else:
            res = ks.fcg_solve(G, net, mass, dev(b), x, p, mfma=True)
            assert res.stats["fallback"] == 0
        torch.cuda.synchronize()
        tr = float(np.linalg.norm(b - oracle.apply_A(g, 4 * mass * mass, host(x))) /
                   np.linalg.norm(b))
        assert res.ok and tr <= 1e-10, (name, tr)
        iters[name] = res.stats["iters"]
    announce("iterations", iters)
    # measured: 395 CG steps, 203 flexible steps
    assert iters["fcg"] <= 0.7 * iters["cg"], iters
    net.free()
    G.free()
