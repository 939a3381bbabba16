"""Pins of the oracle's preconditioner network and flexible CG: gauge equivariance, linearity,
the adjoint identity of every transport and of whole layers, N Hermitian with
<v, N v> = |L v|^2 for the half network computed on its own, the path conventions on a point
source, central finite differences of the loss (an even quartic polynomial in each single
weight, so the differences agree to O(h^2)), the closed-form first Adam step, and flexible CG's
two limits (identity and exact inverse)."""
import numpy as np
import pytest

import oracle
from oracle import network as N
from ksinputs import make_gauge, random_su3, gaussian_source, gaussian_full, GaugeField
from conftest import cvdot, rel_l2
from test_oracle_operator import _gauge_transform


@pytest.fixture(scope="module")
def g6():
    return make_gauge((4, 6, 4, 4), 0.5, 77)


def test_adjoint_identity(g6):
    nb = N.neighbour_tables(g6.dims)
    V = g6.volume
    phi = gaussian_full(V, 1)
    gg = gaussian_full(V, 2)
    for p in range(N.NPATH):
        lhs = cvdot(gg, N.transport(g6.fat, nb, p, phi))
        rhs = cvdot(N.transport_adj(g6.fat, nb, p, gg), phi)
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_path_conventions_point_source(g6):
    """T_{+mu} moves a point source at y to y - mu with V_mu(y - mu) applied; T_{-mu} moves it
    to y + mu with V_mu(y)^+ applied."""
    nb = N.neighbour_tables(g6.dims)
    fwd, bwd = nb
    V = g6.volume
    y = 37
    phi = np.zeros((V, 3), complex)
    phi[y] = [0.2, -1.0j, 0.5]
    for mu in range(4):
        out = N.transport(g6.fat, nb, 1 + mu, phi)
        src = bwd[mu][y]
        assert np.count_nonzero(np.abs(out).sum(1)) == 1
        assert np.allclose(out[src], g6.fat[mu, src] @ phi[y], atol=1e-15)
        out = N.transport(g6.fat, nb, 5 + mu, phi)
        dst = fwd[mu][y]
        assert np.allclose(out[dst], np.conj(g6.fat[mu, y]).T @ phi[y], atol=1e-15)


def test_identity_network_is_identity(g6):
    net = N.Network.identity()
    b = gaussian_source(g6.volume // 2, 4)
    out, _ = N.network_forward(net, g6, b)
    assert np.array_equal(out, b)


def test_linearity(g6):
    net = N.Network.init(5000)
    vh = g6.volume // 2
    b1, b2 = gaussian_source(vh, 5), gaussian_source(vh, 6)
    a = 0.7 - 1.3j
    o1, _ = N.network_forward(net, g6, b1)
    o2, _ = N.network_forward(net, g6, b2)
    o12, _ = N.network_forward(net, g6, a * b1 + b2)
    assert rel_l2(o12, a * o1 + o2) <= 1e-13


def test_gauge_equivariance(g6):
    net = N.Network.init(5000)
    V = g6.volume
    G = random_su3(np.random.default_rng(9), V, 2.0)
    gp = _gauge_transform(g6, G)
    b = gaussian_source(V // 2, 7)
    # gauge matrices of the even sites in checkerboard order
    from ksinputs import lattice_coords
    x, y, z, t = lattice_coords(g6.dims)
    even = np.nonzero(((x + y + z + t) & 1) == 0)[0]
    Gev = G[even]
    out, _ = N.network_forward(net, g6, b)
    outp, _ = N.network_forward(net, gp, np.einsum("vab,vb->va", Gev, b))
    assert rel_l2(outp, np.einsum("vab,vb->va", Gev, out)) <= 1e-13


def test_layer_adjoint_identity(g6):
    """<g, layer(w) phi> = <layer(w')(g), phi> with w' = adjoint_weights(w), channel by channel
    summed, for the 1 -> 8 and 8 -> 8 layers."""
    nb = N.neighbour_tables(g6.dims)
    V = g6.volume
    for w in N.Network.init(5000).weights:
        cout, cin, _ = w.shape
        phi = np.stack([gaussian_full(V, 60 + d) for d in range(cin)])
        gg = np.stack([gaussian_full(V, 70 + c) for c in range(cout)])
        y, _ = N.layer_forward(g6.fat, nb, w, phi)
        ya, _ = N.layer_forward(g6.fat, nb, N.adjoint_weights(w), gg)
        lhs = cvdot(gg, y)
        rhs = cvdot(ya, phi)
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_hermitian_positive(g6):
    """N is Hermitian, and <v, N v> equals |L v|^2 with L v computed by the two free layers
    alone (so Re<N(r), r> > 0 unless L r = 0)."""
    net = N.Network.init(5000)
    vh = g6.volume // 2
    u, v = gaussian_source(vh, 80), gaussian_source(vh, 81)
    Nu, _ = N.network_forward(net, g6, u)
    Nv, _ = N.network_forward(net, g6, v)
    assert abs(cvdot(u, Nv) - np.conj(cvdot(v, Nu))) <= 1e-13 * abs(cvdot(u, Nv))
    Lv = N.half_forward(net, g6, v)
    vNv = cvdot(v, Nv)
    assert abs(vNv.imag) <= 1e-13 * abs(vNv)
    assert abs(vNv.real - np.vdot(Lv.ravel(), Lv.ravel()).real) <= 1e-13 * vNv.real
    assert vNv.real > 0


def test_gradient_central_differences(g6):
    net = N.Network.init(5000)
    vh = g6.volume // 2
    sig = [4 * 0.05 ** 2, 0.3]
    bs = [gaussian_source(vh, 10 + j) for j in range(2)]
    xs = [oracle.cg(g6, s, b, 1e-12)[0] for s, b in zip(sig, bs)]
    loss, grads = N.loss_and_grad(net, g6, sig, bs, xs)
    rng = np.random.default_rng(3)
    h = 1e-4
    for layer in range(2):
        w = net.weights[layer]
        for _ in range(4):
            k = tuple(rng.integers(0, s) for s in w.shape)
            for part, unit in (("re", 1.0), ("im", 1j)):
                saved = w[k]
                w[k] = saved + h * unit
                lp, _ = N.loss_and_grad(net, g6, sig, bs, xs)
                w[k] = saved - h * unit
                lm, _ = N.loss_and_grad(net, g6, sig, bs, xs)
                w[k] = saved
                fd = (lp - lm) / (2 * h)
                an = grads[layer][k].real if part == "re" else grads[layer][k].imag
                assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * abs(loss))


def test_loss_of_exact_pairs():
    """With N = identity the loss is (b - x)^+ A (b - x) / (x^+ A x) by its definition; on a
    free field (unit links times the improvement coefficients) with a plane-wave source b the
    solution is b / lambda: (1 - 1/lambda)^2 lambda |b|^2 over |b|^2 / lambda, i.e.
    (lambda - 1)^2."""
    from test_oracle_operator import free_field, plane_wave
    dims = (4, 6, 4, 8)
    g = free_field(dims, 9.0 / 8.0, -1.0 / 24.0)
    psi, p = plane_wave(dims, (1, 2, 0, 3), np.array([0.3 + 0.1j, -0.7j, 1.1]))
    b = oracle.restrict(dims, 0, psi)
    sigma = 4 * 0.1 ** 2
    s = [9.0 / 8.0 * np.sin(pm) - np.sin(3 * pm) / 24.0 for pm in p]
    lam = sigma + 4 * sum(x * x for x in s)
    x = b / lam
    loss, _ = N.loss_and_grad(N.Network.identity(), g, [sigma], [b], [x])
    assert abs(loss - (lam - 1) ** 2) <= 1e-12 * max(1.0, loss)


def test_adam_first_step_closed_form():
    net = N.Network.init(5000)
    w0 = [w.copy() for w in net.weights]
    grads = [np.full(w.shape, 0.5 - 2.0j) for w in net.weights]
    N.adam_step(net, grads, lr=1e-3)
    # first step: mhat = g, vhat = g^2, so each real moves by -lr * g / (|g| + eps)
    for a, b in zip(net.weights, w0):
        d = a - b
        assert np.allclose(d.real, -1e-3 * 0.5 / (0.5 + 1e-8), rtol=1e-12)
        assert np.allclose(d.imag, -1e-3 * -2.0 / (2.0 + 1e-8), rtol=1e-12)


def test_fcg_identity_equals_cg(g6):
    sigma = 4 * 0.05 ** 2
    b = gaussian_source(g6.volume // 2, 50)
    x, info = oracle.fcg(g6, sigma, b, lambda r: r.copy(), 1e-10)
    xc, ic = oracle.cg(g6, sigma, b, 1e-10)
    assert not info.fallback and info.true_rel_resid <= 1e-10
    assert abs(info.iters - ic.iters) <= 1
    assert rel_l2(x, xc) <= 1e-8


def test_fcg_exact_inverse_one_step(g6):
    sigma = 4 * 0.05 ** 2
    A = oracle.dense_A(g6, sigma)
    Ainv = np.linalg.inv(A)
    b = gaussian_source(g6.volume // 2, 51)
    x, info = oracle.fcg(g6, sigma, b, lambda r: (Ainv @ r.ravel()).reshape(r.shape), 1e-10)
    assert info.iters == 1 and not info.fallback and info.true_rel_resid <= 1e-10


def test_fcg_falls_back_on_bad_preconditioner(g6):
    sigma = 4 * 0.05 ** 2
    b = gaussian_source(g6.volume // 2, 52)
    x, info = oracle.fcg(g6, sigma, b, lambda r: -r, 1e-10)
    assert info.fallback and info.true_rel_resid <= 1e-10
    x, info = oracle.fcg(g6, sigma, b, lambda r: r * np.nan, 1e-10)
    assert info.fallback and info.true_rel_resid <= 1e-10


def test_network_preconditioner_in_fcg(g6):
    """A network preconditioner gives a valid flexible-CG solve."""
    sigma = 4 * 0.05 ** 2
    net = N.Network.init(5000)
    nb = N.neighbour_tables(g6.dims)
    b = gaussian_source(g6.volume // 2, 53)
    x, info = oracle.fcg(g6, sigma, b, lambda r: N.network_forward(net, g6, r, nb)[0], 1e-10)
    assert info.true_rel_resid <= 1e-10
