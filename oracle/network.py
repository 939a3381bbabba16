"""Gauge-covariant preconditioner network, FP64 reference (test infrastructure).

A layer maps c_in channels of colour-vector fields to c_out channels:

    phi'_c(x) = sum_{c', p} w_{c c' p} (T_p phi_{c'})(x)

over nine parallel-transport paths p: the identity T_0, the forward hops
T_{+mu} phi(x) = V_mu(x) phi(x + mu) (p = 1 + mu) and the backward hops
T_{-mu} phi(x) = V_mu(x - mu)^+ phi(x - mu) (p = 5 + mu), with the fat link V of the operator
(phases folded in), so a gauge transform of V and phi commutes with every layer.

The preconditioner is N = L^+ L with L two free layers (channels 1 -> 8 -> 8) and no
activation: applied as four layers 1 -> 8 -> 8 -> 8 -> 1, the last two being the adjoints of
the first two.  The adjoint of a layer, y -> sum_p T_p^+ W_p^H y, is again a layer, with the
channels swapped and the weights w'_{c' c pbar} = conj(w_{c c' p}) (pbar the reversed path,
T_{+mu}^+ = T_{-mu}).  So N is Hermitian and <v, N v> = |L v|^2 >= 0: the flexible CG's descent
condition Re<N(r), r> > 0 holds for every residual L does not annihilate.  The input is the
even-site residual embedded in the full lattice (odd sites zero), the output the even sites of
the last layer.

Loss over pairs (b_j, x_j) with A_j x_j = b_j: the A-norm error relative to the solution's,
    L = (1/B) sum_j (N b_j - x_j)^+ A_j (N b_j - x_j) / (x_j^+ A_j x_j),
the quantity CG minimises over its Krylov space (it weights a mode of A by its eigenvalue, so
the low modes, which set the iteration count, count as much as the A-norm lets them).

Gradients are packed as G = dL/dRe + i dL/dIm.  For y = w u this gives G_w = conj(u) G_y and
G_u = conj(w) G_y; through a linear map M, G_u = M^+ G_y.  A weight that appears both in a
layer and (conjugated) in its adjoint collects G from the first use plus the conjugate of G
from the second.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .core import embed, restrict

CHANNELS = (1, 8, 8)            # the free half L; N applies 1 -> 8 -> 8 -> 8 -> 1
NPATH = 9
PATHS = [("id", -1)] + [("fwd", mu) for mu in range(4)] + [("bwd", mu) for mu in range(4)]


def neighbour_tables(dims):
    """fwd[mu][i] = index of i + mu_hat, bwd[mu][i] = index of i - mu_hat (periodic)."""
    nx, ny, nz, nt = (int(d) for d in dims)
    V = nx * ny * nz * nt
    i = np.arange(V, dtype=np.int64)
    c = [i % nx, (i // nx) % ny, (i // (nx * ny)) % nz, i // (nx * ny * nz)]
    n = [nx, ny, nz, nt]

    def idx(cc):
        return cc[0] + nx * (cc[1] + ny * (cc[2] + nz * cc[3]))

    fwd, bwd = [], []
    for mu in range(4):
        cf = list(c)
        cf[mu] = (c[mu] + 1) % n[mu]
        cb = list(c)
        cb[mu] = (c[mu] - 1) % n[mu]
        fwd.append(idx(cf))
        bwd.append(idx(cb))
    return fwd, bwd


def transport(fat, nb, p: int, phi: np.ndarray) -> np.ndarray:
    """(T_p phi)(x) for phi complex [V][3]."""
    fwd, bwd = nb
    kind, mu = PATHS[p]
    if kind == "id":
        return phi.copy()
    if kind == "fwd":
        return np.einsum("vab,vb->va", fat[mu], phi[fwd[mu]])
    return np.einsum("vba,vb->va", np.conj(fat[mu][bwd[mu]]), phi[bwd[mu]])


def transport_adj(fat, nb, p: int, g: np.ndarray) -> np.ndarray:
    """(T_p^+ g)(x): the identity is self-adjoint and T_{+mu}^+ = T_{-mu}."""
    kind, mu = PATHS[p]
    if kind == "id":
        return g.copy()
    return transport(fat, nb, (5 + mu) if kind == "fwd" else (1 + mu), g)


def layer_forward(fat, nb, w: np.ndarray, phi: np.ndarray):
    """phi complex [c_in][V][3] -> (y [c_out][V][3], T phi [c_in][9][V][3])."""
    tphi = np.stack([np.stack([transport(fat, nb, p, phi[d]) for p in range(NPATH)])
                     for d in range(phi.shape[0])])
    y = np.einsum("cdp,dpvk->cvk", w, tphi)
    return y, tphi


def layer_backward(fat, nb, w: np.ndarray, tphi: np.ndarray, gy: np.ndarray):
    """Given G_y [c_out][V][3]: (G_w [c_out][c_in][9], G_phi [c_in][V][3])."""
    gw = np.einsum("dpvk,cvk->cdp", np.conj(tphi), gy)
    gt = np.einsum("cdp,cvk->dpvk", np.conj(w), gy)
    gphi = np.stack([sum(transport_adj(fat, nb, p, gt[d, p]) for p in range(NPATH))
                     for d in range(gt.shape[0])])
    return gw, gphi


def adjoint_weights(w: np.ndarray) -> np.ndarray:
    """Weights of the adjoint layer: w'[c'][c][pbar] = conj(w[c][c'][p])."""
    cout, cin, _ = w.shape
    wa = np.zeros((cin, cout, NPATH), dtype=np.complex128)
    for p in range(NPATH):
        kind, mu = PATHS[p]
        pb = p if kind == "id" else (5 + mu if kind == "fwd" else 1 + mu)
        wa[:, :, pb] = np.conj(w[:, :, p]).T
    return wa


@dataclass
class Network:
    weights: list                      # the free layers of L: complex128 [c_out][c_in][9]
    adam_m: list = field(default_factory=list)
    adam_v: list = field(default_factory=list)
    step: int = 0

    @staticmethod
    def init(seed: int = 5000) -> "Network":
        """The seeded initial weights of L (drawn by the input module)."""
        from ksinputs import net_init_weights
        return Network([w.copy() for w in net_init_weights(seed)])

    @staticmethod
    def identity() -> "Network":
        """L copies the input into channel 0, so N = L^+ L is the identity."""
        ws = []
        for cin, cout in zip(CHANNELS[:-1], CHANNELS[1:]):
            w = np.zeros((cout, cin, NPATH), dtype=np.complex128)
            w[0, 0, 0] = 1.0
            ws.append(w)
        return Network(ws)

    def layers(self) -> list:
        """The four applied layers: L's two, then their adjoints in reverse order."""
        w1, w2 = self.weights
        return [w1, w2, adjoint_weights(w2), adjoint_weights(w1)]

    def flat(self) -> np.ndarray:
        return np.concatenate([w.ravel() for w in self.weights])

    def set_flat(self, v: np.ndarray) -> None:
        o = 0
        for k, w in enumerate(self.weights):
            self.weights[k] = np.asarray(v[o:o + w.size]).reshape(w.shape).astype(np.complex128)
            o += w.size


def half_forward(net: Network, g, r_e: np.ndarray, nb=None) -> np.ndarray:
    """L r_e: the eight channels on the full lattice, [8][V][3]."""
    nb = nb if nb is not None else neighbour_tables(g.dims)
    phi = embed(g.dims, 0, r_e)[None]
    for w in net.weights:
        phi, _ = layer_forward(g.fat, nb, w, phi)
    return phi


def network_forward(net: Network, g, r_e: np.ndarray, nb=None, keep_cache: bool = True):
    """N(r_e) on even sites, plus the cache of transported activations per applied layer
    (an empty list when keep_cache is False, which keeps large lattices within memory)."""
    nb = nb if nb is not None else neighbour_tables(g.dims)
    phi = embed(g.dims, 0, r_e)[None]
    cache = []
    for w in net.layers():
        phi, tphi = layer_forward(g.fat, nb, w, phi)
        if keep_cache:
            cache.append(tphi)
        del tphi
    return restrict(g.dims, 0, phi[0]), cache


def tied_gradients(grads4) -> list:
    """Gradients of the two free layers from those of the four applied layers."""
    return [grads4[0] + adjoint_weights(grads4[3]), grads4[1] + adjoint_weights(grads4[2])]


def loss_and_grad(net: Network, g, sigmas, bs, xs, nb=None):
    """The A-norm loss over the pairs on lattice g (shift sigmas[j] of A for pair j) and its
    gradient G_w for both free layers."""
    from .core import apply_A
    nb = nb if nb is not None else neighbour_tables(g.dims)
    B = len(bs)
    loss = 0.0
    layers = net.layers()
    grads4 = [np.zeros_like(w) for w in layers]
    for sigma, b, x in zip(sigmas, bs, xs):
        out, cache = network_forward(net, g, b, nb)
        Ad = apply_A(g, sigma, out - x)
        xAx = float(np.vdot(x, apply_A(g, sigma, x)).real)
        loss += float(np.vdot(out - x, Ad).real) / xAx / B
        gy = embed(g.dims, 0, 2.0 * Ad / (xAx * B))[None]
        for layer in range(len(layers) - 1, -1, -1):
            gw, gy = layer_backward(g.fat, nb, layers[layer], cache[layer], gy)
            grads4[layer] += gw
    return loss, tied_gradients(grads4)


def adam_step(net: Network, grads, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8) -> None:
    """One Adam step on the real and imaginary parts of every weight separately."""
    if not net.adam_m:
        net.adam_m = [np.zeros(w.shape + (2,)) for w in net.weights]
        net.adam_v = [np.zeros(w.shape + (2,)) for w in net.weights]
    net.step += 1
    t = net.step
    for k, (w, gw) in enumerate(zip(net.weights, grads)):
        gr = np.stack([gw.real, gw.imag], axis=-1)
        net.adam_m[k] = b1 * net.adam_m[k] + (1 - b1) * gr
        net.adam_v[k] = b2 * net.adam_v[k] + (1 - b2) * gr * gr
        mhat = net.adam_m[k] / (1 - b1 ** t)
        vhat = net.adam_v[k] / (1 - b2 ** t)
        upd = lr * mhat / (np.sqrt(vhat) + eps)
        net.weights[k] = w - (upd[..., 0] + 1j * upd[..., 1])
