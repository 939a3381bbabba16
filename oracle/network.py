"""Gauge-covariant preconditioner network, FP64 reference (test infrastructure).

Layer l maps c_in channels of colour-vector fields to c_out channels:

    phi'_c(x) = sum_{c', p} w_{c c' p} (T_p phi_{c'})(x)

over nine parallel-transport paths p: the identity T_0, the forward hops
T_{+mu} phi(x) = V_mu(x) phi(x + mu) (p = 1 + mu) and the backward hops
T_{-mu} phi(x) = V_mu(x - mu)^+ phi(x - mu) (p = 5 + mu), with the fat link V of the operator
(phases folded in), so a gauge transform of V and phi commutes with every layer.  Four layers
with channels 1 -> 8 -> 8 -> 8 -> 1 and no activation; the input is the even-site residual
embedded in the full lattice (odd sites zero) and the output the even sites of the last layer.

Loss over pairs (b_j, x_j): L = (1/B) sum_j |N(b_j) - x_j|^2 / |x_j|^2.

Gradients are packed as G = dL/dRe + i dL/dIm.  For y = w u this gives G_w = conj(u) G_y and
G_u = conj(w) G_y; through a linear map M, G_u = M^+ G_y, and T_{+mu}^+ = T_{-mu}.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .core import embed, restrict

CHANNELS = (1, 8, 8, 8, 1)
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


@dataclass
class Network:
    weights: list                      # complex128 [c_out][c_in][9] per layer
    adam_m: list = field(default_factory=list)
    adam_v: list = field(default_factory=list)
    step: int = 0

    @staticmethod
    def init(seed: int = 5000) -> "Network":
        """The seeded initial weights (drawn by the input module)."""
        from ksinputs import net_init_weights
        return Network([w.copy() for w in net_init_weights(seed)])

    @staticmethod
    def identity(channels=CHANNELS) -> "Network":
        ws = []
        for cin, cout in zip(channels[:-1], channels[1:]):
            w = np.zeros((cout, cin, NPATH), dtype=np.complex128)
            for c in range(min(cin, cout)):
                w[c, c, 0] = 1.0
            ws.append(w)
        return Network(ws)

    def flat(self) -> np.ndarray:
        return np.concatenate([w.ravel() for w in self.weights])

    def set_flat(self, v: np.ndarray) -> None:
        o = 0
        for k, w in enumerate(self.weights):
            self.weights[k] = np.asarray(v[o:o + w.size]).reshape(w.shape).astype(np.complex128)
            o += w.size


def network_forward(net: Network, g, r_e: np.ndarray, nb=None):
    """N(r_e) on even sites, plus the cache of transported activations per layer."""
    nb = nb if nb is not None else neighbour_tables(g.dims)
    phi = embed(g.dims, 0, r_e)[None]
    cache = []
    for w in net.weights:
        phi, tphi = layer_forward(g.fat, nb, w, phi)
        cache.append(tphi)
    return restrict(g.dims, 0, phi[0]), cache


def loss_and_grad(net: Network, g, bs, xs, nb=None):
    """Loss over the pairs and its gradient G_w for every layer."""
    nb = nb if nb is not None else neighbour_tables(g.dims)
    B = len(bs)
    loss = 0.0
    grads = [np.zeros_like(w) for w in net.weights]
    for b, x in zip(bs, xs):
        out, cache = network_forward(net, g, b, nb)
        diff = out - x
        nx2 = float(np.vdot(x, x).real)
        loss += float(np.vdot(diff, diff).real) / nx2 / B
        gy = embed(g.dims, 0, 2.0 * diff / (nx2 * B))[None]
        for layer in range(len(net.weights) - 1, -1, -1):
            gw, gy = layer_backward(g.fat, nb, net.weights[layer], cache[layer], gy)
            grads[layer] += gw
    return loss, grads


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
