"""Initial weights of the preconditioner network (random draws only).

The free layers of the network's half L have weights w[c_out][c_in][9] (complex): nine
parallel-transport paths, channels 1 -> 8 -> 8.  Entries are CN(0, 1/(9 c_in)) draws
(default_rng(seed), layer by layer, row-major, re before im) plus 1 on the identity path of the
channel diagonal.
"""
import numpy as np

CHANNELS = (1, 8, 8)
NPATH = 9


def net_init_weights(seed: int = 5000, channels=CHANNELS):
    rng = np.random.default_rng(seed)
    ws = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        g = rng.standard_normal((cout, cin, NPATH, 2)) * np.sqrt(0.5 / (NPATH * cin))
        w = g[..., 0] + 1j * g[..., 1]
        for c in range(min(cin, cout)):
            w[c, c, 0] += 1.0
        ws.append(w)
    return ws


def flatten_weights(ws) -> np.ndarray:
    return np.concatenate([np.asarray(w, dtype=np.complex128).ravel() for w in ws])


def unflatten_weights(v, channels=CHANNELS):
    out, o = [], 0
    for cin, cout in zip(channels[:-1], channels[1:]):
        n = cout * cin * NPATH
        out.append(np.asarray(v[o:o + n], dtype=np.complex128).reshape(cout, cin, NPATH))
        o += n
    return out
