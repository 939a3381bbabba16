"""The network checkpoint format (host side): a round trip keeps every value bit for bit, and a
file of another format or a truncated one is refused."""
import numpy as np
import pytest

import paper_1611_00728_amd as ks


def state(seed, n=ks.NET_WEIGHTS):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    m = rng.standard_normal(2 * n)
    v = np.abs(rng.standard_normal(2 * n))
    return w, m, v


def test_round_trip(tmp_path):
    w, m, v = state(1)
    p = tmp_path / "a.ckpt"
    ks.write_checkpoint(p, w, m, v, 123)
    w2, m2, v2, step = ks.read_checkpoint(p)
    assert step == 123
    for a, b in ((w, w2), (m, m2), (v, v2)):
        assert a.dtype == b.dtype and np.array_equal(a, b)
    # little-endian layout: magic, count, step, then the weights' reals
    raw = p.read_bytes()
    assert raw[:8] == b"KSNETCK1"
    assert int.from_bytes(raw[8:12], "little") == ks.NET_WEIGHTS
    assert int.from_bytes(raw[12:16], "little") == 123
    assert np.frombuffer(raw[16:24], dtype="<f8")[0] == w[0].real
    assert len(raw) == 16 + 6 * 8 * ks.NET_WEIGHTS


def test_refuses_other_files(tmp_path):
    w, m, v = state(2)
    p = tmp_path / "b.ckpt"
    ks.write_checkpoint(p, w, m, v, 5)
    raw = p.read_bytes()
    (tmp_path / "short").write_bytes(raw[:-8])
    (tmp_path / "magic").write_bytes(b"XXXXXXXX" + raw[8:])
    for name in ("short", "magic"):
        with pytest.raises(ValueError):
            ks.read_checkpoint(tmp_path / name)
    with pytest.raises(ValueError):
        ks.write_checkpoint(tmp_path / "c", w, m[:-1], v, 0)
    with pytest.raises(ValueError):
        ks.write_checkpoint(tmp_path / "d", w, m, v, -1)
