"""Host-side checks of the seeded inputs and of the host logic around the library: training
blocks cut from a larger lattice, the block tiling, the network's initial weights, the
benchmark's byte models."""
import numpy as np
import pytest

import oracle
from ksinputs import (make_gauge, subblock, gaussian_source, net_init_weights, flatten_weights,
                      unflatten_weights, batch_masses)


@pytest.fixture(scope="module")
def big():
    return make_gauge((8, 8, 8, 8), 0.5, 301, keep_thin=True)


def test_whole_lattice_block_is_the_field(big):
    b = subblock(big, (0, 0, 0, 0), big.dims)
    assert np.array_equal(b.fat, big.fat)
    assert np.allclose(b.naik, big.naik, rtol=0, atol=1e-15)


@pytest.mark.parametrize("origin,bdims", [((0, 0, 0, 0), (4, 4, 4, 4)), ((4, 2, 0, 4), (4, 6, 8, 4))])
def test_block_operator_is_a_staggered_operator(big, origin, bdims):
    """The block's D is anti-Hermitian, and its Naik links are SU(3) times the scalar
    -(1/24) times a sign, as rebuilt from the block's own thin links."""
    b = subblock(big, origin, bdims)
    vh = b.volume // 2
    x, y = gaussian_source(vh, 1), gaussian_source(vh, 2)
    lhs = np.vdot(x, oracle.dslash_eo(b, 0, y))
    rhs = -np.conj(np.vdot(y, oracle.dslash_eo(b, 1, x)))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(x) * np.linalg.norm(y) * 10
    # the block's Naik link is c * phase * SU(3): |det| = (1/24)^3
    d = np.abs(np.linalg.det(b.naik.reshape(-1, 3, 3)))
    assert np.allclose(d, (1.0 / 24) ** 3, rtol=1e-12)


def test_block_fat_links_are_the_big_lattices(big):
    """Away from the block's own boundary signs, the block's fat links are the big lattice's
    links at the shifted sites up to the staggered phase, which an even origin leaves unchanged."""
    origin, bdims = (2, 2, 2, 2), (4, 4, 4, 4)
    b = subblock(big, origin, bdims)
    nx, ny, nz, nt = big.dims
    bx, by, bz, bt = bdims
    for site in (0, 5, 37, 200):
        c = [site % bx, (site // bx) % by, (site // (bx * by)) % bz, site // (bx * by * bz)]
        g = [c[0] + origin[0], c[1] + origin[1], c[2] + origin[2], c[3] + origin[3]]
        gi = g[0] + nx * (g[1] + ny * (g[2] + nz * g[3]))
        for mu in range(3):                  # spatial: no time-boundary sign involved
            assert np.allclose(b.fat[mu, site], big.fat[mu, gi], atol=0, rtol=0)


def test_block_origins_tile_the_lattice():
    from paper_1611_00728_amd.learn import block_origins
    o = block_origins((48, 48, 48, 64), (16, 16, 16, 16))
    assert len(o) == 108 and len(set(o)) == 108
    assert all(all(v % 16 == 0 for v in c) for c in o)


def test_network_initial_weights():
    ws = net_init_weights(5000)
    assert [w.shape for w in ws] == [(8, 1, 9), (8, 8, 9)]
    flat = flatten_weights(ws)
    assert flat.shape == (648,)
    back = unflatten_weights(flat)
    assert all(np.array_equal(a, b) for a, b in zip(ws, back))
    # identity diagonal on the 0-path of the square layers, CN(0, 1/(9 c_in)) noise
    w = ws[1]
    noise = w - np.eye(8)[:, :, None] * (np.arange(9) == 0)
    assert abs(np.var(noise) - 1.0 / 72) <= 0.5 / 72


def test_batch_masses_range_and_seed():
    m1, m2 = batch_masses(64, 0.01, 0.2, 4100), batch_masses(64, 0.01, 0.2, 4100)
    assert np.array_equal(m1, m2) and m1.min() >= 0.01 and m1.max() <= 0.2


def test_bench_byte_models():
    import bench
    assert bench.model_bytes_per_site("f64", 18) == 2400
    assert bench.model_bytes_per_site("f64", 12) == 2016
    assert bench.model_bytes_per_site("f32", 18) == 1200
    assert bench.model_bytes_per_site("f16", 12) == 512
    # batch: a lattice runs as long as its slowest right-hand side
    st = [{"iters": 10, "reliable_updates": 1}, {"iters": 12, "reliable_updates": 2}] * 2
    got = bench.batch_model_bytes(st, [100, 200], nrhs=2)
    per_site = 12 * bench.BATCH_STEP_BYTES + 2 * bench.BATCH_RU_BYTES
    want = (100 + 200) * per_site
    assert got == want


def test_parallel_generation_is_bit_identical(monkeypatch):
    """The chunked generation of a large field gives the same bits with a pool of worker
    processes as computed in one process (same draws in the same order, same operations)."""
    import hashlib
    dims = (16, 16, 16, 128)               # four chunks of 2^17 sites
    monkeypatch.setenv("KS_INPUT_WORKERS", "3")
    a = make_gauge(dims, 0.5, 4321, keep_thin=True)
    monkeypatch.setenv("KS_INPUT_WORKERS", "1")
    b = make_gauge(dims, 0.5, 4321, keep_thin=True)
    for x, y in ((a.thin, b.thin), (a.fat, b.fat), (a.naik, b.naik)):
        assert hashlib.sha256(x.tobytes()).digest() == hashlib.sha256(y.tobytes()).digest()
