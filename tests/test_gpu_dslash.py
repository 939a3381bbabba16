"""GPU parity of the gauge load, the Dslash and the normal operator against the FP64 oracle,
through the C ABI.

Element by element: every output component against the oracle applied to the links and
input exactly as the device stores them (FP32 / binary16 rounding, the 12-real Naik copies of
the link access in use), within the rounding bound of the device's own arithmetic and output
(`dslash_check`: 2^-44 S for FP64, 2^-17 S for FP32, 2^-17 S + 2^-11 n for binary16 output,
S the component's sum of product moduli, n the site maximum).

Relative L2 against the plain FP64 oracle (storage rounding included):
* FP64: 1e-12 (the two sides differ only in summation order; expect ~1e-15);
* FP32: 5e-6; FP16 with per-site FP32 norm: 5e-3.
"""
import numpy as np
import pytest

import oracle
from ksinputs import make_gauge, gaussian_source, GaugeField
from conftest import rel_l2
from gpu_util import dev, host, zeros_dev, announce
import dslash_check as dc

pytestmark = pytest.mark.gpu

DIMS = [(4, 4, 4, 4), (6, 4, 8, 4), (8, 8, 8, 8), (8, 6, 10, 12), (12, 12, 12, 12),
        (16, 16, 16, 16)]


@pytest.fixture(scope="module")
def ks():
    import torch
    import paper_1611_00728_amd as ks
    assert torch.cuda.is_available()
    return ks


_cache = {}


def loaded(ks, dims, scale=0.5, seed=3):
    key = (dims, scale, seed)
    if key not in _cache:
        g = make_gauge(dims, scale, seed)
        _cache[key] = (g, ks.Gauge(dims, g.fat, g.naik))
    return _cache[key]


def run_dslash(ks, G, vh, out_par, psi, prec, recon):
    inp = ks.Field(G, 1 - out_par, prec).load(dev(psi))
    out = ks.Field(G, out_par, prec)
    ks.dslash_eo(G, out, inp, recon)
    res = zeros_dev((vh, 3))
    out.store(res)
    import torch
    torch.cuda.synchronize()
    return host(res)


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("recon", [18, 12])
def test_dslash_f64(ks, dims, recon):
    announce("dslash f64", dims, recon)
    g, G = loaded(ks, dims)
    vh = g.volume // 2
    for out_par in (0, 1):
        psi = gaussian_source(vh, 100 + out_par)
        got = run_dslash(ks, G, vh, out_par, psi, ks.F64, recon)
        ref = oracle.dslash_eo(g, out_par, psi)
        assert rel_l2(got, ref) <= 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 8, 4), (12, 12, 12, 12)])
@pytest.mark.parametrize("recon", [18, 12])
def test_dslash_f32(ks, dims, recon):
    announce("dslash f32", dims, recon)
    g, G = loaded(ks, dims)
    vh = g.volume // 2
    for out_par in (0, 1):
        psi = gaussian_source(vh, 200 + out_par)
        got = run_dslash(ks, G, vh, out_par, psi, ks.F32, recon)
        ref, S = dc.reference(g, "f32", recon, 8, out_par, psi)
        assert dc.worst(got, ref, S, "f32") <= 1.0
        assert rel_l2(got, oracle.dslash_eo(g, out_par, psi)) <= 5e-6


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 8, 4), (12, 12, 12, 12)])
@pytest.mark.parametrize("recon", [18, 12])
def test_dslash_f16(ks, dims, recon):
    announce("dslash f16", dims, recon)
    g, G = loaded(ks, dims)
    vh = g.volume // 2
    for out_par in (0, 1):
        psi = gaussian_source(vh, 300 + out_par) * np.geomspace(1e-3, 10, vh)[:, None]
        got = run_dslash(ks, G, vh, out_par, psi, ks.F16, recon)
        ref, S = dc.reference(g, "f16", recon, 8, out_par, psi)
        assert dc.worst(got, ref, S, "f16") <= 1.0
        assert rel_l2(got, oracle.dslash_eo(g, out_par, psi)) <= 5e-3


def test_field_roundtrip_exact(ks):
    """FP64 import/export is the identity; FP32 and FP16 reproduce the oracle's rounding."""
    announce("field roundtrip")
    g, G = loaded(ks, (6, 4, 8, 4))
    vh = g.volume // 2
    v = gaussian_source(vh, 9) * np.geomspace(1e-4, 1e2, vh)[:, None]
    import torch
    # FP16: the decoded value is n * h rounded to binary32 on the device (exact in FP64 here)
    for prec, ref, tol in ((ks.F64, v, 0.0), (ks.F32, oracle.quantise_f32(v), 0.0),
                           (ks.F16, oracle.quantise_f16_sites(v), 2.0 ** -24)):
        f = ks.Field(G, 0, prec).load(dev(v))
        out = zeros_dev((vh, 3))
        f.store(out)
        torch.cuda.synchronize()
        got = host(out)
        if tol == 0.0:
            assert np.array_equal(got, ref)
        else:
            n = np.max(np.abs(np.stack([v.real, v.imag], -1).reshape(vh, 6)), axis=1)
            assert np.all(np.abs(got.real - ref.real) <= tol * n[:, None])
            assert np.all(np.abs(got.imag - ref.imag) <= tol * n[:, None])


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 6, 10, 12), (16, 16, 16, 16)])
def test_apply_A_f64(ks, dims):
    announce("apply_A f64", dims)
    g, G = loaded(ks, dims)
    vh = g.volume // 2
    x = gaussian_source(vh, 400)
    out = zeros_dev((vh, 3))
    for sigma in (4 * 0.1 ** 2, 0.0, 1.7):
        ks.apply_A(G, sigma, dev(x), out)
        import torch
        torch.cuda.synchronize()
        assert rel_l2(host(out), oracle.apply_A(g, sigma, x)) <= 1e-12


def test_recon12_rejects_non_su3(ks):
    """12-real storage of a Naik field that is not c * phase * SU(3) is refused."""
    announce("recon12 reject")
    g = make_gauge((4, 4, 4, 4), 0.5, 5)
    G = ks.Gauge(g.dims, g.fat, g.fat)   # fat links are not SU(3) times a scalar
    with pytest.raises(ks.KSError) as e:
        G.prepare(ks.F64, 12)
    assert e.value.code == -4
    # the 18-real path still works on it
    G.prepare(ks.F64, 18)


def test_dslash_argument_errors(ks):
    announce("dslash argument errors")
    g, G = loaded(ks, (4, 4, 4, 4))
    a = ks.Field(G, 0, ks.F64)
    b = ks.Field(G, 0, ks.F64)
    c = ks.Field(G, 1, ks.F32)
    for out, inp in ((a, b), (a, a), (a, c)):
        with pytest.raises(ks.KSError) as e:
            ks.dslash_eo(G, out, inp)
        assert e.value.code == -1


def form_built(prec, recon, group, way, staged):
    """The launch forms the library builds (the others would spill registers)."""
    if group == 1:
        return True
    if group == 2:
        return prec != "f64" or (recon == 18 and way == 8 and not staged)
    return prec != "f64" and recon == 18


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("recon", [18, 12])
def test_every_launch_configuration(ks, prec, recon):
    """Every built (staged gathers, link access, links per pass, threads per block, LDS cap)
    form of the kernel gives the oracle's result on a ragged lattice, both parities; unbuilt
    forms are refused."""
    announce("dslash launch configurations", prec, recon)
    dims = (8, 6, 10, 12)
    g, G = loaded(ks, dims)
    vh = g.volume // 2
    P = {"f64": ks.F64, "f32": ks.F32, "f16": ks.F16}[prec]
    bound = {"f64": 1e-12, "f32": 5e-6, "f16": 5e-3}[prec]
    psi = [gaussian_source(vh, 500 + p) for p in (0, 1)]
    ref = [oracle.dslash_eo(g, p, psi[p]) for p in (0, 1)]
    # the quantise-then-FP64 reference of each link access (the 12-real Naik copies differ)
    qref = {(way, p): dc.reference(g, prec, recon, way, p, psi[p]) for way in (8, 4)
            for p in (0, 1)}
    try:
        for staged in (0, 1):
            for way in (8, 4):
                for group in (1, 2, 4):
                    for threads in (64, 128, 256):
                        for lds in (0, 40960):
                            if not form_built(prec, recon, group, way, staged):
                                with pytest.raises(ks.KSError) as e:
                                    G.set_config(P, recon, threads, lds, group, way, staged)
                                assert e.value.code == -1
                                continue
                            G.set_config(P, recon, threads, lds, group, way, staged)
                            cfg = G.config(P, recon)
                            assert (cfg["links_per_pass"], cfg["link_access"],
                                    cfg["staged"]) == (group, way, staged)
                            for out_par in (0, 1):
                                got = run_dslash(ks, G, vh, out_par, psi[out_par], P, recon)
                                form = (staged, way, group, threads, lds)
                                assert rel_l2(got, ref[out_par]) <= bound, form
                                r, S = qref[(way, out_par)]
                                assert dc.worst(got, r, S, prec) <= 1.0, form
        with pytest.raises(ks.KSError):
            G.set_config(P, recon, 96, 0, 1)
        with pytest.raises(ks.KSError):
            G.set_config(P, recon, 64, -1, 1)
        with pytest.raises(ks.KSError):
            G.set_config(P, recon, 64, 0, 1, 6)
        with pytest.raises(ks.KSError):
            G.set_config(P, recon, 64, 0, 1, 8, 2)
    finally:
        G.set_config(P, recon, 256, 0, 1, 8, 0)


@pytest.fixture(scope="module")
def lat32(ks):
    dims = (32, 32, 32, 32)
    g = make_gauge(dims, 0.5, 1002)
    G = ks.Gauge(dims, g.fat, g.naik)
    yield g, G, gaussian_source(g.volume // 2, 2002)
    G.free()


def test_dslash_full_size_32_f64(ks, lat32):
    """32^4 (the benchmark lattice), both parities, every site, FP64 against the oracle."""
    announce("dslash 32^4 f64")
    g, G, psi = lat32
    vh = g.volume // 2
    for out_par in (0, 1):
        ref = oracle.dslash_eo(g, out_par, psi)
        assert rel_l2(run_dslash(ks, G, vh, out_par, psi, ks.F64, 18), ref) <= 1e-12
        assert rel_l2(run_dslash(ks, G, vh, out_par, psi, ks.F64, 12), ref) <= 1e-12


@pytest.mark.parametrize("prec", ["f32", "f16"])
@pytest.mark.parametrize("recon", [18, 12])
def test_dslash_full_size_32(ks, lat32, prec, recon):
    """32^4, both parities, every output component of a reduced-precision variant against its
    quantised reference, with the default 8-way access and with 4-way access and staged
    gathers (boundary rows of 32^4 wrap out of the stage)."""
    g, G, psi = lat32
    vh = g.volume // 2
    P = {"f32": ks.F32, "f16": ks.F16}[prec]
    try:
        for out_par in (0, 1):
            for way, staged in ((8, 0), (4, 1)):
                announce("dslash 32^4", prec, recon, way, staged, out_par)
                G.set_config(P, recon, 256, 0, 1, way, staged)
                got = run_dslash(ks, G, vh, out_par, psi, P, recon)
                r, S = dc.reference(g, prec, recon, way, out_par, psi)
                assert dc.worst(got, r, S, prec) <= 1.0, (prec, recon, way)
                del r, S
    finally:
        G.set_config(P, recon, 256, 0, 1, 8, 0)


def test_tune_cache(ks, tmp_path, monkeypatch):
    """KS_TUNE_CACHE: tuning records the variant's configuration in the file; a new handle on
    the same lattice takes an entry from there as written (an edited one included) and its
    Dslash still equals the oracle's; an unusable entry is tuned again and replaced; entries of
    other variants and lines the library cannot read are kept."""
    import json
    announce("tune cache")
    path = tmp_path / "tune.jsonl"
    path.write_text("not an entry\n")
    monkeypatch.setenv("KS_TUNE_CACHE", str(path))
    dims = (8, 8, 8, 8)
    g = make_gauge(dims, 0.5, 3)
    vh = g.volume // 2
    G1 = ks.Gauge(dims, g.fat, g.naik)
    c1 = G1.tune(ks.F64, 18)
    lines = path.read_text().splitlines()
    assert len(lines) == 2 and lines[0] == "not an entry"
    e = json.loads(lines[1])
    assert e["dims"] == list(dims) and e["prec"] == 0 and e["naik"] == 18
    assert [e[k] for k in ("threads", "lds_bytes", "links_per_pass", "link_access", "staged")] == \
        [c1[k] for k in ("threads", "lds_bytes", "links_per_pass", "link_access", "staged")]
    # an entry edited to another built form is taken as written, without timing
    e.update(threads=128, lds_bytes=0, links_per_pass=1, link_access=4, staged=0, us=12.5)
    path.write_text(lines[0] + "\n" + json.dumps(e) + "\n")
    G2 = ks.Gauge(dims, g.fat, g.naik)
    c2 = G2.tune(ks.F64, 18)
    assert (c2["threads"], c2["link_access"], c2["links_per_pass"], c2["staged"]) == (128, 4, 1, 0)
    assert c2["tuned_us"] == pytest.approx(12.5)
    psi = gaussian_source(vh, 808)
    got = run_dslash(ks, G2, vh, 0, psi, ks.F64, 18)
    assert rel_l2(got, oracle.dslash_eo(g, 0, psi)) <= 1e-12
    # an unusable entry (96 threads) is tuned again and replaced
    e.update(threads=96)
    path.write_text(lines[0] + "\n" + json.dumps(e) + "\n")
    G3 = ks.Gauge(dims, g.fat, g.naik)
    c3 = G3.tune(ks.F64, 18)
    assert c3["threads"] in (64, 128, 256)
    lines = path.read_text().splitlines()
    assert len(lines) == 2 and lines[0] == "not an entry"
    assert json.loads(lines[1])["threads"] == c3["threads"]
    # another variant is added beside it
    G3.tune(ks.F32, 18)
    lines = path.read_text().splitlines()
    assert len(lines) == 3 and sorted(json.loads(x)["prec"] for x in lines[1:]) == [0, 1]
    for G in (G1, G2, G3):
        G.free()
