"""GPU CG and multi-shift CG through the C ABI, judged by the FP64 oracle on the CPU:

* the true relative residual |b - A x| / |b| of the returned x, recomputed by the oracle's
  operator, must be <= the requested tolerance;
* the solution must agree with the oracle's own CG solution within 2 tol kappa, kappa taken
  from the oracle's Lanczos estimate (a solution with residual <= tol is within tol kappa of
  the exact one, for both sides).
"""
import numpy as np
import pytest

import oracle
from ksinputs import make_gauge, gaussian_source, SEEDS
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
def cfg1(ks):
    """8^4, s = 0.3, m = 0.1: the small plain-FP64 workload."""
    g = make_gauge((8, 8, 8, 8), 0.3, SEEDS["gauge"](1))
    b = gaussian_source(g.volume // 2, SEEDS["source"](1))
    x, info = oracle.cg(g, 4 * 0.1 ** 2, b, 1e-12)
    lo, hi = oracle.lanczos_extremes(info.alpha, info.beta)
    return g, ks.Gauge(g.dims, g.fat, g.naik), b, x, hi / lo


def true_rel(g, sigma, b, x):
    return float(np.linalg.norm(b - oracle.apply_A(g, sigma, x)) / np.linalg.norm(b))


def solve(ks, G, mass, b, x0=None, **kw):
    import torch
    xd = zeros_dev(b.shape) if x0 is None else dev(x0)
    res = ks.cg_solve(G, mass, dev(b), xd, ks.default_params(**kw), raise_on_error=False)
    torch.cuda.synchronize()
    return host(xd), res


@pytest.mark.parametrize("inner,recon", [("f64", 18), ("f64", 12), ("f32", 18), ("f32", 12),
                                         ("f16", 18), ("f16", 12)])
def test_cg_config1(ks, cfg1, inner, recon):
    announce("cg 8^4", inner, recon)
    g, G, b, xo, kappa = cfg1
    x, res = solve(ks, G, 0.1, b, tol=1e-10, inner=inner, recon=recon, check_every=8)
    assert res.ok, res
    tr = true_rel(g, 0.04, b, x)
    assert tr <= 1e-10
    assert abs(res.stats["true_rel_resid"] - tr) <= 1e-3 * tr + 1e-15
    assert rel_l2(x, xo) <= 2 * 1e-10 * kappa
    if inner != "f64":
        assert res.stats["reliable_updates"] >= 1


def test_cg_f64_iterations_match_oracle(ks, cfg1):
    """FP64 GPU CG takes the oracle's iteration count (rounding order aside)."""
    g, G, b, _, _ = cfg1
    announce("cg iteration count")
    _, info = oracle.cg(g, 0.04, b, 1e-10)
    x, res = solve(ks, G, 0.1, b, tol=1e-10, check_every=1)
    assert abs(res.stats["iters"] - info.iters) <= 1


def test_cg_coefficients_match_oracle(ks, cfg1):
    """The FP64 run's recorded alpha_k, beta_k are the oracle CG's (the two differ only in
    summation order), so their Lanczos extremes agree; a reduced-precision run marks the
    steps that ended in a reliable update with beta = NaN."""
    g, G, b, _, _ = cfg1
    announce("cg coefficients")
    _, info = oracle.cg(g, 0.04, b, 1e-10)
    x, res = solve(ks, G, 0.1, b, tol=1e-10, check_every=4)
    alpha, beta = G.cg_coefficients()
    assert len(alpha) == res.stats["iters"]
    k = min(len(alpha), len(info.alpha)) - 1
    assert np.allclose(alpha[:20], info.alpha[:20], rtol=1e-10, atol=0)
    assert np.allclose(beta[:20], info.beta[:20], rtol=1e-10, atol=0)
    lo, hi = oracle.lanczos_extremes(alpha[:k], beta[:k])
    lo_o, hi_o = oracle.lanczos_extremes(info.alpha[:k], info.beta[:k])
    assert abs(lo - lo_o) <= 1e-6 * lo_o and abs(hi - hi_o) <= 1e-6 * hi_o
    assert 0.04 * (1 - 1e-9) <= lo < hi
    x, res = solve(ks, G, 0.1, b, tol=1e-10, inner="f32", check_every=4)
    alpha, beta = G.cg_coefficients()
    assert len(alpha) == res.stats["iters"]
    assert np.all(np.isfinite(alpha))
    assert np.isnan(beta).sum() == res.stats["reliable_updates"] + res.stats["restarts"] + 1


def test_cg_initial_guess(ks, cfg1):
    g, G, b, xo, _ = cfg1
    announce("cg initial guess")
    x, res = solve(ks, G, 0.1, b, x0=xo, tol=1e-10)
    assert res.ok and res.stats["iters"] <= 2
    x, res = solve(ks, G, 0.1, b, x0=0.5 * xo, tol=1e-10)
    assert res.ok and true_rel(g, 0.04, b, x) <= 1e-10


def test_cg_zero_source(ks, cfg1):
    g, G, b, _, _ = cfg1
    announce("cg zero source")
    x, res = solve(ks, G, 0.1, np.zeros_like(b), x0=b)
    assert res.ok and np.all(x == 0)


@pytest.mark.parametrize("inner", ["f64", "f32", "f16"])
def test_cg_not_converged(ks, cfg1, inner):
    """At max_iter the solver returns the last iterate (in reduced precision with its FP32
    increments added in) and that iterate's own true residual."""
    g, G, b, _, _ = cfg1
    announce("cg max_iter", inner)
    x, res = solve(ks, G, 0.1, b, tol=1e-10, max_iter=5, check_every=2, inner=inner)
    assert res.status == -5
    assert res.stats["iters"] == 5
    tr = true_rel(g, 0.04, b, x)
    assert 1e-6 < tr < 1.0
    assert abs(res.stats["true_rel_resid"] - tr) <= 1e-6


def test_cg_nonfinite_source(ks, cfg1):
    g, G, b, _, _ = cfg1
    announce("cg nonfinite")
    bad = b.copy()
    bad[3, 1] = np.nan
    x, res = solve(ks, G, 0.1, bad, tol=1e-10)
    assert res.status == -7


@pytest.mark.parametrize("dims", [(6, 4, 8, 4), (12, 12, 12, 12)])
def test_cg_ragged_lattices(ks, dims):
    announce("cg ragged", dims)
    g = make_gauge(dims, 0.5, 31)
    G = ks.Gauge(dims, g.fat, g.naik)
    b = gaussian_source(g.volume // 2, 32)
    for inner in ("f64", "f32", "f16"):
        x, res = solve(ks, G, 0.05, b, tol=1e-10, inner=inner, recon=12)
        assert res.ok and true_rel(g, 0.01, b, x) <= 1e-10


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_cg_16_agrees_with_oracle_solution(ks, inner):
    """16^4, m = 0.01: the solution agrees with the oracle's own CG solution within
    2 tol kappa (kappa from the oracle's Lanczos estimate)."""
    announce("cg 16^4 vs oracle solution", inner)
    g = make_gauge((16, 16, 16, 16), 0.5, 51)
    G = ks.Gauge(g.dims, g.fat, g.naik)
    b = gaussian_source(g.volume // 2, 52)
    xo, info = oracle.cg(g, 4 * 0.01 ** 2, b, 1e-12)
    lo, hi = oracle.lanczos_extremes(info.alpha, info.beta)
    x, res = solve(ks, G, 0.01, b, tol=1e-10, inner=inner)
    assert res.ok and true_rel(g, 4e-4, b, x) <= 1e-10
    assert rel_l2(x, xo) <= 2 * (1e-10 + 1e-12) * hi / lo


@pytest.mark.parametrize("inner,recon", [("f64", 18), ("f32", 18), ("f16", 12)])
def test_cg_runs_are_bit_identical(ks, inner, recon):
    """Every reduction has a fixed order (in the fused step kernels every block re-adds the
    partials in the same order), so two runs return the same x bit for bit: a cheap check for
    races.  12^4 spans several hundred blocks per launch."""
    announce("cg repeatability", inner, recon)
    g = make_gauge((12, 12, 12, 12), 0.5, 61)
    G = ks.Gauge(g.dims, g.fat, g.naik)
    b = gaussian_source(g.volume // 2, 62)
    x1, r1 = solve(ks, G, 0.05, b, tol=1e-10, inner=inner, recon=recon, check_every=3)
    x2, r2 = solve(ks, G, 0.05, b, tol=1e-10, inner=inner, recon=recon, check_every=7)
    assert r1.ok and r2.ok
    assert r1.stats["iters"] == r2.stats["iters"]
    assert r1.stats["reliable_updates"] == r2.stats["reliable_updates"]
    assert np.array_equal(x1, x2)


def test_multishift_runs_are_bit_identical(ks, cfg1):
    announce("multishift repeatability")
    g, G, b, _, _ = cfg1
    sig = 4 * np.geomspace(0.002, 0.5, 9) ** 2
    out = []
    for _ in range(2):
        xs = [zeros_dev(b.shape) for _ in sig]
        rc, stats = ks.multishift_cg_solve(G, sig, dev(b), xs, 1e-9,
                                           ks.default_params(inner=ks.F32, check_every=4))
        assert rc == 0
        out.append(([host(x) for x in xs], [st["iters"] for st in stats]))
    assert out[0][1] == out[1][1]
    for a, c in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, c)


@pytest.mark.parametrize("inner", ["f64", "f32", "f16"])
def test_multishift(ks, cfg1, inner):
    announce("multishift 8^4", inner)
    g, G, b, _, _ = cfg1
    masses = np.geomspace(0.002, 0.5, 9)
    sig = 4 * masses ** 2
    xs = [zeros_dev(b.shape) for _ in sig]
    rc, stats = ks.multishift_cg_solve(G, sig, dev(b), xs, 1e-9,
                                       ks.default_params(inner=ks.PREC[inner], check_every=4),
                                       raise_on_error=False)
    assert rc == 0
    if inner != "f64":
        # the base residual is recomputed in FP64 during the shared iteration
        assert stats[0]["reliable_updates"] >= 1
        # several shifts need refinement after the reduced-precision phase: they are refined
        # together by the batched CG (one right-hand side per shift)
        assert sum(1 for st in stats if st["restarts"]) >= 2
    xo, _, _, st = oracle.multishift_cg(g, sig, b, 1e-11)
    for i, s in enumerate(sig):
        x = host(xs[i])
        tr = true_rel(g, s, b, x)
        assert tr <= 1e-9, (i, tr)
        assert abs(stats[i]["true_rel_resid"] - tr) <= 1e-3 * tr + 1e-15
        # -D_eo D_oe is positive semi-definite with norm below 16, so kappa_i <= (16 + s) / s
        assert rel_l2(x, xo[i]) <= 2e-9 * (16.0 + s) / s


def test_multishift_loose_base_tolerance(ks, cfg1):
    """The base (smallest) shift may reach a looser tolerance first: its solution keeps being
    updated while the heavier shifts iterate, so the base reliable updates stay consistent and
    the shared iteration takes about the steps of the uniform-tolerance run; every x_i is
    judged by the oracle against its own tolerance."""
    announce("multishift loose base tolerance")
    g, G, b, _, _ = cfg1
    sig = 4 * np.geomspace(0.002, 0.5, 9) ** 2
    shared = {}
    for name, tols in (("uniform", [1e-10] * 9), ("loose", [1e-6] + [1e-10] * 8)):
        xs = [zeros_dev(b.shape) for _ in sig]
        rc, stats = ks.multishift_cg_solve(G, sig, dev(b), xs, tols,
                                           ks.default_params(inner=ks.F32, check_every=4),
                                           raise_on_error=False)
        assert rc == 0, name
        shared[name] = min(st["iters"] for st in stats)
        for i, s in enumerate(sig):
            assert true_rel(g, s, b, host(xs[i])) <= tols[i], (name, i)
    # the heavier shifts converge before the base would reach 1e-10: the loose run stops
    # earlier, never later
    assert shared["loose"] <= shared["uniform"] + 4, shared


@pytest.mark.parametrize("delta", [0.03, 0.01, 0.003])
def test_multishift_f16_small_delta(ks, delta):
    """FP16 shared iterations with rare reliable updates: whether or not the binary16
    recursion breaks down, the solve succeeds (a broken-down shared phase falls back to the
    last reliable update and refines every shift); each x_i judged by the oracle."""
    announce("multishift f16 delta", delta)
    dims = (16, 16, 16, 16)
    g = make_gauge(dims, 0.5, 1003)
    G = ks.Gauge(dims, g.fat, g.naik)
    b = gaussian_source(g.volume // 2, 2003)
    sig = 4 * np.geomspace(0.002, 0.5, 9) ** 2
    xs = [zeros_dev(b.shape) for _ in sig]
    rc, stats = ks.multishift_cg_solve(G, sig, dev(b), xs, 1e-9,
                                       ks.default_params(inner=ks.F16, check_every=8, delta=delta),
                                       raise_on_error=False)
    assert rc == 0
    for i, s in enumerate(sig):
        assert true_rel(g, s, b, host(xs[i])) <= 1e-9, i
    G.free()


def test_multishift_single_shift_equals_cg(ks, cfg1):
    announce("multishift one shift")
    g, G, b, _, _ = cfg1
    xs = [zeros_dev(b.shape)]
    rc, stats = ks.multishift_cg_solve(G, [0.04], dev(b), xs, 1e-10)
    x, res = solve(ks, G, 0.1, b, tol=1e-10)
    assert rc == 0 and abs(stats[0]["iters"] - res.stats["iters"]) <= 1
    assert rel_l2(host(xs[0]), x) <= 1e-8


def test_multishift_argument_errors(ks, cfg1):
    g, G, b, _, _ = cfg1
    announce("multishift args")
    with pytest.raises(ks.KSError):
        ks.multishift_cg_solve(G, [-1.0], dev(b), [zeros_dev(b.shape)], 1e-9)
    with pytest.raises(ks.KSError):
        ks.multishift_cg_solve(G, [0.1] * 33, dev(b), [zeros_dev(b.shape)] * 33, 1e-9)


def test_tuned_launches_keep_results(ks):
    """After autotuning every Dslash variant (other block sizes, LDS caps, partial counts),
    the Dslash and the solvers give the same answers."""
    announce("autotuned launches")
    dims = (12, 12, 12, 12)
    g = make_gauge(dims, 0.5, 41)
    G = ks.Gauge(dims, g.fat, g.naik)
    vh = g.volume // 2
    b = gaussian_source(vh, 42)
    for p in (ks.F64, ks.F32, ks.F16):
        for r in (18, 12):
            cfg = G.tune(p, r)
            assert cfg["threads"] in (64, 128, 256) and cfg["tuned_us"] > 0
    import torch
    inp = ks.Field(G, 1, ks.F64).load(dev(b))
    out = ks.Field(G, 0, ks.F64)
    ks.dslash_eo(G, out, inp)
    res = zeros_dev((vh, 3))
    out.store(res)
    torch.cuda.synchronize()
    assert rel_l2(host(res), oracle.dslash_eo(g, 0, b)) <= 1e-12
    for inner in ("f64", "f32", "f16"):
        x, r = solve(ks, G, 0.05, b, tol=1e-10, inner=inner, recon=12)
        assert r.ok and true_rel(g, 0.01, b, x) <= 1e-10


@pytest.mark.parametrize("inner,recon", [("f64", 18), ("f32", 18), ("f16", 12)])
@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 8, 4)])
def test_full_solve(ks, dims, inner, recon):
    """M x = b on both parities (M = 2m + D): the oracle's FP64 |b - M x| / |b| of the returned
    x is within tol, the reported residual matches it, and x agrees with the oracle's own full
    solve within 2 tol cond(M).  D is anti-Hermitian, so M is normal with singular values
    |2m + i lambda|: cond(M) = sqrt(lambda_max(A)) / (2m), A = 4m^2 - D_eo D_oe, lambda_max(A)
    from the oracle's Lanczos estimate."""
    announce("full solve", dims, inner, recon)
    import torch
    g = make_gauge(dims, 0.3, 61)
    G = ks.Gauge(dims, g.fat, g.naik)
    vh = g.volume // 2
    m, tol = 0.1, 1e-10
    b_e, b_o = gaussian_source(vh, 62), gaussian_source(vh, 63)
    xe, xo = zeros_dev((vh, 3)), zeros_dev((vh, 3))
    res = ks.full_solve(G, m, dev(b_e), dev(b_o), xe, xo,
                        ks.default_params(tol=tol, inner=ks.PREC[inner], recon=recon))
    torch.cuda.synchronize()
    assert res.ok
    he, ho = host(xe), host(xo)
    me, mo = oracle.apply_M(g, m, he, ho)
    nb = np.sqrt(np.linalg.norm(b_e) ** 2 + np.linalg.norm(b_o) ** 2)
    tr = np.sqrt(np.linalg.norm(b_e - me) ** 2 + np.linalg.norm(b_o - mo) ** 2) / nb
    assert tr <= tol
    assert abs(res.stats["true_rel_resid"] - tr) <= 1e-3 * tr + 1e-15
    oe, oo, _ = oracle.full_solve(g, m, b_e, b_o, 1e-12)
    _, info = oracle.cg(g, 4 * m * m, b_e, 1e-10)
    _, hi = oracle.lanczos_extremes(info.alpha, info.beta)
    cond = np.sqrt(1.01 * hi) / (2 * m)
    x = np.concatenate([he, ho])
    xo_ = np.concatenate([oe, oo])
    assert rel_l2(x, xo_) <= 2 * tol * cond


def test_full_solve_special_cases(ks, cfg1):
    """b_o = 0 gives x_e = 2m A^-1 b_e (the even-odd CG's solution scaled); b = 0 gives x = 0;
    a non-positive mass is refused."""
    announce("full solve special cases")
    import torch
    g, G, b, xo, kappa = cfg1
    m = 0.1
    z = np.zeros_like(b)
    xe, xod = zeros_dev(b.shape), zeros_dev(b.shape)
    res = ks.full_solve(G, m, dev(b), dev(z), xe, xod, ks.default_params(tol=1e-11))
    torch.cuda.synchronize()
    assert res.ok
    assert rel_l2(host(xe), 2 * m * xo) <= 2 * (1e-11 + 1e-12) * kappa
    res = ks.full_solve(G, m, dev(z), dev(z), xe, xod, ks.default_params(tol=1e-11))
    torch.cuda.synchronize()
    assert res.ok and np.all(host(xe) == 0) and np.all(host(xod) == 0)
    with pytest.raises(ks.KSError) as e:
        ks.full_solve(G, 0.0, dev(b), dev(z), xe, xod)
    assert e.value.code == -1


def test_ks_log_solve_summary(ks):
    """KS_LOG = 1: a tuning prints its result and a solve one summary line with its status,
    steps and FP64 residual (in a child process, whose environment sets the level)."""
    import os
    import subprocess
    import sys
    announce("KS_LOG solve summary")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import torch, paper_1611_00728_amd as ks\n"
            "from ksinputs import make_gauge, gaussian_source\n"
            "g = make_gauge((4, 4, 4, 8), 0.5, 5)\n"
            "G = ks.Gauge(g.dims, g.fat, g.naik)\n"
            "G.tune(ks.F32, 18)\n"
            "b = torch.from_numpy(gaussian_source(g.volume // 2, 6)).cuda()\n"
            "x = torch.zeros_like(b)\n"
            "r = ks.cg_solve(G, 0.1, b, x, ks.default_params(tol=1e-10, inner=ks.F32))\n"
            "print('iters', r.stats['iters'])\n") % root
    env = dict(os.environ, KS_LOG="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=110)
    assert out.returncode == 0, out.stderr[-2000:]
    iters = int(out.stdout.split("iters")[1])
    assert "[ks] tuned FP32 18-real Dslash at 4x4x4x8:" in out.stderr
    line = [l for l in out.stderr.splitlines() if l.startswith("[ks] cg: ")]
    assert len(line) == 1 and line[0].startswith("[ks] cg: status 0, %d steps," % iters)
