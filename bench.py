"""Benchmark of the improved-staggered solver on one MI355X.

Workload: the 32^4 lattice (thin-link scale 0.5, gauge seed 1002, source seed 2002, m = 0.01).
One step is one pass of the hot path:
  1. timed bursts of Dslash_eo launches of all six variants (FP64 / FP32 / FP16, 18- and
     12-real Naik; HIP events around every launch, on the stream the library launches on);
  2. the batched solve (64 lattices of 8^4, 12^4, 16^4 x 4 right-hand sides, FP32 + RU, then
     binary16 + RU);
  3. the multi-shift solve on 32^3 x 48 (9 shifts; FP64, FP32 + RU and FP16 + RU, 18-real
     Naik, and FP64 and FP32 with 12-real Naik) and the force from its solutions;
  4. network bursts and the learned flexible CG;
  5. the full-system solve M x = b and the link construction from thin links;
  6. the plain FP64 GPU CG and the mixed-precision CG solves (FP32 inner with 18- and 12-real
     Naik, FP16 inner with 12-real Naik) to FP64 true relative residual 1e-10.
After the timed steps, once: every returned solution's residual recomputed by the FP64 oracle
on the host (and the 32^4 FP64 solution's distance to the oracle's own CG solution, which a
host thread computes while the GPU runs), and the 48^3 x 64, m = 0.002 learned-preconditioner
workload (training pairs, training, FP64 / mixed / learned solves).
`value` is the FP64 Dslash_eo's algorithmic HBM bandwidth (least-data model: 2400 bytes per
output site) averaged over every launch of the timed steps; the other rows report their own
figures in the same JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload default|learned48|sweep]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DIMS = (32, 32, 32, 32)
MASS = 0.01
TOL = 1e-10
BURST = 50


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def model_bytes_per_site(prec: str, recon: int) -> int:
    real = {"f64": 8, "f32": 4, "f16": 2}[prec]
    spinor = {"f64": 48, "f32": 24, "f16": 16}[prec]
    links = (8 * 18 + 8 * 12) * real if recon == 12 else 16 * 18 * real
    return links + 2 * spinor


# one batched CG step for 4 right-hand sides, FP32 vectors and links, FP64 x, per even site:
# two multi-RHS hopping terms (links 1152 + 4 x 24 in + 4 x 24 out, the second also reading
# 4 x 24 of p), the x/r update (p, q, r read, r written: 4 x 4 x 24; x's FP32 increments read
# and written: 2 x 4 x 24) and p = r + beta p (3 x 4 x 24)
BATCH_STEP_BYTES = 1344 + 1440 + 576 + 288
# the same with binary16 links and vectors (16-byte records per site and right-hand side; x's
# increments stay FP32): hopping terms 576 + 4 x 16 in + 4 x 16 out (+ 4 x 16 p), the update
# 3 x 4 x 16 read, 4 x 16 written, 2 x 4 x 24 increments, p = r + beta p 3 x 4 x 16
BATCH_STEP_BYTES_F16 = 704 + 768 + 448 + 192
# binary16 inner iterations take reliable updates at a 33-fold drop (at 0.01 the binary16
# recursion needs more steps, at 0.1 more updates)
BATCH_DELTA_F16 = 0.03
# reliable-update threshold of the batch: its updates are lattice-synchronous FP64 multi-RHS
# A-applies (the fastest of a lattice's four residuals sets their rate), so it takes them at a
# 100-fold drop; the FP32 recursion keeps the same step counts there (single-mass CG keeps 0.1)
BATCH_DELTA = 0.01
# one FP64 reliable update for 4 right-hand sides (a step of its own for the lattice): the
# increments added into the FP64 x (x read and written 2 x 4 x 48, increments read and cleared
# 2 x 4 x 24), the odd FP64 hopping term (links 2304, x gathered 4 x 48, t written 4 x 48), the
# even one with r = b - (sigma x - D t) (links 2304, t, x, b read and r written: 4 x 4 x 48),
# and the restart of the inner vectors (r64 read 4 x 48, r and p read and written 4 x 4 x 24)
BATCH_RU_BYTES = (2 * 4 * 48 + 2 * 4 * 24) + (2304 + 2 * 4 * 48) + (2304 + 4 * 4 * 48) + \
    (4 * 48 + 4 * 4 * 24)
# network (per site of the full lattice), applied to the solver's FP32 even-site fields (24 B
# per even site), as the flexible CG applies it.  FP32 path: four layers 1->8, 8->8, 8->8,
# 8->1, each reading its site's 8 stored FP32 fat links (8 x 72 B) and its input channels and
# writing its output channels (FP32 complex colour vectors, 24 B each), plus the input embedded
# on both parities (even input read, both parities written: 12 + 24 B per site) and the even
# output read back into the field (12 + 12 B).  Matrix-core path: binary16 links (8 x 36 B) and
# activations (96 B per site for 8 channels); the first layer reads the even input and the odd
# sites' links and writes both parities, the middle two read and write every site, the last
# reads all activations and the even sites' links and writes the even output.
_NET_F32 = sum(576 + 24 * (ci + co) for ci, co in ((1, 8), (8, 8), (8, 8), (8, 1))) + 36 + 24
_NET_MFMA = (12 + 144 + 96) + 2 * (96 + 288 + 96) + (96 + 144 + 12)
NET_BYTES_PER_SITE = {"f32": _NET_F32, "mfma": _NET_MFMA}
# link construction, per site: the 3x3 complex products of the two smearing levels as nested
# (per direction 6 three-link staples and 6 outer terms of 4 inner staples, 2 products each:
# 72; Lepage adds loads, no products), the Naik products (2 per direction), 198 flops each,
# and the U(3) projection counted as 8 Newton steps of ~300 flops per link.  Its least data is
# the thin links read (576 B) and the fat and Naik links written (2 x 576 B).
HISQ_FLOPS_PER_SITE = (2 * 4 * 72 + 4 * 2) * 198 + 4 * 8 * 300
HISQ_BYTES_PER_SITE = 3 * 576
FP64_PEAK_TFLOPS = 78.6


def batch_model_bytes(stats, vhs, nrhs=4, step_bytes=BATCH_STEP_BYTES):
    """Algorithmic bytes of one batched solve: a lattice takes CG steps while any of its
    right-hand sides iterates, and reliable updates while any is due."""
    total = 0.0
    for l, vh in enumerate(vhs):
        st = stats[l * nrhs:(l + 1) * nrhs]
        total += vh * (max(x["iters"] for x in st) * step_bytes +
                       max(x["reliable_updates"] for x in st) * BATCH_RU_BYTES)
    return total


def lanczos_spectrum(alpha, beta):
    """(lambda_min, lambda_max, kappa) of the Lanczos tridiagonal of one unbroken CG run:
    diagonal 1/alpha_k + beta_{k-1}/alpha_{k-1}, off-diagonal sqrt(beta_k)/alpha_k (the last
    step's beta, NaN after the final check, is not used)."""
    import numpy as np
    k = len(alpha)
    if k < 2:
        return None
    a = np.asarray(alpha, dtype=float)
    bt = np.asarray(beta[:k - 1], dtype=float)
    if not (np.all(np.isfinite(a)) and np.all(np.isfinite(bt))):
        return None
    diag = 1.0 / a
    diag[1:] += bt / a[:-1]
    off = np.sqrt(bt) / a[:-1]
    w = np.linalg.eigvalsh(np.diag(diag) + np.diag(off, 1) + np.diag(off, -1))
    return {"lambda_min": float(w[0]), "lambda_max": float(w[-1]), "kappa": float(w[-1] / w[0]),
            "steps": k}


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "dslash_32x32x32x32_hbm_traffic.md")
KERNEL_SOURCES = ["dslash.hip", "ks_device.h", "ks_common.h"]


def measured_traffic(variant: str, threads: int, group: int, way: int, staged: int):
    """HBM bytes per launch of one kernel instantiation (variant, threads per block, links per
    pass, link access, staged gathers) from the committed counter summary, or None once the
    kernel sources differ from the
    ones the counters were taken on."""
    import hashlib
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1611_00728_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    values, recorded = {}, None
    for line in open(TRAFFIC_SUMMARY):
        parts = line.split()
        if len(parts) == 7 and parts[0] == "traffic_bytes_per_launch":
            values[(parts[1], int(parts[2]), int(parts[3]), int(parts[4]), int(parts[5]))] = \
                float(parts[6])
        elif len(parts) == 2 and parts[0] == "source_hash":
            recorded = parts[1]
    if recorded != h.hexdigest()[:16]:
        return None
    return values.get((variant, threads, group, way, staged))


def cpu_baseline(g, b, budget_s: float = 12.0):
    """The FP64 oracle timed on the host: Dslash_eo calls over the same 32^4 field.  The oracle
    computes D on the whole lattice and keeps one parity, twice the work of D_eo, so its
    GB/s counts the D_eo model bytes over the time of that double work."""
    import oracle
    threads = oracle.max_threads()
    oracle.set_threads(threads)
    vh = g.volume // 2
    oracle.dslash_eo(g, 0, b)   # warm
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        oracle.dslash_eo(g, 0, b)
        n += 1
    dt = (time.perf_counter() - t0) / n
    return {"value": model_bytes_per_site("f64", 18) * vh / dt / 1e9, "unit": "GB/s",
            "cores": threads, "kind": "oracle",
            "sample": "%d FP64 oracle Dslash_eo calls on the 32^4 field (%.3f s each); the oracle "
                      "applies the full-lattice D and restricts it to one parity, twice the "
                      "work of D_eo, and the rate counts D_eo's 2400 bytes per output site"
                      % (n, dt)}


def oracle_resid(g, sigma, b, x):
    """|b - A x| / |b| with the FP64 oracle's A on the host, x a device tensor."""
    import numpy as np
    import oracle
    xh = x.detach().cpu().numpy()
    return float(np.linalg.norm(b - oracle.apply_A(g, sigma, xh)) / np.linalg.norm(b))


class OracleSolve:
    """The oracle's FP64 CG solution of one system, computed by a host thread (the oracle's C
    loops run without the interpreter lock) while the GPU works."""

    def __init__(self, g, sigma, b, tol, threads):
        import threading
        self.result = None
        self.seconds = None

        def run():
            import oracle
            oracle.set_threads(threads)
            t = time.perf_counter()
            self.result = oracle.cg(g, sigma, b, tol)
            self.seconds = time.perf_counter() - t
        self.thread = threading.Thread(target=run, daemon=True)
        self.thread.start()
        self.threads = threads

    def join(self):
        self.thread.join()
        return self.result


L5_DIMS, L5_MASS = (48, 48, 48, 64), 0.002


def learned_inputs():
    """The 48^3 x 64 field (thin-link scale 0.5, gauge seed 1005, thin links kept) and the
    108 16^4 blocks cut from it, the source and the training sources (input preparation, not
    timed)."""
    from ksinputs import make_gauge, gaussian_source, subblock, SEEDS
    from paper_1611_00728_amd import learn
    t0 = time.time()
    g5 = make_gauge(L5_DIMS, 0.5, SEEDS["gauge"](5), keep_thin=True)
    log("48^3x64 field generated in %.1f s" % (time.time() - t0))
    t1 = time.time()
    blocks = [subblock(g5, o, (16, 16, 16, 16))
              for o in learn.block_origins(L5_DIMS, (16, 16, 16, 16))]
    log("%d 16^4 blocks cut in %.1f s" % (len(blocks), time.time() - t1))
    return g5, blocks


def config5(g5, blocks):
    """48^3 x 64 lattice, thin-link scale 0.5, m = 0.002: 252 training pairs on 16^4 blocks cut
    from the field (two sources on each of the 108 blocks, two more on the first 18) plus 4 on
    the full lattice (FP64 CG solutions), 1000 Adam steps on the A-norm loss, then flexible CG
    with the network (matrix-core mixing) against FP32-inner CG with reliable updates and plain
    FP64 CG, all to FP64 true relative residual 1e-10, each solution's residual recomputed by
    the FP64 oracle; mixed and learned again on three more held-out sources.  Returns the JSON
    row."""
    import numpy as np
    import torch
    import paper_1611_00728_amd as ks
    from paper_1611_00728_amd import learn
    from ksinputs import gaussian_source, net_init_weights, flatten_weights, SEEDS
    dims, mass, tol = L5_DIMS, L5_MASS, 1e-10
    vh = g5.volume // 2
    t0 = time.time()
    G = ks.Gauge(dims, g5.fat, g5.naik)
    for p in (ks.F64, ks.F32):
        G.prepare(p, 18)
        G.tune(p, 18)
    G.prepare(ks.F16, 18)
    log("48^3x64 gauge loaded and tuned in %.1f s" % (time.time() - t0))
    k = 0
    groups = []
    for sel in (range(len(blocks)), range(252 // 2 - len(blocks))):
        srcs = []
        for j in sel:
            srcs.append([gaussian_source(blocks[j].volume // 2, SEEDS["train_source"](k + r))
                         for r in range(2)])
            k += 2
        groups.append(([blocks[j] for j in sel], srcs))
    pairs, t_blocks = [], 0.0
    for fields, srcs in groups:
        pp, dt, st = learn.solve_pairs_batched(fields, srcs, mass)
        pairs += pp
        t_blocks += dt
        log("%d block pairs in %.1f s (batched FP64 CG, iterations %d-%d)"
            % (len(pp), dt, min(x["iters"] for x in st), max(x["iters"] for x in st)))
    t_gen0 = time.perf_counter()
    full = learn.solve_pairs(G, mass, [gaussian_source(vh, SEEDS["train_source"](10000 + r))
                                       for r in range(4)])
    pairs += full
    t_gen = t_blocks + time.perf_counter() - t_gen0
    net = ks.Net(flatten_weights(net_init_weights(SEEDS["net_init"])))
    steps, batch, lr = 1000, 8, 1e-2
    hist, t_train = learn.train(net, pairs, steps=steps, batch=batch, lr=lr)
    log("trained: loss %.4f -> %.4f in %.1f s" % (hist[0], hist[-1], t_train))
    bh = gaussian_source(vh, SEEDS["source"](5))
    b = torch.from_numpy(bh).cuda()
    rows, xs = {}, {}
    spectrum = None
    for name, fn in (("fp64_cg", lambda x: ks.cg_solve(G, mass, b, x, ks.default_params(tol=tol))),
                     ("mixed_f32_cg", lambda x: ks.cg_solve(
                         G, mass, b, x, ks.default_params(tol=tol, inner=ks.F32))),
                     ("learned_fcg", lambda x: ks.fcg_solve(
                         G, net, mass, b, x, ks.default_params(tol=tol, inner=ks.F32), mfma=True))):
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = fn(x)
        torch.cuda.synchronize()
        xs[name] = x
        rows[name] = {"seconds": time.perf_counter() - t, "iters": res.stats["iters"],
                      "true_rel_resid_gpu": res.stats["true_rel_resid"],
                      "fallback_code": res.stats["fallback"],
                      "flexible_steps": res.stats["iters"] - res.stats["restarts"]
                      if res.stats["fallback"] else res.stats["iters"]}
        if name == "fp64_cg":
            spectrum = lanczos_spectrum(*G.cg_coefficients())
        log("%s: %s" % (name, json.dumps(rows[name])))
    for name, x in xs.items():
        rows[name]["true_rel_resid_oracle"] = oracle_resid(g5, 4 * mass * mass, bh, x)
    # three more held-out sources, mixed and learned, each judged by the oracle
    held = {"sources": 4, "mixed_iters": [rows["mixed_f32_cg"]["iters"]],
            "learned_iters": [rows["learned_fcg"]["iters"]],
            "mixed_s": [rows["mixed_f32_cg"]["seconds"]],
            "learned_s": [rows["learned_fcg"]["seconds"]], "learned_fallbacks": 0,
            "max_true_rel_resid_oracle": max(rows[k]["true_rel_resid_oracle"]
                                             for k in ("mixed_f32_cg", "learned_fcg"))}
    for r in range(3):
        hb = gaussian_source(vh, SEEDS["source"](5) + 100 + r)
        hd = torch.from_numpy(hb).cuda()
        for key, fn in (("mixed", lambda x: ks.cg_solve(
                            G, mass, hd, x, ks.default_params(tol=tol, inner=ks.F32))),
                        ("learned", lambda x: ks.fcg_solve(
                            G, net, mass, hd, x, ks.default_params(tol=tol, inner=ks.F32),
                            mfma=True))):
            x = torch.zeros_like(hd)
            torch.cuda.synchronize()
            t = time.perf_counter()
            res = fn(x)
            torch.cuda.synchronize()
            held[key + "_s"].append(time.perf_counter() - t)
            held[key + "_iters"].append(res.stats["iters"])
            if key == "learned" and res.stats["fallback"]:
                held["learned_fallbacks"] += 1
            held["max_true_rel_resid_oracle"] = max(held["max_true_rel_resid_oracle"],
                                                    oracle_resid(g5, 4 * mass * mass, hb, x))
    held["iteration_ratio_mean"] = float(np.mean(np.array(held["learned_iters"]) /
                                                 np.array(held["mixed_iters"])))
    held["time_ratio_mean"] = float(np.mean(np.array(held["learned_s"]) /
                                            np.array(held["mixed_s"])))
    log("held-out sources: %s" % json.dumps(held))
    tm, tl = rows["mixed_f32_cg"]["seconds"], rows["learned_fcg"]["seconds"]
    im, il = rows["mixed_f32_cg"]["iters"], rows["learned_fcg"]["iters"]
    net.free()
    G.free()
    return {
        "workload": "learned preconditioner, 48^3x64, H scale 0.5, m=0.002, tol 1e-10",
        "solves": rows,
        "spectrum_of_A": spectrum,
        "training": {"pairs": len(pairs), "block_pairs": len(pairs) - len(full),
                     "full_lattice_pairs": len(full), "pair_generation_s": t_gen,
                     "adam_steps": steps, "batch": batch, "lr": lr, "training_s": t_train,
                     "loss": "A-norm error relative to the solution's",
                     "loss_first": float(hist[0]), "loss_last": float(hist[-1])},
        "held_out_sources": held,
        "learned_vs_mixed_iterations": il / im,
        "learned_vs_mixed_speedup": tm / tl,
        "break_even_solves": ((t_gen + t_train) / (tm - tl)) if tl < tm else None,
        "amortised_training_per_solve_s_over_100": (t_gen + t_train) / 100.0}


def learned48(args):
    """The 48^3 x 64 learned-preconditioner workload on its own (one JSON line)."""
    g5, blocks = learned_inputs()
    import torch
    torch.cuda.set_device(0)
    print(json.dumps(config5(g5, blocks)), flush=True)


def multishift_workload(args):
    """The multi-shift workload alone: 32^3 x 48 (thin-link scale 0.5), nine shifts
    sigma_i = 4 m_i^2 with m_i log-spaced over [0.002, 0.5], per-shift target 1e-9; FP64, FP32 and
    FP16 inner with 18-real Naik, each variant tuned first, `--warmup` untimed and `--steps`
    timed solves.  One JSON line (seconds per solve, steps per shift, largest GPU residual)."""
    import numpy as np
    import torch
    import paper_1611_00728_amd as ks
    from ksinputs import make_gauge, gaussian_source, SEEDS
    dims = (32, 32, 32, 48)
    g = make_gauge(dims, 0.5, SEEDS["gauge"](3))
    b_h = gaussian_source(g.volume // 2, SEEDS["source"](3))
    torch.cuda.set_device(0)
    G = ks.Gauge(dims, g.fat, g.naik)
    del g
    b = torch.from_numpy(b_h).cuda()
    sig = 4 * np.geomspace(0.002, 0.5, 9) ** 2
    xs = [torch.zeros_like(b) for _ in sig]
    rows = {}
    for name, p_ in (("f64", ks.F64), ("f32", ks.F32), ("f16", ks.F16)):
        G.prepare(p_, 18)
        G.tune(p_, 18)
        times = []
        for k in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            time.sleep(0.05)   # an idle gap that marks the solve's start in a kernel trace
            t = time.perf_counter()
            rc, st = ks.multishift_cg_solve(G, sig, b, xs, 1e-9,
                                            ks.default_params(inner=p_, check_every=16))
            torch.cuda.synchronize()
            if k >= args.warmup:
                times.append(time.perf_counter() - t)
        torch.cuda.synchronize()
        time.sleep(0.05)   # and its end, before the next variant's set-up
        rows[name] = {"seconds": float(np.median(times)), "solves": len(times),
                      "iters_per_shift": [x["iters"] for x in st],
                      "reliable_updates_per_shift": [x["reliable_updates"] for x in st],
                      "max_true_rel_resid_gpu": max(x["true_rel_resid"] for x in st)}
        log("multishift %s: %.4f s" % (name, rows[name]["seconds"]))
    print(json.dumps({"workload": "multi-shift CG, 32^3x48, 9 shifts, tol 1e-9",
                      "lattice": list(dims), "shifts": [float(x) for x in sig],
                      "variants": rows}), flush=True)
    G.free()


def sweep(args):
    """Dslash_eo bandwidth over lattice sizes (L^4 for L = 8 ... 48 and the paper's 20^3 x 64 and
    24^3 x 60), every precision and Naik storage, each variant autotuned per lattice; and the
    FP64 oracle on the host: Dslash_eo per site at 8^4, 16^4 and 32^4 on one thread and on all,
    full CG solves at 8^4 and 16^4, and the 32^4 solve extrapolated from the time of 20 steps
    times the GPU's step count.  One JSON line."""
    import numpy as np
    import torch
    import paper_1611_00728_amd as ks
    import oracle
    from ksinputs import make_gauge, gaussian_source
    lattices = [(L, L, L, L) for L in (8, 12, 16, 20, 24, 28, 32, 40, 48)] + \
               [(20, 20, 20, 64), (24, 24, 24, 60)]
    pmap = {"f64": ks.F64, "f32": ks.F32, "f16": ks.F16}
    variants = [("f64", 18), ("f64", 12), ("f32", 18), ("f32", 12), ("f16", 18), ("f16", 12)]
    stream = torch.cuda.current_stream()
    rows = []
    for dims in lattices:
        seed = 1100 + dims[0] if dims[3] == dims[0] else 1200 + dims[0]
        t0 = time.time()
        g = make_gauge(dims, 0.5, seed)
        vh = g.volume // 2
        G = ks.Gauge(dims, g.fat, g.naik)
        b = torch.from_numpy(gaussian_source(vh, seed + 1000)).cuda()
        del g
        row = {"lattice": list(dims), "even_sites": vh,
               "cache_resident": vh * 2400 * 2 < 256e6}
        for prec, rc in variants:
            G.prepare(pmap[prec], rc)
            cfg = G.tune(pmap[prec], rc)
            ein = ks.Field(G, ks.EVEN, pmap[prec]).load(b)
            eout = ks.Field(G, ks.ODD, pmap[prec])
            for _ in range(3):
                ks.dslash_eo(G, eout, ein, rc)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(BURST):
                ks.dslash_eo(G, eout, ein, rc)
            e1.record(stream)
            stream.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / BURST
            gbs = model_bytes_per_site(prec, rc) * vh / (us * 1e-6) / 1e9
            row["%s_r%d" % (prec, rc)] = {"us": us, "GBps": gbs, "frac_of_8TBps": gbs / HBM_PEAK_GBS,
                                          "launch": cfg}
            del ein, eout
        G.free()
        torch.cuda.synchronize()
        rows.append(row)
        log("sweep %s: FP64 %.0f GB/s, FP16-12 %.0f GB/s (%.0f s)"
            % ("x".join(map(str, dims)), row["f64_r18"]["GBps"], row["f16_r12"]["GBps"],
               time.time() - t0))
    # the oracle on the host cores
    nthreads = oracle.max_threads()
    cpu = {"threads_all": nthreads, "dslash_s_per_site": {}, "cg": {}}
    for dims in ((8, 8, 8, 8), (16, 16, 16, 16), (32, 32, 32, 32)):
        g = make_gauge(dims, 0.5, 1100 + dims[0])
        vh = g.volume // 2
        psi = gaussian_source(vh, 7)
        entry = {}
        for nt in (1, nthreads):
            oracle.set_threads(nt)
            oracle.dslash_eo(g, 0, psi)
            n, t1 = 0, time.perf_counter()
            while time.perf_counter() - t1 < 1.0 or n < 2:
                oracle.dslash_eo(g, 0, psi)
                n += 1
            entry["threads_%d" % nt] = (time.perf_counter() - t1) / n / vh
        cpu["dslash_s_per_site"]["x".join(map(str, dims))] = entry
        oracle.set_threads(nthreads)
        if dims[0] <= 16:
            mass = 0.1 if dims[0] == 8 else 0.01
            b = gaussian_source(vh, 8)
            t1 = time.perf_counter()
            _, info = oracle.cg(g, 4 * mass * mass, b, 1e-10)
            cpu["cg"]["x".join(map(str, dims))] = {"seconds": time.perf_counter() - t1,
                                                   "iters": info.iters, "mass": mass}
        else:
            b = gaussian_source(vh, 2002)
            t1 = time.perf_counter()
            oracle.cg(g, 4 * MASS * MASS, b, 1e-30, max_iter=20, max_restarts=0)
            per = (time.perf_counter() - t1) / 20
            cpu["cg"]["32x32x32x32"] = {"seconds_per_step": per, "extrapolated_seconds": per * 601,
                                        "note": "20 timed steps x the GPU's 601 steps (extrapolated)"}
        log("oracle %s done" % "x".join(map(str, dims)))
    print(json.dumps({"workload": "Dslash_eo sweep over lattice sizes (H scale 0.5) and the FP64 "
                                  "oracle's host timings", "rows": rows, "cpu_oracle": cpu}),
          flush=True)


def counters_pass(N, ks, G, g, bd, fields, variants, gm, mb_h):
    """One short pass over every hot kernel, for rocprofv3 counter runs (the calibration copy
    first).  Prints the launch sizes the per-kernel byte models need."""
    import numpy as np
    import torch
    from ksinputs import make_gauge, gaussian_source, flatten_weights, net_init_weights, SEEDS
    vh = g.volume // 2
    # a plain copy of known size (1 GiB read + 1 GiB written) calibrates the byte counters
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    ks.stream_copy(dst, src)
    torch.cuda.synchronize()
    del src, dst
    for v in variants:
        ein, eout = fields[v[0]]
        for _ in range(N):
            ks.dslash_eo(G, eout, ein, v[1])
    # FP32-inner CG on the 32^4 system: N fused steps (and the reliable updates among them)
    x = torch.zeros_like(bd)
    ks.cg_solve(G, MASS, bd, x, ks.default_params(tol=TOL, inner=ks.F32, max_iter=N),
                raise_on_error=False)
    # the network on the solver's FP32 fields, both paths
    net = ks.Net(flatten_weights(net_init_weights(SEEDS["net_init"])))
    nin, nout = ks.Field(G, ks.EVEN, ks.F32).load(bd), ks.Field(G, ks.EVEN, ks.F32)
    for _ in range(N):
        net.apply_field(nin, nout, mfma=True)
        net.apply_field(nin, nout, mfma=False)
    torch.cuda.synchronize()
    del nin, nout, net
    # link construction from the 32^4 thin links
    thin_d = torch.from_numpy(np.ascontiguousarray(g.thin).reshape(-1)).cuda()
    hf, hn = torch.empty_like(thin_d), torch.empty_like(thin_d)
    ks.hisq_links(g.dims, thin_d, hf, hn)
    torch.cuda.synchronize()
    del thin_d, hf, hn
    ks.hisq_release()
    # 32^3 x 48: FP32-inner multi-shift, N shared steps, then the force from its iterates
    GM = ks.Gauge(gm.dims, gm.fat, gm.naik)
    GM.prepare(ks.F32, 18)
    mb = torch.from_numpy(mb_h).cuda()
    sig = 4 * np.geomspace(0.002, 0.5, 9) ** 2
    xs = [torch.zeros_like(mb) for _ in sig]
    ks.multishift_cg_solve(GM, sig, mb, xs, 1e-9, ks.default_params(inner=ks.F32, max_iter=N),
                           raise_on_error=False)
    fv = torch.empty(36 * gm.volume, dtype=torch.complex128, device="cuda")
    fw = torch.empty_like(fv)
    ks.force(GM, [1.0 / (i + 1) for i in range(len(sig))], xs, fv, fw)
    torch.cuda.synchronize()
    del GM, xs, fv, fw
    # batch: 8 lattices of 16^4 x 4 right-hand sides, N steps
    bdims = [(16, 16, 16, 16)] * 8
    bg = [make_gauge(d, 0.4, SEEDS["batch_gauge"](j)) for j, d in enumerate(bdims)]
    B = ks.Batch(bdims, [x_.fat for x_ in bg], [x_.naik for x_ in bg], 4, ks.F32)
    bb = [torch.from_numpy(gaussian_source(x_.volume // 2, SEEDS["batch_rhs"](j, r))).cuda()
          for j, x_ in enumerate(bg) for r in range(4)]
    bx = [torch.zeros_like(v) for v in bb]
    B.solve([0.05] * len(bdims), bb, bx, ks.default_params(tol=TOL, max_iter=N, check_every=8,
                                                           delta=BATCH_DELTA),
            raise_on_error=False)
    torch.cuda.synchronize()
    # the same batch with binary16 inner iterations
    B16 = ks.Batch(bdims, [x_.fat for x_ in bg], [x_.naik for x_ in bg], 4, ks.F16)
    bx = [torch.zeros_like(v) for v in bb]
    B16.solve([0.05] * len(bdims), bb, bx, ks.default_params(tol=TOL, max_iter=N, check_every=8,
                                                             delta=BATCH_DELTA_F16),
              raise_on_error=False)
    torch.cuda.synchronize()
    print(json.dumps({"counters": N, "sites_32x32x32x32": g.volume,
                      "sites_32x32x32x48": gm.volume, "batch": "8 x 16^4 x 4 RHS, FP32 and binary16",
                      "copy_bytes": 2 * (1 << 27) * 8,
                      "dslash_model_bytes": {"%s_r%d" % v: model_bytes_per_site(*v) * vh
                                             for v in variants}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned48", action="store_true",
                    help="skip the 48^3 x 64 learned-preconditioner workload after the steps")
    ap.add_argument("--workload", default="default",
                    choices=["default", "learned48", "sweep", "multishift"],
                    help="learned48: the 48^3 x 64, m = 0.002 learned-preconditioner workload "
                         "(training pairs, training, flexible CG vs mixed CG); sweep: Dslash_eo "
                         "over lattice sizes and the oracle's host timings; multishift: the "
                         "32^3 x 48 multi-shift solves alone (FP64, FP32, FP16 inner, --steps "
                         "timed solves each); each its own JSON line")
    ap.add_argument("--counters", type=int, default=0, metavar="N",
                    help="counter runs: one plain 1 GiB device copy (calibration), N launches "
                         "of each tuned Dslash_eo variant, then N steps or launches of each "
                         "other hot kernel (FP32 CG, network layers, 32^3x48 multi-shift and "
                         "force, a 16^4 batch, link construction), then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path (the lattice is "
              "not domain-decomposed here); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from ksinputs import make_gauge, gaussian_source, SEEDS

    if args.workload == "learned48":
        learned48(args)
        return
    if args.workload == "sweep":
        import torch
        torch.cuda.set_device(0)
        sweep(args)
        return
    if args.workload == "multishift":
        multishift_workload(args)
        return
    # every input is generated before the GPU is touched: large fields are computed by forked
    # worker processes
    t0 = time.time()
    g = make_gauge(DIMS, 0.5, 1002, keep_thin=True)
    vh = g.volume // 2
    b = gaussian_source(vh, 2002)
    MS_DIMS = (32, 32, 32, 48)
    gm = make_gauge(MS_DIMS, 0.5, SEEDS["gauge"](3))
    mb_h = gaussian_source(gm.volume // 2, SEEDS["source"](3))
    log("32^4 and 32^3x48 inputs generated in %.1f s" % (time.time() - t0))
    g5 = blocks5 = None
    if not args.counters and not args.no_learned48:
        g5, blocks5 = learned_inputs()
    # the oracle's own FP64 CG solution of the 32^4 system, on host threads meanwhile
    oracle_ref = None
    if not args.counters:
        import oracle
        ncpu = oracle.max_threads()
        oracle_ref = OracleSolve(g, 4 * MASS * MASS, b, 1e-12, max(1, ncpu - 4))
        log("oracle FP64 CG of the 32^4 system started on %d host threads" % oracle_ref.threads)

    import torch
    import paper_1611_00728_amd as ks
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    G = ks.Gauge(DIMS, g.fat, g.naik)
    for p in (ks.F64, ks.F32, ks.F16):
        for r in (18, 12):
            G.prepare(p, r)
    torch.cuda.synchronize()
    log("gauge loaded, %.2f GB on the device" % (G.device_bytes() / 1e9))

    bd = torch.from_numpy(b).cuda()
    fields = {}
    for name, p in (("f64", ks.F64), ("f32", ks.F32), ("f16", ks.F16)):
        fields[name] = (ks.Field(G, ks.EVEN, p).load(bd), ks.Field(G, ks.ODD, p))
    stream = torch.cuda.current_stream()

    variants = [("f64", 18), ("f64", 12), ("f32", 18), ("f32", 12), ("f16", 18), ("f16", 12)]
    times = {v: [] for v in variants}
    pmap = {"f64": ks.F64, "f32": ks.F32, "f16": ks.F16}
    tuned = {}
    for v in variants:
        tuned["%s_r%d" % v] = G.tune(pmap[v[0]], v[1])
    log("autotuned: %s" % json.dumps(tuned))

    def time_variant(v, reps=20):
        ein, eout = fields[v[0]]
        for _ in range(3):
            ks.dslash_eo(G, eout, ein, v[1])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            ks.dslash_eo(G, eout, ein, v[1])
        e1.record(stream)
        stream.synchronize()
        return e0.elapsed_time(e1) * 1e3 / reps

    # 8-way vs 4-way link access (the storage question Sec. 3 leaves open), and neighbour
    # gathers through the caches vs staged in LDS: the best launch shape of each combination
    # per variant; the tuned configuration is restored afterwards
    link_study = {}
    if not args.counters:
        for v in variants:
            key = "%s_r%d" % v
            cfg = tuned[key]
            row = {}
            for way in (8, 4):
                for staged in (0, 1):
                    best = None
                    for group in (1, 2, 4):
                        for nt in (64, 128, 256):
                            for lds in (0, 13312, 20224, 32512, 54272):
                                try:
                                    G.set_config(pmap[v[0]], v[1], nt, lds, group, way, staged)
                                except ks.KSError:
                                    continue        # a form that is not built
                                us = time_variant(v, reps=5)
                                if best is None or us < best[0]:
                                    best = (us, nt, lds, group)
                    G.set_config(pmap[v[0]], v[1], best[1], best[2], best[3], way, staged)
                    name = "%d-way_%s" % (way, "staged" if staged else "cached")
                    row[name + "_us"] = time_variant(v)
                    row[name + "_shape"] = {"threads": best[1], "lds_bytes": best[2],
                                            "links_per_pass": best[3]}
            G.set_config(pmap[v[0]], v[1], cfg["threads"], cfg["lds_bytes"], cfg["links_per_pass"],
                         cfg["link_access"], cfg["staged"])
            link_study[key] = row
        log("link access study: %s" % json.dumps(link_study))

    if args.counters:
        counters_pass(args.counters, ks, G, g, bd, fields, variants, gm, mb_h)
        return

    def burst(v, record):
        ein, eout = fields[v[0]]
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(BURST)]
        for k in range(BURST):
            evs[k][0].record(stream)
            ks.dslash_eo(G, eout, ein, v[1])
            evs[k][1].record(stream)
        stream.synchronize()
        if record:
            times[v].extend(a.elapsed_time(c) * 1e-3 for a, c in evs)

    # batched workload: 64 lattices of three sizes x 4 right-hand sides, FP32 inner iterations
    from ksinputs import batch_masses, SEEDS
    bdims = [(8, 8, 8, 8)] * 24 + [(12, 12, 12, 12)] * 24 + [(16, 16, 16, 16)] * 16
    t1 = time.time()
    bg = [make_gauge(d, 0.4, SEEDS["batch_gauge"](j)) for j, d in enumerate(bdims)]
    bmass = batch_masses(len(bdims), 0.01, 0.2, SEEDS["batch_mass"])
    B = ks.Batch(bdims, [x.fat for x in bg], [x.naik for x in bg], 4, ks.F32)
    bb_h = [gaussian_source(x.volume // 2, SEEDS["batch_rhs"](j, r))
            for j, x in enumerate(bg) for r in range(4)]
    bb = [torch.from_numpy(v).cuda() for v in bb_h]
    bx = [torch.zeros_like(v) for v in bb]
    bvh = [x.volume // 2 for x in bg]
    batch_cfg = B.tune()
    # the same batch with binary16 inner iterations
    B16 = ks.Batch(bdims, [x.fat for x in bg], [x.naik for x in bg], 4, ks.F16)
    batch16_cfg = B16.tune()
    bx16 = [torch.zeros_like(v) for v in bb]
    log("batch of %d lattices x 4 RHS ready in %.1f s, schedule %s, binary16 %s"
        % (len(bdims), time.time() - t1, json.dumps(batch_cfg), json.dumps(batch16_cfg)))
    batch_runs, batch16_runs = [], []

    def batch_solve(record):
        for B_, xs_, delta_, runs_ in ((B, bx, BATCH_DELTA, batch_runs),
                                       (B16, bx16, BATCH_DELTA_F16, batch16_runs)):
            for v in xs_:
                v.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            rc, st = B_.solve(bmass, bb, xs_, ks.default_params(tol=TOL, check_every=8,
                                                                delta=delta_))
            torch.cuda.synchronize()
            if record:
                runs_.append((time.perf_counter() - t, st))

    # multi-shift workload: 32^3 x 48, nine shifts sigma_i = 4 m_i^2, m_i log-spaced 0.002..0.5
    t1 = time.time()
    GM = ks.Gauge(MS_DIMS, gm.fat, gm.naik)
    for p_, rc_ in ((ks.F64, 18), (ks.F64, 12), (ks.F32, 18), (ks.F32, 12), (ks.F16, 18)):
        GM.prepare(p_, rc_)
        GM.tune(p_, rc_)
    mb_ = torch.from_numpy(mb_h).cuda()
    ms_sigma = 4 * np.geomspace(0.002, 0.5, 9) ** 2
    ms_x = [torch.zeros_like(mb_) for _ in ms_sigma]
    ms_vh = gm.volume // 2
    ms_last = {}
    log("32^3x48 multi-shift field ready in %.1f s" % (time.time() - t1))
    ms_runs = {"f64": [], "f64_r12": [], "f32": [], "f32_r12": [], "f16": []}

    # link derivative of sum_i r_i b^+ A_i^-1 b from the nine solutions (residues 1/(i+1))
    ms_res = [1.0 / (i + 1) for i in range(len(ms_sigma))]
    fvol = 2 * ms_vh
    force_v = torch.empty(36 * fvol, dtype=torch.complex128, device="cuda")
    force_w = torch.empty_like(force_v)
    force_runs = []

    def multishift(record):
        for name, p_, rc_ in (("f64", ks.F64, 18), ("f64_r12", ks.F64, 12), ("f32", ks.F32, 18),
                              ("f32_r12", ks.F32, 12), ("f16", ks.F16, 18)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            rc, st = ks.multishift_cg_solve(GM, ms_sigma, mb_, ms_x, 1e-9,
                                            ks.default_params(inner=p_, recon=rc_,
                                                              check_every=16))
            torch.cuda.synchronize()
            if record:
                ms_runs[name].append((time.perf_counter() - t, st))
                ms_last[name] = [x.clone() for x in ms_x]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ks.force(GM, ms_res, ms_x, force_v, force_w)
        e1.record(stream)
        stream.synchronize()
        if record:
            force_runs.append(e0.elapsed_time(e1) * 1e-3)

    # learned preconditioner: (source, FP64-CG solution) pairs on the sixteen 16^4 blocks of
    # the 32^4 field (4 sources each) and 4 on the full lattice, Adam on the GPU kernels
    from paper_1611_00728_amd import learn
    from ksinputs import subblock, net_init_weights, flatten_weights
    blocks = [subblock(g, o, (16, 16, 16, 16)) for o in learn.block_origins(DIMS, (16, 16, 16, 16))]
    srcs = [[gaussian_source(bk.volume // 2, SEEDS["train_source"](4 * j + r)) for r in range(4)]
            for j, bk in enumerate(blocks)]
    pairs, t_blocks, _ = learn.solve_pairs_batched(blocks, srcs, MASS)
    t_gen0 = time.perf_counter()
    pairs += learn.solve_pairs(G, MASS, [gaussian_source(vh, SEEDS["train_source"](1000 + r))
                                         for r in range(4)])
    t_gen = t_blocks + time.perf_counter() - t_gen0
    del blocks
    net = ks.Net(flatten_weights(net_init_weights(SEEDS["net_init"])))
    NET_STEPS, NET_LR = 1000, 1e-2
    loss_hist, t_train = learn.train(net, pairs, steps=NET_STEPS, batch=8, lr=NET_LR)
    log("learned preconditioner: %d pairs in %.1f s, %d Adam steps in %.1f s, loss %.4f -> %.4f"
        % (len(pairs), t_gen, NET_STEPS, t_train, loss_hist[0], loss_hist[-1]))
    last_x = {}
    learned_runs = []
    net_times = {"f32": [], "mfma": []}
    net_in = ks.Field(G, 0, ks.F32).load(bd)
    net_out = ks.Field(G, 0, ks.F32)

    def net_burst(record):
        for name in ("f32", "mfma"):
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(5)]
            for e0, e1 in evs:
                e0.record(stream)
                net.apply_field(net_in, net_out, mfma=(name == "mfma"))
                e1.record(stream)
            stream.synchronize()
            if record:
                net_times[name].extend(a.elapsed_time(c) * 1e-3 for a, c in evs)

    def learned(record):
        xd = torch.zeros_like(bd)
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = ks.fcg_solve(G, net, MASS, bd, xd, ks.default_params(tol=TOL, inner=ks.F32),
                           mfma=True)
        torch.cuda.synchronize()
        if record:
            learned_runs.append((time.perf_counter() - t, res.stats))
            last_x["learned_fcg_f32"] = xd

    # link construction from the thin links of the same 32^4 field (two smearing levels, U(3)
    # projection, Naik): its flops (3x3 complex products, HISQ_FLOPS_PER_SITE) against the FP64
    # peak, and its least data (thin links in, fat and Naik links out) against HBM
    thin_d = torch.from_numpy(np.ascontiguousarray(g.thin).reshape(-1)).cuda()
    hisq_fat = torch.empty_like(thin_d)
    hisq_naik = torch.empty_like(thin_d)
    hisq_runs = []

    def link_construction(record):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ks.hisq_links(DIMS, thin_d, hisq_fat, hisq_naik)
        torch.cuda.synchronize()
        if record:
            hisq_runs.append(time.perf_counter() - t)

    # full system M x = b on both parities (odd source: seed 2102), FP32 inner iterations
    bod = torch.from_numpy(gaussian_source(vh, 2102)).cuda()
    full_runs = []

    def full_solve(record):
        xe, xo = torch.zeros_like(bd), torch.zeros_like(bd)
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = ks.full_solve(G, MASS, bd, bod, xe, xo, ks.default_params(tol=TOL, inner=ks.F32))
        torch.cuda.synchronize()
        if record:
            full_runs.append((time.perf_counter() - t, res.stats))
            last_x["full_system_f32"] = (xe, xo)

    solves = {"f64": [], "f32": [], "f32_r12": [], "f16_r12": []}
    spectrum = {}
    solve_cfg = {"f64": dict(inner=ks.F64, recon=18), "f32": dict(inner=ks.F32, recon=18),
                 "f32_r12": dict(inner=ks.F32, recon=12), "f16_r12": dict(inner=ks.F16, recon=12)}

    def step(record):
        for v in variants:
            burst(v, record)
        batch_solve(record)
        multishift(record)
        net_burst(record)
        learned(record)
        full_solve(record)
        link_construction(record)
        for name, kw in solve_cfg.items():
            xd = torch.zeros_like(bd)
            torch.cuda.synchronize()
            t = time.perf_counter()
            res = ks.cg_solve(G, MASS, bd, xd, ks.default_params(tol=TOL, **kw))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            if record:
                solves[name].append((dt, res.stats))
                last_x[name] = xd
                if name == "f64":
                    spectrum["f64"] = lanczos_spectrum(*G.cg_coefficients())

    for _ in range(args.warmup):
        step(False)
    log("warmup done")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        step(True)
        log("step %d done" % k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    # the FP64 oracle on the host judges every returned solution: its residual b - A x
    # recomputed with the oracle's A, and the 32^4 FP64 solution's distance to the oracle's own
    # CG solution (tolerance 1e-12)
    import oracle
    ref = oracle_ref.join()
    oracle.set_threads(oracle.max_threads())
    t_or = time.time()
    sig = 4 * MASS * MASS
    orc = {name: oracle_resid(g, sig, b, x) for name, x in last_x.items()
           if name != "full_system_f32"}
    from oracle.solvers import apply_M
    xe_h, xo_h = (t_.detach().cpu().numpy() for t_ in last_x["full_system_f32"])
    bo_h = gaussian_source(vh, 2102)
    me, mo = apply_M(g, MASS, xe_h, xo_h)
    orc["full_system_f32"] = float(np.sqrt(np.linalg.norm(b - me) ** 2 + np.linalg.norm(bo_h - mo) ** 2) /
                                   np.sqrt(np.linalg.norm(b) ** 2 + np.linalg.norm(bo_h) ** 2))
    x_or, info_or = ref
    x64 = last_x["f64"].detach().cpu().numpy()
    f64_x_err = float(np.linalg.norm(x64 - x_or) / np.linalg.norm(x_or))
    ms_orc = {name: [oracle_resid(gm, s_, mb_h, x) for s_, x in zip(ms_sigma, xs)]
              for name, xs in ms_last.items()}
    batch_orc = [oracle_resid(bg[p_ // 4], 4 * bmass[p_ // 4] ** 2, bb_h[p_], bx[p_])
                 for p_ in range(len(bb))]
    batch16_orc = [oracle_resid(bg[p_ // 4], 4 * bmass[p_ // 4] ** 2, bb_h[p_], bx16[p_])
                   for p_ in range(len(bb))]
    log("oracle residuals of every solution in %.1f s (32^4 oracle CG: %d steps, %.1f s on %d "
        "threads)" % (time.time() - t_or, info_or.iters, oracle_ref.seconds, oracle_ref.threads))

    dsl = {}
    for v, ts in times.items():
        avg = float(np.mean(ts))
        mb = model_bytes_per_site(*v) * vh
        dsl["%s_r%d" % v] = {"avg_us": avg * 1e6, "model_GBps": mb / avg / 1e9,
                             "frac_of_8TBps": mb / avg / 1e9 / HBM_PEAK_GBS,
                             "gflops": 1146.0 * vh / avg / 1e9,
                             "launch": tuned["%s_r%d" % v]}
    head = dsl["f64_r18"]
    tts = {}
    base = float(np.median([d for d, _ in solves["f64"]]))
    for name, rs in solves.items():
        med = float(np.median([d for d, _ in rs]))
        st = rs[-1][1]
        tts[name] = {"seconds": med, "iters": st["iters"], "reliable_updates": st["reliable_updates"],
                     "true_rel_resid_gpu": st["true_rel_resid"],
                     "true_rel_resid_oracle": orc[name], "speedup_vs_f64": base / med,
                     "model_GBps": st["model_bytes"] / st["seconds"] / 1e9,
                     "frac_of_8TBps": st["model_bytes"] / st["seconds"] / 1e9 / HBM_PEAK_GBS}
    tts["f64"]["solution_rel_error_vs_oracle_cg"] = f64_x_err
    tts["f64"]["oracle_cg"] = {"tol": 1e-12, "iters": info_or.iters, "seconds": oracle_ref.seconds,
                               "threads": oracle_ref.threads}
    fst = full_runs[-1][1]
    fmed = float(np.median([d for d, _ in full_runs]))
    tts["full_system_f32"] = {
        "seconds": fmed, "iters": fst["iters"], "reliable_updates": fst["reliable_updates"],
        "true_rel_resid_of_Mx_eq_b_gpu": fst["true_rel_resid"],
        "true_rel_resid_of_Mx_eq_b_oracle": orc["full_system_f32"],
        "model_GBps": fst["model_bytes"] / fst["seconds"] / 1e9,
        "note": "M = 2m + D on both parities: even Schur system by FP32-inner CG, odd sites "
                "reconstructed in FP64"}
    hsec = float(np.median(hisq_runs))
    hflops = HISQ_FLOPS_PER_SITE * g.volume / hsec / 1e12
    links = {"seconds": hsec,
             "roofline": {"bound": "alu", "achieved": hflops, "peak": FP64_PEAK_TFLOPS,
                          "unit": "TFLOP/s", "frac": hflops / FP64_PEAK_TFLOPS,
                          "flops_per_site": HISQ_FLOPS_PER_SITE},
             "least_data_GBps": HISQ_BYTES_PER_SITE * g.volume / hsec / 1e9,
             "note": "fat and Naik links from the 32^4 thin links: fat7, U(3) projection, "
                     "fat7 + Lepage, Naik, signs (FP64): far below both its FP64 and its HBM "
                     "roofline; its passes are bound by the latency of cached neighbour-matrix "
                     "gathers"}
    walls = [w for w, _ in batch_runs]
    per_solve = [x["seconds"] for _, st in batch_runs for x in st]
    worst = max(x["true_rel_resid"] for _, st in batch_runs for x in st)
    batch = {"lattices": "24 x 8^4 + 24 x 12^4 + 16 x 16^4, H scale 0.4, m ~ U[0.01, 0.2]",
             "rhs_per_lattice": 4, "solves": len(bb), "inner": "f32 + FP64 reliable updates",
             "reliable_update_delta": BATCH_DELTA,
             "wall_seconds": float(np.median(walls)),
             "solves_per_second": len(bb) / float(np.median(walls)),
             "p50_seconds_per_solve": float(np.percentile(per_solve, 50)),
             "p99_seconds_per_solve": float(np.percentile(per_solve, 99)),
             "max_true_rel_resid_gpu": worst,
             "max_true_rel_resid_oracle": max(batch_orc),
             "model_GBps": batch_model_bytes(batch_runs[-1][1], bvh) / float(np.median(walls)) / 1e9,
             "iters_range": [min(x["iters"] for _, st in batch_runs for x in st),
                             max(x["iters"] for _, st in batch_runs for x in st)],
             "schedule": batch_cfg}
    walls16 = [w for w, _ in batch16_runs]
    per16 = [x["seconds"] for _, st in batch16_runs for x in st]
    batch["binary16_inner"] = {
        "inner": "binary16 links and vectors (FP32 arithmetic) + FP64 reliable updates",
        "reliable_update_delta": BATCH_DELTA_F16,
        "wall_seconds": float(np.median(walls16)),
        "solves_per_second": len(bb) / float(np.median(walls16)),
        "p50_seconds_per_solve": float(np.percentile(per16, 50)),
        "p99_seconds_per_solve": float(np.percentile(per16, 99)),
        "max_true_rel_resid_gpu": max(x["true_rel_resid"] for _, st in batch16_runs for x in st),
        "max_true_rel_resid_oracle": max(batch16_orc),
        "model_GBps": batch_model_bytes(batch16_runs[-1][1], bvh,
                                        step_bytes=BATCH_STEP_BYTES_F16) /
                      float(np.median(walls16)) / 1e9,
        "iters_range": [min(x["iters"] for _, st in batch16_runs for x in st),
                        max(x["iters"] for _, st in batch16_runs for x in st)],
        "schedule": batch16_cfg}

    msr = {}
    for name, rs in ms_runs.items():
        med = float(np.median([d for d, _ in rs]))
        st = rs[-1][1]
        shared = min(x["iters"] for x in st)
        # model flops: shared steps (two hopping terms, xpay, r update and nine shift
        # updates per site) plus the per-shift refinement steps of a single-mass CG
        flops = ms_vh * (shared * (2 * 1146 + 12 + 12 + 9 * 24 + 12) +
                         sum(x["iters"] - shared for x in st) * (2 * 1146 + 72))
        mbytes = sum(x["model_bytes"] for x in st)
        msr[name] = {"seconds": med, "shared_iters": shared,
                     "total_iters_per_shift": [x["iters"] for x in st],
                     "max_true_rel_resid_gpu": max(x["true_rel_resid"] for x in st),
                     "true_rel_resid_oracle_per_shift": ms_orc[name],
                     "model_gflops": flops / med / 1e9,
                     "model_GBps": mbytes / med / 1e9,
                     "frac_of_8TBps": mbytes / med / 1e9 / HBM_PEAK_GBS}
    msr["lattice"] = list(MS_DIMS)
    fsec = float(np.median(force_runs))
    # per term: import (48 B read + 48 written per even site) and its share of the multi-vector
    # FP64 hopping term (links, 2304 B per odd site, read once per pass of up to five terms; the
    # term's input and output, 96 B); outer products: both forces written (2 x 4 x 144 B per
    # site) and each term's vector read once per site (48 B)
    nt_ = len(ms_sigma)
    fpasses = -(-nt_ // 5)
    fbytes = (nt_ * ms_vh * (96 + 96) + fpasses * ms_vh * 2304 +
              fvol * (2 * 4 * 144 + nt_ * 48))
    # least data: the odd-site links once (2304 B per odd site), each term's solution once
    # (48 B per even site) and both forces written once (2 x 4 x 144 B per site)
    fleast = ms_vh * 2304 + nt_ * ms_vh * 48 + fvol * 2 * 4 * 144
    msr["force"] = {"seconds": fsec, "terms": nt_,
                    "roofline": {"bound": "hbm", "achieved": fleast / fsec / 1e9,
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": fleast / fsec / 1e9 / HBM_PEAK_GBS,
                                 "least_data_bytes": fleast},
                    "access_model_GBps": fbytes / fsec / 1e9,
                    "note": "link derivative of the nine-term rational action from the "
                            "multi-shift solutions, fat and Naik links, FP64; the access model "
                            "also counts the odd images of the solutions written and read back "
                            "and the links read once per pass of five terms"}
    msr["shifts"] = "sigma_i = 4 m_i^2, m_i = geomspace(0.002, 0.5, 9), tol 1e-9 per shift"

    lmed = float(np.median([d for d, _ in learned_runs]))
    lst = learned_runs[-1][1]
    t_mixed = tts["f32"]["seconds"]
    overhead = t_gen + t_train
    tts["learned_fcg_f32"] = {
        "seconds": lmed, "iters": lst["iters"], "fallback": bool(lst["fallback"]),
        "fallback_reason": {0: None, 1: "N(r) not finite", 2: "Re<N(r), r> <= 0",
                            3: "<p, Ap> <= 0", 4: "|r| not halved in 50 steps",
                            5: "max_iter"}[lst["fallback"]],
        "fallback_iters": lst["restarts"], "reliable_updates": lst["reliable_updates"],
        "true_rel_resid_gpu": lst["true_rel_resid"],
        "true_rel_resid_oracle": orc["learned_fcg_f32"], "speedup_vs_f64": base / lmed,
        "speedup_vs_mixed_f32": t_mixed / lmed,
        "iterations_vs_mixed_f32": lst["iters"] / tts["f32"]["iters"],
        "training": {"pairs": len(pairs), "pair_generation_s": t_gen, "adam_steps": NET_STEPS,
                     "lr": NET_LR, "loss": "A-norm error relative to the solution's",
                     "training_s": t_train, "loss_first": float(loss_hist[0]),
                     "loss_last": float(loss_hist[-1]),
                     "break_even_solves_vs_mixed": (overhead / (t_mixed - lmed))
                     if lmed < t_mixed else None,
                     "amortised_per_solve_s_over_100_solves": overhead / 100.0}}

    network = {}
    for name, ts in net_times.items():
        avg = float(np.mean(ts))
        nb_ = NET_BYTES_PER_SITE[name]
        network[name] = {"avg_us": avg * 1e6, "model_bytes_per_site": nb_,
                         "model_GBps": nb_ * 2 * vh / avg / 1e9,
                         "frac_of_8TBps": nb_ * 2 * vh / avg / 1e9 / HBM_PEAK_GBS}
    network["lattice"] = list(DIMS)

    # achievable-bandwidth references (1 GiB read + 1 GiB written): the library's streaming
    # copy kernel and torch's elementwise add
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)

    def copy_rate(fn):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            fn()
        e1.record(stream)
        stream.synchronize()
        return 2 * src.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9

    copy_gbps = copy_rate(lambda: ks.stream_copy(dst, src))
    torch_gbps = copy_rate(lambda: torch.add(src, 1.0, out=dst))
    # the Dslash's bytes are ~98 % reads: the library's streaming read of the same 1 GiB is its
    # closer ceiling (copy_rate counts 2 GiB per call, so halve it)
    read_gbps = copy_rate(lambda: ks.stream_read(src)) / 2
    del src, dst
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(g, b)
    out = {
        "metric": "Dslash HBM GB/s; CG time-to-1e-10 residual, mixed/learned vs FP64, 32^4",
        "value": head["model_GBps"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "32^4 improved-staggered Dslash_eo + CG, m=0.01, H scale 0.5",
                   "lattice": list(DIMS), "mass": MASS, "tol": TOL, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": head["model_GBps"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": head["model_GBps"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic("f64_r18", tuned["f64_r18"]["threads"],
                                                 tuned["f64_r18"]["links_per_pass"],
                                                 tuned["f64_r18"]["link_access"],
                                                 tuned["f64_r18"]["staged"]),
                     "kernel": "dslash_kernel<F64,18,false,%d,%d,%s,%s>" % (
                         tuned["f64_r18"]["threads"], tuned["f64_r18"]["links_per_pass"],
                         "4-way" if tuned["f64_r18"]["link_access"] == 4 else "8-way",
                         "staged" if tuned["f64_r18"]["staged"] else "cached"),
                     "bytes_per_launch": model_bytes_per_site("f64", 18) * vh,
                     "copy_GBps": copy_gbps, "frac_of_copy": head["model_GBps"] / copy_gbps,
                     "read_GBps": read_gbps, "frac_of_read": head["model_GBps"] / read_gbps,
                     "torch_elementwise_GBps": torch_gbps},
        "dslash": dsl,
        "link_access_study": link_study,
        "link_construction": links,
        "time_to_solution": tts,
        "spectrum_32x32x32x32_m0.01": spectrum.get("f64"),
        "batch": batch,
        "multishift": msr,
        "network": network,
        "cpu_baseline": cpu,
    }
    if g5 is not None:
        del g, gm, bg
        t5 = time.time()
        out["learned_48x48x48x64"] = config5(g5, blocks5)
        log("48^3x64 learned workload in %.1f s" % (time.time() - t5))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
