// Conjugate-gradient solvers of (sigma - D_eo D_oe) x = b on even sites: single-mass CG with
// optional reduced-precision inner iterations under FP64 reliable updates, and multi-mass
// (multi-shift) CG (the routines of Sec. 3, benchmarked in Sec. 4).
//
// All scalars live on the device; the host only reads a small status block every
// `check_every` steps, so the queue of kernels never drains inside a solve.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "ks_batch.h"
#include "ks_blas.h"
#include "ks_device.h"
#include "ks_solvers.h"

namespace ks {

namespace {

size_t spinor_bytes(ks_prec_t p) { return p == KS_F64 ? 48 : p == KS_F32 ? 24 : 16; }

template <class T>
T* ws_vec(Workspace& w, T*& slot, size_t bytes)
{
    if (!slot) {
        slot = static_cast<T*>(device_alloc(bytes));
        w.bytes += bytes;
    }
    return slot;
}

}  // namespace

double dslash_model_bytes(ks_prec_t p, ks_recon_t r)
{
    const double real = p == KS_F64 ? 8 : p == KS_F32 ? 4 : 2;
    const double links = (r == KS_RECON_12) ? (8 * 18 + 8 * 12) * real : 16 * 18 * real;
    return links + 2 * (double)spinor_bytes(p);
}

double cg_iter_model_bytes(ks_prec_t p, ks_recon_t r)
{
    // two hopping terms, the xpay read of p, x read+write (FP64, or its FP32 increment in
    // reduced precision), r/p/q reads and the r write of the update, r/p reads and the p
    // write of p = r + beta p
    return 2 * dslash_model_bytes(p, r) + 8 * (double)spinor_bytes(p) + (p == KS_F64 ? 96 : 48);
}

Workspace& workspace(ks_gauge_t g)
{
    if (!g->ws) g->ws = new Workspace();
    Workspace& w = *g->ws;
    const int vh = g->geom.Vh;
    if (!w.partials) {
        w.npart = blocks_for(vh);
        const int cap = std::max(w.npart, dslash_max_blocks(g->geom));
        w.partials = static_cast<double*>(device_alloc(sizeof(double) * (cap + 64)));
        w.scal = w.partials + cap;
        w.bytes += sizeof(double) * (cap + 64);
        const int nrr = blocks_for(vh, kCgFuse);
        w.rr_part = static_cast<double*>(device_alloc(sizeof(double) * nrr));
        w.bytes += sizeof(double) * nrr;
        w.st = static_cast<CGState*>(device_alloc(sizeof(CGState)));
        KS_HIP(hipHostMalloc(reinterpret_cast<void**>(&w.st_host), sizeof(CGState)));
        KS_HIP(hipHostMalloc(reinterpret_cast<void**>(&w.host_scal), sizeof(double) * 64));
    }
    const size_t f64 = field_bytes(g->geom, KS_F64);
    ws_vec(w, w.b64, f64);
    ws_vec(w, w.x64, f64);
    ws_vec(w, w.r64, f64);
    ws_vec(w, w.t64, f64);
    ws_vec(w, w.ax64, f64);
    return w;
}

static void sloppy_vectors(ks_gauge_t g, Workspace& w, ks_prec_t p)
{
    const size_t b = field_bytes(g->geom, p);
    ws_vec(w, w.rs[p], b);
    ws_vec(w, w.ps[p], b);
    ws_vec(w, w.qs[p], b);
    ws_vec(w, w.ts[p], b);
    if (p != KS_F64) ws_vec(w, w.dx32, field_bytes(g->geom, KS_F32));
}

void workspace_free(Workspace* w)
{
    if (!w) return;
    device_free(w->partials);
    device_free(w->rr_part);
    device_free(w->cg_coef);
    device_free(w->st);
    if (w->st_host) (void)hipHostFree(w->st_host);
    if (w->host_scal) (void)hipHostFree(w->host_scal);
    device_free(w->b64);
    device_free(w->x64);
    device_free(w->r64);
    device_free(w->t64);
    device_free(w->ax64);
    for (int p = 0; p < 3; ++p) {
        device_free(w->rs[p]);
        device_free(w->ps[p]);
        device_free(w->qs[p]);
        device_free(w->ts[p]);
    }
    device_free(w->dx32);
    for (void* v : w->ms_x) device_free(v);
    for (void* v : w->ms_p) device_free(v);
    for (void* v : w->ms_dx) device_free(v);
    device_free(w->ms_r);
    device_free(w->ms_pb);
    device_free(w->ms_q);
    device_free(w->ms_t);
    device_free(w->ms_st);
    for (double* v : w->full) device_free(v);
    for (double* v : w->force_psi) device_free(v);
    for (BatchCtx* c : w->ms_batch) batch_free(c);
    for (double* v : w->ms_io) device_free(v);
    if (w->ms_st_host) (void)hipHostFree(w->ms_st_host);
    delete w;
}

// |v|^2 of an FP64 field, read back to the host (synchronises the stream).
double norm2_host(ks_gauge_t g, const double* v, hipStream_t s)
{
    Workspace& w = workspace(g);
    norm2_partials(g->geom.Vh, v, w.partials, s);
    finish_to(w.partials, w.npart, w.scal, s);
    KS_HIP(hipMemcpyAsync(w.host_scal, w.scal, sizeof(double), hipMemcpyDeviceToHost, s));
    KS_HIP(hipStreamSynchronize(s));
    return w.host_scal[0];
}

// ax = A_sigma x in FP64 (t64 as the odd temporary)
void apply_A64(ks_gauge_t g, double sigma, const double* x, double* ax, hipStream_t s,
               const int* gate)
{
    Workspace& w = workspace(g);
    DslashArgs a1;
    a1.out_parity = 1;
    a1.in = x;
    a1.out = w.t64;
    a1.gate = gate;
    dslash(g, KS_F64, KS_RECON_18, a1, s);
    DslashArgs a2;
    a2.out_parity = 0;
    a2.in = w.t64;
    a2.out = ax;
    a2.x = x;
    a2.a = sigma;
    a2.gate = gate;
    dslash(g, KS_F64, KS_RECON_18, a2, s);
}

// |b - A_sigma x|^2 on the host (r64 receives the residual).
double true_resid2(ks_gauge_t g, double sigma, const double* b, const double* x, hipStream_t s)
{
    Workspace& w = workspace(g);
    apply_A64(g, sigma, x, w.ax64, s, nullptr);
    sub_norm_partials(g->geom.Vh, b, w.ax64, w.r64, w.partials, s);
    finish_to(w.partials, w.npart, w.scal, s);
    KS_HIP(hipMemcpyAsync(w.host_scal, w.scal, sizeof(double), hipMemcpyDeviceToHost, s));
    KS_HIP(hipStreamSynchronize(s));
    return w.host_scal[0];
}

namespace {

void read_state(Workspace& w, hipStream_t s)
{
    KS_HIP(hipMemcpyAsync(w.st_host, w.st, sizeof(CGState), hipMemcpyDeviceToHost, s));
    KS_HIP(hipStreamSynchronize(s));
}

}  // namespace

// CG on internal FP64 planes: b (read), x (initial guess in, solution out).
void cg_coefficients(ks_gauge_t g, int n_max, double* alpha, double* beta, int* n)
{
    *n = 0;
    if (!g->ws || !g->ws->cg_coef) return;
    Workspace& w = *g->ws;
    const int k = std::min(n_max, w.cg_coef_n);
    if (k <= 0) return;
    std::vector<double> tmp(2 * (size_t)k);
    KS_HIP(hipMemcpy(tmp.data(), w.cg_coef, sizeof(double) * 2 * (size_t)k, hipMemcpyDeviceToHost));
    for (int j = 0; j < k; ++j) {
        alpha[j] = tmp[2 * j];
        beta[j] = tmp[2 * j + 1];
    }
    *n = k;
}

ks_status_t cg_core(ks_gauge_t g, double sigma, const double* b, double* x,
                    const ks_solver_params& prm, ks_solver_stats& stats, hipStream_t s)
{
    const auto t0 = std::chrono::steady_clock::now();
    Workspace& w = workspace(g);
    const Geom& G = g->geom;
    const int vh = G.Vh;
    const ks_prec_t P = prm.inner;
    const ks_recon_t RC = prm.recon;
    gauge_prepare(g, P, RC, s);
    sloppy_vectors(g, w, P);
    void* rs = (P == KS_F64) ? static_cast<void*>(w.r64) : w.rs[P];
    void* ps = w.ps[P];
    void* qs = w.qs[P];
    void* ts = w.ts[P];

    stats = ks_solver_stats();
    const double b2 = norm2_host(g, b, s);
    const double bnorm = std::sqrt(b2);
    if (bnorm == 0.0) {
        KS_HIP(hipMemsetAsync(x, 0, field_bytes(G, KS_F64), s));
        KS_HIP(hipStreamSynchronize(s));
        stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return KS_SUCCESS;
    }
    CGState init{};
    init.stop2 = (prm.tol * bnorm) * (prm.tol * bnorm);
    init.delta = (P == KS_F64) ? 0.0 : prm.delta;
    init.max_iter = prm.max_iter;
    init.gate = 1;
    *w.st_host = init;
    KS_HIP(hipMemcpyAsync(w.st, w.st_host, sizeof(CGState), hipMemcpyHostToDevice, s));

    // alpha_k, beta_k of every step (up to 2^20 of them), for the Lanczos estimate of the
    // spectrum from an unbroken FP64 run
    const int want = std::min(prm.max_iter, 1 << 20);
    if (w.cg_coef_cap < want) {
        device_free(w.cg_coef);
        w.cg_coef = nullptr;
        w.cg_coef_cap = 0;
        w.cg_coef = static_cast<double*>(device_alloc(sizeof(double) * 2 * (size_t)want));
        w.cg_coef_cap = want;
    }
    w.cg_coef_n = 0;
    // reduced precision: x's increments accumulate in FP32 and are added into the FP64 x
    // before every reliable update and at the end
    const bool sloppy = P != KS_F64;
    if (sloppy) KS_HIP(hipMemsetAsync(w.dx32, 0, field_bytes(G, KS_F32), s));
    void* xu = sloppy ? w.dx32 : static_cast<void*>(x);
    auto flush = [&]() {
        if (sloppy) flush_dx(vh, w.dx32, x, s);
    };
    auto reliable = [&](int initial) {
        flush();
        apply_A64(g, sigma, x, w.ax64, s, nullptr);
        sub_norm_partials(vh, b, w.ax64, w.r64, w.partials, s);
        cg_reliable(w.partials, w.npart, w.st, initial, s);
        if (P != KS_F64) convert_field(vh, KS_F64, w.r64, P, rs, nullptr, s);
    };
    auto iteration = [&]() {
        DslashArgs a1;
        a1.out_parity = 1;
        a1.in = ps;
        a1.out = ts;
        a1.gate = &w.st->gate;
        dslash(g, P, RC, a1, s);
        DslashArgs a2;
        a2.out_parity = 0;
        a2.in = ts;
        a2.out = qs;
        a2.x = ps;
        a2.a = sigma;
        a2.dot_partials = w.partials;
        a2.gate = &w.st->gate;
        dslash(g, P, RC, a2, s);
        cg_update(vh, P, xu, ps, qs, rs, w.st, w.partials, dslash_blocks(g, P, RC), w.rr_part,
                  w.cg_coef, w.cg_coef_cap, s);
        cg_beta_xpay(vh, P, rs, ps, w.st, w.rr_part, w.cg_coef, w.cg_coef_cap, s);
    };

    reliable(1);
    convert_field(vh, P, rs, P, ps, &w.st->gate, s);   // p = r
    int ru = 0, restarts = 0;
    ks_status_t result = KS_SUCCESS;
    const int chunk = std::max(1, prm.check_every);
    for (;;) {
        read_state(w, s);
        const CGState& h = *w.st_host;
        if (h.status != 0) {
            result = static_cast<ks_status_t>(h.status);
            set_error(result == KS_ERR_BREAKDOWN ? "CG breakdown: <p, A p> <= 0 at step %d"
                                                 : "non-finite value in CG at step %d",
                      h.iter);
            break;
        }
        if (h.done) break;
        if (h.ru_pending) {
            // the inner residual met the target (final check) or fell by delta: recompute
            // r = b - A x in FP64 and continue with beta = |r|^2 / rho
            const bool final_check = h.rho_new <= h.stop2;
            reliable(0);
            read_state(w, s);
            if (w.st_host->done || w.st_host->status != 0) continue;
            if (final_check) {
                if (++restarts > prm.max_restarts) {
                    result = KS_ERR_NOT_CONVERGED;
                    set_error("CG: true residual above tolerance after %d restarts", restarts - 1);
                    break;
                }
            } else {
                ++ru;
            }
            xpay(vh, P, rs, ps, w.st, s);
            continue;
        }
        if (h.iter >= prm.max_iter) {
            reliable(0);
            read_state(w, s);
            if (!w.st_host->done) {
                result = KS_ERR_NOT_CONVERGED;
                set_error("CG did not converge in %d steps", prm.max_iter);
            }
            break;
        }
        for (int k = 0; k < chunk; ++k) iteration();
    }
    flush();   // x = the last iterate also when the loop ended on an error
    read_state(w, s);
    const CGState& h = *w.st_host;
    w.cg_coef_n = std::min(h.iter, w.cg_coef_cap);
    stats.iters = h.iter;
    stats.reliable_updates = ru;
    stats.restarts = restarts;
    stats.true_rel_resid = std::sqrt(h.true_r2) / bnorm;
    stats.model_bytes = (double)h.iter * cg_iter_model_bytes(P, RC) * vh +
                        (ru + restarts + 1) * (2 * dslash_model_bytes(KS_F64, KS_RECON_18) + 192) * vh;
    stats.model_flops = (double)h.iter * (2 * 1146.0 + 12 + 60) * vh;
    stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return result;
}

}  // namespace ks
