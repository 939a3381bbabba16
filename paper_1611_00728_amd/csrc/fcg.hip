// Flexible CG preconditioned by the network N = L^+ L (Notay's flexible CG truncated to one
// previous direction), with the inner operator and vectors in FP32 (or FP64), x accumulated in
// FP64 (through FP32 increments between reliable updates in reduced precision), FP64 reliable
// updates, and plain CG as the fallback:
//
//   r = b - A x, z = N(r), p = z
//   repeat: q = A p, alpha = <p, r> / <p, q>, x += alpha p, r -= alpha q,
//           z = N(r), beta = -<z, q> / <p, q>, p = z + beta p
//
// A and N are Hermitian, so alpha and beta are real (the real parts of the products are
// taken); with N the identity this is CG step for step.  Every scalar lives on the device:
// the kernels of a step read a gate flag and do nothing once it is set (converged, reliable
// update due, or a fallback condition), so the host queues `check_every` steps at a time and
// reads a small status block per chunk.  Fallback to ks_cg_solve's method from the current x
// when N(r) is not finite, when <z, r> <= 0, when <p, A p> <= 0, when |r| has not halved over
// 50 steps, or at max_iter.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <utility>

#include "ks_blas.h"
#include "ks_device.h"
#include "ks_net.h"
#include "ks_solvers.h"

namespace ks {

namespace {

constexpr int kNT = 256;
constexpr int kFin = 1024;

// fallback reasons (ks_solver_stats.fallback)
enum { kNonFinite = 1, kNoDescent = 2, kBreakdown = 3, kStall = 4, kMaxIter = 5 };

struct FcgState {
    double pq;         // <p, A p>
    double alpha, beta;
    double rho;        // |r|^2 of the inner residual after the last step (as stored)
    double rho_new;
    double maxr;       // max |r| since the last reliable update
    double stop2;      // (tol |b|)^2
    double delta;      // reliable-update threshold (0: only the final check)
    double scale;      // network input scale sqrt(3 Vh / rho): O(1) entries for binary16
    double zr;         // <z, r>
    double true_r2;    // |b - A x|^2 of the last FP64 recomputation
    int vh;
    int iter, max_iter, gate, ru_pending, done, reason;
};

// Every block sums the partials itself in one fixed order, so all blocks agree bit for bit.
__device__ __forceinline__ double block_fused_sum(const double* __restrict__ in, int n)
{
    __shared__ double total;
    double t = 0.0;
    for (int k = threadIdx.x; k < n; k += kCgFuse) t += in[k];
    t = block_sum<kCgFuse>(t);
    if (threadIdx.x == 0) total = t;
    __syncthreads();
    return total;
}

__device__ __forceinline__ double one_block_sum(const double* __restrict__ in, int n)
{
    double t = 0.0;
    for (int k = threadIdx.x; k < n; k += kFin) t += in[k];
    return block_sum<kFin>(t);
}

// alpha = <p, r> / <p, q> from the partials of the previous p update and of the xpay Dslash;
// x += alpha p, r -= alpha q; partials of |r|^2 as stored.
template <int P>
__global__ __launch_bounds__(kCgFuse) void fcg_update_kernel(int vh, void* __restrict__ x,
                                                             const void* __restrict__ p,
                                                             const void* __restrict__ q,
                                                             void* __restrict__ r,
                                                             FcgState* __restrict__ st,
                                                             const double* __restrict__ pq_part,
                                                             int npq,
                                                             const double* __restrict__ pr_part,
                                                             int npr, double* __restrict__ rr_part)
{
    using R = typename St<P>::R;
    constexpr int kX = P == KS_F64 ? KS_F64 : KS_F32;
    using XR = typename St<kX>::R;
    __shared__ int gated;
    if (threadIdx.x == 0) gated = st->gate;
    __syncthreads();
    if (gated) return;
    const double pq = block_fused_sum(pq_part, npq);
    const double pr = block_fused_sum(pr_part, npr);
    const bool ok = isfinite(pq) && pq > 0.0 && isfinite(pr);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (lead) {
        st->pq = pq;
        if (ok) {
            st->alpha = pr / pq;
        } else {
            st->reason = isfinite(pq) && isfinite(pr) ? kBreakdown : kNonFinite;
            st->gate = 1;
        }
    }
    if (!ok) return;
    const double alpha = pr / pq;
    const int h = blockIdx.x * kCgFuse + threadIdx.x;
    double s = 0.0;
    if (h < vh) {
        cx<R> pv[3], qv[3], rv[3];
        cx<XR> xv[3];
        Spinor<P>::load(p, vh, h, pv);
        Spinor<P>::load(q, vh, h, qv);
        Spinor<P>::load(r, vh, h, rv);
        Spinor<kX>::load(x, vh, h, xv);
        const XR ax = (XR)alpha;
        const R a = (R)alpha;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            xv[k].r = fma(ax, (XR)pv[k].r, xv[k].r);
            xv[k].i = fma(ax, (XR)pv[k].i, xv[k].i);
            rv[k].r = fma(-a, qv[k].r, rv[k].r);
            rv[k].i = fma(-a, qv[k].i, rv[k].i);
        }
        Spinor<kX>::store(x, vh, h, xv);
        Spinor<P>::store(r, vh, h, rv);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            s += (double)rv[k].r * (double)rv[k].r + (double)rv[k].i * (double)rv[k].i;
    }
    s = block_sum<kCgFuse>(s);
    if (threadIdx.x == 0) rr_part[blockIdx.x] = s;
}

// |r|^2 after the update: stop for a reliable update (or the final check), at max_iter, or go
// on with the network's input scale for this r.
__global__ __launch_bounds__(kFin) void fcg_check_kernel(const double* __restrict__ rr_part, int n,
                                                         FcgState* __restrict__ st)
{
    if (st->gate) return;
    const double rn = one_block_sum(rr_part, n);
    if (threadIdx.x != 0) return;
    st->iter += 1;
    st->rho_new = rn;
    if (!isfinite(rn)) {
        st->reason = kNonFinite;
        st->gate = 1;
        return;
    }
    const double s = sqrt(rn);
    if (rn <= st->stop2 || s < st->delta * st->maxr) {
        st->ru_pending = 1;
        st->gate = 1;
        return;
    }
    st->rho = rn;
    st->maxr = fmax(st->maxr, s);
    st->scale = rn > 0.0 ? sqrt(3.0 * st->vh / rn) : 1.0;
    if (st->iter >= st->max_iter) {
        st->reason = kMaxIter;
        st->gate = 1;
    }
}

// partials of Re<z, r> and Re<z, q>
template <int P>
__global__ __launch_bounds__(kNT) void fcg_dots_kernel(int vh, const void* __restrict__ z,
                                                       const void* __restrict__ r,
                                                       const void* __restrict__ q,
                                                       const FcgState* __restrict__ st,
                                                       double* __restrict__ zr_part,
                                                       double* __restrict__ zq_part)
{
    using R = typename St<P>::R;
    if (st->gate) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (h < vh) {
        cx<R> zv[3], rv[3], qv[3];
        Spinor<P>::load(z, vh, h, zv);
        Spinor<P>::load(r, vh, h, rv);
        Spinor<P>::load(q, vh, h, qv);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            a += (double)zv[k].r * rv[k].r + (double)zv[k].i * rv[k].i;
            b += (double)zv[k].r * qv[k].r + (double)zv[k].i * qv[k].i;
        }
    }
    a = block_sum<kNT>(a);
    __syncthreads();
    b = block_sum<kNT>(b);
    if (threadIdx.x == 0) {
        zr_part[blockIdx.x] = a;
        zq_part[blockIdx.x] = b;
    }
}

// beta = -<z, q> / <p, q> (0 on the first step), p = z + beta p, and partials of Re<p, r> for
// the next step's alpha.  <z, r> must be finite and positive (N positive on r).
template <int P>
__global__ __launch_bounds__(kCgFuse) void fcg_p_kernel(int vh, const void* __restrict__ z,
                                                        const void* __restrict__ r,
                                                        void* __restrict__ p,
                                                        FcgState* __restrict__ st,
                                                        const double* __restrict__ zr_part,
                                                        const double* __restrict__ zq_part, int nz,
                                                        double* __restrict__ pr_part, int first)
{
    using R = typename St<P>::R;
    __shared__ int gated;
    if (threadIdx.x == 0) gated = st->gate;
    __syncthreads();
    if (gated) return;
    const double zr = block_fused_sum(zr_part, nz);
    const double zq = block_fused_sum(zq_part, nz);
    const double pq = st->pq;
    // on the first step q holds no A p yet: p = z, and <z, q> is not used
    const bool finite = isfinite(zr) && (first || isfinite(zq));
    const bool ok = finite && zr > 0.0;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const double beta = first ? 0.0 : -zq / pq;
    if (lead) {
        st->zr = zr;
        if (ok) {
            st->beta = beta;
        } else {
            st->reason = finite ? kNoDescent : kNonFinite;
            st->gate = 1;
        }
    }
    if (!ok) return;
    const int h = blockIdx.x * kCgFuse + threadIdx.x;
    double s = 0.0;
    if (h < vh) {
        cx<R> zv[3], rv[3], pv[3];
        Spinor<P>::load(z, vh, h, zv);
        Spinor<P>::load(r, vh, h, rv);
        if (first) {
#pragma unroll
            for (int k = 0; k < 3; ++k) pv[k] = zv[k];
        } else {
            Spinor<P>::load(p, vh, h, pv);
            const R b = (R)beta;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                pv[k].r = fma(b, pv[k].r, zv[k].r);
                pv[k].i = fma(b, pv[k].i, zv[k].i);
            }
        }
        Spinor<P>::store(p, vh, h, pv);
#pragma unroll
        for (int k = 0; k < 3; ++k) s += (double)pv[k].r * rv[k].r + (double)pv[k].i * rv[k].i;
    }
    s = block_sum<kCgFuse>(s);
    if (threadIdx.x == 0) pr_part[blockIdx.x] = s;
}

// After r = b - A x in FP64: converged, or go on from this residual.
__global__ __launch_bounds__(kFin) void fcg_reliable_kernel(const double* __restrict__ part, int n,
                                                            FcgState* __restrict__ st)
{
    const double r2 = one_block_sum(part, n);
    if (threadIdx.x != 0) return;
    st->true_r2 = r2;
    st->ru_pending = 0;
    if (!isfinite(r2)) {
        st->reason = kNonFinite;
        st->gate = 1;
        return;
    }
    if (r2 <= st->stop2) {
        st->done = 1;
        st->gate = 1;
        return;
    }
    st->rho = r2;
    st->maxr = sqrt(r2);
    st->scale = sqrt(3.0 * st->vh / r2);
    st->gate = 0;
    if (st->iter >= st->max_iter) {
        st->reason = kMaxIter;
        st->gate = 1;
    }
}

struct FcgBufs {
    void* z = nullptr;
    double* zr_part = nullptr;
    double* zq_part = nullptr;
    double* pr_part = nullptr;
    FcgState* st = nullptr;
    FcgState* st_host = nullptr;   // pinned
    int vh = 0;
    int prec = -1;
};

std::map<ks_gauge_t, FcgBufs> g_fcg;   // per gauge handle (freed with the handle)

void free_bufs(FcgBufs& fb)
{
    device_free(fb.z);
    device_free(fb.zr_part);
    device_free(fb.zq_part);
    device_free(fb.pr_part);
    device_free(fb.st);
    if (fb.st_host) (void)hipHostFree(fb.st_host);
    fb = FcgBufs();
}

template <int P>
void launch_step_kernels(int vh, void* xu, void* ps, void* qs, void* rs, FcgBufs& fb,
                         Workspace& w, int npq, hipStream_t s)
{
    const int nf = blocks_for(vh, kCgFuse);
    fcg_update_kernel<P><<<nf, kCgFuse, 0, s>>>(vh, xu, ps, qs, rs, fb.st, w.partials, npq,
                                                 fb.pr_part, nf, w.rr_part);
    fcg_check_kernel<<<1, kFin, 0, s>>>(w.rr_part, nf, fb.st);
    KS_HIP(hipGetLastError());
}

template <int P>
void launch_tail_kernels(int vh, void* zs, void* rs, void* qs, void* ps, FcgBufs& fb, int first,
                         hipStream_t s)
{
    const int nb = blocks_for(vh, kNT);
    const int nf = blocks_for(vh, kCgFuse);
    fcg_dots_kernel<P><<<nb, kNT, 0, s>>>(vh, zs, rs, qs, fb.st, fb.zr_part, fb.zq_part);
    fcg_p_kernel<P><<<nf, kCgFuse, 0, s>>>(vh, zs, rs, ps, fb.st, fb.zr_part, fb.zq_part, nb,
                                           fb.pr_part, first);
    KS_HIP(hipGetLastError());
}

}  // namespace

void fcg_release(ks_gauge_t g)
{
    auto it = g_fcg.find(g);
    if (it == g_fcg.end()) return;
    free_bufs(it->second);
    g_fcg.erase(it);
}

ks_status_t fcg_core(ks_gauge_t g, NetCtx& net, double sigma, const double* b, double* x,
                     const ks_solver_params& prm, int use_mfma, ks_solver_stats& stats,
                     hipStream_t s)
{
    const auto t0 = std::chrono::steady_clock::now();
    Workspace& w = workspace(g);
    const Geom& G = g->geom;
    const int vh = G.Vh;
    const ks_prec_t P = prm.inner == KS_F16 ? KS_F32 : prm.inner;   // network output is FP32
    const ks_recon_t RC = prm.recon;
    gauge_prepare(g, P, RC, s);
    gauge_prepare(g, KS_F32, KS_RECON_18, s);
    FcgBufs& fb = g_fcg[g];
    if (fb.vh != vh || fb.prec != (int)P) {
        free_bufs(fb);
        fb.z = device_alloc(field_bytes(G, P));
        fb.zr_part = static_cast<double*>(device_alloc(sizeof(double) * blocks_for(vh, kNT)));
        fb.zq_part = static_cast<double*>(device_alloc(sizeof(double) * blocks_for(vh, kNT)));
        fb.pr_part = static_cast<double*>(device_alloc(sizeof(double) * blocks_for(vh, kCgFuse)));
        fb.st = static_cast<FcgState*>(device_alloc(sizeof(FcgState)));
        KS_HIP(hipHostMalloc(reinterpret_cast<void**>(&fb.st_host), sizeof(FcgState)));
        fb.vh = vh;
        fb.prec = (int)P;
    }
    const size_t fbytes = field_bytes(G, P);
    for (void** v : {&w.rs[P], &w.ps[P], &w.qs[P], &w.ts[P]})
        if (!*v) {
            *v = device_alloc(fbytes);
            w.bytes += fbytes;
        }
    const bool sloppy = P != KS_F64;
    if (sloppy && !w.dx32) {
        w.dx32 = device_alloc(field_bytes(G, KS_F32));
        w.bytes += field_bytes(G, KS_F32);
    }
    void* rs = (P == KS_F64) ? static_cast<void*>(w.r64) : w.rs[P];
    void* ps = w.ps[P];
    void* qs = w.qs[P];
    void* ts = w.ts[P];
    void* zs = fb.z;
    void* xu = sloppy ? w.dx32 : static_cast<void*>(x);
    FcgState* st = fb.st;
    FcgState* hs = fb.st_host;

    stats = ks_solver_stats();
    const double b2 = norm2_host(g, b, s);
    const double bnorm = std::sqrt(b2);
    if (bnorm == 0.0) {
        KS_HIP(hipMemsetAsync(x, 0, field_bytes(G, KS_F64), s));
        KS_HIP(hipStreamSynchronize(s));
        return KS_SUCCESS;
    }
    FcgState init{};
    init.stop2 = prm.tol * prm.tol * b2;
    init.delta = sloppy ? prm.delta : 0.0;
    init.max_iter = prm.max_iter;
    init.vh = vh;
    init.gate = 1;
    *hs = init;
    KS_HIP(hipMemcpyAsync(st, hs, sizeof(FcgState), hipMemcpyHostToDevice, s));
    if (sloppy) KS_HIP(hipMemsetAsync(w.dx32, 0, field_bytes(G, KS_F32), s));

    auto read_state = [&]() {
        KS_HIP(hipMemcpyAsync(hs, st, sizeof(FcgState), hipMemcpyDeviceToHost, s));
        KS_HIP(hipStreamSynchronize(s));
    };
    auto flush = [&]() {
        if (sloppy) flush_dx(vh, w.dx32, x, s);
    };
    // r = b - A x in FP64 (after adding x's FP32 increments), into the inner r
    auto reliable = [&]() {
        flush();
        apply_A64(g, sigma, x, w.ax64, s, nullptr);
        sub_norm_partials(vh, b, w.ax64, w.r64, w.partials, s);
        fcg_reliable_kernel<<<1, kFin, 0, s>>>(w.partials, w.npart, st);
        KS_HIP(hipGetLastError());
        if (sloppy) convert_field(vh, KS_F64, w.r64, P, rs, &st->gate, s);
    };
    // z = N(r), the dot products, and the new direction
    auto tail = [&](int first) {
        net_apply_spinor(net, g, P, rs, zs, &st->scale, &st->gate, use_mfma, s);
        if (P == KS_F64) launch_tail_kernels<KS_F64>(vh, zs, rs, qs, ps, fb, first, s);
        else launch_tail_kernels<KS_F32>(vh, zs, rs, qs, ps, fb, first, s);
    };
    auto step = [&]() {
        DslashArgs a1;
        a1.out_parity = 1;
        a1.in = ps;
        a1.out = ts;
        a1.gate = &st->gate;
        dslash(g, P, RC, a1, s);
        DslashArgs a2;
        a2.out_parity = 0;
        a2.in = ts;
        a2.out = qs;
        a2.x = ps;
        a2.a = sigma;
        a2.dot_partials = w.partials;
        a2.gate = &st->gate;
        dslash(g, P, RC, a2, s);
        const int npq = dslash_blocks(g, P, RC);
        if (P == KS_F64) launch_step_kernels<KS_F64>(vh, xu, ps, qs, rs, fb, w, npq, s);
        else launch_step_kernels<KS_F32>(vh, xu, ps, qs, rs, fb, w, npq, s);
        tail(0);
    };

    reliable();
    tail(1);
    int ru = 0, restarts = 0;
    ks_status_t rc = KS_SUCCESS;
    int reason = 0;
    const int chunk = std::max(1, prm.check_every);
    std::deque<std::pair<int, double>> hist;   // (step, |r|) at each host read
    for (;;) {
        read_state();
        if (hs->done) break;
        if (hs->reason) {
            reason = hs->reason;
            break;
        }
        if (hs->ru_pending) {
            const bool final_check = hs->rho_new <= hs->stop2;
            reliable();
            read_state();
            if (hs->done) break;
            if (hs->reason) {
                reason = hs->reason;
                break;
            }
            if (final_check) {
                if (++restarts > prm.max_restarts) {
                    rc = KS_ERR_NOT_CONVERGED;
                    set_error("flexible CG: true residual above tolerance after %d restarts",
                              restarts - 1);
                    break;
                }
            } else {
                ++ru;
            }
            hist.clear();
            tail(0);
            continue;
        }
        // |r| must halve over any 50 steps
        hist.emplace_back(hs->iter, std::sqrt(hs->rho));
        while (hist.size() > 1 && hist.back().first - hist[1].first >= 50) hist.pop_front();
        if (hist.back().first - hist.front().first >= 50 &&
            hist.back().second > 0.5 * hist.front().second) {
            reason = kStall;
            break;
        }
        for (int k = 0; k < chunk; ++k) step();
    }
    flush();   // x = the last iterate also when the loop stopped for a fallback
    read_state();
    const int it = hs->iter;
    double true_r2 = hs->true_r2;
    int fb_iters = 0;
    if (reason && rc == KS_SUCCESS) {
        ks_solver_params q = prm;
        q.max_iter = std::max(1, prm.max_iter - it);
        ks_solver_stats cs;
        rc = cg_core(g, sigma, b, x, q, cs, s);
        fb_iters = cs.iters;
        ru += cs.reliable_updates;
        true_r2 = cs.true_rel_resid * cs.true_rel_resid * b2;
    }
    stats.iters = it + fb_iters;
    stats.reliable_updates = ru;
    stats.restarts = fb_iters;        // steps taken by the fallback CG
    stats.fallback = reason;
    stats.true_rel_resid = std::sqrt(true_r2 / b2);
    // per flexible step: the CG step's bytes, one network application (with its input and
    // output vectors) and the two dot products (z, r, q) and the p update (z, r, p read, p
    // written)
    const double sb = (double)field_bytes(G, P) / vh;
    stats.model_bytes = (double)it * vh *
                            (cg_iter_model_bytes(P, RC) + net_model_bytes(use_mfma, sb) + 3 * sb +
                             4 * sb) +
                        (ru + restarts + 1) * (2 * dslash_model_bytes(KS_F64, KS_RECON_18) + 192) * vh;
    stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

}  // namespace ks
