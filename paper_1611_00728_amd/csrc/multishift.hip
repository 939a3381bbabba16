// Multi-mass (multi-shift) CG: (sigma_i - D_eo D_oe) x_i = b for all shifts in one Krylov
// space (the multi-mass CG of Sec. 3 and Sec. 4), then FP64-checked per-shift refinement.
//
// Base system A_0 = sigma_0 - D_eo D_oe with sigma_0 = min sigma_i; delta_i = sigma_i - sigma_0.
// Per step, with the base CG's alpha, beta:
//   zeta_i' = zeta_i zeta_i^- alpha^- / (alpha beta^- (zeta_i^- - zeta_i)
//                                        + zeta_i^- alpha^- (1 + delta_i alpha))
//   alpha_i = alpha zeta_i' / zeta_i,  beta_i = beta (zeta_i' / zeta_i)^2,
//   x_i += alpha_i p_i,  p_i = zeta_i' r + beta_i p_i  (one fused kernel for all shifts),
// which keeps r_i = zeta_i r.  Shift i freezes once zeta_i^2 |r|^2 <= (tol_i |b|)^2.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "ks_batch.h"
#include "ks_blas.h"
#include "ks_device.h"
#include "ks_solvers.h"
#include "ks_stream.h"

namespace ks {

namespace {

constexpr int kMaxShift = 32;

struct MSState {
    double rho, alpha, alpha_prev, beta, beta_prev, pAp;
    double maxr, ru_delta;   // reliable updates of the base residual (ru_delta 0: none)
    int iter, max_iter, gate, stop_next, status, nactive, nshift, ru_pending, base;
    double delta[kMaxShift], stop2[kMaxShift];
    double zeta[kMaxShift], zeta_prev[kMaxShift];
    double alpha_i[kMaxShift];
    int active[kMaxShift], upd[kMaxShift];
    // taken by the residual kernel's lead for the update kernel, whose own lead rewrites the
    // live fields while its other blocks still read these: rho, the step's gate and count,
    // zeta_i before and after the step
    double s_rho;
    int s_gate, s_iter;
    double s_zeta[kMaxShift], s_zn[kMaxShift];
};

struct ShiftPtrs {
    double2* x[kMaxShift];
    void* p[kMaxShift];    // p[base] is the base direction
    void* dx[kMaxShift];   // FP32 increments of x_i since the last flush (reduced precision)
    int base;              // index of the smallest shift, whose system is the base system
};

// Every block adds up the previous kernel's partial sums itself (thread t adds t, t + NT, ...,
// then the fixed block tree), so all blocks hold the same total bit for bit.
template <int NT>
__device__ __forceinline__ double block_total(const double* __restrict__ in, int n)
{
    __shared__ double total;
    double t = 0.0;
    for (int k = threadIdx.x; k < n; k += NT) t += in[k];
    t = block_sum<NT>(t);
    if (threadIdx.x == 0) total = t;
    __syncthreads();
    return total;
}

// alpha = rho / <p, A p> from the hopping term's partials, r -= alpha q, partials of |r|^2 as
// stored.  The lead thread alone writes the state: per shift the step's zeta', alpha_i and
// whether the shift is updated, and the copies that the update kernel decides from.
template <int P>
__global__ __launch_bounds__(kCgFuse) void ms_r_kernel(int vh, const void* __restrict__ q,
                                                       void* __restrict__ r,
                                                       MSState* __restrict__ st,
                                                       const double* __restrict__ pap_part,
                                                       int npap, double* __restrict__ rr_part)
{
    using R = typename St<P>::R;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    // one read of the gate per block: only this kernel's lead can set it (on breakdown), and
    // a block that sees that skips the step as the breakdown test would
    __shared__ int gated;
    if (threadIdx.x == 0) gated = st->gate;
    __syncthreads();
    if (gated) {
        if (lead) st->s_gate = 1;
        return;
    }
    const double pap = block_total<kCgFuse>(pap_part, npap);
    const double rho = st->rho;
    const bool ok = isfinite(pap) && pap > 0.0;
    if (lead) {
        st->pAp = pap;
        st->s_gate = ok ? 0 : 1;
        if (!ok) {
            st->status = isfinite(pap) ? KS_ERR_BREAKDOWN : KS_ERR_NONFINITE;
            st->gate = 1;
        } else {
            const double a = rho / pap;
            st->alpha = a;
            st->s_rho = rho;
            st->s_iter = st->iter;
            for (int i = 0; i < st->nshift; ++i) {
                // the base shift's solution keeps being updated while any shift iterates: the
                // base reliable update recomputes r from it, and every shifted residual is
                // zeta_i r
                st->upd[i] = st->active[i] || i == st->base;
                if (!st->upd[i]) continue;
                const double z = st->zeta[i], zp = st->zeta_prev[i];
                const double zn =
                    z * zp * st->alpha_prev /
                    (a * st->beta_prev * (zp - z) + zp * st->alpha_prev * (1.0 + st->delta[i] * a));
                st->alpha_i[i] = a * zn / z;
                st->s_zeta[i] = z;
                st->s_zn[i] = zn;
            }
        }
    }
    if (!ok) return;
    const R a = (R)(rho / pap);
    const int h = blockIdx.x * kCgFuse + threadIdx.x;
    double sum = 0.0;
    if (h < vh) {
        cx<R> qv[3], rv[3];
        Spinor<P>::load(q, vh, h, qv);
        Spinor<P>::load(r, vh, h, rv);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            rv[k].r = fma(-a, qv[k].r, rv[k].r);
            rv[k].i = fma(-a, qv[k].i, rv[k].i);
        }
        Spinor<P>::store(r, vh, h, rv);
        Spinor<P>::round(rv);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            sum += (double)rv[k].r * (double)rv[k].r + (double)rv[k].i * (double)rv[k].i;
    }
    sum = block_sum<kCgFuse>(sum);
    if (threadIdx.x == 0) rr_part[blockIdx.x] = sum;
}

// x_i += alpha_i p_i; p_i = zeta_i r + beta_i p_i for every shift updated this step, and the
// base direction p = r + beta p.  r and p are read once per site for all shifts.  The base
// shift (delta = 0) keeps zeta = 1, alpha_i = alpha and beta_i = beta exactly, so its p_i is
// the base p itself: it is neither loaded nor stored separately.  Loads of a group of shifts
// are issued before any of the group's stores, so that a wave has several in flight.  In
// reduced precision the x_i increments go to FP32 fields that are added into the FP64 x_i at
// every reliable update of the base and at the end (half the bytes of an FP64
// read-modify-write).  The shifts' own vectors (x_i or its increments, p_i) are touched once
// per step: read and written streamed, they do not push the base direction p, which the next
// hopping term gathers from its 16 neighbours, out of the caches.
// The step's scalars come first: every block sums the residual kernel's |r|^2 partials
// itself and forms beta = |r|^2 / rho and per shift beta_i = beta (zeta_i' / zeta_i)^2 from
// the copies that kernel's lead took; the lead thread alone commits the live state (zeta_i,
// frozen shifts, the step count, the base's reliable-update and stop decisions, the gate).
template <int P>
__global__ __launch_bounds__(kBlock) void ms_update_kernel(int vh, const void* __restrict__ r,
                                                           void* __restrict__ pb, ShiftPtrs sp,
                                                           MSState* __restrict__ st,
                                                           const double* __restrict__ rr_part,
                                                           int nrr)
{
    using R = typename St<P>::R;
    constexpr bool kSloppy = P != KS_F64;
    constexpr int kX = kSloppy ? KS_F32 : KS_F64;
    using XR = typename St<kX>::R;
    constexpr int G = kSloppy ? 4 : 3;
    if (st->s_gate) return;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const double rn = block_total<kBlock>(rr_part, nrr);
    if (!isfinite(rn)) {
        if (lead) {
            st->status = KS_ERR_NONFINITE;
            st->gate = 1;
        }
        return;
    }
    const int ns = st->nshift;
    const double beta = rn / st->s_rho;
    __shared__ XR sh_ai[kMaxShift];
    __shared__ R sh_bi[kMaxShift], sh_zi[kMaxShift];
    __shared__ int sh_upd[kMaxShift];
    if (threadIdx.x < ns) {
        const int i = threadIdx.x;
        const int u = st->upd[i];
        sh_upd[i] = u;
        if (u) {
            const double zn = st->s_zn[i];
            const double ratio = zn / st->s_zeta[i];
            sh_ai[i] = (XR)st->alpha_i[i];
            sh_bi[i] = (R)(beta * ratio * ratio);
            sh_zi[i] = (R)zn;
        }
    }
    if (lead) {
        const int iter = st->s_iter + 1;
        st->beta = beta;
        st->iter = iter;
        for (int i = 0; i < ns; ++i) {
            if (!st->upd[i]) continue;
            const double zn = st->s_zn[i];
            st->zeta_prev[i] = st->s_zeta[i];
            st->zeta[i] = zn;
            if (st->active[i] && zn * zn * rn <= st->stop2[i]) {
                st->active[i] = 0;
                st->nactive -= 1;
            }
        }
        st->alpha_prev = st->alpha;
        st->beta_prev = beta;
        st->rho = rn;
        if (st->nactive == 0 || iter >= st->max_iter) st->stop_next = 1;
        // reliable update of the base residual when it fell by ru_delta since the last one
        const double sr = sqrt(rn);
        if (st->ru_delta > 0.0 && sr < st->ru_delta * st->maxr) st->ru_pending = 1;
        st->maxr = fmax(st->maxr, sr);
        if (st->stop_next || st->ru_pending) st->gate = 1;
    }
    __syncthreads();
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
    cx<R> rv[3], bv[3];
    Spinor<P>::load(r, vh, h, rv);
    Spinor<P>::load(pb, vh, h, bv);
    for (int i0 = 0; i0 < ns; i0 += G) {
        cx<R> pv[G][3];
        cx<XR> xv[G][3];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int i = i0 + j;
            if (i >= ns || !sh_upd[i]) continue;
            if (i == sp.base) {
#pragma unroll
                for (int k = 0; k < 3; ++k) pv[j][k] = bv[k];
            } else {
                Streamed<P>::load(sp.p[i], vh, h, pv[j]);
            }
            Streamed<kX>::load(kSloppy ? sp.dx[i] : sp.x[i], vh, h, xv[j]);
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int i = i0 + j;
            if (i >= ns || !sh_upd[i]) continue;
            const XR ai = sh_ai[i];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                xv[j][k].r = fma(ai, (XR)pv[j][k].r, xv[j][k].r);
                xv[j][k].i = fma(ai, (XR)pv[j][k].i, xv[j][k].i);
            }
            Streamed<kX>::store(kSloppy ? sp.dx[i] : sp.x[i], vh, h, xv[j]);
            if (i == sp.base) continue;
            const R bi = sh_bi[i], zi = sh_zi[i];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                pv[j][k].r = fma(bi, pv[j][k].r, zi * rv[k].r);
                pv[j][k].i = fma(bi, pv[j][k].i, zi * rv[k].i);
            }
            Streamed<P>::store(sp.p[i], vh, h, pv[j]);
        }
    }
    const R b = (R)beta;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        bv[k].r = fma(b, bv[k].r, rv[k].r);
        bv[k].i = fma(b, bv[k].i, rv[k].i);
    }
    Spinor<P>::store(pb, vh, h, bv);
}

// x_i += dx_i (FP64), dx_i = 0, for every shift
__global__ __launch_bounds__(kBlock) void ms_flush_kernel(int vh, int nshift, ShiftPtrs sp)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
    const cx<float> zero[3] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
    for (int i = 0; i < nshift; ++i) {
        cx<float> d[3];
        Spinor<KS_F32>::load(sp.dx[i], vh, h, d);
        double2* x = sp.x[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double2 t = x[k * vh + h];
            t.x += (double)d[k].r;
            t.y += (double)d[k].i;
            x[k * vh + h] = t;
        }
        Spinor<KS_F32>::store(sp.dx[i], vh, h, zero);
    }
}

template <int P>
void launch_r(int vh, const void* q, void* r, MSState* st, const double* pap_part, int npap,
              double* rr_part, hipStream_t s)
{
    ms_r_kernel<P><<<blocks_for(vh, kCgFuse), kCgFuse, 0, s>>>(vh, q, r, st, pap_part, npap,
                                                                rr_part);
}

template <int P>
void launch_upd(int vh, const void* r, void* pb, const ShiftPtrs& sp, MSState* st,
                const double* rr_part, hipStream_t s)
{
    ms_update_kernel<P><<<blocks_for(vh), kBlock, 0, s>>>(vh, r, pb, sp, st, rr_part,
                                                          blocks_for(vh, kCgFuse));
}

}  // namespace

double multishift_iter_model_bytes(ks_prec_t p, ks_recon_t r, int nactive, bool base_active)
{
    const double sb = p == KS_F64 ? 48 : p == KS_F32 ? 24 : 16;
    // A-apply (two hopping terms + xpay read), r update (q, r read, r write), fused update
    // (r, p read, p write; per shift p_i read/write and x_i read/write: FP64, or its FP32
    // increments in reduced precision; the base shift's p_i is p)
    const double xb = p == KS_F64 ? 96 : 48;
    const int np = nactive - (base_active ? 1 : 0);
    return 2 * dslash_model_bytes(p, r) + sb + 3 * sb + 3 * sb + nactive * xb + np * 2 * sb;
}

ks_status_t multishift_core(ks_gauge_t g, int nshift, const double* sigma, const double* b,
                            double* const* x, const double* tol, const ks_solver_params& prm,
                            ks_solver_stats* stats, hipStream_t s)
{
    const auto t0 = std::chrono::steady_clock::now();
    KS_REQUIRE(nshift >= 1 && nshift <= kMaxShift, KS_ERR_ARG, "nshift must be in [1, %d]",
               kMaxShift);
    for (int i = 0; i < nshift; ++i) {
        KS_REQUIRE(sigma[i] >= 0 && std::isfinite(sigma[i]), KS_ERR_ARG, "shift %d is negative", i);
        KS_REQUIRE(tol[i] > 0, KS_ERR_ARG, "tolerance of shift %d must be positive", i);
        KS_REQUIRE(x[i] != nullptr, KS_ERR_ARG, "solution pointer %d is null", i);
    }
    Workspace& w = workspace(g);
    const Geom& G = g->geom;
    const int vh = G.Vh;
    const ks_prec_t P = prm.inner;
    const ks_recon_t RC = prm.recon;
    gauge_prepare(g, P, RC, s);
    const size_t fb = field_bytes(G, P);
    if (w.ms_prec != (int)P) {
        for (void* v : w.ms_p) device_free(v);
        w.ms_p.clear();
        device_free(w.ms_r);
        device_free(w.ms_pb);
        device_free(w.ms_q);
        device_free(w.ms_t);
        w.ms_r = device_alloc(fb);
        w.ms_pb = device_alloc(fb);
        w.ms_q = device_alloc(fb);
        w.ms_t = device_alloc(fb);
        w.ms_prec = (int)P;
    }
    while ((int)w.ms_p.size() < nshift) w.ms_p.push_back(device_alloc(fb));
    const bool sloppy = P != KS_F64;
    if (sloppy)
        while ((int)w.ms_dx.size() < nshift) w.ms_dx.push_back(device_alloc(field_bytes(G, KS_F32)));
    if (!w.ms_st) {
        w.ms_st = device_alloc(sizeof(MSState));
        KS_HIP(hipHostMalloc(&w.ms_st_host, sizeof(MSState)));
    }
    MSState* st = static_cast<MSState*>(w.ms_st);
    MSState* hs = static_cast<MSState*>(w.ms_st_host);

    double s0 = sigma[0];
    int i0 = 0;
    for (int i = 1; i < nshift; ++i)
        if (sigma[i] < s0) {
            s0 = sigma[i];
            i0 = i;
        }

    // r = p = p_i = b in the inner precision, x_i = 0
    convert_field(vh, KS_F64, b, P, w.ms_r, nullptr, s);
    convert_field(vh, KS_F64, b, P, w.ms_pb, nullptr, s);
    ShiftPtrs sp{};
    sp.base = i0;
    for (int i = 0; i < nshift; ++i) {
        if (i != i0) convert_field(vh, KS_F64, b, P, w.ms_p[i], nullptr, s);
        KS_HIP(hipMemsetAsync(x[i], 0, field_bytes(G, KS_F64), s));
        sp.x[i] = reinterpret_cast<double2*>(x[i]);
        sp.p[i] = i == i0 ? w.ms_pb : w.ms_p[i];
        if (sloppy) {
            sp.dx[i] = w.ms_dx[i];
            KS_HIP(hipMemsetAsync(w.ms_dx[i], 0, field_bytes(G, KS_F32), s));
        }
    }
    auto flush = [&]() {
        if (!sloppy) return;
        ms_flush_kernel<<<blocks_for(vh), kBlock, 0, s>>>(vh, nshift, sp);
        KS_HIP(hipGetLastError());
    };
    const double b2 = norm2_host(g, b, s);
    convert_field(vh, P, w.ms_r, KS_F64, w.r64, nullptr, s);
    const double r2 = norm2_host(g, static_cast<const double*>(w.r64), s);

    std::memset(hs, 0, sizeof(MSState));
    hs->rho = r2;
    hs->alpha_prev = 1.0;
    hs->beta_prev = 0.0;
    hs->maxr = std::sqrt(r2);
    hs->ru_delta = (P == KS_F64) ? 0.0 : prm.delta;
    hs->max_iter = prm.max_iter;
    hs->nshift = nshift;
    hs->nactive = nshift;
    hs->base = i0;
    for (int i = 0; i < nshift; ++i) {
        hs->delta[i] = sigma[i] - s0;
        hs->stop2[i] = tol[i] * tol[i] * b2;
        hs->zeta[i] = hs->zeta_prev[i] = 1.0;
        hs->active[i] = 1;
    }
    if (b2 == 0.0) {
        hs->gate = 1;
        hs->nactive = 0;
    }
    KS_HIP(hipMemcpyAsync(st, hs, sizeof(MSState), hipMemcpyHostToDevice, s));

    const int chunk = std::max(1, prm.check_every);
    ks_status_t result = KS_SUCCESS;
    auto iteration = [&]() {
        DslashArgs a1;
        a1.out_parity = 1;
        a1.in = w.ms_pb;
        a1.out = w.ms_t;
        a1.gate = &st->gate;
        dslash(g, P, RC, a1, s);
        DslashArgs a2;
        a2.out_parity = 0;
        a2.in = w.ms_t;
        a2.out = w.ms_q;
        a2.x = w.ms_pb;
        a2.a = s0;
        a2.dot_partials = w.partials;
        a2.gate = &st->gate;
        dslash(g, P, RC, a2, s);
        const int npap = dslash_blocks(g, P, RC);
        if (P == KS_F64) launch_r<KS_F64>(vh, w.ms_q, w.ms_r, st, w.partials, npap, w.rr_part, s);
        else if (P == KS_F32) launch_r<KS_F32>(vh, w.ms_q, w.ms_r, st, w.partials, npap, w.rr_part, s);
        else launch_r<KS_F16>(vh, w.ms_q, w.ms_r, st, w.partials, npap, w.rr_part, s);
        if (P == KS_F64) launch_upd<KS_F64>(vh, w.ms_r, w.ms_pb, sp, st, w.rr_part, s);
        else if (P == KS_F32) launch_upd<KS_F32>(vh, w.ms_r, w.ms_pb, sp, st, w.rr_part, s);
        else launch_upd<KS_F16>(vh, w.ms_r, w.ms_pb, sp, st, w.rr_part, s);
        KS_HIP(hipGetLastError());
    };
    double model_bytes = 0.0;
    int last_iter = 0;
    int ms_ru = 0;
    bool rolled_back = false;
    for (;;) {
        KS_HIP(hipMemcpyAsync(hs, st, sizeof(MSState), hipMemcpyDeviceToHost, s));
        KS_HIP(hipStreamSynchronize(s));
        // the base shift's vectors are updated while any shift iterates
        const int nupd = hs->nactive + (hs->nactive > 0 && !hs->active[i0] ? 1 : 0);
        model_bytes += (hs->iter - last_iter) * multishift_iter_model_bytes(P, RC, nupd, true) * vh;
        last_iter = hs->iter;
        if (hs->status != 0) {
            if (sloppy) {
                // the reduced-precision recursion broke down (a non-finite value, or
                // <p, A p> <= 0 from rounding): the x_i increments since the last reliable
                // update are dropped, every x_i goes back to its FP64 value at that update, and
                // the FP64 check below sends each shift to the refinement
                rolled_back = true;
                break;
            }
            result = static_cast<ks_status_t>(hs->status);
            set_error("multi-shift CG: %s at step %d",
                      result == KS_ERR_BREAKDOWN ? "breakdown" : "non-finite value", hs->iter);
            break;
        }
        if (hs->stop_next) break;
        if (hs->ru_pending) {
            // r = b - A_0 x_0 in FP64 for the base (smallest) shift; the shifted systems keep
            // r_i = zeta_i r with the recomputed r
            flush();
            apply_A64(g, s0, x[i0], w.ax64, s, nullptr);
            sub_norm_partials(vh, b, w.ax64, w.r64, w.partials, s);
            finish_to(w.partials, w.npart, w.scal, s);
            convert_field(vh, KS_F64, w.r64, P, w.ms_r, nullptr, s);
            KS_HIP(hipMemcpyAsync(w.host_scal, w.scal, sizeof(double), hipMemcpyDeviceToHost, s));
            KS_HIP(hipStreamSynchronize(s));
            hs->rho = w.host_scal[0];
            hs->maxr = std::sqrt(hs->rho);
            hs->ru_pending = 0;
            hs->gate = 0;
            ++ms_ru;
            KS_HIP(hipMemcpyAsync(st, hs, sizeof(MSState), hipMemcpyHostToDevice, s));
        } else if (hs->gate) {
            break;
        }
        for (int k = 0; k < chunk; ++k) iteration();
    }
    const int ms_iters = hs->iter;
    if (!rolled_back) flush();

    // FP64 verdict per shift; refine the ones above target from x_i.  In reduced precision with
    // at least two shifts besides the base, those go to the batched refinement unchecked: its
    // first step computes every pair's FP64 residual anyway and finishes the pairs already at
    // target, so a separate FP64 A-apply per shift here would only repeat it.
    const bool batch_all = P != KS_F64 && nshift >= 3 && b2 > 0;
    std::vector<int> need;
    for (int i = 0; i < nshift; ++i) {
        ks_solver_stats& o = stats[i];
        o = ks_solver_stats();
        o.iters = ms_iters;
        o.reliable_updates = ms_ru;
        o.model_bytes = model_bytes / nshift;
        if (result != KS_SUCCESS) continue;
        if (batch_all && i != i0) {
            need.push_back(i);
            continue;
        }
        const double tr2 = true_resid2(g, sigma[i], b, x[i], s);
        o.true_rel_resid = b2 > 0 ? std::sqrt(tr2 / b2) : 0.0;
        if (b2 > 0 && tr2 > tol[i] * tol[i] * b2) need.push_back(i);
    }
    if (need.size() >= 2 && P != KS_F64) {
        // reduced-precision refinement of several shifts at once: a batched CG on this lattice
        // with one right-hand side per shift (its own shift, scalars and FP64 reliable
        // updates) loads every link once for all of them.  Lighter shifts (the slowest) go
        // first so that each group's members take similar step counts.  Its inner iterations
        // are binary16 whatever the shared phase's precision: from the shared phase's
        // residual they take the same step counts as FP32 ones (32^3x48, nine shifts) on
        // half the bytes (FP32 solve 0.425 -> 0.396 s)
        constexpr ks_prec_t RP = KS_F16;
        const double rsb = 16;          // bytes of one binary16 colour vector record
        std::sort(need.begin(), need.end(), [&](int a, int c) { return sigma[a] < sigma[c]; });
        const size_t fb = field_bytes(G, KS_F64);
        while (w.ms_io.size() < 6) {
            w.ms_io.push_back(static_cast<double*>(device_alloc(fb)));
            w.bytes += fb;
        }
        double* bb = w.ms_io[0];        // b in the boundary layout
        double* zero = w.ms_io[1];      // padding pair: zero source, scratch solution
        export_field(G, KS_F64, b, bb, s);
        for (size_t g0 = 0; g0 < need.size(); g0 += 4) {
            const int n = (int)std::min<size_t>(4, need.size() - g0);
            const int R = n <= 2 ? 2 : 4;
            const int ri = R == 2 ? 1 : 2;
            if (!w.ms_batch[ri]) {
                w.ms_batch[ri] = batch_create_on(g, R, RP, s);
                // 256-site tiles: one large lattice fills the device with them, and the
                // update kernels' capped grid covers 4x the sites per wave (measured at
                // 32^3x48, FP32: 0.441 -> 0.423 s for the whole solve)
                w.ms_batch[ri]->set_tiles(2, s);
            }
            KS_HIP(hipMemsetAsync(zero, 0, fb, s));
            std::vector<const double*> bp(R);
            std::vector<double*> xp(R);
            std::vector<double> sg(R), tl(R);
            for (int k = 0; k < R; ++k) {
                if (k < n) {
                    const int i = need[g0 + k];
                    export_field(G, KS_F64, x[i], w.ms_io[2 + k], s);
                    bp[k] = bb;
                    xp[k] = w.ms_io[2 + k];
                    sg[k] = sigma[i];
                    tl[k] = tol[i];
                } else {
                    bp[k] = zero;       // a zero source starts finished
                    xp[k] = w.ms_io[2 + k];
                    sg[k] = sigma[need[g0]];
                    tl[k] = 1.0;
                }
            }
            ks_solver_params q = prm;
            q.inner = RP;
            // the group's FP64 updates are synchronous (the fastest shift sets their rate):
            // from an FP32 shared phase (two decades to go) take them at a ten times deeper
            // drop, where the step counts stay the same; from a binary16 one (five decades) the
            // binary16 recursion needs them at the caller's drop (32^3x48, nine shifts: FP16
            // solve 0.488 -> 0.444 s; FP32 within 1 % either way)
            q.delta = P == KS_F16 ? prm.delta : prm.delta * 0.1;
            std::vector<ks_batch_stats> bs(R);
            const ks_status_t rc = batch_solve_pairs(*w.ms_batch[ri], sg.data(), tl.data(),
                                                     bp.data(), xp.data(), q, bs.data(), s);
            for (int k = 0; k < n; ++k) {
                const int i = need[g0 + k];
                import_field(G, KS_F64, w.ms_io[2 + k], x[i], s);
                ks_solver_stats& o = stats[i];
                o.iters += bs[k].iters;
                o.reliable_updates += bs[k].reliable_updates;
                o.restarts = 1;
                o.true_rel_resid = bs[k].true_rel_resid;
                // per step: two multi-RHS binary16 hopping terms (links once for the group,
                // each term's vector in and out per right-hand side) and the per-RHS vector
                // traffic of a mixed CG step with x's FP32 increments (read + write)
                o.model_bytes += (double)bs[k].iters * vh *
                                 ((2 * dslash_model_bytes(RP, KS_RECON_18) - 4 * rsb) / R +
                                  4 * rsb + 8 * rsb + 48);
                if (bs[k].status != KS_SUCCESS && result == KS_SUCCESS)
                    result = static_cast<ks_status_t>(bs[k].status);
            }
            if (rc != KS_SUCCESS && result == KS_SUCCESS) result = rc;
            KS_HIP(hipStreamSynchronize(s));
        }
    } else {
        for (int i : need) {
            ks_solver_stats& o = stats[i];
            ks_solver_params q = prm;
            q.tol = tol[i];
            ks_solver_stats rs;
            const ks_status_t rc = cg_core(g, sigma[i], b, x[i], q, rs, s);
            o.iters += rs.iters;
            o.reliable_updates += rs.reliable_updates;
            o.restarts = rs.restarts + 1;
            o.true_rel_resid = rs.true_rel_resid;
            o.model_bytes += rs.model_bytes;
            if (rc != KS_SUCCESS && result == KS_SUCCESS) result = rc;
        }
    }
    const double total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < nshift; ++i) {
        stats[i].seconds = total;
        stats[i].model_flops = (double)stats[i].iters * (2 * 1146.0 + 100) * vh;
    }
    return result;
}

}  // namespace ks
