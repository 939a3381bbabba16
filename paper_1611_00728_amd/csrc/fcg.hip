// Flexible CG preconditioned by the network (Notay's flexible CG truncated to one previous
// direction), with FP32 (or FP64) inner operator and vectors, FP64 solution accumulation,
// FP64 reliable updates, and plain CG as the fallback:
//
//   r = b - A x, z = N(r), p = z
//   repeat: q = A p, alpha = <p, r> / <p, q>, x += alpha p, r -= alpha q,
//           z = N(r), beta = -<q, z> / <p, q>, p = z + beta p
//
// (complex alpha, beta: N need not be Hermitian).  With N the identity this is CG step for
// step.  Fallback to ks_cg_solve's method from the current x when z is not finite, when
// Re<z, r> <= 0, when |r| has not halved over the last 50 steps, or at max_iter.
#include <chrono>
#include <cmath>
#include <complex>
#include <deque>
#include <map>

#include "ks_blas.h"
#include "ks_device.h"
#include "ks_net.h"
#include "ks_solvers.h"

namespace ks {

namespace {

constexpr int kNT = 256;

// partial sums of <a, b> = sum conj(a) b (re, im in two arrays)
template <int P>
__global__ __launch_bounds__(kNT) void cdot_kernel(int vh, const void* __restrict__ a,
                                                   const void* __restrict__ b,
                                                   double* __restrict__ pre,
                                                   double* __restrict__ pim)
{
    using R = typename St<P>::R;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double sr = 0.0, si = 0.0;
    if (h < vh) {
        cx<R> av[3], bv[3];
        Spinor<P>::load(a, vh, h, av);
        Spinor<P>::load(b, vh, h, bv);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            sr += (double)av[k].r * bv[k].r + (double)av[k].i * bv[k].i;
            si += (double)av[k].r * bv[k].i - (double)av[k].i * bv[k].r;
        }
    }
    sr = block_sum<kNT>(sr);
    __syncthreads();
    si = block_sum<kNT>(si);
    if (threadIdx.x == 0) {
        pre[blockIdx.x] = sr;
        pim[blockIdx.x] = si;
    }
}

// x (FP64) += alpha p; r -= alpha q (complex alpha); partial sums of |r|^2 as stored
template <int P>
__global__ __launch_bounds__(kNT) void fcg_update_kernel(int vh, double2* __restrict__ x,
                                                         const void* __restrict__ p,
                                                         const void* __restrict__ q,
                                                         void* __restrict__ r, double ar, double ai,
                                                         double* __restrict__ partials)
{
    using R = typename St<P>::R;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (h < vh) {
        cx<R> pv[3], qv[3], rv[3];
        Spinor<P>::load(p, vh, h, pv);
        Spinor<P>::load(q, vh, h, qv);
        Spinor<P>::load(r, vh, h, rv);
        const cx<R> a = {(R)ar, (R)ai};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double2 t = x[(size_t)k * vh + h];
            t.x += ar * (double)pv[k].r - ai * (double)pv[k].i;
            t.y += ar * (double)pv[k].i + ai * (double)pv[k].r;
            x[(size_t)k * vh + h] = t;
            const cx<R> d = cmul(a, qv[k]);
            rv[k].r -= d.r;
            rv[k].i -= d.i;
        }
        Spinor<P>::store(r, vh, h, rv);
        Spinor<P>::round(rv);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            s += (double)rv[k].r * rv[k].r + (double)rv[k].i * rv[k].i;
    }
    s = block_sum<kNT>(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// p = z + beta p (complex beta)
template <int P>
__global__ __launch_bounds__(kNT) void fcg_p_kernel(int vh, const void* __restrict__ z,
                                                    void* __restrict__ p, double br, double bi)
{
    using R = typename St<P>::R;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
    cx<R> zv[3], pv[3];
    Spinor<P>::load(z, vh, h, zv);
    Spinor<P>::load(p, vh, h, pv);
    const cx<R> b = {(R)br, (R)bi};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const cx<R> d = cmul(b, pv[k]);
        pv[k] = {zv[k].r + d.r, zv[k].i + d.i};
    }
    Spinor<P>::store(p, vh, h, pv);
}

struct FcgBufs {
    double* aos_in = nullptr;    // complex128 [Vh][3] network input / output staging
    double* aos_out = nullptr;
    void* z = nullptr;
    double* pim = nullptr;       // second partial array for complex dots
    int vh = 0;
    int prec = -1;
};

std::map<ks_gauge_t, FcgBufs> g_fcg;   // per gauge handle (freed with the handle's workspace)

}  // namespace

void fcg_release(ks_gauge_t g)
{
    auto it = g_fcg.find(g);
    if (it == g_fcg.end()) return;
    device_free(it->second.aos_in);
    device_free(it->second.aos_out);
    device_free(it->second.z);
    device_free(it->second.pim);
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
        device_free(fb.aos_in);
        device_free(fb.aos_out);
        device_free(fb.z);
        device_free(fb.pim);
        fb = FcgBufs();
        fb.aos_in = static_cast<double*>(device_alloc((size_t)vh * 48));
        fb.aos_out = static_cast<double*>(device_alloc((size_t)vh * 48));
        fb.z = device_alloc(field_bytes(G, P));
        fb.pim = static_cast<double*>(device_alloc(sizeof(double) * (w.npart + 8)));
        fb.vh = vh;
        fb.prec = (int)P;
    }
    // inner vectors
    const size_t fbytes = field_bytes(G, P);
    if (!w.rs[P]) w.rs[P] = device_alloc(fbytes);
    if (!w.ps[P]) w.ps[P] = device_alloc(fbytes);
    if (!w.qs[P]) w.qs[P] = device_alloc(fbytes);
    if (!w.ts[P]) w.ts[P] = device_alloc(fbytes);
    void* rs = (P == KS_F64) ? static_cast<void*>(w.r64) : w.rs[P];
    void* ps = w.ps[P];
    void* qs = w.qs[P];
    void* ts = w.ts[P];
    void* zs = fb.z;
    const int nb = blocks_for(vh, kNT);
    double* hs = w.host_scal;

    auto sync_read = [&](int n) {
        KS_HIP(hipMemcpyAsync(hs, w.scal, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        KS_HIP(hipStreamSynchronize(s));
    };
    auto cdot = [&](const void* a, const void* bb, int slot) {
        if (P == KS_F64) cdot_kernel<KS_F64><<<nb, kNT, 0, s>>>(vh, a, bb, w.partials, fb.pim);
        else cdot_kernel<KS_F32><<<nb, kNT, 0, s>>>(vh, a, bb, w.partials, fb.pim);
        KS_HIP(hipGetLastError());
        reduce_sum(w.partials, nb, w.scal + slot, s);
        reduce_sum(fb.pim, nb, w.scal + slot + 1, s);
    };
    // true residual into r64 and the inner r; returns |r|^2
    auto reliable = [&]() {
        apply_A64(g, sigma, x, w.ax64, s, nullptr);
        sub_norm_partials(vh, b, w.ax64, w.r64, w.partials, s);
        reduce_sum(w.partials, w.npart, w.scal, s);
        if (P != KS_F64) convert_field(vh, KS_F64, w.r64, P, rs, nullptr, s);
        sync_read(1);
        return hs[0];
    };
    auto precondition = [&](double rho) {
        // z = N(r): the network is linear, so the input is scaled to O(1) entries and the
        // output scaled back
        export_field(G, P, rs, fb.aos_in, s);
        const double sc = rho > 0 ? std::sqrt((double)vh / rho) : 1.0;
        if (use_mfma) net_apply_mfma(net, g, fb.aos_in, fb.aos_out, sc, s);
        else net_apply_f32(net, g, fb.aos_in, fb.aos_out, sc, s);
        import_field(G, P, fb.aos_out, zs, s);
    };

    stats = ks_solver_stats();
    const double b2 = norm2_host(g, b, s);
    const double bnorm = std::sqrt(b2);
    if (bnorm == 0.0) {
        KS_HIP(hipMemsetAsync(x, 0, field_bytes(G, KS_F64), s));
        KS_HIP(hipStreamSynchronize(s));
        return KS_SUCCESS;
    }
    const double stop2 = prm.tol * prm.tol * b2;
    const double delta = (P == KS_F64) ? 0.0 : prm.delta;
    double rho = reliable();
    double maxr = std::sqrt(rho);
    double true_r2 = rho;
    int it = 0, ru = 0;
    bool done = rho <= stop2, fallback = false;
    int reason = 0;   // why the flexible iteration stopped (see ks_solver_stats.fallback)
    std::deque<double> hist;
    hist.push_back(std::sqrt(rho));
    std::complex<double> zr;
    if (!done) {
        precondition(rho);
        convert_field(vh, P, zs, P, ps, nullptr, s);   // p = z
        cdot(zs, rs, 0);
        sync_read(2);
        zr = {hs[0], hs[1]};
    }
    while (!done) {
        if (!std::isfinite(zr.real()) || !std::isfinite(zr.imag())) reason = 1;
        else if (zr.real() <= 0.0) reason = 2;
        else if (it >= prm.max_iter) reason = 5;
        if (reason) {
            fallback = true;
            break;
        }
        DslashArgs a1;
        a1.out_parity = 1;
        a1.in = ps;
        a1.out = ts;
        dslash(g, P, RC, a1, s);
        DslashArgs a2;
        a2.out_parity = 0;
        a2.in = ts;
        a2.out = qs;
        a2.x = ps;
        a2.a = sigma;
        a2.dot_partials = w.partials;
        dslash(g, P, RC, a2, s);
        reduce_sum(w.partials, dslash_blocks(g, P, RC), w.scal + 2, s);
        if (P == KS_F64) cdot_kernel<KS_F64><<<nb, kNT, 0, s>>>(vh, ps, rs, w.partials, fb.pim);
        else cdot_kernel<KS_F32><<<nb, kNT, 0, s>>>(vh, ps, rs, w.partials, fb.pim);
        KS_HIP(hipGetLastError());
        reduce_sum(w.partials, nb, w.scal + 0, s);
        reduce_sum(fb.pim, nb, w.scal + 1, s);
        sync_read(3);
        const double pap = hs[2];
        const std::complex<double> pr(hs[0], hs[1]);
        if (!(pap > 0.0) || !std::isfinite(pap)) {
            fallback = true;
            reason = 3;
            break;
        }
        const std::complex<double> alpha = pr / pap;
        if (P == KS_F64)
            fcg_update_kernel<KS_F64><<<nb, kNT, 0, s>>>(vh, reinterpret_cast<double2*>(x), ps, qs, rs,
                                                         alpha.real(), alpha.imag(), w.partials);
        else
            fcg_update_kernel<KS_F32><<<nb, kNT, 0, s>>>(vh, reinterpret_cast<double2*>(x), ps, qs, rs,
                                                         alpha.real(), alpha.imag(), w.partials);
        KS_HIP(hipGetLastError());
        reduce_sum(w.partials, nb, w.scal, s);
        sync_read(1);
        double rn = hs[0];
        ++it;
        if (rn <= stop2 || std::sqrt(rn) < delta * maxr) {
            rn = reliable();
            true_r2 = rn;
            ++ru;
            maxr = std::sqrt(rn);
            if (rn <= stop2) {
                done = true;
                break;
            }
        }
        maxr = std::max(maxr, std::sqrt(rn));
        hist.push_back(std::sqrt(rn));
        if (hist.size() > 51) hist.pop_front();
        if (hist.size() == 51 && hist.back() > 0.5 * hist.front()) {
            fallback = true;
            reason = 4;
            break;
        }
        rho = rn;
        precondition(rho);
        cdot(qs, zs, 0);   // <q, z>
        cdot(zs, rs, 2);   // <z, r>
        sync_read(4);
        const std::complex<double> qz(hs[0], hs[1]);
        zr = {hs[2], hs[3]};
        const std::complex<double> beta = -qz / pap;
        if (P == KS_F64) fcg_p_kernel<KS_F64><<<nb, kNT, 0, s>>>(vh, zs, ps, beta.real(), beta.imag());
        else fcg_p_kernel<KS_F32><<<nb, kNT, 0, s>>>(vh, zs, ps, beta.real(), beta.imag());
        KS_HIP(hipGetLastError());
    }
    ks_status_t rc = KS_SUCCESS;
    int fb_iters = 0;
    if (fallback) {
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
    stats.fallback = fallback ? reason : 0;
    stats.true_rel_resid = std::sqrt(true_r2 / b2);
    stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

}  // namespace ks
