// Solve of the full staggered system M x = b, M = 2m + D on both parities, through its even-odd
// Schur complement (the even-odd preconditioned CG of Sec. 3 with the odd sites reconstructed):
// in parity blocks M = [[2m, D_eo], [D_oe, 2m]], so
//     (4 m^2 - D_eo D_oe) x_e = 2m b_e - D_eo b_o,      x_o = (b_o - D_oe x_e) / (2m).
// The even residual of M x = b is the even system's residual over 2m and the odd one vanishes,
// so the even system is solved to |r_e| <= 2m tol |b|; the FP64 residual of M x = b over both
// parities is recomputed at the end.
#include <chrono>
#include <cmath>

#include "ks_blas.h"
#include "ks_device.h"
#include "ks_solvers.h"

namespace ks {

namespace {

// v *= f over an FP64 field [3][Vh] of double2
__global__ __launch_bounds__(kBlock) void scale_kernel(int vh, double2* __restrict__ v, double f)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double2 u = v[k * vh + h];
        v[k * vh + h] = make_double2(f * u.x, f * u.y);
    }
}

// per-block partial sums of |b - a x - t|^2
__global__ __launch_bounds__(kBlock) void resid_axt_kernel(int vh, const double2* __restrict__ b,
                                                           const double2* __restrict__ x,
                                                           const double2* __restrict__ t, double a,
                                                           double* __restrict__ partials)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (h < vh) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double2 u = b[k * vh + h], xv = x[k * vh + h], tv = t[k * vh + h];
            const double re = u.x - a * xv.x - tv.x, im = u.y - a * xv.y - tv.y;
            s += re * re + im * im;
        }
    }
    s = block_sum<kBlock>(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

double finish_host(Workspace& w, hipStream_t s)
{
    finish_to(w.partials, w.npart, w.scal, s);
    KS_HIP(hipMemcpyAsync(w.host_scal, w.scal, sizeof(double), hipMemcpyDeviceToHost, s));
    KS_HIP(hipStreamSynchronize(s));
    return w.host_scal[0];
}

}  // namespace

ks_status_t full_solve_core(ks_gauge_t g, double mass, const double* b_e, const double* b_o,
                            double* x_e, double* x_o, const ks_solver_params& prm,
                            ks_solver_stats& stats, hipStream_t s)
{
    const auto t0 = std::chrono::steady_clock::now();
    Workspace& w = workspace(g);
    const int vh = g->geom.Vh;
    const size_t fb = field_bytes(g->geom, KS_F64);
    for (int k = 0; k < 3; ++k)
        if (!w.full[k]) {
            w.full[k] = static_cast<double*>(device_alloc(fb));
            w.bytes += fb;
        }
    double* bp = w.full[0];     // even: 2m b_e - D_eo b_o
    double* te = w.full[1];     // even temporary
    double* to = w.full[2];     // odd temporary
    const double two_m = 2.0 * mass;

    // bp = 2m b_e - D_eo b_o  (the fused xpay form of the hopping term)
    DslashArgs a;
    a.out_parity = 0;
    a.in = b_o;
    a.out = bp;
    a.x = b_e;
    a.a = two_m;
    dslash(g, KS_F64, KS_RECON_18, a, s);
    const double b2 = norm2_host(g, b_e, s) + norm2_host(g, b_o, s);
    const double bp2 = norm2_host(g, bp, s);
    const double bnorm = std::sqrt(b2);

    stats = ks_solver_stats();
    ks_status_t rc = KS_SUCCESS;
    if (bp2 > 0.0) {
        ks_solver_params inner = prm;
        inner.tol = two_m * prm.tol * bnorm / std::sqrt(bp2);
        rc = cg_core(g, two_m * two_m, bp, x_e, inner, stats, s);
    } else {
        KS_HIP(hipMemsetAsync(x_e, 0, fb, s));
    }
    // x_o = (b_o - D_oe x_e) / (2m)
    DslashArgs c;
    c.out_parity = 1;
    c.in = x_e;
    c.out = x_o;
    c.x = b_o;
    c.a = 1.0;
    dslash(g, KS_F64, KS_RECON_18, c, s);
    scale_kernel<<<blocks_for(vh), kBlock, 0, s>>>(vh, reinterpret_cast<double2*>(x_o), 1.0 / two_m);
    KS_HIP(hipGetLastError());

    // FP64 residual of M x = b: even b_e - 2m x_e - D_eo x_o, odd b_o - 2m x_o - D_oe x_e
    double r2 = 0.0;
    if (bnorm > 0.0) {
        DslashArgs d1;
        d1.out_parity = 0;
        d1.in = x_o;
        d1.out = te;
        dslash(g, KS_F64, KS_RECON_18, d1, s);
        resid_axt_kernel<<<blocks_for(vh), kBlock, 0, s>>>(
            vh, reinterpret_cast<const double2*>(b_e), reinterpret_cast<const double2*>(x_e),
            reinterpret_cast<const double2*>(te), two_m, w.partials);
        KS_HIP(hipGetLastError());
        r2 += finish_host(w, s);
        DslashArgs d2;
        d2.out_parity = 1;
        d2.in = x_e;
        d2.out = to;
        dslash(g, KS_F64, KS_RECON_18, d2, s);
        resid_axt_kernel<<<blocks_for(vh), kBlock, 0, s>>>(
            vh, reinterpret_cast<const double2*>(b_o), reinterpret_cast<const double2*>(x_o),
            reinterpret_cast<const double2*>(to), two_m, w.partials);
        KS_HIP(hipGetLastError());
        r2 += finish_host(w, s);
    }
    stats.true_rel_resid = bnorm > 0.0 ? std::sqrt(r2) / bnorm : 0.0;
    stats.model_bytes += 4 * dslash_model_bytes(KS_F64, KS_RECON_18) * vh + 6 * 48.0 * vh;
    if (rc == KS_SUCCESS && stats.true_rel_resid > prm.tol) {
        rc = KS_ERR_NOT_CONVERGED;
        set_error("full solve: residual of M x = b is %.3e > tol %.3e", stats.true_rel_resid,
                  prm.tol);
    }
    stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

}  // namespace ks
