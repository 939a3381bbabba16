// Scalar state and vector steps of the CG solvers.
#pragma once

#include "ks_common.h"

namespace ks {

// Device-resident scalars of one CG solve.  Kernels of one iteration skip their work while
// `gate` is nonzero: after convergence, after an error, or while a reliable update is due.
struct CGState {
    double rho;        // |r|^2 of the inner residual
    double rho_new;
    double alpha, beta;
    double pAp;
    double maxr;       // max |r| since the last reliable update
    double stop2;      // (tol |b|)^2
    double delta;      // reliable-update threshold (0 = only the final check)
    double true_r2;    // |b - A x|^2 of the last FP64 recomputation
    int iter;
    int max_iter;
    int gate;
    int ru_pending;
    int done;
    int status;
    // copies taken by the update kernel for the next kernel of the same step, whose lead
    // thread rewrites the live fields while its other blocks still decide from these
    double s_rho, s_maxr;
    int s_iter, s_gate;
};

void convert_field(int vh, ks_prec_t pin, const void* in, ks_prec_t pout, void* out,
                   const int* gate, hipStream_t s);
void norm2_partials(int vh, const double* v, double* partials, hipStream_t s);
void sub_norm_partials(int vh, const double* b, const double* ax, double* r, double* partials,
                       hipStream_t s);
// x (FP64 planes) += dx (FP32 field); dx = 0
void flush_dx(int vh, void* dx, double* x, hipStream_t s);
// Threads per block of the two fused CG step kernels (one site per thread).
constexpr int kCgFuse = 1024;
// One CG step after q = A p and the <p, q> partials (npap of them) are written: every block
// sums the partials in the same order and takes alpha = rho / <p, q>; then x += alpha p (x:
// FP64 planes, or in reduced precision x's FP32 increment field, see flush_dx),
// r -= alpha q, and the |r|^2 partials to rr_part (blocks_for(vh, kCgFuse) of them).
// Breakdown and a non-finite <p, q> gate the solver.  Step k's alpha goes to coef[2k]
// (k < coef_cap).
void cg_update(int vh, ks_prec_t prec, void* x, const void* p, const void* q, void* r,
               CGState* st, const double* pap_part, int npap, double* rr_part, double* coef,
               int coef_cap, hipStream_t s);
// The rest of the step: every block sums the |r|^2 partials; beta, the stopping and
// reliable-update decisions, and p = r + beta p when the step goes on.  Step k's beta goes to
// coef[2k + 1] (NaN when the step ends in a reliable update or the final check).
void cg_beta_xpay(int vh, ks_prec_t prec, const void* r, void* p, CGState* st,
                  const double* rr_part, double* coef, int coef_cap, hipStream_t s);
void xpay(int vh, ks_prec_t prec, const void* r, void* p, const CGState* st, hipStream_t s);
void cg_reliable(const double* part, int n, CGState* st, int initial, hipStream_t s);
void finish_to(const double* part, int n, double* out, hipStream_t s);
// dst = src, bytes a multiple of 16, both 16-byte aligned (a streaming copy: the
// achievable-bandwidth reference of the memory-bound kernels)
void stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// reads src (bytes a multiple of 16, 16-byte aligned): the achievable read bandwidth
void stream_read(const void* src, size_t bytes, hipStream_t s);

}  // namespace ks
