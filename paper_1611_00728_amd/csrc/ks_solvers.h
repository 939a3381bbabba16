// Solver workspaces and internal solver entry points.
#pragma once

#include <vector>

#include "ks_blas.h"

namespace ks {

// Per-gauge-handle solver buffers, allocated on first use and kept until ks_gauge_free.
struct Workspace {
    size_t bytes = 0;
    int npart = 0;
    double* partials = nullptr;   // per-block partial sums
    double* rr_part = nullptr;    // |r|^2 partials of the fused CG step (blocks_for(Vh, kCgFuse))
    double* cg_coef = nullptr;    // alpha_k, beta_k of the last CG run, interleaved
    int cg_coef_cap = 0;          // steps it holds
    int cg_coef_n = 0;            // steps recorded by the last run
    double* scal = nullptr;       // device scalars (after the partials)
    double* host_scal = nullptr;  // pinned
    CGState* st = nullptr;
    CGState* st_host = nullptr;   // pinned
    // FP64 planes [3][Vh] (t64 has the odd parity)
    double* b64 = nullptr;
    double* x64 = nullptr;
    double* r64 = nullptr;
    double* t64 = nullptr;
    double* ax64 = nullptr;
    // inner-precision vectors per precision (ts odd)
    void* rs[3] = {nullptr, nullptr, nullptr};
    void* ps[3] = {nullptr, nullptr, nullptr};
    void* qs[3] = {nullptr, nullptr, nullptr};
    void* ts[3] = {nullptr, nullptr, nullptr};
    void* dx32 = nullptr;         // FP32 increments of x between reliable updates (reduced precision)
    // multi-shift
    std::vector<void*> ms_x;      // FP64 solutions
    std::vector<void*> ms_p;      // shifted directions, inner precision
    std::vector<void*> ms_dx;     // FP32 increments of the shifted solutions (reduced precision)
    int ms_prec = -1;
    void* ms_r = nullptr;
    void* ms_pb = nullptr;
    void* ms_q = nullptr;
    void* ms_t = nullptr;
    void* ms_st = nullptr;
    void* ms_st_host = nullptr;
    // full-lattice solve, FP64 planes: even right-hand side of the Schur system, even and odd
    // temporaries, and the odd b and x of the boundary call
    double* full[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    // force: per term the even solution and its odd hopping image, FP64 planes
    std::vector<double*> force_psi;
    // multi-shift refinement of several shifts at once: batched CG contexts on this gauge
    // (1, 2 or 4 right-hand sides) and boundary-layout vectors for them
    struct BatchCtx* ms_batch[3] = {nullptr, nullptr, nullptr};
    std::vector<double*> ms_io;
};

Workspace& workspace(ks_gauge_t g);
void workspace_free(Workspace* w);

double dslash_model_bytes(ks_prec_t p, ks_recon_t r);
double cg_iter_model_bytes(ks_prec_t p, ks_recon_t r);
double norm2_host(ks_gauge_t g, const double* v, hipStream_t s);
void apply_A64(ks_gauge_t g, double sigma, const double* x, double* ax, hipStream_t s,
               const int* gate);
double true_resid2(ks_gauge_t g, double sigma, const double* b, const double* x, hipStream_t s);

// alpha_k, beta_k (host arrays of n_max) of the last CG run on g; *n = steps copied
void cg_coefficients(ks_gauge_t g, int n_max, double* alpha, double* beta, int* n);
ks_status_t cg_core(ks_gauge_t g, double sigma, const double* b, double* x,
                    const ks_solver_params& prm, ks_solver_stats& stats, hipStream_t s);
// M x = b with M = 2m + D on both parities (internal FP64 planes; x_e: initial guess in)
ks_status_t full_solve_core(ks_gauge_t g, double mass, const double* b_e, const double* b_o,
                            double* x_e, double* x_o, const ks_solver_params& prm,
                            ks_solver_stats& stats, hipStream_t s);
// link derivative of sum_i r_i phi^+ A_i^-1 phi from X_i = A_i^-1 phi (boundary layout)
int force_max_terms();
void force_core(ks_gauge_t g, int nterm, const double* residues, const double* const* x_even,
                double* force_fat, double* force_naik, hipStream_t s);
ks_status_t multishift_core(ks_gauge_t g, int nshift, const double* sigma, const double* b,
                            double* const* x, const double* tol, const ks_solver_params& prm,
                            ks_solver_stats* stats, hipStream_t s);

}  // namespace ks
