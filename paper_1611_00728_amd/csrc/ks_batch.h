// Batched multi-lattice, multi-RHS CG: internal state.
#pragma once

#include <vector>

#include "ks_common.h"

namespace ks {

// One lattice of a batch, as the kernels see it.
struct LatDesc {
    Geom g;
    const void* fat32[2];     // inner-precision link planes per output parity
    const void* naik32[2];
    float fat_scale, naik_scale;   // value = stored * scale (binary16 stores; 1 otherwise)
    const void* fat64[2];     // FP64 link planes (reliable updates)
    const void* naik64[2];
    size_t vec_off;           // site offset of this lattice in every vector arena
    int tile_begin, tile_end; // its range in the active tile table
    int pair0;                // first (lattice, RHS) pair index
};

// CG scalars of one (lattice, RHS) pair.  One step is four launches (two hopping terms, the
// update, the direction update); every block of a lattice takes the same decisions from the
// same sums, and each kernel writes only fields that no block of the same kernel reads: the
// live fields are committed by the last kernel of the step (its lead block), the shadows s_*
// carry the third kernel's results to it, and s_mode (first pair of a lattice) the step's mode
// from the second hopping term to both.
struct BatchPair {
    double sigma;                // shift of this pair's operator, sigma - D_eo D_oe
    double rho, alpha, beta, maxr, stop2, delta, true_r2;
    unsigned long long t_done;   // device wall clock at convergence
    int iter, max_iter, ru, done, status;
    int ru_now;                  // reliable update due in the next step (1: target met, step cap,
                                 // forced by the lattice or initial; 2: |r| fell by delta)
    int first;                   // the next reliable update is the initial residual (beta = 0)
    // shadows written by the update kernel for the direction-update kernel
    double s_alpha, s_beta, s_rho, s_maxr, s_true_r2;
    int s_done, s_status, s_iter, s_ru, s_finished;
    int s_mode;                  // first pair of a lattice: 0 idle, 1 CG step, 2 reliable update
};

struct BatchCtx {
    int nrhs = 1;
    int npairs = 0;
    ks_prec_t prec = KS_F32;
    size_t total_vh = 0;
    std::vector<ks_gauge_t> gauges;
    bool owns_gauges = true;   // false: built on a caller's gauge handle, which keeps its stores
    std::vector<LatDesc> lats_host;
    LatDesc* lats_dev = nullptr;
    std::vector<int2> tile_tables[3];
    int2* tiles[3] = {nullptr, nullptr, nullptr};
    int ntiles[3] = {0, 0, 0};
    int tile_idx = 0;          // 0: 64, 1: 128, 2: 256 sites per tile
    int persistent = 0;        // >0: grid of this many blocks striding over the tiles
    float tuned_us = 0.f;
    double* partials = nullptr;   // per tile and RHS: <p, A p> of a step, or |b - A x|^2
    double* partials2 = nullptr;  // per tile and RHS: |r|^2 after the update
    BatchPair* pairs = nullptr;
    BatchPair* pairs_host = nullptr;
    unsigned long long* clock = nullptr;
    int* census = nullptr;
    int* census_host = nullptr;
    // vector arenas: inner precision p, q, t (odd), r; FP64 x, b, r, t (odd), A x
    char *ps = nullptr, *qs = nullptr, *ts = nullptr, *rs = nullptr;
    char *x64 = nullptr, *b64 = nullptr, *r64 = nullptr, *t64 = nullptr, *ax64 = nullptr;
    // FP32 inner: x's FP32 increments since the pair's last reliable update (zero otherwise)
    char* dx32 = nullptr;
    size_t dx32_bytes = 0;
    size_t inner_bytes = 0;   // bytes of each inner-precision arena (p, q, t, r)
    void** io_ptrs = nullptr;  // device table of the caller's per-pair vectors
    double* b2 = nullptr;      // |b|^2 per pair
    double* pair_param = nullptr;     // device [2][npairs]: shift and tolerance of each pair
    hipStream_t stream = nullptr;     // the batch's own stream (default priority)
    hipEvent_t order = nullptr;       // orders it after the caller's stream
    hipGraphExec_t graph_exec = nullptr;
    int graph_chunk = 0;
    double last_seconds = 0.0;

    int grid(int ntiles_now) const;
    void set_tiles(int k, hipStream_t s);
};

BatchCtx* batch_create(int nlat, const int* dims, const double* const* fat,
                       const double* const* naik, int on_device, int nrhs, ks_prec_t inner,
                       hipStream_t s);
void batch_free(BatchCtx* c);
ks_status_t batch_solve(BatchCtx& c, const double* masses, const double* const* b,
                        double* const* x, const ks_solver_params& prm, ks_batch_stats* stats,
                        hipStream_t s);
void batch_tune(BatchCtx& c, hipStream_t s);
// one lattice with nrhs right-hand sides on an existing gauge handle (its stores are shared)
BatchCtx* batch_create_on(ks_gauge_t g, int nrhs, ks_prec_t inner, hipStream_t s);
// solve with a shift and a tolerance per pair (host arrays of npairs); b, x as in batch_solve
ks_status_t batch_solve_pairs(BatchCtx& c, const double* sigma, const double* tol,
                              const double* const* b, double* const* x,
                              const ks_solver_params& prm, ks_batch_stats* stats, hipStream_t s);

}  // namespace ks

struct ks_batch_s {
    ks::BatchCtx* ctx;
};
