/*
 * ks.h -- C ABI of the MI355X (gfx950) improved-staggered solver library, libks.so.
 *
 * The library solves the even-odd preconditioned normal equations of the improved-staggered
 * (HISQ-style) Dirac operator,
 *
 *     A_sigma x_e = (sigma - D_eo D_oe) x_e = b_e,   sigma = 4 m^2 for one mass,
 *
 * by conjugate gradient, single-mass and multi-mass (the "staggered CG" and "multi-mass CG"
 * of Sec. 3, benchmarked in double precision in Sec. 4), with
 *
 *     (D psi)(x) = sum_mu [ V_mu(x) psi(x+mu) - V_mu(x-mu)^+ psi(x-mu)
 *                         + W_mu(x) psi(x+3mu) - W_mu(x-3mu)^+ psi(x-3mu) ]
 *
 * for the fat one-link V and the Naik three-link W, staggered phases and boundary signs
 * folded into the links by the caller.  No factor 1/2: the full operator is M = 2m + D.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice: dims = {Nx, Ny, Nz, Nt}, each even and >= 4; V = Nx Ny Nz Nt, Vh = V / 2.
 * Sites are lexicographic, i = x + Nx (y + Ny (z + Nz t)); parity (x+y+z+t) mod 2 (even = 0).
 * One-parity ("checkerboard") colour-vector fields are complex128 [Vh][3], interleaved
 * (re, im), colour fastest; the site i of that parity is row i >> 1.
 * Links are complex128 [4][V][3][3] (mu, site, row, column).
 * Pointers named *_dev are device pointers (hipMalloc or torch CUDA tensors); the caller owns
 * them.  Handles (ks_gauge_t, ks_field_t) are owned by the library and hold device memory in
 * the library's internal layout; free them with the matching *_free call.
 * Streams: all device work is queued on the caller's stream.  ks_dslash_eo and ks_apply_A
 * return without waiting; the solvers wait for their stream before returning.
 * Concurrency: calls on one gauge handle (or one batch or network handle) must not overlap in
 * time, from several host threads or on several streams: they share the handle's solver
 * workspace.  Different handles are independent.
 * Errors: every call returns a ks_status_t and never aborts; ks_last_error() gives a message
 * for the calling thread's last failure.
 * Diagnostics: with the environment variable KS_LOG at 1 or more, each solve prints a summary
 * line (status, steps, reliable updates, FP64 residual, seconds, model GB/s), each tuning its
 * result and each failing call its error on stderr, prefixed "[ks]"; unset or 0, the library
 * prints nothing.
 */
#ifndef KS_H
#define KS_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ks_gauge_s* ks_gauge_t;
typedef struct ks_field_s* ks_field_t;

typedef enum { KS_F64 = 0, KS_F32 = 1, KS_F16 = 2 } ks_prec_t;
/* storage of the Naik link W: 18 reals, or the two first rows of W / c (12 reals) with the
 * real scale c and the third row rebuilt in the kernel (exact only when W = c * SU(3)). */
typedef enum { KS_RECON_18 = 18, KS_RECON_12 = 12 } ks_recon_t;
typedef enum { KS_EVEN = 0, KS_ODD = 1 } ks_parity_t;

typedef enum {
    KS_SUCCESS = 0,
    KS_ERR_ARG = -1,            /* invalid argument (dims, null pointer, parity, aliasing) */
    KS_ERR_HIP = -2,            /* a HIP runtime call failed */
    KS_ERR_NOMEM = -3,          /* device (or host) allocation failed */
    KS_ERR_NOT_SU3 = -4,        /* 12-real storage asked for links that are not c * SU(3) */
    KS_ERR_NOT_CONVERGED = -5,  /* max_iter reached; x holds the last iterate, stats filled */
    KS_ERR_BREAKDOWN = -6,      /* <p, A p> <= 0 */
    KS_ERR_NONFINITE = -7       /* a NaN or Inf appeared in the iteration */
} ks_status_t;

typedef struct {
    double tol;           /* target true relative residual |b - A x| / |b| */
    int max_iter;         /* cap on Krylov steps (all restarts included) */
    ks_prec_t inner;      /* precision of the inner operator and Krylov vectors */
    ks_recon_t recon;     /* Naik-link storage of the inner operator */
    double delta;         /* reliable update when |r_inner| < delta * max |r| since the last */
    int check_every;      /* Krylov steps between host reads of the device status */
    int max_restarts;     /* FP64 true-residual checks that may send the loop back */
} ks_solver_params;

typedef struct {
    int iters;                 /* Krylov steps taken */
    int reliable_updates;      /* FP64 recomputations of r = b - A x */
    int restarts;              /* FP64 checks that failed and continued the loop */
    int fallback;              /* flexible CG only: 0, or why it fell back to plain CG: 1 N(r) not
                                  finite, 2 Re<N(r), r> <= 0, 3 <p, A p> <= 0, 4 |r| not halved
                                  in 50 steps, 5 max_iter */
    double true_rel_resid;     /* FP64 |b - A x| / |b| at return, computed on the GPU */
    double seconds;            /* wall time of the call */
    double model_bytes;        /* least-data model bytes of the work done */
    double model_flops;        /* model flops of the work done */
} ks_solver_stats;

/* Defaults: tol 1e-10, max_iter 100000, FP64 inner, 18-real Naik, delta 0.1, check every 16
 * steps, 5 restarts. */
void ks_default_params(ks_solver_params* p);

/* ------------------------------------------------------------------ gauge field */

/* Loads V (fat) and W (naik), complex128 [4][V][3][3] each, host (on_device = 0) or device
 * (on_device = 1) memory, into a new handle (the gauge fields the solver of Sec. 3 reads).
 * Only the FP64 18-real store is built here; the reduced-precision and 12-real stores are
 * built by ks_gauge_prepare (or on first use), so the Naik storage is chosen per store and per
 * call rather than once at load.  The library keeps, for both output parities,
 * the 16 matrices of every site {V_mu(x), -V_mu(x-mu)^+, W_mu(x), -W_mu(x-3mu)^+} as FP64
 * site-major planes (the 8-way forward-plus-backward storage of Sec. 3).  Synchronises the
 * stream before returning; the caller may free its arrays afterwards.
 * KS_ERR_ARG for bad dims or null pointers, KS_ERR_NOMEM, KS_ERR_HIP. */
ks_status_t ks_gauge_load(ks_gauge_t* out, const int dims[4], const double* fat,
                          const double* naik, int on_device, hipStream_t stream);

/* Builds (once) the link store of precision `prec` and Naik storage `recon` from the FP64
 * store; every later call with that pair reuses it.  FP16 stores each link class scaled by a
 * power of two so that its largest real lies in [0.5, 1).  12-real storage requires every
 * stored Naik matrix to be c * eta_mu(x) * bc(x) * SU(3) for one real c, the staggered phases
 * eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z), and bc = -1 exactly
 * on the three-links that cross the antiperiodic time boundary; otherwise KS_ERR_NOT_SU3 and
 * no store is kept.  Synchronises the stream. */
ks_status_t ks_gauge_prepare(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon,
                             hipStream_t stream);

ks_status_t ks_gauge_free(ks_gauge_t g);

/* Device bytes held by the handle (all stores and solver workspaces). */
size_t ks_gauge_device_bytes(ks_gauge_t g);

/* ------------------------------------------------------------------ fields */

/* A one-parity colour-vector field of the handle's lattice in the library's layout (the
 * colour vectors of one checkerboard that the staggered dslash and CG of Sec. 3 act on, laid
 * out site-major for coalesced loads as Sec. 3's data-layout discussion asks of its vector
 * unit): FP64 and FP32 as three site-major complex planes, FP16 as one 16-byte record per site
 * (FP32 scale n, then three binary16 complex numbers of v / n, n = max |real| of the site). */
ks_status_t ks_field_create(ks_field_t* f, ks_gauge_t g, ks_parity_t parity, ks_prec_t prec);
ks_status_t ks_field_free(ks_field_t f);
/* Copies complex128 [Vh][3] (device memory) into / out of the field, rounding to nearest
 * even into FP32 / FP16.  Asynchronous on `stream`. */
ks_status_t ks_field_import(ks_field_t f, const double* src_dev, hipStream_t stream);
ks_status_t ks_field_export(ks_field_t f, double* dst_dev, hipStream_t stream);

/* ------------------------------------------------------------------ operator */

/* The staggered dslash of Sec. 3 restricted to one output parity (its even-odd form, the
 * kernel whose memory bandwidth Sec. 4 measures): out = D_{p,1-p} in, p = parity of `out`;
 * `in` must have the other parity and both fields the same precision, and `recon` selects the
 * Naik storage (the link store of that precision and `recon` is built on first use, as
 * ks_gauge_prepare would).
 * KS_ERR_ARG if parities or precisions do not match, if out == in, or if the fields belong
 * to another lattice.  Asynchronous. */
ks_status_t ks_dslash_eo(ks_gauge_t g, ks_field_t out, ks_field_t in, ks_recon_t recon,
                         hipStream_t stream);

/* Autotuner: times the Dslash of precision `prec` / Naik storage `recon` on this lattice
 * over candidate launch configurations (64, 128 or 256 threads per block; blocks per CU
 * capped through the LDS request) and keeps the fastest for every later launch through this
 * handle (ks_dslash_eo and the solvers).  Untuned variants use 256 threads, no cap.  Allocates
 * two scratch fields for the duration of the call; synchronises the stream.  Must not be
 * called while the stream is being captured into a graph.
 * With the environment variable KS_TUNE_CACHE naming a file, the configuration is taken from
 * that file when it holds a usable entry for this device (architecture, compute units),
 * lattice extents, precision and Naik storage, without any timing; otherwise the tuned result
 * is recorded there (one JSON object per line, the file replaced atomically; lines of other
 * keys, readable or not, are kept).  KS_LOG >= 1 prints each tuning result on stderr, >= 2
 * also the cache's hit or miss. */
ks_status_t ks_tune_dslash(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon, hipStream_t stream);

/* Launch configuration of one Dslash variant:
 *   threads         64, 128 or 256 threads per block (one output site per thread);
 *   lds_bytes       dynamic LDS requested per block (0 to the device's LDS per workgroup);
 *                   it caps how many blocks share a CU, and the staged form uses at least
 *                   what its staging needs;
 *   links_per_pass  1, 2 or 4 link matrices loaded per pass of the per-site loop (4 only for
 *                   FP32 and FP16 with 18-real Naik; FP64 takes 2 only with 18-real Naik,
 *                   8-way access and unstaged gathers);
 *   link_access     8: every site reads its own 16 stored matrices, the 8-way storage of
 *                   Sec. 3; 4: the backward matrices are formed from the forward links of the
 *                   neighbour sites, so only the forward half of the storage is read (the
 *                   4-way alternative Sec. 3 leaves untested);
 *   staged          0: neighbour vectors read through the caches; 1: the vectors of the
 *                   block's x and y neighbourhood are first staged in LDS by one coalesced read
 *                   and those gathers read LDS;
 *   tuned_us        time per launch measured by the autotuner (0 if never tuned; ignored by
 *                   ks_dslash_set_config). */
typedef struct {
    int threads;
    int lds_bytes;
    int links_per_pass;
    int link_access;
    int staged;
    float tuned_us;
} ks_dslash_launch;

/* The configuration in use for a variant. */
ks_status_t ks_dslash_config(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon,
                             ks_dslash_launch* out);

/* Sets a variant's configuration by hand, replacing the tuned one; KS_ERR_ARG for a value
 * outside the ranges above. */
ks_status_t ks_dslash_set_config(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon,
                                 const ks_dslash_launch* cfg);

/* out_dev = (sigma - D_eo D_oe) in_dev in FP64 on even sites, complex128 [Vh][3] device
 * arrays (in_dev != out_dev).  Asynchronous. */
ks_status_t ks_apply_A(ks_gauge_t g, double sigma, const double* in_dev, double* out_dev,
                       hipStream_t stream);

/* ks_apply_A without any device allocation, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments and
 * result as ks_apply_A (the same kernels run); out_dev also stages the input's internal
 * planes.  Its temporaries live in a fixed 48 MiB device array of the library, one per GPU,
 * held until the process ends: lattices of up to 524288 even sites (32^4) are accepted, larger
 * ones return KS_ERR_ARG before any device work.  The FP64 link store is built by
 * ks_gauge_load, so nothing is allocated on the way.  Calls that overlap in time on one GPU
 * (several host threads or streams) share that array and race.  Asynchronous on `stream`. */
ks_status_t ks_apply_A_noalloc(ks_gauge_t g, double sigma, const double* in_dev, double* out_dev,
                               hipStream_t stream);

/* ------------------------------------------------------------------ solvers */

/* The single-mass staggered CG of Sec. 3 on the even-odd normal equations:
 * solves (4 m^2 - D_eo D_oe) x = b, b_dev and x_dev complex128 [Vh][3] device arrays.
 * x_dev holds the initial guess on entry (zero it for x0 = 0) and the solution on return.
 * With p->inner = KS_F64 this is plain FP64 CG; with KS_F32 / KS_F16 the Krylov vectors and
 * the inner operator are FP32 / FP16; x's increments are summed in FP32 and added into the
 * FP64 x, and r = b - A x is recomputed in FP64 (reliable update), whenever the inner residual
 * falls below delta times its maximum since the last update, and before returning.
 * Reductions are FP64 throughout.
 * Success means the FP64 true relative residual is <= p->tol. */
ks_status_t ks_cg_solve(ks_gauge_t g, double mass, const double* b_dev, double* x_dev,
                        const ks_solver_params* p, ks_solver_stats* st, hipStream_t stream);

/* The CG coefficients alpha_k, beta_k of every step of the last CG run on this handle
 * (ks_cg_solve, or the CG inside ks_full_solve and the flexible-CG fallback): up to n_max of
 * them into the host arrays alpha and beta, *n = how many (at most the run's steps, and at most
 * 2^20).  beta_k is NaN for a step that ended in a reliable update or the final check.  With
 * p->inner = KS_F64 and no restart they belong to one unbroken CG run, so they define its
 * Lanczos tridiagonal (diagonal 1/alpha_k + beta_{k-1}/alpha_{k-1}, off-diagonal
 * sqrt(beta_k)/alpha_k), whose extreme eigenvalues estimate those of A (the solver's condition
 * number).  Synchronous.  KS_ERR_ARG for a null handle or pointer or n_max < 0. */
ks_status_t ks_cg_coefficients(ks_gauge_t g, int n_max, double* alpha, double* beta, int* n);

/* Solves (sigma_i - D_eo D_oe) x_i = b for nshift (<= 32) shifts in one Krylov space (the
 * multi-mass CG of Sec. 3 and Sec. 4); sigma (host, length nshift) >= 0, x_dev a host array
 * of nshift device pointers (complex128 [Vh][3], overwritten; the initial guess is zero),
 * tol (host, length nshift) the per-shift targets.  The shared iteration runs in p->inner
 * precision with x_i accumulated in FP64 (in reduced precision through FP32 increments added
 * in at every reliable update of the base system); every shift whose FP64 true residual is
 * then above its target is refined from x_i by ks_cg_solve's method (several at once, one
 * right-hand side each, FP32 inner, reliable updates at p->delta / 10, when the inner precision
 * is reduced).  In reduced precision a shared iteration that breaks down (a non-finite value,
 * or <p, A p> <= 0) is not an error: every x_i returns to its FP64 value at the last reliable
 * update and is refined like the others.  The base (smallest) shift's solution is updated for
 * as long as any shift iterates, whatever its own tolerance.  st: nshift entries. */
ks_status_t ks_multishift_cg_solve(ks_gauge_t g, int nshift, const double* sigma,
                                   const double* b_dev, double* const* x_dev,
                                   const double* tol, const ks_solver_params* p,
                                   ks_solver_stats* st, hipStream_t stream);

/* Solves the full staggered system M x = b on both parities, M = 2m + D (mass > 0), by the
 * even-odd reduction of Sec. 3 with the odd sites reconstructed: the even system
 * (4 m^2 - D_eo D_oe) x_e = 2m b_e - D_eo b_o is solved by ks_cg_solve's method (p->inner,
 * p->recon, reliable updates, restarts) to the tolerance that makes |b - M x| <= p->tol |b|,
 * then x_o = (b_o - D_oe x_e) / (2m) in FP64.  b_even, b_odd: device complex128 [Vh][3] of the
 * two parities; x_even: initial guess in, solution out; x_odd: output.  No argument may alias
 * another.  st->true_rel_resid is the FP64 |b - M x| / |b| over both parities, recomputed at
 * the end; KS_ERR_NOT_CONVERGED if it exceeds p->tol.  Synchronises the stream. */
ks_status_t ks_full_solve(ks_gauge_t g, double mass, const double* b_even, const double* b_odd,
                          double* x_even, double* x_odd, const ks_solver_params* p,
                          ks_solver_stats* st, hipStream_t stream);

/* Link derivative ("fermion force") of S = sum_i r_i phi^+ (sigma_i - D_eo D_oe)^-1 phi from
 * the solutions X_i of ks_multishift_cg_solve: the next consumer of the multi-mass solver's
 * output in molecular dynamics (the fermion force named as future work in Sec. 5).  With
 * Y_i = D_oe X_i and Psi_i = X_i on even, Y_i on odd sites, a change of the links changes S by
 * sum_{x,mu} 2 Re Tr[dV_mu(x) FV_mu(x) + dW_mu(x) FW_mu(x)], where
 *     FV_mu(x) = eps(x) sum_i r_i Psi_i(x+mu) Psi_i(x)^+,
 *     FW_mu(x) = eps(x) sum_i r_i Psi_i(x+3mu) Psi_i(x)^+,   eps = +1 even, -1 odd sites,
 * with respect to the links as loaded (phases and boundary signs folded in); the chain rule
 * through the construction of V and W from thin links is the caller's.  nterm in [1, 32];
 * residues: host [nterm]; x_even: host array of nterm device complex128 [Vh][3] pointers;
 * force_fat, force_naik: device complex128 [4][V][3][3] in the layout of ks_gauge_load.  FP64
 * throughout.  Asynchronous on `stream`. */
ks_status_t ks_force(ks_gauge_t g, int nterm, const double* residues, const double* const* x_even,
                     double* force_fat, double* force_naik, hipStream_t stream);

/* Fat and Naik links from unsigned thin links U (SU(3), periodic): the link construction that
 * precedes the solve in production (HISQ-type).  With staples of a field M on mu-links in a
 * signed transverse direction a, S_a[M](x) = L_a(x) M(x+a) L_a(x+mu)^+ (L_a the thin link from
 * x toward a), a smearing with coefficients c = (c1, c3, c5, c7, cL) is
 *     F_mu = c1 U_mu + c3 sum S_a[U_mu] + c5 sum S_a S_b[U_mu] + c7 sum S_a S_b S_c[U_mu]
 *            + cL sum S_a S_a[U_mu]   (a, b, c on distinct transverse axes).
 * Output: V = F(U; level1), W = V (V^+ V)^-1/2 (U(3) projection, Newton polar iteration),
 * fat = F(W; level2), naik_mu(x) = c_naik W_mu(x) W_mu(x+mu) W_mu(x+2mu), then the staggered
 * phases eta_mu(x) and the antiperiodic time sign folded in as ks_gauge_load expects.
 * level1 = NULL: (1/8, 1/16, 1/64, 1/384, 0); level2 = NULL: (1, 1/16, 1/64, 1/384, -1/8)
 * (fat = 9/8 for unit links, so 9/8 - 3/24 = 1 normalises the free derivative); c_naik: -1/24
 * for HISQ.  thin_dev, fat_dev, naik_dev: device complex128 [4][V][3][3] (layout of
 * ks_gauge_load), distinct.  KS_ERR_NONFINITE when a level-1 link is singular.  Its scratch
 * (14 link fields, 2.1 GB at 32^4) is allocated on the first call on a device and kept for
 * later calls (grown for a larger lattice) until ks_hisq_release; calls that overlap in time
 * on one device share it and race.  Synchronises the stream. */
ks_status_t ks_hisq_links(const int dims[4], const double* thin_dev, double* fat_dev,
                          double* naik_dev, const double* level1, const double* level2,
                          double c_naik, hipStream_t stream);

/* Frees the scratch that ks_hisq_links keeps on every device (waits for each device). */
ks_status_t ks_hisq_release(void);

/* ------------------------------------------------------------------ batched solves */

/* Many independent lattices (uneven sizes allowed), each with nrhs right-hand sides, solved
 * by CG together (the single-mass CG of Sec. 3 applied to a whole batch at once). */
typedef struct ks_batch_s* ks_batch_t;

typedef struct {
    int iters;                 /* Krylov steps of this (lattice, RHS) pair */
    int reliable_updates;      /* FP64 recomputations of r = b - A x */
    int status;                /* KS_SUCCESS, KS_ERR_NOT_CONVERGED, KS_ERR_BREAKDOWN, ... */
    double true_rel_resid;     /* FP64 |b - A x| / |b| of the last recomputation */
    double seconds;            /* device clock from the start of the batch to this pair's
                                  convergence (-1 if it did not converge) */
} ks_batch_stats;

/* nlat lattices; dims: nlat x 4 extents (each even, >= 4); fat[l], naik[l]: the links of
 * lattice l in the layout of ks_gauge_load, host (on_device = 0) or device memory; nrhs: 1, 2
 * or 4 right-hand sides per lattice; inner: KS_F32 (FP32 inner iterations, FP64 reliable
 * updates), KS_F16 (binary16 links and vectors with an FP32 scale per site and right-hand
 * side, FP32 arithmetic, the solution's increments in FP32, FP64 reliable updates) or KS_F64.
 * Links are held in the library's per-lattice stores; vectors in arenas that keep the nrhs
 * values of a site adjacent, so one link load serves all of them.  Synchronises the
 * stream. */
ks_status_t ks_batch_create(ks_batch_t* out, int nlat, const int* dims, const double* const* fat,
                            const double* const* naik, int on_device, int nrhs, ks_prec_t inner,
                            hipStream_t stream);

/* Solves (4 m_l^2 - D_eo D_oe) x = b for every (lattice l, RHS r) pair, pair index p = l *
 * nrhs + r.  masses: host [nlat]; b_dev, x_dev: host arrays of nlat*nrhs device pointers to
 * complex128 [Vh_l][3] (x holds the initial guess, then the solution).  Every pair has its own
 * CG scalars on the device; FP64 reliable updates are taken per lattice (when one pair's
 * residual has met its target or fallen by p->delta, the lattice's other unfinished pairs take
 * the update with it in the next step, since it costs the lattice one multi-RHS A-apply either
 * way).  A step is four launches over the whole batch (two multi-RHS hopping terms, the update,
 * the direction update; a lattice taking a reliable update spends that step on it in FP64);
 * the host replays a HIP graph of p->check_every steps (captured on the first call, replayed
 * by later ones) until every pair has finished.  st: nlat*nrhs entries.  Returns KS_SUCCESS if every pair reached
 * p->tol, else the first failing pair's code (all stats filled).  p->inner and p->recon are
 * ignored (the batch's inner precision and 18-real links are used). */
ks_status_t ks_batch_solve(ks_batch_t b, const double* masses, const double* const* b_dev,
                           double* const* x_dev, const ks_solver_params* p, ks_batch_stats* st,
                           hipStream_t stream);

/* Autotuner of the batch: sites per tile (64, 128, 256) and schedule (one workgroup per tile,
 * or a persistent grid of 1-8 workgroups per CU striding over the tile table), timed on the
 * batch's multi-RHS Dslash; the fastest is kept.  Must not run during graph capture. */
ks_status_t ks_batch_tune(ks_batch_t b, hipStream_t stream);

/* Current schedule: sites per tile, persistent grid size (0 = one workgroup per tile), tuned
 * time of one multi-RHS Dslash in microseconds (0 if never tuned), wall seconds of the last
 * ks_batch_solve.  Any output may be NULL. */
ks_status_t ks_batch_config(ks_batch_t b, int* tile_sites, int* persistent_blocks,
                            float* tuned_us, double* last_solve_seconds);

ks_status_t ks_batch_free(ks_batch_t b);

/* ------------------------------------------------------------------ learned preconditioner */

/* A gauge-covariant network used as the preconditioner of flexible CG (the paper leaves the
 * solver's preconditioning open; this one is learned).  A layer maps c_in to c_out channels of
 * colour-vector fields on the full lattice:
 *     y_c(x) = sum_{c', p} w_{c c' p} (T_p phi_{c'})(x),
 * nine paths p: the identity (p = 0), T_{+mu} phi(x) = V_mu(x) phi(x+mu) (p = 1+mu) and
 * T_{-mu} phi(x) = V_mu(x-mu)^+ phi(x-mu) (p = 5+mu), V the fat link of the gauge handle, so
 * the network commutes with gauge transformations.  The network is N = L^+ L, L two free
 * layers with channels 1 -> 8 -> 8 and no activation: it applies four layers
 * 1 -> 8 -> 8 -> 8 -> 1, the last two the adjoints of the first two (channels swapped, weights
 * w'_{c' c pbar} = conj(w_{c c' p}), pbar the reversed path), so N is Hermitian and
 * <v, N v> = |L v|^2 >= 0.  Input: an even-site vector (odd sites zero); output: the even sites
 * of the last layer.  Weights: KS_NET_WEIGHTS complex numbers, L's first layer then its
 * second, each w[c_out][c_in][9], complex128 (re, im) on the host. */
#define KS_NET_WEIGHTS 648
typedef struct ks_net_s* ks_net_t;

ks_status_t ks_net_create(ks_net_t* out, const double* weights);
ks_status_t ks_net_set_weights(ks_net_t n, const double* weights);   /* also resets Adam */
ks_status_t ks_net_get_weights(ks_net_t n, double* weights);
ks_status_t ks_net_free(ks_net_t n);

/* Training state, for checkpoints: the free weights (complex128 [KS_NET_WEIGHTS]), Adam's first
 * and second moments (double [2 * KS_NET_WEIGHTS] each, one per real and imaginary part, in the
 * order of the weights' reals) and the number of Adam steps taken, all on the host.
 * ks_net_set_state restores a state that ks_net_get_state returned, after which ks_net_train
 * continues exactly as the saved network would have (bias correction included).  Synchronous.
 * KS_ERR_ARG for null pointers, a negative step count or non-finite values. */
ks_status_t ks_net_get_state(ks_net_t n, double* weights, double* adam_m, double* adam_v,
                             int* step);
ks_status_t ks_net_set_state(ks_net_t n, const double* weights, const double* adam_m,
                             const double* adam_v, int step);

/* out_dev = N(in_dev), complex128 [Vh][3] device arrays of the handle's lattice.  use_mfma = 0:
 * FP32 channel mixing on the vector ALUs, transports with the FP32 fat links; 1: every layer
 * mixes its channels on the matrix cores (binary16 operands, FP32 accumulation), transports
 * with the binary16 fat-link store (built on first use) by FP32-accumulated dot products, and
 * keeps the activations between layers in binary16.  Asynchronous on `stream`. */
ks_status_t ks_net_apply(ks_net_t n, ks_gauge_t g, const double* in_dev, double* out_dev,
                         int use_mfma, hipStream_t stream);

/* out = N(in) on two even-parity fields of one gauge handle in the solver's storage (KS_F64 or
 * KS_F32, both the same): the application that ks_fcg_solve makes each step, reading and
 * writing the fields directly.  use_mfma as in ks_net_apply.  KS_ERR_ARG for null or aliased
 * fields, fields of other handles or parities, differing or binary16 precisions.
 * Asynchronous on `stream`. */
ks_status_t ks_net_apply_field(ks_net_t n, ks_field_t out, ks_field_t in, int use_mfma,
                               hipStream_t stream);

/* Loss over npairs = B pairs (b_j, x_j), A_j x_j = b_j with A_j = sigma_j - D_eo D_oe on
 * lattice gauges[j] (b_j, x_j complex128 [Vh_j][3] device arrays, sigma host [npairs]): the
 * A-norm error of N b_j relative to that of x_j, the quantity CG minimises,
 *     L = (1/B) sum_j (N b_j - x_j)^+ A_j (N b_j - x_j) / (x_j^+ A_j x_j)
 * (x_j^+ A_j x_j taken as Re<x_j, b_j>), and its gradient with respect to the free weights,
 * G = dL/dRe w + i dL/dIm w, written to grad (host, complex128 [KS_NET_WEIGHTS]) when not NULL.
 * FP32 forward and backward kernels, FP64 A-apply and reductions.  Synchronises the stream.
 * KS_ERR_ARG for null entries, a negative shift or Re<x_j, b_j> <= 0. */
ks_status_t ks_net_loss_grad(ks_net_t n, int npairs, const ks_gauge_t* gauges,
                             const double* sigma, const double* const* b_dev,
                             const double* const* x_dev, double* loss, double* grad,
                             hipStream_t stream);

/* steps Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr, on the real and
 * imaginary parts separately); step k uses the minibatch of `batch` pairs starting at pair
 * (k * batch) mod npairs, cyclically.  loss_history (host, [steps]) receives the minibatch
 * loss before each step when not NULL.  Synchronises the stream. */
ks_status_t ks_net_train(ks_net_t n, int npairs, const ks_gauge_t* gauges, const double* sigma,
                         const double* const* b_dev, const double* const* x_dev, int steps,
                         int batch, double lr, double* loss_history, hipStream_t stream);

/* Flexible CG (Notay's, truncated to one previous direction) for (4 m^2 - D_eo D_oe) x = b
 * preconditioned by the network (z = N(r)), with the inner operator and vectors in p->inner
 * precision (KS_F16 is taken as KS_F32), x in FP64 (FP32 increments between reliable updates
 * in reduced precision), FP64 reliable updates as in ks_cg_solve; A and N are Hermitian, so
 * alpha = <p, r> / <p, A p> and beta = -<z, A p> / <p, A p> are real.  All scalars stay on the
 * device (the host reads a status block every p->check_every steps).  Falls back to
 * ks_cg_solve's method from the current x when N(r) is not finite, when <N(r), r> <= 0, when
 * <p, A p> <= 0, when |r| has not halved over 50 steps, or at p->max_iter (st->fallback = the
 * reason's code, st->restarts = steps of the fallback).  b_dev, x_dev as in ks_cg_solve. */
ks_status_t ks_fcg_solve(ks_gauge_t g, ks_net_t n, double mass, const double* b_dev,
                         double* x_dev, const ks_solver_params* p, int use_mfma,
                         ks_solver_stats* st, hipStream_t stream);

/* ------------------------------------------------------------------ measurement */

/* dst_dev = src_dev: a streaming device copy (one 16-byte non-temporal load and one store per
 * thread), the achievable-HBM-bandwidth reference that the memory-bound kernels
 * above are measured against (Sec. 4 judges the solver by its memory bandwidth).  bytes and
 * both addresses must be multiples of 16 and the buffers must not overlap, else KS_ERR_ARG.
 * Asynchronous on `stream`. */
ks_status_t ks_stream_copy(void* dst_dev, const void* src_dev, size_t bytes, hipStream_t stream);

/* Reads bytes of src_dev (one 16-byte non-temporal load per thread; nothing is written that
 * the caller can see): the achievable read bandwidth, the reference of the hopping term,
 * whose bytes are ~98 % reads.  bytes and the address must be multiples of 16, else
 * KS_ERR_ARG.  Asynchronous on `stream`. */
ks_status_t ks_stream_read(const void* src_dev, size_t bytes, hipStream_t stream);

/* Message of the calling thread's last failure ("" if none). */
const char* ks_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KS_H */
