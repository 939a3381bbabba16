/*
 * ks_oracle.c -- plain FP64 CPU oracle for the even-odd preconditioned improved-staggered
 * (HISQ-style) operator and its conjugate-gradient solvers.
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this file; the GPU library never does, and the two share no code.
 *
 * The paper names the computation (Sec. 3: the staggered dslash, single- and multi-mass CG;
 * Sec. 4: the double-precision multi-mass CG that takes most of the production time) but
 * never writes the operator down.  This file writes out the standard definitions:
 *
 *   (D psi)(x) = sum_mu [ V_mu(x) psi(x+mu) - V_mu(x-mu)^+ psi(x-mu)
 *                       + W_mu(x) psi(x+3mu) - W_mu(x-3mu)^+ psi(x-3mu) ]
 *
 * with the fat link V and the Naik link W carrying the staggered phases and the boundary
 * signs, no factor 1/2 (so M = 2m + D and M^+ M = 4m^2 - D^2), and
 *
 *   A_sigma x_e = sigma x_e - D_eo (D_oe x_e),   sigma = 4 m^2 for the single-mass system.
 *
 * Layouts: links complex128 [4][V][3][3] (row before column), full-lattice colour vectors
 * complex128 [V][3], one-parity vectors complex128 [Vh][3] in checkerboard order (site i of
 * that parity at row i >> 1).  Sites are lexicographic, i = x + Nx (y + Ny (z + Nz t)).
 *
 * Every routine is a direct transcription of its definition: one site at a time, modulo
 * neighbour arithmetic, no blocking or fusion.  OpenMP only splits the site loop.
 */
#include <complex.h>
#include <omp.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zc;

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_BREAKDOWN = 2, ORC_BAD_ARG = 3, ORC_NOMEM = 4 };

/* ---------------------------------------------------------------- geometry */

static long volume(const int n[4]) { return (long)n[0] * n[1] * n[2] * n[3]; }

static void coords_of(const int n[4], long i, int c[4])
{
    c[0] = (int)(i % n[0]); i /= n[0];
    c[1] = (int)(i % n[1]); i /= n[1];
    c[2] = (int)(i % n[2]); i /= n[2];
    c[3] = (int)i;
}

static long index_of(const int n[4], const int c[4])
{
    return c[0] + (long)n[0] * (c[1] + (long)n[1] * (c[2] + (long)n[2] * c[3]));
}

/* site reached from i by k steps along mu, periodic */
static long hop(const int n[4], long i, int mu, int k)
{
    int c[4];
    coords_of(n, i, c);
    c[mu] = ((c[mu] + k) % n[mu] + n[mu]) % n[mu];
    return index_of(n, c);
}

static int parity_of(const int n[4], long i)
{
    int c[4];
    coords_of(n, i, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

static int dims_ok(const int n[4])
{
    for (int mu = 0; mu < 4; ++mu)
        if (n[mu] < 4 || (n[mu] & 1)) return 0;
    return 1;
}

/* ---------------------------------------------------------------- SU(3) algebra */

static const zc* link_at(const zc* L, long V, int mu, long i) { return L + ((long)mu * V + i) * 9; }

/* y += s * M v */
static void add_mv(zc y[3], const zc* M, const zc* v, double s)
{
    for (int a = 0; a < 3; ++a) {
        zc acc = 0;
        for (int b = 0; b < 3; ++b) acc += M[a * 3 + b] * v[b];
        y[a] += s * acc;
    }
}

/* y += s * M^+ v */
static void add_mdv(zc y[3], const zc* M, const zc* v, double s)
{
    for (int a = 0; a < 3; ++a) {
        zc acc = 0;
        for (int b = 0; b < 3; ++b) acc += conj(M[b * 3 + a]) * v[b];
        y[a] += s * acc;
    }
}

/* ---------------------------------------------------------------- the operator */

/* (D psi) on every site of the full lattice. */
int orc_dslash_full(const int n[4], const double* fat, const double* naik, const double* in,
                    double* out)
{
    if (!dims_ok(n)) return ORC_BAD_ARG;
    const long V = volume(n);
    const zc* Vl = (const zc*)fat;
    const zc* Wl = (const zc*)naik;
    const zc* psi = (const zc*)in;
    zc* res = (zc*)out;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < V; ++i) {
        zc acc[3] = {0, 0, 0};
        for (int mu = 0; mu < 4; ++mu) {
            long f1 = hop(n, i, mu, +1), b1 = hop(n, i, mu, -1);
            long f3 = hop(n, i, mu, +3), b3 = hop(n, i, mu, -3);
            add_mv(acc, link_at(Vl, V, mu, i), psi + 3 * f1, +1.0);
            add_mdv(acc, link_at(Vl, V, mu, b1), psi + 3 * b1, -1.0);
            add_mv(acc, link_at(Wl, V, mu, i), psi + 3 * f3, +1.0);
            add_mdv(acc, link_at(Wl, V, mu, b3), psi + 3 * b3, -1.0);
        }
        for (int a = 0; a < 3; ++a) res[3 * i + a] = acc[a];
    }
    return ORC_OK;
}

/* Copy a one-parity vector into a full-lattice vector (other parity zero), and back. */
int orc_embed(const int n[4], int parity, const double* cb, double* full)
{
    const long V = volume(n);
    const zc* s = (const zc*)cb;
    zc* d = (zc*)full;
    for (long i = 0; i < V; ++i)
        for (int a = 0; a < 3; ++a)
            d[3 * i + a] = (parity_of(n, i) == parity) ? s[3 * (i >> 1) + a] : 0;
    return ORC_OK;
}

int orc_restrict(const int n[4], int parity, const double* full, double* cb)
{
    const long V = volume(n);
    const zc* s = (const zc*)full;
    zc* d = (zc*)cb;
    for (long i = 0; i < V; ++i)
        if (parity_of(n, i) == parity)
            for (int a = 0; a < 3; ++a) d[3 * (i >> 1) + a] = s[3 * i + a];
    return ORC_OK;
}

/* D_{p,1-p}: one-parity input of parity 1-p, one-parity output of parity p.  Written as
 * embed -> full D -> restrict, which is its definition. */
int orc_dslash_eo(const int n[4], const double* fat, const double* naik, int out_parity,
                  const double* in_cb, double* out_cb)
{
    if (!dims_ok(n) || (out_parity != 0 && out_parity != 1)) return ORC_BAD_ARG;
    const long V = volume(n);
    double* a = malloc(sizeof(zc) * 3 * V);
    double* b = malloc(sizeof(zc) * 3 * V);
    if (!a || !b) { free(a); free(b); return ORC_NOMEM; }
    orc_embed(n, 1 - out_parity, in_cb, a);
    orc_dslash_full(n, fat, naik, a, b);
    orc_restrict(n, out_parity, b, out_cb);
    free(a);
    free(b);
    return ORC_OK;
}

/* A_sigma x = sigma x - D_eo D_oe x on even sites. */
int orc_apply_A(const int n[4], const double* fat, const double* naik, double sigma,
                const double* x, double* out)
{
    if (!dims_ok(n)) return ORC_BAD_ARG;
    const long Vh = volume(n) / 2;
    double* t = malloc(sizeof(zc) * 3 * Vh);
    if (!t) return ORC_NOMEM;
    orc_dslash_eo(n, fat, naik, 1, x, t);
    orc_dslash_eo(n, fat, naik, 0, t, out);
    zc* o = (zc*)out;
    const zc* xi = (const zc*)x;
    for (long k = 0; k < 3 * Vh; ++k) o[k] = sigma * xi[k] - o[k];
    free(t);
    return ORC_OK;
}

/* ---------------------------------------------------------------- vector algebra */

static zc dot(const zc* a, const zc* b, long n)       /* <a,b> = sum conj(a) b */
{
    zc s = 0;
    for (long k = 0; k < n; ++k) s += conj(a[k]) * b[k];
    return s;
}

static double norm2(const zc* a, long n)
{
    double s = 0;
    for (long k = 0; k < n; ++k) s += creal(a[k]) * creal(a[k]) + cimag(a[k]) * cimag(a[k]);
    return s;
}

/* r = b - A_sigma x, returns |r| */
static double residual(const int n[4], const double* fat, const double* naik, double sigma,
                       const zc* b, const zc* x, zc* r, long len)
{
    orc_apply_A(n, fat, naik, sigma, (const double*)x, (double*)r);
    for (long k = 0; k < len; ++k) r[k] = b[k] - r[k];
    return sqrt(norm2(r, len));
}

/* ---------------------------------------------------------------- CG */

typedef struct {
    int iters;              /* total CG steps, all restarts included */
    int restarts;           /* times the loop restarted from the true residual */
    double true_rel_resid;  /* |b - A x| / |b| at return */
} orc_cg_info;

/*
 * Hestenes-Stiefel CG on A_sigma from the x passed in:
 *   r = b - A x, p = r, rho = |r|^2;
 *   repeat: q = A p, alpha = rho / Re<p,q>, x += alpha p, r -= alpha q, rho' = |r|^2,
 *           stop when sqrt(rho') <= tol |b|, beta = rho'/rho, p = r + beta p;
 * then the true residual b - A x decides: accept, or restart from x (at most max_restarts).
 * If alpha_out/beta_out are given, the step coefficients of the first max_iter steps are
 * stored (they define the Lanczos tridiagonal of A).
 */
int orc_cg(const int n[4], const double* fat, const double* naik, double sigma, const double* bd,
           double* xd, double tol, int max_iter, int max_restarts, orc_cg_info* info,
           double* alpha_out, double* beta_out)
{
    if (!dims_ok(n) || tol <= 0 || max_iter < 1) return ORC_BAD_ARG;
    const long len = 3 * (volume(n) / 2);
    const zc* b = (const zc*)bd;
    zc* x = (zc*)xd;
    zc* r = malloc(sizeof(zc) * len);
    zc* p = malloc(sizeof(zc) * len);
    zc* q = malloc(sizeof(zc) * len);
    if (!r || !p || !q) { free(r); free(p); free(q); return ORC_NOMEM; }
    const double bnorm = sqrt(norm2(b, len));
    int status = ORC_NOT_CONVERGED, iters = 0, restarts = 0;
    double rel = 0;
    if (bnorm == 0) {
        memset(x, 0, sizeof(zc) * len);
        status = ORC_OK;
        goto done;
    }
    for (;;) {
        double rn = residual(n, fat, naik, sigma, b, x, r, len);
        rel = rn / bnorm;
        if (rn <= tol * bnorm) { status = ORC_OK; break; }
        if (iters >= max_iter) break;
        if (iters > 0) {
            if (restarts >= max_restarts) break;
            ++restarts;
        }
        memcpy(p, r, sizeof(zc) * len);
        double rho = rn * rn;
        while (iters < max_iter) {
            orc_apply_A(n, fat, naik, sigma, (const double*)p, (double*)q);
            double pq = creal(dot(p, q, len));
            if (!(pq > 0)) { status = ORC_BREAKDOWN; goto done; }
            double alpha = rho / pq;
            for (long k = 0; k < len; ++k) { x[k] += alpha * p[k]; r[k] -= alpha * q[k]; }
            double rho_new = norm2(r, len);
            double beta = rho_new / rho;
            if (alpha_out) alpha_out[iters] = alpha;
            if (beta_out) beta_out[iters] = beta;
            ++iters;
            if (sqrt(rho_new) <= tol * bnorm) break;
            for (long k = 0; k < len; ++k) p[k] = r[k] + beta * p[k];
            rho = rho_new;
        }
    }
done:
    if (info) { info->iters = iters; info->restarts = restarts; info->true_rel_resid = rel; }
    free(r); free(p); free(q);
    return status;
}

/* ---------------------------------------------------------------- multi-shift CG */

/*
 * Solves (A_{sigma_min} + delta_i) x_i = b with delta_i = sigma_i - sigma_min >= 0, i.e.
 * (sigma_i - D_eo D_oe) x_i = b, from x_i = 0, all in one Krylov space (the multi-mass CG
 * of Sec. 3 and Sec. 4).  Base CG coefficients alpha, beta as in orc_cg; for each shift
 *   zeta_new = zeta zeta_prev alpha_prev /
 *              (alpha beta_prev (zeta_prev - zeta) + zeta_prev alpha_prev (1 + delta alpha)),
 *   alpha_i = alpha zeta_new / zeta,  x_i += alpha_i p_i,
 *   beta_i = beta (zeta_new / zeta)^2,  p_i = zeta_new r + beta_i p_i,
 * with zeta = zeta_prev = 1, alpha_prev = 1, beta_prev = 0 at the start, so the shifted
 * residuals stay r_i = zeta_i r.  Shift i freezes once |zeta_i| |r| <= tol_i |b|; the loop
 * ends when every shift is frozen.  true_rel_resid[i] is |b - A_i x_i| / |b| at return.
 */
int orc_multishift_cg(const int n[4], const double* fat, const double* naik, int nshift,
                      const double* sigma, const double* bd, double* xd, const double* tol,
                      int max_iter, int* iters_out, double* true_rel_resid)
{
    if (!dims_ok(n) || nshift < 1 || nshift > 64 || max_iter < 1) return ORC_BAD_ARG;
    const long len = 3 * (volume(n) / 2);
    double s0 = sigma[0];
    for (int i = 1; i < nshift; ++i) if (sigma[i] < s0) s0 = sigma[i];
    const zc* b = (const zc*)bd;
    zc* x = (zc*)xd;
    zc* r = malloc(sizeof(zc) * len);
    zc* p = malloc(sizeof(zc) * len);
    zc* q = malloc(sizeof(zc) * len);
    zc* ps = malloc(sizeof(zc) * len * nshift);
    double* zeta = malloc(sizeof(double) * nshift);
    double* zeta_prev = malloc(sizeof(double) * nshift);
    int* frozen = calloc(nshift, sizeof(int));
    if (!r || !p || !q || !ps || !zeta || !zeta_prev || !frozen) {
        free(r); free(p); free(q); free(ps); free(zeta); free(zeta_prev); free(frozen);
        return ORC_NOMEM;
    }
    const double bnorm = sqrt(norm2(b, len));
    memcpy(r, b, sizeof(zc) * len);
    memcpy(p, b, sizeof(zc) * len);
    memset(x, 0, sizeof(zc) * len * nshift);
    for (int i = 0; i < nshift; ++i) {
        memcpy(ps + i * len, b, sizeof(zc) * len);
        zeta[i] = zeta_prev[i] = 1.0;
        frozen[i] = (bnorm == 0);
    }
    double rho = bnorm * bnorm, alpha_prev = 1.0, beta_prev = 0.0;
    int iters = 0, status = ORC_OK, active = (bnorm != 0) ? nshift : 0;
    while (active > 0) {
        if (iters >= max_iter) { status = ORC_NOT_CONVERGED; break; }
        orc_apply_A(n, fat, naik, s0, (const double*)p, (double*)q);
        double pq = creal(dot(p, q, len));
        if (!(pq > 0)) { status = ORC_BREAKDOWN; break; }
        double alpha = rho / pq;
        double zeta_new[64], ratio[64];
        for (int i = 0; i < nshift; ++i) {
            if (frozen[i]) continue;
            double delta = sigma[i] - s0;
            zeta_new[i] = zeta[i] * zeta_prev[i] * alpha_prev /
                          (alpha * beta_prev * (zeta_prev[i] - zeta[i]) +
                           zeta_prev[i] * alpha_prev * (1.0 + delta * alpha));
            ratio[i] = zeta_new[i] / zeta[i];
            double ai = alpha * ratio[i];
            zc* pi = ps + i * len;
            zc* xi = x + i * len;
            for (long k = 0; k < len; ++k) xi[k] += ai * pi[k];
        }
        for (long k = 0; k < len; ++k) r[k] -= alpha * q[k];
        double rho_new = norm2(r, len);
        double beta = rho_new / rho;
        ++iters;
        for (int i = 0; i < nshift; ++i) {
            if (frozen[i]) continue;
            double bi = beta * ratio[i] * ratio[i];
            zc* pi = ps + i * len;
            for (long k = 0; k < len; ++k) pi[k] = zeta_new[i] * r[k] + bi * pi[k];
            zeta_prev[i] = zeta[i];
            zeta[i] = zeta_new[i];
            if (fabs(zeta[i]) * sqrt(rho_new) <= tol[i] * bnorm) { frozen[i] = 1; --active; }
        }
        for (long k = 0; k < len; ++k) p[k] = r[k] + beta * p[k];
        rho = rho_new;
        alpha_prev = alpha;
        beta_prev = beta;
    }
    if (iters_out) *iters_out = iters;
    if (true_rel_resid) {
        for (int i = 0; i < nshift; ++i) {
            double rn = residual(n, fat, naik, sigma[i], b, x + i * len, q, len);
            true_rel_resid[i] = (bnorm > 0) ? rn / bnorm : 0.0;
        }
    }
    free(r); free(p); free(q); free(ps); free(zeta); free(zeta_prev); free(frozen);
    return status;
}

/* Thread count of the OpenMP loops (harness control for timing the oracle on n host cores). */
int orc_set_threads(int n)
{
    if (n < 1) return ORC_BAD_ARG;
    omp_set_num_threads(n);
    return ORC_OK;
}

int orc_max_threads(void) { return omp_get_max_threads(); }
