/* Host-side check of the FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
 * compiles the oracle's own source and drives every entry point on small lattices (one of them
 * ragged), so that an out-of-bounds neighbour index, a use of freed or uninitialised memory
 * or undefined arithmetic in it stops the run.  Also checks two properties that do not depend
 * on the random links: A is Hermitian and the solvers return their success codes.
 * Exit status 0 when every check passes. */
#include "../../oracle/ks_oracle.c"

#include <stdio.h>

static unsigned long long rng_state = 88172645463325252ULL;

static double uniform(void)   /* xorshift64, then [-1, 1) */
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) / 4503599627370496.0 - 1.0;
}

static void fill(double* v, long n, double scale)
{
    for (long k = 0; k < n; ++k) v[k] = scale * uniform();
}

static int check_lattice(const int n[4])
{
    const long V = (long)n[0] * n[1] * n[2] * n[3], Vh = V / 2;
    double* fat = malloc(sizeof(double) * 2 * 4 * V * 9);
    double* naik = malloc(sizeof(double) * 2 * 4 * V * 9);
    double* x = malloc(sizeof(double) * 2 * 3 * Vh);
    double* y = malloc(sizeof(double) * 2 * 3 * Vh);
    double* ax = malloc(sizeof(double) * 2 * 3 * Vh);
    double* ay = malloc(sizeof(double) * 2 * 3 * Vh);
    double* xs = malloc(sizeof(double) * 2 * 3 * Vh * 3);
    if (!fat || !naik || !x || !y || !ax || !ay || !xs) return 10;
    fill(fat, 2 * 4 * V * 9, 0.1);
    fill(naik, 2 * 4 * V * 9, 0.05);
    fill(x, 2 * 3 * Vh, 1.0);
    fill(y, 2 * 3 * Vh, 1.0);
    const double sigma = 0.5;
    if (orc_apply_A(n, fat, naik, sigma, x, ax) != ORC_OK) return 11;
    if (orc_apply_A(n, fat, naik, sigma, y, ay) != ORC_OK) return 12;
    /* Hermitian: <y, A x> = conj(<x, A y>) */
    const zc yax = dot((const zc*)y, (const zc*)ax, 3 * Vh);
    const zc xay = dot((const zc*)x, (const zc*)ay, 3 * Vh);
    if (cabs(yax - conj(xay)) > 1e-11 * (cabs(yax) + 1.0)) return 13;
    /* the single- and multi-mass solvers on this (well conditioned) system */
    orc_cg_info info;
    memset(y, 0, sizeof(double) * 2 * 3 * Vh);
    static double alpha[500], beta[500];   /* the first max_iter steps' coefficients */
    const int rc = orc_cg(n, fat, naik, sigma, x, y, 1e-10, 500, 3, &info, alpha, beta);
    if (rc != ORC_OK) return 14;
    const double sg[3] = {sigma, sigma + 0.25, sigma + 1.0};
    const double tl[3] = {1e-10, 1e-10, 1e-10};
    int iters = 0;
    double res[3];
    if (orc_multishift_cg(n, fat, naik, 3, sg, x, xs, tl, 500, &iters, res) != ORC_OK) return 15;
    for (int i = 0; i < 3; ++i)
        if (!(res[i] <= 1e-9)) return 16;
    free(fat);
    free(naik);
    free(x);
    free(y);
    free(ax);
    free(ay);
    free(xs);
    return 0;
}

int main(void)
{
    const int dims[2][4] = {{4, 4, 4, 4}, {6, 4, 4, 8}};
    for (int k = 0; k < 2; ++k) {
        const int rc = check_lattice(dims[k]);
        if (rc) {
            fprintf(stderr, "lattice %d: check %d failed\n", k, rc);
            return rc;
        }
    }
    printf("oracle checks passed\n");
    return 0;
}
