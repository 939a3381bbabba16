// Link derivative ("force") of the multi-shift pseudofermion action
//     S = sum_i r_i phi^+ (sigma_i - D_eo D_oe)^-1 phi
// from the shifted solutions X_i = (sigma_i - D_eo D_oe)^-1 phi, the quantity the multi-mass
// solver's output feeds in molecular-dynamics evolution (the fermion force of Sec. 5's outlook).
// With Y_i = D_oe X_i and Psi_i = X_i on even sites, Y_i on odd sites, a change of the links
// changes S by sum_{x,mu} 2 Re Tr[dV_mu(x) FV_mu(x) + dW_mu(x) FW_mu(x)] with
//     FV_mu(x) = eps(x) sum_i r_i Psi_i(x+mu) Psi_i(x)^+,
//     FW_mu(x) = eps(x) sum_i r_i Psi_i(x+3mu) Psi_i(x)^+,      eps = +1 even, -1 odd sites.
// The Y_i come from the FP64 hopping term; one pass over (direction, site) pairs then builds
// both outer-product sums in registers and writes them in the canonical link layout.
#include <vector>

#include "ks_blas.h"
#include "ks_device.h"
#include "ks_solvers.h"

namespace ks {

namespace {

constexpr int kMaxTerms = 32;

struct Terms {
    const double2* psi[2][kMaxTerms];   // [parity][term]: FP64 planes [3][Vh]
    double r[kMaxTerms];
    int n;
};

__device__ __forceinline__ void load_psi(const double2* p, int vh, int h, cx<double> v[3])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double2 t = p[(size_t)k * vh + h];
        v[k] = {t.x, t.y};
    }
}

// thread per (direction mu, lexicographic site x): t = mu V + x
__global__ __launch_bounds__(kBlock) void force_outer_kernel(Geom g, Terms terms,
                                                             double2* __restrict__ fv,
                                                             double2* __restrict__ fw)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4L * g.V) return;
    const int mu = (int)(t / g.V);
    const int x = (int)(t - (long)mu * g.V);
    int c[4];
    int r = x;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c[d] = r % g.n[d];
        r /= g.n[d];
    }
    c[3] = r;
    const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
    const int h = x >> 1;
    const int n1 = hop_cb(g, x, c, mu, +1);
    const int n3 = hop_cb(g, x, c, mu, +3);
    const int vh = g.Vh;
    cx<double> a1[9], a3[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        a1[e] = {0.0, 0.0};
        a3[e] = {0.0, 0.0};
    }
    for (int i = 0; i < terms.n; ++i) {
        cx<double> p0[3], p1[3], p3[3];
        load_psi(terms.psi[par][i], vh, h, p0);
        load_psi(terms.psi[1 - par][i], vh, n1, p1);
        load_psi(terms.psi[1 - par][i], vh, n3, p3);
        const double ri = terms.r[i];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const cx<double> u1 = {ri * p1[a].r, ri * p1[a].i};
            const cx<double> u3 = {ri * p3[a].r, ri * p3[a].i};
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                // u conj(p0_b)
                a1[a * 3 + b].r = fma(u1.r, p0[b].r, fma(u1.i, p0[b].i, a1[a * 3 + b].r));
                a1[a * 3 + b].i = fma(u1.i, p0[b].r, fma(-u1.r, p0[b].i, a1[a * 3 + b].i));
                a3[a * 3 + b].r = fma(u3.r, p0[b].r, fma(u3.i, p0[b].i, a3[a * 3 + b].r));
                a3[a * 3 + b].i = fma(u3.i, p0[b].r, fma(-u3.r, p0[b].i, a3[a * 3 + b].i));
            }
        }
    }
    const double eps = par ? -1.0 : 1.0;
    double2* o1 = fv + (size_t)t * 9;
    double2* o3 = fw + (size_t)t * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        o1[e] = make_double2(eps * a1[e].r, eps * a1[e].i);
        o3[e] = make_double2(eps * a3[e].r, eps * a3[e].i);
    }
}

}  // namespace

int force_max_terms() { return kMaxTerms; }

void force_core(ks_gauge_t g, int nterm, const double* residues, const double* const* x_even,
                double* force_fat, double* force_naik, hipStream_t s)
{
    Workspace& w = workspace(g);
    const Geom& G = g->geom;
    const size_t fb = field_bytes(G, KS_F64);
    while ((int)w.force_psi.size() < 2 * nterm) {
        w.force_psi.push_back(static_cast<double*>(device_alloc(fb)));
        w.bytes += fb;
    }
    Terms terms{};
    terms.n = nterm;
    for (int i = 0; i < nterm; ++i) {
        double* xe = w.force_psi[2 * i];
        double* yo = w.force_psi[2 * i + 1];
        import_field(G, KS_F64, x_even[i], xe, s);
        DslashArgs a;
        a.out_parity = 1;
        a.in = xe;
        a.out = yo;
        dslash(g, KS_F64, KS_RECON_18, a, s);
        terms.psi[0][i] = reinterpret_cast<const double2*>(xe);
        terms.psi[1][i] = reinterpret_cast<const double2*>(yo);
        terms.r[i] = residues[i];
    }
    const long n = 4L * G.V;
    force_outer_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        G, terms, reinterpret_cast<double2*>(force_fat), reinterpret_cast<double2*>(force_naik));
    KS_HIP(hipGetLastError());
}

}  // namespace ks
