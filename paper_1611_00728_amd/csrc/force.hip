// Link derivative ("force") of the multi-shift pseudofermion action
//     S = sum_i r_i phi^+ (sigma_i - D_eo D_oe)^-1 phi
// from the shifted solutions X_i = (sigma_i - D_eo D_oe)^-1 phi, the quantity the multi-mass
// solver's output feeds in molecular-dynamics evolution (the fermion force of Sec. 5's outlook).
// With Y_i = D_oe X_i and Psi_i = X_i on even sites, Y_i on odd sites, a change of the links
// changes S by sum_{x,mu} 2 Re Tr[dV_mu(x) FV_mu(x) + dW_mu(x) FW_mu(x)] with
//     FV_mu(x) = eps(x) sum_i r_i Psi_i(x+mu) Psi_i(x)^+,
//     FW_mu(x) = eps(x) sum_i r_i Psi_i(x+3mu) Psi_i(x)^+,      eps = +1 even, -1 odd sites.
// The Y_i come from a multi-vector FP64 hopping term (links read once for up to five X_i);
// one pass over (direction, site) pairs then builds both outer-product sums in registers and
// writes them in the canonical link layout.
#include <algorithm>
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

// y_k = D_{par} x_k for K vectors at once (FP64, 18-real, 8-way links of the output parity):
// each of a site's 16 link matrices is loaded once and applied to the K vectors, so the
// links' bytes are read once per K outputs instead of once per output.
constexpr int kMultiMax = 5;   // nine terms in two passes (measured: 5 beats 3 and 4 per pass)

struct MultiVec {
    const double2* in[kMultiMax];
    double2* out[kMultiMax];
};

// Two lanes per output site: lane 0 of the pair takes the eight one-link matrices, lane 1 the
// eight Naik matrices (twice the waves, half of each lane's chain of dependent loads); one
// shuffle adds the halves and lane 0 stores.
template <int K>
__global__ __launch_bounds__(kBlock) void dslash_multi_kernel(Geom g, int par,
                                                              const void* __restrict__ fat,
                                                              const void* __restrict__ naik,
                                                              MultiVec mv, float fat_scale,
                                                              float naik_scale)
{
    const int vh = g.Vh;
    const int t = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int h = t >> 1;
    const int kind = t & 1;                 // 0: one-link, 1: Naik
    const bool live = h < vh;
    const int hs = live ? h : vh - 1;       // a dead lane shadows a live site (no store)
    int c[4];
    cb_coords(g, hs, par, c);
    const int i = site_index(g, c);
    cx<double> res[K][3];
#pragma unroll
    for (int q = 0; q < K; ++q)
#pragma unroll
        for (int a = 0; a < 3; ++a) res[q][a] = {0.0, 0.0};
    const void* links = kind ? naik : fat;
    const double sc = kind ? (double)naik_scale : (double)fat_scale;
#pragma unroll 1
    for (int s = 0; s < 8; ++s) {
        // slots 0-3: +mu, 4-7: -mu; backward slots hold the negated adjoint of the link
        const int dist = (s & 4) ? (kind ? -3 : -1) : (kind ? 3 : 1);
        const int nb = hop_cb(g, i, c, s & 3, dist);
        cx<double> m[9];
        load_link<KS_F64, 9>(links, s, g.lp, hs, m);
#pragma unroll
        for (int q = 0; q < K; ++q) {
            cx<double> v[3];
            load_psi(mv.in[q], vh, nb, v);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                cx<double> u = {0.0, 0.0};
#pragma unroll
                for (int b = 0; b < 3; ++b) cfma(u, m[a * 3 + b], v[b]);
                res[q][a].r = fma(sc, u.r, res[q][a].r);
                res[q][a].i = fma(sc, u.i, res[q][a].i);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < K; ++q)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            res[q][a].r += __shfl_xor(res[q][a].r, 1, 64);
            res[q][a].i += __shfl_xor(res[q][a].i, 1, 64);
        }
    if (!live || kind) return;
#pragma unroll
    for (int q = 0; q < K; ++q)
#pragma unroll
        for (int a = 0; a < 3; ++a) mv.out[q][(size_t)a * vh + h] = make_double2(res[q][a].r, res[q][a].i);
}

template <int K>
void launch_multi_k(int k, unsigned nb, const Geom& G, const LinkStore& st, const MultiVec& mv,
                    hipStream_t s)
{
    if constexpr (K > 1) {
        if (k < K) {
            launch_multi_k<K - 1>(k, nb, G, st, mv, s);
            return;
        }
    }
    dslash_multi_kernel<K><<<nb, kBlock, 0, s>>>(G, 1, st.fat[1], st.naik[1], mv, st.fat_scale,
                                                st.naik_scale);
}

void launch_multi(int k, unsigned nb, const Geom& G, const LinkStore& st, const MultiVec& mv,
                  hipStream_t s)
{
    launch_multi_k<kMultiMax>(k, nb, G, st, mv, s);
}

// One block: kOuterSites consecutive lexicographic sites x the four directions (wave w takes
// mu = w), so the four waves that read a site's vectors share them through one CU's L1; blocks
// are remapped so that each XCD walks one contiguous range of sites.  Thread (mu, x) writes
// link t = mu V + x.
constexpr int kOuterSites = 64;

__global__ __launch_bounds__(4 * kOuterSites) void force_outer_kernel(Geom g, Terms terms,
                                                                      double2* __restrict__ fv,
                                                                      double2* __restrict__ fw)
{
    const int mu = threadIdx.x / kOuterSites;
    const int lane = threadIdx.x % kOuterSites;
    const long x0 = (long)xcd_tile(blockIdx.x, gridDim.x) * kOuterSites;
    const bool full = x0 + kOuterSites <= g.V;   // uniform over the block
    const long xl = x0 + lane;
    if (!full && xl >= g.V) return;               // only in a ragged last block
    const int x = (int)(xl < g.V ? xl : g.V - 1);
    const long t = (long)mu * g.V + x;
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
    if (full) {
        // stage each wave's 64 consecutive links in LDS, then store them as one contiguous,
        // streamed run (a lane's own 144 bytes at a 144-byte lane stride, stored directly,
        // measured slower; streamed without staging, far slower)
        __shared__ dvec2 stage[4][kOuterSites * 9];
        dvec2* sw = stage[mu];
        dvec2* o1 = reinterpret_cast<dvec2*>(fv + ((size_t)mu * g.V + x0) * 9);
        dvec2* o3 = reinterpret_cast<dvec2*>(fw + ((size_t)mu * g.V + x0) * 9);
#pragma unroll
        for (int e = 0; e < 9; ++e) sw[lane * 9 + e] = dvec2{eps * a1[e].r, eps * a1[e].i};
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 9; ++k)
            __builtin_nontemporal_store(sw[k * kOuterSites + lane], o1 + k * kOuterSites + lane);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 9; ++e) sw[lane * 9 + e] = dvec2{eps * a3[e].r, eps * a3[e].i};
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 9; ++k)
            __builtin_nontemporal_store(sw[k * kOuterSites + lane], o3 + k * kOuterSites + lane);
        return;
    }
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
        import_field(G, KS_F64, x_even[i], w.force_psi[2 * i], s);
        terms.psi[0][i] = reinterpret_cast<const double2*>(w.force_psi[2 * i]);
        terms.psi[1][i] = reinterpret_cast<const double2*>(w.force_psi[2 * i + 1]);
        terms.r[i] = residues[i];
    }
    // Y_i = D_oe X_i, up to kMultiMax terms per pass over the odd sites' links
    const LinkStore& st = g->store[KS_F64][recon_index(KS_RECON_18)];
    if (!st.ready) gauge_prepare(g, KS_F64, KS_RECON_18, s);
    for (int i0 = 0; i0 < nterm; i0 += kMultiMax) {
        const int k = std::min(kMultiMax, nterm - i0);
        MultiVec mv{};
        for (int q = 0; q < k; ++q) {
            mv.in[q] = terms.psi[0][i0 + q];
            mv.out[q] = reinterpret_cast<double2*>(w.force_psi[2 * (i0 + q) + 1]);
        }
        const unsigned nb = (unsigned)blocks_for(2L * G.Vh);   // two lanes per site
        launch_multi(k, nb, G, st, mv, s);
        KS_HIP(hipGetLastError());
    }
    force_outer_kernel<<<(unsigned)((G.V + kOuterSites - 1) / kOuterSites), 4 * kOuterSites, 0, s>>>(
        G, terms, reinterpret_cast<double2*>(force_fat), reinterpret_cast<double2*>(force_naik));
    KS_HIP(hipGetLastError());
}

}  // namespace ks
