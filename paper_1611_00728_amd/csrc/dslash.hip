// Improved-staggered hopping term on one parity (the staggered dslash of Sec. 3):
//   (D psi)(x) = sum_mu [ V_mu(x) psi(x+mu) - V_mu(x-mu)^+ psi(x-mu)
//                       + W_mu(x) psi(x+3mu) - W_mu(x-3mu)^+ psi(x-3mu) ]
// One thread per output site.  The 16 matrices of a site stream from site-major planes
// (perfectly coalesced, read once: the bulk of the bytes); the 16 neighbour vectors are
// gathers that the XCD-aware tile order keeps inside one XCD's L2 for most hops.
#include "ks_device.h"
#include "ks_naik.h"

namespace ks {

namespace {

template <class R>
__device__ __forceinline__ void matvec_acc(cx<R> acc[3], const cx<R> m[9], const cx<R> v[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) cfma(acc[a], m[a * 3 + b], v[b]);
}

template <int P>
__device__ __forceinline__ void load_link18(const void* base, int slot, int vh, int h,
                                            cx<typename St<P>::R> m[9])
{
#pragma unroll
    for (int e = 0; e < 9; ++e) m[e] = load_entry<P>(plane_ptr<P>(base, slot * 9 + e, vh), h);
}

// rows 0, 1 stored; row 2 = conj(row0 x row1)
template <int P>
__device__ __forceinline__ void load_link12(const void* base, int slot, int vh, int h,
                                            cx<typename St<P>::R> m[9])
{
    using R = typename St<P>::R;
#pragma unroll
    for (int e = 0; e < 6; ++e) m[e] = load_entry<P>(plane_ptr<P>(base, slot * 6 + e, vh), h);
    const cx<R> a0 = m[0], a1 = m[1], a2 = m[2], b0 = m[3], b1 = m[4], b2 = m[5];
    cx<R> t;
    t = cmul(a1, b2);
    cfma(t, {-a2.r, -a2.i}, b1);
    m[6] = {t.r, -t.i};
    t = cmul(a2, b0);
    cfma(t, {-a0.r, -a0.i}, b2);
    m[7] = {t.r, -t.i};
    t = cmul(a0, b1);
    cfma(t, {-a1.r, -a1.i}, b0);
    m[8] = {t.r, -t.i};
}

template <int P, int RECON, bool XPAY>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void dslash_kernel(Geom g, int par, const void* __restrict__ fat,
                                                        const void* __restrict__ naik,
                                                        const void* __restrict__ in,
                                                        void* __restrict__ out,
                                                        const void* __restrict__ xv, double a,
                                                        double* __restrict__ partials,
                                                        const int* __restrict__ gate,
                                                        float fat_scale, float naik_scale,
                                                        double naik_c0)
{
    using R = typename St<P>::R;
    if (gate && *gate) return;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int h = tile * kBlock + threadIdx.x;
    const int vh = g.Vh;
    double dot = 0.0;
    if (h < vh) {
        int c[4];
        cb_coords(g, h, par, c);
        const int i = site_index(g, c);
        int nb[16];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            nb[mu] = hop_cb(g, i, c, mu, +1);
            nb[4 + mu] = hop_cb(g, i, c, mu, -1);
            nb[8 + mu] = hop_cb(g, i, c, mu, +3);
            nb[12 + mu] = hop_cb(g, i, c, mu, -3);
        }
        cx<R> res[3] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll 1
        for (int s = 0; s < 16; ++s) {
            cx<R> m[9], v[3], t[3] = {{0, 0}, {0, 0}, {0, 0}};
            R sc;
            if (s < 8) {
                load_link18<P>(fat, s, vh, h, m);
                sc = (R)fat_scale;
            } else if (RECON == 12) {
                load_link12<P>(naik, s - 8, vh, h, m);
                sc = (R)(naik_c0 * naik_sign(c, s - 8, g.n[3]));
            } else {
                load_link18<P>(naik, s - 8, vh, h, m);
                sc = (R)naik_scale;
            }
            Spinor<P>::load(in, vh, nb[s], v);
            matvec_acc(t, m, v);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                res[k].r = fma(sc, t[k].r, res[k].r);
                res[k].i = fma(sc, t[k].i, res[k].i);
            }
        }
        if (XPAY) {
            cx<R> xs[3];
            Spinor<P>::load(xv, vh, h, xs);
            const R aa = (R)a;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                res[k].r = aa * xs[k].r - res[k].r;
                res[k].i = aa * xs[k].i - res[k].i;
            }
            Spinor<P>::store(out, vh, h, res);
            if (partials) {
                // Re<x, out> of the output as stored
                Spinor<P>::round(res);
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    dot += (double)xs[k].r * (double)res[k].r + (double)xs[k].i * (double)res[k].i;
            }
        } else {
            Spinor<P>::store(out, vh, h, res);
        }
    }
    if (partials) {
        const double s = block_sum<kBlock>(dot);
        if (threadIdx.x == 0) partials[tile] = s;
    }
}

template <int P, int RECON>
void launch_p(const LinkStore& st, const Geom& G, double c0, const DslashArgs& a, hipStream_t s)
{
    const int nb = dslash_blocks(G);
    const void* fat = st.fat[a.out_parity];
    const void* naik = st.naik[a.out_parity];
    if (a.x)
        dslash_kernel<P, RECON, true><<<nb, kBlock, 0, s>>>(G, a.out_parity, fat, naik, a.in, a.out,
                                                            a.x, a.a, a.dot_partials, a.gate,
                                                            st.fat_scale, st.naik_scale, c0);
    else
        dslash_kernel<P, RECON, false><<<nb, kBlock, 0, s>>>(G, a.out_parity, fat, naik, a.in, a.out,
                                                             nullptr, 0.0, nullptr, a.gate,
                                                             st.fat_scale, st.naik_scale, c0);
    KS_HIP(hipGetLastError());
}

}  // namespace

int dslash_blocks(const Geom& g) { return blocks_for(g.Vh); }

void dslash(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon, const DslashArgs& a, hipStream_t s)
{
    const int ri = recon_index(recon);
    if (!g->store[prec][ri].ready) gauge_prepare(g, prec, recon, s);
    const LinkStore& st = g->store[prec][ri];
    const Geom& G = g->geom;
    if (prec == KS_F64)
        ri ? launch_p<KS_F64, 12>(st, G, g->naik_c0, a, s) : launch_p<KS_F64, 18>(st, G, 0.0, a, s);
    else if (prec == KS_F32)
        ri ? launch_p<KS_F32, 12>(st, G, g->naik_c0, a, s) : launch_p<KS_F32, 18>(st, G, 0.0, a, s);
    else
        ri ? launch_p<KS_F16, 12>(st, G, g->naik_c0, a, s) : launch_p<KS_F16, 18>(st, G, 0.0, a, s);
}

}  // namespace ks
