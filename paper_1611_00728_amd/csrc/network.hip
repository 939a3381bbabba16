// Gauge-covariant preconditioner network on the GPU: forward (inference), adjoint and
// weight-gradient passes, A-norm loss, Adam.
//
// Layer:  y_c(x) = sum_{c', p} w_{c c' p} (T_p phi_{c'})(x), nine paths p: the identity,
// T_{+mu} phi(x) = V_mu(x) phi(x+mu) (p = 1+mu) and T_{-mu} phi(x) = V_mu(x-mu)^+ phi(x-mu)
// (p = 5+mu), with the operator's fat link V.  The network is N = L^+ L, L two free layers
// (1 -> 8 -> 8): it applies four layers 1 -> 8 -> 8 -> 8 -> 1, the last two the adjoints of
// the first two, so N is Hermitian and <v, N v> = |L v|^2 (no activation).
// Activations live on the full lattice as two checkerboard halves, [parity][channel][colour][Vh]
// complex FP32.  The FP32 channel mixing runs on the vector ALUs (training, and the reference
// inference path); the inference path also has an MFMA form (network_mfma.hip).
//
// The adjoint of a layer, y -> sum_p T_p^+ W_p^H y, is again a layer: channels swapped,
// weights w'_{c' c pbar} = conj(w_{c c' p}), pbar the reversed path (T_{+mu}^+ = T_{-mu}).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ks_device.h"
#include "ks_net.h"
#include "ks_solvers.h"

namespace ks {

namespace {

constexpr int kNT = 256;

template <int C>
__device__ __forceinline__ const float2* act_ptr(const float2* a, int par, int c, int k, int vh)
{
    return a + ((size_t)(par * C + c) * 3 + k) * vh;
}

// one thread per site of the full lattice (t < Vh: even, else odd)
template <int CIN, int COUT>
__global__ __launch_bounds__(kNT) void net_layer_kernel(Geom g, const float2* __restrict__ in,
                                                        float2* __restrict__ out,
                                                        const void* __restrict__ fat_e,
                                                        const void* __restrict__ fat_o,
                                                        const float2* __restrict__ w,
                                                        const int* __restrict__ gate)
{
    if (gate && *gate) return;
    const int vh = g.Vh;
    // each XCD takes one contiguous range of sites, so its L2 holds most neighbour activations
    const int t = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (t >= 2 * vh) return;
    const int par = t >= vh ? 1 : 0;
    const int h = t - par * vh;
    const void* fat = par ? fat_o : fat_e;
    int c[4];
    cb_coords(g, h, par, c);
    const int i = site_index(g, c);
    cx<float> y[COUT][3];
#pragma unroll
    for (int o = 0; o < COUT; ++o)
#pragma unroll
        for (int k = 0; k < 3; ++k) y[o][k] = {0.f, 0.f};
    // identity path
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci) {
        cx<float> v[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float2 q = act_ptr<CIN>(in, par, ci, k, vh)[h];
            v[k] = {q.x, q.y};
        }
#pragma unroll
        for (int o = 0; o < COUT; ++o) {
            const float2 ww = w[(o * CIN + ci) * 9];
            const cx<float> wc = {ww.x, ww.y};
#pragma unroll
            for (int k = 0; k < 3; ++k) cfma(y[o][k], wc, v[k]);
        }
    }
#pragma unroll 1
    for (int s = 0; s < 8; ++s) {
        const int mu = s & 3;
        const bool bwd = s >= 4;
        const int nbh = hop_cb(g, i, c, mu, bwd ? -1 : +1);
        const int p = bwd ? 5 + mu : 1 + mu;
        cx<float> m[9];
        load_link<KS_F32, 9>(fat, s, g.lp, h, m);
        if (bwd) {   // stored -V_mu(x-mu)^+
#pragma unroll
            for (int e = 0; e < 9; ++e) m[e] = {-m[e].r, -m[e].i};
        }
#pragma unroll
        for (int ci = 0; ci < CIN; ++ci) {
            cx<float> v[3], tv[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float2 q = act_ptr<CIN>(in, 1 - par, ci, k, vh)[nbh];
                v[k] = {q.x, q.y};
                tv[k] = {0.f, 0.f};
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) cfma(tv[a], m[a * 3 + b], v[b]);
#pragma unroll
            for (int o = 0; o < COUT; ++o) {
                const float2 ww = w[(o * CIN + ci) * 9 + p];
                const cx<float> wc = {ww.x, ww.y};
#pragma unroll
                for (int k = 0; k < 3; ++k) cfma(y[o][k], wc, tv[k]);
            }
        }
    }
#pragma unroll
    for (int o = 0; o < COUT; ++o)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            const_cast<float2*>(act_ptr<COUT>(out, par, o, k, vh))[h] = make_float2(y[o][k].r, y[o][k].i);
}

// G_w[c][c'][p] += sum over sites and colours of conj((T_p phi_c')(x)_a) G_c(x)_a.
// A block walks tiles of kWTile sites.  Per tile it stages G (all output channels) in LDS once,
// then per path the transported inputs u = T_p phi (all input channels, two per thread); every
// thread owns one (c, c') pair and a slice of the tile's sites and accumulates its conj(u) G
// products per path in FP64 registers across all tiles.  At the end the slices of each pair
// are summed in a fixed order and the block writes one partial per value.
constexpr int kWTile = 64;
constexpr int kWPitch = 3 * kWTile + 4;    // float2 per channel row of a stage (bank spread)

template <int CIN, int COUT>
__global__ __launch_bounds__(kNT) void net_wgrad_kernel(Geom g, const float2* __restrict__ in,
                                                        const float2* __restrict__ gy,
                                                        const void* __restrict__ fat_e,
                                                        const void* __restrict__ fat_o,
                                                        double* __restrict__ partials)
{
    constexpr int NPAIR = COUT * CIN;
    constexpr int TPP = kNT / NPAIR;            // threads per (c, c') pair
    constexpr int SPT = kWTile / TPP;           // sites per thread and tile
    static_assert(kNT % NPAIR == 0 && kWTile % TPP == 0, "wgrad tiling");
    __shared__ float2 gs[COUT * kWPitch];
    __shared__ float2 us[CIN * kWPitch];
    __shared__ double red[2 * 9 * kNT];
    const int vh = g.Vh;
    const int tid = threadIdx.x;
    const int pair = tid % NPAIR, slice = tid / NPAIR;
    const int co = pair / CIN, ci = pair % CIN;
    double ar[9], ai[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) ar[p] = ai[p] = 0.0;
    const int ntiles = (2 * vh + kWTile - 1) / kWTile;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        // ---- G of the tile's sites, every output channel
        for (int e = tid; e < COUT * 3 * kWTile; e += kNT) {
            const int site = e % kWTile, k = (e / kWTile) % 3, o = e / (3 * kWTile);
            const int t = tile * kWTile + site;
            float2 v = make_float2(0.f, 0.f);
            if (t < 2 * vh) {
                const int par = t >= vh ? 1 : 0;
                v = act_ptr<COUT>(gy, par, o, k, vh)[t - par * vh];
            }
            gs[o * kWPitch + k * kWTile + site] = v;
        }
        // ---- per path: u = T_p phi for every input channel, then the products
        const int site = tid % kWTile, cgrp = tid / kWTile;     // 4 groups of input channels
        const int t = tile * kWTile + site;
        const bool live = t < 2 * vh;
        const int par = (live && t >= vh) ? 1 : 0;
        const int h = live ? t - par * vh : 0;
        int c[4];
        cb_coords(g, h, par, c);
        const int i = site_index(g, c);
        const void* fat = par ? fat_o : fat_e;
#pragma unroll 1
        for (int p = 0; p < 9; ++p) {
            __syncthreads();     // the previous path's products are done with us (and gs is in)
            cx<float> m[9];
            int nbh = h, spar = par;
            if (p > 0) {
                const int s = p - 1;
                nbh = hop_cb(g, i, c, s & 3, s >= 4 ? -1 : +1);
                spar = 1 - par;
                load_link<KS_F32, 9>(fat, s, g.lp, h, m);
                if (s >= 4)   // the store holds -V(x-mu)^+
#pragma unroll
                    for (int e = 0; e < 9; ++e) m[e] = {-m[e].r, -m[e].i};
            }
            for (int q = cgrp; q < CIN; q += kNT / kWTile) {
                cx<float> v[3], u[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const float2 x = live ? act_ptr<CIN>(in, spar, q, k, vh)[nbh]
                                          : make_float2(0.f, 0.f);
                    v[k] = {x.x, x.y};
                }
                if (p == 0) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) u[k] = v[k];
                } else {
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        u[a] = {0.f, 0.f};
#pragma unroll
                        for (int b = 0; b < 3; ++b) cfma(u[a], m[a * 3 + b], v[b]);
                    }
                }
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    us[q * kWPitch + k * kWTile + site] = make_float2(u[k].r, u[k].i);
            }
            __syncthreads();
            float sr = 0.f, si = 0.f;
#pragma unroll 4
            for (int j = 0; j < SPT; ++j) {
                const int st = slice * SPT + j;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const float2 u = us[ci * kWPitch + k * kWTile + st];
                    const float2 gv = gs[co * kWPitch + k * kWTile + st];
                    // conj(u) g
                    sr = fmaf(u.x, gv.x, fmaf(u.y, gv.y, sr));
                    si = fmaf(u.x, gv.y, fmaf(-u.y, gv.x, si));
                }
            }
            ar[p] += sr;
            ai[p] += si;
        }
        __syncthreads();         // gs is rewritten by the next tile
    }
    // ---- sum the TPP slices of each pair in slice order, one partial per value
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        red[(2 * p) * kNT + tid] = ar[p];
        red[(2 * p + 1) * kNT + tid] = ai[p];
    }
    __syncthreads();
    constexpr int NV = NPAIR * 9 * 2;
    for (int k = tid; k < NV; k += kNT) {
        // k in the weight order ((o*CIN + ci)*9 + p)*2 + reim
        const int reim = k & 1;
        const int p = (k >> 1) % 9;
        const int pr = (k >> 1) / 9;           // = o * CIN + ci
        double s = 0.0;
        for (int sl = 0; sl < TPP; ++sl) s += red[(2 * p + reim) * kNT + sl * NPAIR + pr];
        partials[(size_t)blockIdx.x * NV + k] = s;
    }
}

// grad[k] += sum_b partials[b][k]: one block per value, strided thread sums and a block tree
// (fixed order)
__global__ __launch_bounds__(kNT) void net_grad_finish_kernel(const double* __restrict__ partials,
                                                              int nblocks, int nv,
                                                              double* __restrict__ grad)
{
    const int k = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kNT) s += partials[(size_t)b * nv + k];
    s = block_sum<kNT>(s);
    if (threadIdx.x == 0) grad[k] += s;
}

// w'[c'][c][pbar] = conj(w[c][c'][p])
__global__ void net_adjoint_weights_kernel(const float2* __restrict__ w, float2* __restrict__ wa,
                                           int cin, int cout)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cin * cout * 9) return;
    const int p = k % 9, ci = (k / 9) % cin, o = k / (9 * cin);
    const int pb = p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4);
    const float2 v = w[k];
    wa[(ci * cout + o) * 9 + pb] = make_float2(v.x, -v.y);
}

// network input: even sites from a complex128 [Vh][3] vector times `scale`, odd sites zero
__global__ void net_embed_kernel(int vh, const double2* __restrict__ src, double scale,
                                 float2* __restrict__ act)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double2 v = src[(size_t)h * 3 + k];
        act[(size_t)k * vh + h] = make_float2((float)(v.x * scale), (float)(v.y * scale));
        act[(size_t)(3 + k) * vh + h] = make_float2(0.f, 0.f);
    }
}

// network output (even sites of the last layer) times `scale` into complex128 [Vh][3]
__global__ void net_extract_kernel(int vh, const float2* __restrict__ act, double scale,
                                   double2* __restrict__ dst)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float2 v = act[(size_t)k * vh + h];
        dst[(size_t)h * 3 + k] = make_double2(v.x * scale, v.y * scale);
    }
}

// A-norm loss term of one pair and the output gradient: with y = N(b) (even sites of the last
// layer) and ay = A y (FP64 planes), partial sums of Re<y - x, A y - b> = (y - x)^+ A (y - x)
// (A x = b) and G = coef (A y - b) on even sites, 0 on odd ones (the Wirtinger gradient of
// the pair's loss is 2 A (y - x) over its normalisation).
__global__ __launch_bounds__(kNT) void net_anorm_loss_kernel(int vh, const float2* __restrict__ y,
                                                             const double2* __restrict__ ay,
                                                             const double2* __restrict__ b,
                                                             const double2* __restrict__ x,
                                                             double coef, float2* __restrict__ gy,
                                                             double* __restrict__ partials)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (h < vh) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float2 o = y[(size_t)k * vh + h];
            const double2 a = ay[(size_t)k * vh + h];
            const double2 bv = b[(size_t)h * 3 + k];
            const double2 xv = x[(size_t)h * 3 + k];
            const double rr = a.x - bv.x, ri = a.y - bv.y;
            s += (o.x - xv.x) * rr + (o.y - xv.y) * ri;
            gy[(size_t)k * vh + h] = make_float2((float)(coef * rr), (float)(coef * ri));
            gy[(size_t)(3 + k) * vh + h] = make_float2(0.f, 0.f);
        }
    }
    s = block_sum<kNT>(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// even sites of the last layer (FP32 planes) -> FP64 planes [3][Vh]
__global__ void net_out_f64_kernel(int vh, const float2* __restrict__ y, double2* __restrict__ out)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float2 v = y[(size_t)k * vh + h];
        out[(size_t)k * vh + h] = make_double2(v.x, v.y);
    }
}

// partials of Re<x, b> of two complex128 [Vh][3] vectors
__global__ __launch_bounds__(kNT) void net_rdot_kernel(int vh, const double2* __restrict__ x,
                                                       const double2* __restrict__ b,
                                                       double* __restrict__ partials)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (h < vh)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double2 u = x[(size_t)h * 3 + k], v = b[(size_t)h * 3 + k];
            s += u.x * v.x + u.y * v.y;
        }
    s = block_sum<kNT>(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__device__ __forceinline__ int reversed_path(int p) { return p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4); }

// FP32 weights of the four applied layers from the FP64 free weights: layers 1 and 2 as they
// are, layer 3 = adjoint of layer 2, layer 4 = adjoint of layer 1
// (w'[c'][c][pbar] = conj(w[c][c'][p])).
__global__ void net_expand_kernel(const double2* __restrict__ w, float2* __restrict__ w32)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    constexpr int n1 = 8 * 1 * 9, n2 = 8 * 8 * 9;
    if (k >= kNetLayerWeights) return;
    double2 v;
    if (k < n1 + n2) {
        v = w[k];
    } else if (k < n1 + 2 * n2) {
        const int j = k - n1 - n2;                        // layer 3: [c'][c][q], 8 x 8
        const int q = j % 9, c = (j / 9) % 8, cp = j / 72;
        const double2 u = w[n1 + (c * 8 + cp) * 9 + reversed_path(q)];
        v = make_double2(u.x, -u.y);
    } else {
        const int j = k - n1 - 2 * n2;                    // layer 4: [0][c][q]
        const int q = j % 9, c = j / 9;
        const double2 u = w[c * 9 + reversed_path(q)];
        v = make_double2(u.x, -u.y);
    }
    w32[k] = make_float2((float)v.x, (float)v.y);
}

// Gradient of the free weights from the four layers' gradients: a free weight collects its
// own layer's G plus the conjugate of G at its place in the adjoint layer.
__global__ void net_fold_kernel(const double2* __restrict__ g4, double2* __restrict__ g)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    constexpr int n1 = 8 * 1 * 9, n2 = 8 * 8 * 9;
    if (k >= kNetWeights) return;
    double2 a = g4[k], t;
    if (k < n1) {                                          // w1[c][0][p]
        const int p = k % 9, c = k / 9;
        t = g4[n1 + 2 * n2 + c * 9 + reversed_path(p)];    // layer 4 [0][c][pbar]
    } else {                                               // w2[c][c'][p]
        const int j = k - n1;
        const int p = j % 9, cp = (j / 9) % 8, c = j / 72;
        t = g4[n1 + n2 + (cp * 8 + c) * 9 + reversed_path(p)];   // layer 3 [c'][c][pbar]
    }
    g[k] = make_double2(a.x + t.x, a.y - t.y);
}

// network input from an inner-precision field: even sites r * scale (scale null: 1), odd sites
// zero
template <int P>
__global__ void net_embed_spinor_kernel(int vh, const void* __restrict__ r,
                                        const double* __restrict__ scale, float2* __restrict__ act,
                                        const int* __restrict__ gate)
{
    if (gate && *gate) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
    const float sc = scale ? (float)*scale : 1.f;
    cx<typename St<P>::R> v[3];
    Spinor<P>::load(r, vh, h, v);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        act[(size_t)k * vh + h] = make_float2(sc * (float)v[k].r, sc * (float)v[k].i);
        act[(size_t)(3 + k) * vh + h] = make_float2(0.f, 0.f);
    }
}

// network output (even sites of the last layer) divided by scale (null: 1) into an
// inner-precision field
template <int P>
__global__ void net_extract_spinor_kernel(int vh, const float2* __restrict__ act,
                                          const double* __restrict__ scale, void* __restrict__ z,
                                          const int* __restrict__ gate)
{
    if (gate && *gate) return;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
    const float inv = (float)(1.0 / (scale ? *scale : 1.0));
    using R = typename St<P>::R;
    cx<R> v[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float2 a = act[(size_t)k * vh + h];
        v[k] = {(R)(inv * a.x), (R)(inv * a.y)};
    }
    Spinor<P>::store(z, vh, h, v);
}

// One Adam step on every real of the FP64 master weights.
__global__ void net_adam_kernel(double* __restrict__ w, double* __restrict__ m,
                                double* __restrict__ v, const double* __restrict__ grad, int n,
                                double lr, double b1, double b2, double eps, double c1, double c2)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double gk = grad[k];
    const double mk = b1 * m[k] + (1.0 - b1) * gk;
    const double vk = b2 * v[k] + (1.0 - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const double mh = mk / c1, vhat = vk / c2;
    w[k] = w[k] - lr * mh / (sqrt(vhat) + eps);
}

template <int CIN, int COUT>
void layer(ks_gauge_t g, const float2* in, float2* out, const float2* w, hipStream_t s,
           const int* gate = nullptr)
{
    const LinkStore& st = g->store[KS_F32][0];
    net_layer_kernel<CIN, COUT><<<blocks_for(2L * g->geom.Vh, kNT), kNT, 0, s>>>(
        g->geom, in, out, st.fat[0], st.fat[1], w, gate);
    KS_HIP(hipGetLastError());
}

void expand_weights(NetCtx& n, hipStream_t s)
{
    net_expand_kernel<<<blocks_for(kNetLayerWeights, 256), 256, 0, s>>>(
        reinterpret_cast<const double2*>(n.w64), reinterpret_cast<float2*>(n.w32));
    KS_HIP(hipGetLastError());
}

template <int CIN, int COUT>
void wgrad(NetCtx& n, NetBuffers& B, ks_gauge_t g, const float2* in, const float2* gy,
           double* grad, hipStream_t s)
{
    const LinkStore& st = g->store[KS_F32][0];
    constexpr int NV = COUT * CIN * 9 * 2;
    const int nb = std::min(blocks_for(2L * g->geom.Vh, kWTile), kWgradBlocks);
    net_wgrad_kernel<CIN, COUT><<<nb, kNT, 0, s>>>(g->geom, in, gy, st.fat[0], st.fat[1], B.wpart);
    net_grad_finish_kernel<<<NV, kNT, 0, s>>>(B.wpart, nb, NV, grad);
    KS_HIP(hipGetLastError());
}

}  // namespace

const int kLayerIn[4] = {1, 8, 8, 8};

double net_model_bytes(int use_mfma, double vec_bytes)
{
    if (use_mfma) return 2.0 * net_mfma_model_bytes_per_site(vec_bytes);
    // per site of the full lattice each FP32 layer reads its site's eight stored links and
    // its input channels and writes its output channels (FP32 complex colour vectors); the
    // input is embedded on both parities and the output read back on the even sites
    double total = 0.0;
    for (int l = 0; l < 4; ++l) total += 8 * 72 + 24.0 * (kLayerIn[l] + kLayerOut[l]);
    return 2.0 * total + vec_bytes + 2 * 24.0 + 24.0 + vec_bytes;
}
const int kLayerOut[4] = {8, 8, 8, 1};

size_t layer_weight_offset(int l)
{
    size_t o = 0;
    for (int k = 0; k < l; ++k) o += (size_t)kLayerIn[k] * kLayerOut[k] * 9;
    return o;
}

NetBuffers& net_buffers(NetCtx& n, const Geom& g)
{
    NetBuffers& B = n.bufs[g.Vh];
    if (!B.act[0]) {
        const size_t site = (size_t)2 * 3 * g.Vh * sizeof(float2);   // one channel, both parities
        const int ch[5] = {1, 8, 8, 8, 1};
        for (int l = 0; l < 5; ++l) {
            B.act[l] = static_cast<float2*>(device_alloc(site * ch[l]));
            B.grad[l] = static_cast<float2*>(device_alloc(site * ch[l]));
        }
        B.npart = blocks_for(g.Vh, kNT);
        B.part = static_cast<double*>(device_alloc(sizeof(double) * (B.npart + 8)));
        B.wpart = static_cast<double*>(device_alloc(sizeof(double) * kWgradBlocks * 8 * 8 * 9 * 2));
        B.vh = g.Vh;
    }
    return B;
}

void net_free(NetCtx* n)
{
    if (!n) return;
    for (auto& kv : n->bufs) {
        for (int l = 0; l < 5; ++l) {
            device_free(kv.second.act[l]);
            device_free(kv.second.grad[l]);
            device_free(kv.second.act16[l]);
        }
        device_free(kv.second.part);
        device_free(kv.second.wpart);
    }
    device_free(n->w64);
    device_free(n->w32);
    device_free(n->wadj);
    device_free(n->adam_m);
    device_free(n->adam_v);
    device_free(n->grad);
    device_free(n->grad4);
    device_free(n->scal);
    device_free(n->wmma);
    if (n->host) (void)hipHostFree(n->host);
    delete n;
}

NetCtx* net_create(const double* w_host)
{
    NetCtx* n = new NetCtx();
    try {
        const size_t nr = 2 * (size_t)kNetWeights;
        const size_t nl = 2 * (size_t)kNetLayerWeights;
        n->w64 = static_cast<double*>(device_alloc(sizeof(double) * nr));
        n->w32 = static_cast<float*>(device_alloc(sizeof(float) * nl));
        n->wadj = static_cast<float*>(device_alloc(sizeof(float) * nl));
        n->adam_m = static_cast<double*>(device_alloc(sizeof(double) * nr));
        n->adam_v = static_cast<double*>(device_alloc(sizeof(double) * nr));
        n->grad = static_cast<double*>(device_alloc(sizeof(double) * nr));
        n->grad4 = static_cast<double*>(device_alloc(sizeof(double) * nl));
        n->scal = static_cast<double*>(device_alloc(sizeof(double) * 64));
        KS_HIP(hipHostMalloc(reinterpret_cast<void**>(&n->host), sizeof(double) * 64));
        net_set_weights(*n, w_host, nullptr);
    } catch (...) {
        net_free(n);
        throw;
    }
    return n;
}

void net_set_weights(NetCtx& n, const double* w_host, hipStream_t s)
{
    const int nr = 2 * kNetWeights;
    KS_HIP(hipMemcpyAsync(n.w64, w_host, sizeof(double) * nr, hipMemcpyHostToDevice, s));
    KS_HIP(hipMemsetAsync(n.adam_m, 0, sizeof(double) * nr, s));
    KS_HIP(hipMemsetAsync(n.adam_v, 0, sizeof(double) * nr, s));
    expand_weights(n, s);
    KS_HIP(hipStreamSynchronize(s));
    n.step = 0;
    n.version += 1;
}

void net_get_weights(NetCtx& n, double* w_host, hipStream_t s)
{
    KS_HIP(hipMemcpyAsync(w_host, n.w64, sizeof(double) * 2 * kNetWeights, hipMemcpyDeviceToHost, s));
    KS_HIP(hipStreamSynchronize(s));
}

void net_get_state(NetCtx& n, double* w, double* m, double* v, int* step, hipStream_t s)
{
    const size_t nb = sizeof(double) * 2 * kNetWeights;
    KS_HIP(hipMemcpyAsync(w, n.w64, nb, hipMemcpyDeviceToHost, s));
    KS_HIP(hipMemcpyAsync(m, n.adam_m, nb, hipMemcpyDeviceToHost, s));
    KS_HIP(hipMemcpyAsync(v, n.adam_v, nb, hipMemcpyDeviceToHost, s));
    KS_HIP(hipStreamSynchronize(s));
    *step = n.step;
}

void net_set_state(NetCtx& n, const double* w, const double* m, const double* v, int step,
                   hipStream_t s)
{
    const size_t nb = sizeof(double) * 2 * kNetWeights;
    KS_HIP(hipMemcpyAsync(n.w64, w, nb, hipMemcpyHostToDevice, s));
    KS_HIP(hipMemcpyAsync(n.adam_m, m, nb, hipMemcpyHostToDevice, s));
    KS_HIP(hipMemcpyAsync(n.adam_v, v, nb, hipMemcpyHostToDevice, s));
    expand_weights(n, s);
    KS_HIP(hipStreamSynchronize(s));
    n.step = step;
    n.version += 1;
}

// Forward through the four layers, input already in act[0]; activations of every layer kept.
void net_forward(NetCtx& n, NetBuffers& B, ks_gauge_t g, hipStream_t s)
{
    const float2* w = reinterpret_cast<const float2*>(n.w32);
    layer<1, 8>(g, B.act[0], B.act[1], w + layer_weight_offset(0), s);
    layer<8, 8>(g, B.act[1], B.act[2], w + layer_weight_offset(1), s);
    layer<8, 8>(g, B.act[2], B.act[3], w + layer_weight_offset(2), s);
    layer<8, 1>(g, B.act[3], B.act[4], w + layer_weight_offset(3), s);
}

// out_dev = N(in_dev) (complex128 [Vh][3], even sites); FP32 vector-ALU mixing.
void net_apply_f32(NetCtx& n, ks_gauge_t g, const double* in, double* out, double in_scale,
                   hipStream_t s)
{
    gauge_prepare(g, KS_F32, KS_RECON_18, s);
    NetBuffers& B = net_buffers(n, g->geom);
    const int vh = g->geom.Vh;
    net_embed_kernel<<<blocks_for(vh), kBlock, 0, s>>>(vh, reinterpret_cast<const double2*>(in),
                                                       in_scale, B.act[0]);
    net_forward(n, B, g, s);
    net_extract_kernel<<<blocks_for(vh), kBlock, 0, s>>>(vh, B.act[4], 1.0 / in_scale,
                                                         reinterpret_cast<double2*>(out));
    KS_HIP(hipGetLastError());
}

void net_apply_spinor(NetCtx& n, ks_gauge_t g, ks_prec_t prec, const void* r, void* z,
                      const double* in_scale, const int* gate, int use_mfma, hipStream_t s)
{
    KS_REQUIRE(prec == KS_F64 || prec == KS_F32, KS_ERR_ARG,
               "network: the solver's vectors must be FP64 or FP32");
    if (use_mfma) {
        net_apply_mfma_spinor(n, g, prec, r, z, in_scale, gate, s);
        return;
    }
    gauge_prepare(g, KS_F32, KS_RECON_18, s);
    NetBuffers& B = net_buffers(n, g->geom);
    const int vh = g->geom.Vh;
    const int nb = blocks_for(vh);
    const float2* w = reinterpret_cast<const float2*>(n.w32);
    if (prec == KS_F64)
        net_embed_spinor_kernel<KS_F64><<<nb, kBlock, 0, s>>>(vh, r, in_scale, B.act[0], gate);
    else
        net_embed_spinor_kernel<KS_F32><<<nb, kBlock, 0, s>>>(vh, r, in_scale, B.act[0], gate);
    layer<1, 8>(g, B.act[0], B.act[1], w + layer_weight_offset(0), s, gate);
    layer<8, 8>(g, B.act[1], B.act[2], w + layer_weight_offset(1), s, gate);
    layer<8, 8>(g, B.act[2], B.act[3], w + layer_weight_offset(2), s, gate);
    layer<8, 1>(g, B.act[3], B.act[4], w + layer_weight_offset(3), s, gate);
    if (prec == KS_F64)
        net_extract_spinor_kernel<KS_F64><<<nb, kBlock, 0, s>>>(vh, B.act[4], in_scale, z, gate);
    else
        net_extract_spinor_kernel<KS_F32><<<nb, kBlock, 0, s>>>(vh, B.act[4], in_scale, z, gate);
    KS_HIP(hipGetLastError());
}

// A-norm loss of the pairs and its gradient: the four applied layers' gradients accumulate in
// n.grad4 (zeroed first), then fold into the free weights' gradient n.grad.
double net_loss_grad(NetCtx& n, int npairs, const ks_gauge_t* gauges, const double* sigma,
                     const double* const* b, const double* const* x, hipStream_t s)
{
    KS_HIP(hipMemsetAsync(n.grad4, 0, sizeof(double) * 2 * kNetLayerWeights, s));
    const float2* w = reinterpret_cast<const float2*>(n.w32);
    float2* wa = reinterpret_cast<float2*>(n.wadj);
    for (int l = 1; l < 4; ++l) {
        const size_t o = layer_weight_offset(l);
        net_adjoint_weights_kernel<<<blocks_for(kLayerIn[l] * kLayerOut[l] * 9, 256), 256, 0, s>>>(
            w + o, wa + o, kLayerIn[l], kLayerOut[l]);
    }
    KS_HIP(hipGetLastError());
    double loss = 0.0;
    for (int j = 0; j < npairs; ++j) {
        ks_gauge_t g = gauges[j];
        gauge_prepare(g, KS_F32, KS_RECON_18, s);
        Workspace& ws = workspace(g);
        NetBuffers& B = net_buffers(n, g->geom);
        const int vh = g->geom.Vh;
        const int nb = blocks_for(vh, kNT);
        const double2* bj = reinterpret_cast<const double2*>(b[j]);
        const double2* xj = reinterpret_cast<const double2*>(x[j]);
        // x^+ A x = Re<x, b>
        net_rdot_kernel<<<nb, kNT, 0, s>>>(vh, xj, bj, B.part);
        reduce_sum(B.part, nb, n.scal, s);
        KS_HIP(hipMemcpyAsync(n.host, n.scal, sizeof(double), hipMemcpyDeviceToHost, s));
        KS_HIP(hipStreamSynchronize(s));
        const double xax = n.host[0];
        KS_REQUIRE(xax > 0, KS_ERR_ARG, "network training: pair %d has Re<x, b> <= 0", j);
        net_embed_kernel<<<blocks_for(vh), kBlock, 0, s>>>(vh, bj, 1.0, B.act[0]);
        net_forward(n, B, g, s);
        // A y in FP64 on the pair's lattice
        net_out_f64_kernel<<<blocks_for(vh), kBlock, 0, s>>>(vh, B.act[4],
                                                             reinterpret_cast<double2*>(ws.r64));
        apply_A64(g, sigma[j], ws.r64, ws.ax64, s, nullptr);
        net_anorm_loss_kernel<<<nb, kNT, 0, s>>>(vh, B.act[4],
                                                 reinterpret_cast<const double2*>(ws.ax64), bj, xj,
                                                 2.0 / (xax * npairs), B.grad[4], B.part);
        reduce_sum(B.part, nb, n.scal + 1, s);
        KS_HIP(hipMemcpyAsync(n.host + 1, n.scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        // backward: weight gradients and the adjoint layers
        double* gr = n.grad4;
        wgrad<8, 1>(n, B, g, B.act[3], B.grad[4], gr + 2 * layer_weight_offset(3), s);
        layer<1, 8>(g, B.grad[4], B.grad[3], wa + layer_weight_offset(3), s);
        wgrad<8, 8>(n, B, g, B.act[2], B.grad[3], gr + 2 * layer_weight_offset(2), s);
        layer<8, 8>(g, B.grad[3], B.grad[2], wa + layer_weight_offset(2), s);
        wgrad<8, 8>(n, B, g, B.act[1], B.grad[2], gr + 2 * layer_weight_offset(1), s);
        layer<8, 8>(g, B.grad[2], B.grad[1], wa + layer_weight_offset(1), s);
        wgrad<1, 8>(n, B, g, B.act[0], B.grad[1], gr + 2 * layer_weight_offset(0), s);
        KS_HIP(hipStreamSynchronize(s));
        loss += n.host[1] / (xax * npairs);
    }
    net_fold_kernel<<<blocks_for(kNetWeights, 256), 256, 0, s>>>(
        reinterpret_cast<const double2*>(n.grad4), reinterpret_cast<double2*>(n.grad));
    KS_HIP(hipGetLastError());
    return loss;
}

void net_adam(NetCtx& n, double lr, hipStream_t s)
{
    const int nr = 2 * kNetWeights;
    n.step += 1;
    const double b1 = 0.9, b2 = 0.999;
    net_adam_kernel<<<blocks_for(nr, 256), 256, 0, s>>>(n.w64, n.adam_m, n.adam_v, n.grad, nr, lr,
                                                       b1, b2, 1e-8, 1.0 - std::pow(b1, n.step),
                                                       1.0 - std::pow(b2, n.step));
    KS_HIP(hipGetLastError());
    expand_weights(n, s);
    n.version += 1;
}

}  // namespace ks
