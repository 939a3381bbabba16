// Batched CG: many independent lattices of uneven sizes, each with R right-hand sides, solved
// together.  One launch of each step covers every (lattice, site tile) of the batch through a
// tile table; the multi-RHS Dslash loads each link once and applies it to all R vectors of
// the site.  Every (lattice, RHS) pair keeps its own CG scalars on the device, with FP32 (or
// FP64) inner iterations, FP64 solution accumulation (through FP32 increments added in at
// each reliable update when the inner iterations are FP32) and per-pair FP64 reliable updates
// decided on the device, so a fixed sequence of kernels makes up one step and a run of steps
// is captured once into a HIP graph and replayed until every pair has converged.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "ks_batch.h"
#include "ks_device.h"

namespace ks {

namespace {

constexpr int kFin = 256;

// ---------------------------------------------------------------- multi-RHS vectors
// Lattice l's part of a vector arena: [3 colours][Vh_l][R] complex, starting at site offset
// vec_off_l (sum of the Vh of the lattices before it).  The R complex numbers of one site and
// colour are contiguous, so a lane loads them with 16-byte vector loads.

template <int P, int R>
struct MVec {
    using T = typename St<P>::R;
    static constexpr int CS = P == KS_F64 ? 16 : 8;   // bytes of one complex
    __device__ static __forceinline__ size_t off(size_t vec_off, int vh, int k, int h)
    {
        return ((vec_off * 3 + (size_t)k * vh + h) * R) * CS;
    }
    __device__ static __forceinline__ void load(const char* base, size_t vec_off, int vh, int h,
                                                cx<T> v[3][R])
    {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const char* p = base + off(vec_off, vh, k, h);
            if constexpr (P == KS_F64) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double2 t = reinterpret_cast<const double2*>(p)[r];
                    v[k][r] = {t.x, t.y};
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; r += 2) {
                    if (r + 1 < R) {
                        const float4 t = reinterpret_cast<const float4*>(p)[r / 2];
                        v[k][r] = {t.x, t.y};
                        v[k][r + 1] = {t.z, t.w};
                    } else {
                        const float2 t = reinterpret_cast<const float2*>(p)[r];
                        v[k][r] = {t.x, t.y};
                    }
                }
            }
        }
    }
    __device__ static __forceinline__ void store(char* base, size_t vec_off, int vh, int h,
                                                 const cx<T> v[3][R])
    {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            char* p = base + off(vec_off, vh, k, h);
            if constexpr (P == KS_F64) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    reinterpret_cast<double2*>(p)[r] = make_double2(v[k][r].r, v[k][r].i);
            } else {
#pragma unroll
                for (int r = 0; r < R; r += 2) {
                    if (r + 1 < R)
                        reinterpret_cast<float4*>(p)[r / 2] =
                            make_float4(v[k][r].r, v[k][r].i, v[k][r + 1].r, v[k][r + 1].i);
                    else
                        reinterpret_cast<float2*>(p)[r] = make_float2(v[k][r].r, v[k][r].i);
                }
            }
        }
    }
};

// R <= 4: the flags of all pairs are loaded together, not one after another
__device__ __forceinline__ bool lattice_busy(const BatchPair* pairs, int p0, int R, bool ru)
{
    bool busy = false;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (r < R) {
            const BatchPair& q = pairs[p0 + r];
            busy = busy || (ru ? (q.ru_now && !q.done) : !q.done);
        }
    }
    return busy;
}

// out_r = D in_r for every RHS r of the site (XPAY: out_r = sigma_r x_r - D in_r, with
// per-tile partial sums of Re<x_r, out_r>), on lattices with a pair still iterating.
template <int P, int R, bool XPAY, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void batch_dslash_kernel(
    const LatDesc* __restrict__ lats, const int2* __restrict__ tiles, int ntiles, int par,
    const char* __restrict__ in, char* __restrict__ out, const char* __restrict__ xv,
    const BatchPair* __restrict__ pairs, double* __restrict__ partials)
{
    using T = typename St<P>::R;
    using V = MVec<P, R>;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int2 tl = tiles[t];
        const LatDesc& L = lats[tl.x];
        const bool busy = lattice_busy(pairs, L.pair0, R, false);
        if (!busy) {
            if (XPAY && threadIdx.x < R) partials[(size_t)t * R + threadIdx.x] = 0.0;
            continue;
        }
        const Geom& g = L.g;
        const int vh = g.Vh;
        const int h = tl.y + threadIdx.x;
        double dot[R];
#pragma unroll
        for (int r = 0; r < R; ++r) dot[r] = 0.0;
        if (h < vh) {
            const void* fat = (P == KS_F64) ? L.fat64[par] : L.fat32[par];
            const void* naik = (P == KS_F64) ? L.naik64[par] : L.naik32[par];
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
            cx<T> res[3][R];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int r = 0; r < R; ++r) res[k][r] = {0, 0};
            // FP32: four hops per pass keep four link and neighbour loads in flight
            // (measured best; a full unroll is slower); FP64 at four hops would spill
            constexpr int kHopUnroll = P == KS_F64 ? 1 : 4;
#pragma unroll kHopUnroll
            for (int s = 0; s < 16; ++s) {
                cx<T> m[9];
                if (s < 8) load_link<P, 9>(fat, s, vh, h, m);
                else load_link<P, 9>(naik, s - 8, vh, h, m);
                cx<T> v[3][R];
                V::load(in, L.vec_off, vh, nb[s], v);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b)
#pragma unroll
                        for (int r = 0; r < R; ++r) cfma(res[a][r], m[a * 3 + b], v[b][r]);
            }
            if (XPAY) {
                cx<T> xs[3][R];
                V::load(xv, L.vec_off, vh, h, xs);
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const T sg = (T)pairs[L.pair0 + r].sigma;
                        res[k][r].r = sg * xs[k][r].r - res[k][r].r;
                        res[k][r].i = sg * xs[k][r].i - res[k][r].i;
                        dot[r] += (double)xs[k][r].r * (double)res[k][r].r +
                                  (double)xs[k][r].i * (double)res[k][r].i;
                    }
            }
            V::store(out, L.vec_off, vh, h, res);
        }
        if (XPAY) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double s = block_sum<NT>(dot[r]);
                if (threadIdx.x == 0) partials[(size_t)t * R + r] = s;
                __syncthreads();
            }
        }
    }
}

// FP64 reliable-update form of the multi-RHS hopping term (out_r = D in_r, or with XPAY
// out_r = sigma_r x_r - D in_r), for the few lattices whose update is due.  Such a launch has
// little work, so the tile walk of the inner-precision kernel would leave most of the chip
// idle and each site's chain of 16 dependent link and neighbour loads would set the time.
// Here every block first finds, with one parallel scan, the lattices with an update due and
// numbers their 64-site chunks; the chunks are spread over the whole grid; and four lanes
// share a site, each taking the four matrices of one hop kind (forward one-link, backward
// one-link, forward Naik, backward Naik): four times the waves and a quarter of the chain.
// A two-step butterfly adds the four sums (every lane ends with the same total) and lanes 0-2
// store one colour each.  No partial sums: the residual kernel that follows computes its own.
constexpr int kRuLanes = 4;                // lanes per site (8 ties, 16 is slower)
constexpr int kRuSites = 256 / kRuLanes;   // sites per chunk (one block's pass)
constexpr int kRuGrid = 1024;              // blocks of a reliable-update launch

template <int R, bool XPAY>
__global__ __launch_bounds__(256) void batch_dslash_ru_kernel(
    const LatDesc* __restrict__ lats, int nlat, int par, const char* __restrict__ in,
    char* __restrict__ out, const char* __restrict__ xv, const BatchPair* __restrict__ pairs)
{
    using V = MVec<KS_F64, R>;
    __shared__ int pref[257];   // pref[j]: chunks of the chunk-group's lattices before j
    constexpr int kM = 16 / kRuLanes;   // matrices per lane, all of one hop kind
    const int part = threadIdx.x & (kRuLanes - 1);
    const int sl = threadIdx.x / kRuLanes;
    const int kind = (part * kM) >> 2;  // 0: +1, 1: -1 (one-link), 2: +3, 3: -3 (Naik)
    const int dist = (kind & 1) ? ((kind & 2) ? -3 : -1) : ((kind & 2) ? 3 : 1);
    const int mu0 = (part * kM) & 3;
    for (int l0 = 0; l0 < nlat; l0 += 256) {
        const int l = l0 + threadIdx.x;
        int n = 0;
        if (l < nlat && lattice_busy(pairs, lats[l].pair0, R, true))
            n = (lats[l].g.Vh + kRuSites - 1) / kRuSites;
        if (threadIdx.x == 0) pref[0] = 0;
        pref[threadIdx.x + 1] = n;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {   // inclusive scan of pref[1..256]
            const int v = threadIdx.x >= off ? pref[threadIdx.x + 1 - off] : 0;
            __syncthreads();
            pref[threadIdx.x + 1] += v;
            __syncthreads();
        }
        const int total = pref[256];
        for (int u = blockIdx.x; u < total; u += gridDim.x) {
            int lo = 0, hi = 256;   // the lattice j with pref[j] <= u < pref[j + 1]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (pref[mid] <= u) lo = mid;
                else hi = mid;
            }
            const LatDesc& L = lats[l0 + lo];
            const Geom& g = L.g;
            const int vh = g.Vh;
            const int h = (u - pref[lo]) * kRuSites + sl;
            const void* links = kind < 2 ? L.fat64[par] : L.naik64[par];
            cx<double> res[3][R];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int r = 0; r < R; ++r) res[k][r] = {0.0, 0.0};
            if (h < vh) {
                int c[4];
                cb_coords(g, h, par, c);
                const int i = site_index(g, c);
#pragma unroll 1
                for (int mu = mu0; mu < mu0 + kM; ++mu) {
                    cx<double> m[9];
                    load_link<KS_F64, 9>(links, (kind & 1) * 4 + mu, vh, h, m);
                    cx<double> v[3][R];
                    V::load(in, L.vec_off, vh, hop_cb(g, i, c, mu, dist), v);
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b)
#pragma unroll
                            for (int r = 0; r < R; ++r) cfma(res[a][r], m[a * 3 + b], v[b][r]);
                }
            }
#pragma unroll
            for (int off = 1; off < kRuLanes; off <<= 1)
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        res[k][r].r += __shfl_xor(res[k][r].r, off);
                        res[k][r].i += __shfl_xor(res[k][r].i, off);
                    }
            if (h >= vh) continue;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (part != k) continue;
                const size_t o = V::off(L.vec_off, vh, k, h);
                double2* dst = reinterpret_cast<double2*>(out + o);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    double2 w = make_double2(res[k][r].r, res[k][r].i);
                    if (XPAY) {
                        const double2 x = reinterpret_cast<const double2*>(xv + o)[r];
                        const double sg = pairs[L.pair0 + r].sigma;
                        w = make_double2(sg * x.x - w.x, sg * x.y - w.y);
                    }
                    dst[r] = w;
                }
            }
        }
        __syncthreads();   // pref is rewritten by the next group of lattices
    }
}

// x += alpha p (FP64 x, or with FP32 inner iterations its FP32 increments); r -= alpha q;
// partial sums of |r|^2 per RHS
template <int P, int R, int NT>
__global__ __launch_bounds__(NT) void batch_update_kernel(const LatDesc* __restrict__ lats,
                                                         const int2* __restrict__ tiles, int ntiles,
                                                         char* __restrict__ x, const char* __restrict__ p,
                                                         const char* __restrict__ q, char* __restrict__ r,
                                                         const BatchPair* __restrict__ pairs,
                                                         double* __restrict__ partials)
{
    using T = typename St<P>::R;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int2 tl = tiles[t];
        const LatDesc& L = lats[tl.x];
        if (!lattice_busy(pairs, L.pair0, R, false)) {
            if (threadIdx.x < R) partials[(size_t)t * R + threadIdx.x] = 0.0;
            continue;
        }
        const int vh = L.g.Vh;
        const int h = tl.y + threadIdx.x;
        double nrm[R];
#pragma unroll
        for (int k = 0; k < R; ++k) nrm[k] = 0.0;
        if (h < vh) {
            // xv: x itself (FP64), or x's FP32 increments since the last reliable update
            cx<T> pv[3][R], qv[3][R], rv[3][R], xv[3][R];
            MVec<P, R>::load(p, L.vec_off, vh, h, pv);
            MVec<P, R>::load(q, L.vec_off, vh, h, qv);
            MVec<P, R>::load(r, L.vec_off, vh, h, rv);
            MVec<P, R>::load(x, L.vec_off, vh, h, xv);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const BatchPair& pp = pairs[L.pair0 + k];
                // a finished pair keeps x and r as they are: its direction p is no longer
                // maintained (never written for a pair that starts finished), so it must not
                // enter even with a zero step
                if (pp.done) continue;
                const T af = (T)pp.alpha;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xv[c][k].r = fma(af, pv[c][k].r, xv[c][k].r);
                    xv[c][k].i = fma(af, pv[c][k].i, xv[c][k].i);
                    rv[c][k].r = fma(-af, qv[c][k].r, rv[c][k].r);
                    rv[c][k].i = fma(-af, qv[c][k].i, rv[c][k].i);
                    nrm[k] += (double)rv[c][k].r * rv[c][k].r + (double)rv[c][k].i * rv[c][k].i;
                }
            }
            MVec<P, R>::store(x, L.vec_off, vh, h, xv);
            MVec<P, R>::store(r, L.vec_off, vh, h, rv);
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const double s = block_sum<NT>(nrm[k]);
            if (threadIdx.x == 0) partials[(size_t)t * R + k] = s;
            __syncthreads();
        }
    }
}

// FP32 inner: x += dx, dx = 0 on the lattices with a reliable update due (all = 1: every
// lattice, at the end of a solve)
template <int R, int NT>
__global__ __launch_bounds__(NT) void batch_flush_kernel(const LatDesc* __restrict__ lats,
                                                        const int2* __restrict__ tiles, int ntiles,
                                                        char* __restrict__ x, char* __restrict__ dx,
                                                        const BatchPair* __restrict__ pairs, int all)
{
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int2 tl = tiles[t];
        const LatDesc& L = lats[tl.x];
        if (!all && !lattice_busy(pairs, L.pair0, R, true)) continue;
        const int vh = L.g.Vh;
        const int h = tl.y + threadIdx.x;
        if (h >= vh) continue;
        cx<double> xv[3][R];
        cx<float> dv[3][R], zero[3][R];
        MVec<KS_F64, R>::load(x, L.vec_off, vh, h, xv);
        MVec<KS_F32, R>::load(dx, L.vec_off, vh, h, dv);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < R; ++k) {
                xv[c][k].r += (double)dv[c][k].r;
                xv[c][k].i += (double)dv[c][k].i;
                zero[c][k] = {0.f, 0.f};
            }
        MVec<KS_F64, R>::store(x, L.vec_off, vh, h, xv);
        MVec<KS_F32, R>::store(dx, L.vec_off, vh, h, zero);
    }
}

// FP64: r64 = b - Ax for lattices with an update due; partial sums of |r|^2
template <int R, int NT>
__global__ __launch_bounds__(NT) void batch_resid_kernel(const LatDesc* __restrict__ lats,
                                                        const int2* __restrict__ tiles, int ntiles,
                                                        const char* __restrict__ b,
                                                        const char* __restrict__ ax,
                                                        char* __restrict__ r64,
                                                        const BatchPair* __restrict__ pairs,
                                                        double* __restrict__ partials)
{
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int2 tl = tiles[t];
        const LatDesc& L = lats[tl.x];
        if (!lattice_busy(pairs, L.pair0, R, true)) {
            if (threadIdx.x < R) partials[(size_t)t * R + threadIdx.x] = 0.0;
            continue;
        }
        const int vh = L.g.Vh;
        const int h = tl.y + threadIdx.x;
        double nrm[R];
#pragma unroll
        for (int k = 0; k < R; ++k) nrm[k] = 0.0;
        if (h < vh) {
            cx<double> bv[3][R], av[3][R];
            MVec<KS_F64, R>::load(b, L.vec_off, vh, h, bv);
            MVec<KS_F64, R>::load(ax, L.vec_off, vh, h, av);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    bv[c][k].r -= av[c][k].r;
                    bv[c][k].i -= av[c][k].i;
                    nrm[k] += bv[c][k].r * bv[c][k].r + bv[c][k].i * bv[c][k].i;
                }
            MVec<KS_F64, R>::store(r64, L.vec_off, vh, h, bv);
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const double s = block_sum<NT>(nrm[k]);
            if (threadIdx.x == 0) partials[(size_t)t * R + k] = s;
            __syncthreads();
        }
    }
}

// r_inner = r64 for pairs whose reliable update ran this step and that continue
template <int P, int R, int NT>
__global__ __launch_bounds__(NT) void batch_load_r_kernel(const LatDesc* __restrict__ lats,
                                                         const int2* __restrict__ tiles, int ntiles,
                                                         const char* __restrict__ r64,
                                                         char* __restrict__ rs,
                                                         const BatchPair* __restrict__ pairs)
{
    using T = typename St<P>::R;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int2 tl = tiles[t];
        const LatDesc& L = lats[tl.x];
        if (!lattice_busy(pairs, L.pair0, R, true)) continue;
        const int vh = L.g.Vh;
        const int h = tl.y + threadIdx.x;
        if (h >= vh) continue;
        cx<double> a[3][R];
        cx<T> o[3][R];
        MVec<KS_F64, R>::load(r64, L.vec_off, vh, h, a);
        MVec<P, R>::load(rs, L.vec_off, vh, h, o);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const BatchPair& pp = pairs[L.pair0 + k];
            if (!pp.ru_now) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) o[c][k] = {(T)a[c][k].r, (T)a[c][k].i};
        }
        MVec<P, R>::store(rs, L.vec_off, vh, h, o);
    }
}

// p = r + beta p for pairs still iterating (p = r where beta is 0 after the initial update)
template <int P, int R, int NT>
__global__ __launch_bounds__(NT) void batch_xpay_kernel(const LatDesc* __restrict__ lats,
                                                       const int2* __restrict__ tiles, int ntiles,
                                                       const char* __restrict__ rs, char* __restrict__ ps,
                                                       const BatchPair* __restrict__ pairs, int fresh)
{
    using T = typename St<P>::R;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int2 tl = tiles[t];
        const LatDesc& L = lats[tl.x];
        if (!lattice_busy(pairs, L.pair0, R, false)) continue;
        const int vh = L.g.Vh;
        const int h = tl.y + threadIdx.x;
        if (h >= vh) continue;
        cx<T> rv[3][R], pv[3][R];
        MVec<P, R>::load(rs, L.vec_off, vh, h, rv);
        MVec<P, R>::load(ps, L.vec_off, vh, h, pv);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const BatchPair& pp = pairs[L.pair0 + k];
            if (pp.done) continue;
            const T b = (T)pp.beta;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (fresh) {
                    pv[c][k] = rv[c][k];
                } else {
                    pv[c][k].r = fma(b, pv[c][k].r, rv[c][k].r);
                    pv[c][k].i = fma(b, pv[c][k].i, rv[c][k].i);
                }
            }
        }
        MVec<P, R>::store(ps, L.vec_off, vh, h, pv);
    }
}

// ---------------------------------------------------------------- per-pair scalar steps
// One block per pair; it sums its lattice's tile partials in tile order.

__device__ __forceinline__ double pair_sum(const LatDesc& L, const double* part, int R, int r)
{
    double s = 0.0;
    for (int t = L.tile_begin + threadIdx.x; t < L.tile_end; t += kFin) s += part[(size_t)t * R + r];
    return block_sum<kFin>(s);
}

// The scalar steps run one block of kLat threads per lattice: one pass over the lattice's tile
// partials gives the sums of all its R pairs (thread j adds tiles j, j + kLat, ... in order,
// then wave sums and the waves in order, for all pairs in one LDS round), so a lattice with
// many tiles is summed as fast as a small one.
constexpr int kLat = 1024;

__device__ __forceinline__ void lattice_sums(const LatDesc& L, const double* __restrict__ part,
                                             int R, double* tot)
{
    __shared__ double red[kLat / 64][4];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = L.tile_begin + threadIdx.x; t < L.tile_end; t += kLat)
        for (int r = 0; r < R; ++r) s[r] += part[(size_t)t * R + r];
    // every pair's wave sums in one LDS round; thread r then adds pair r's waves in order
#pragma unroll
    for (int r = 0; r < 4; ++r) s[r] = wave_sum(s[r]);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[threadIdx.x >> 6][r] = s[r];
    __syncthreads();
    if (threadIdx.x < R) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < kLat / 64; ++k) v += red[k][threadIdx.x];
        tot[threadIdx.x] = v;
    }
    __syncthreads();
}

// alpha = rho / <p, A p> per pair (thread r of the lattice's block takes pair r)
__global__ __launch_bounds__(kLat) void batch_alpha_kernel(const LatDesc* __restrict__ lats, int R,
                                                           BatchPair* __restrict__ pairs,
                                                           const double* __restrict__ part)
{
    const LatDesc& L = lats[blockIdx.x];
    if (!lattice_busy(pairs, L.pair0, R, false)) return;
    __shared__ double tot[4];
    lattice_sums(L, part, R, tot);
    if (threadIdx.x >= R) return;
    BatchPair& q = pairs[L.pair0 + threadIdx.x];
    if (q.done) return;
    const double pap = tot[threadIdx.x];
    q.ru_now = 0;
    if (!isfinite(pap) || !(pap > 0.0)) {
        q.status = isfinite(pap) ? KS_ERR_BREAKDOWN : KS_ERR_NONFINITE;
        q.done = 1;
        q.t_done = wall_clock64();
        q.alpha = 0.0;
        return;
    }
    q.alpha = q.rho / pap;
}

// One block per lattice.  Each pair's |r|^2 of the step (its tile partials in tile order) and
// the pair's own decision (update due: target met or step cap; or |r| fell by delta), then
// the lattice's: a reliable update costs the lattice one FP64 multi-RHS A-apply whatever the
// number of its pairs that take part, so when one pair's residual has fallen by delta every
// unfinished pair takes the update with it (the right-hand sides then stay in step instead of
// each paying its own).  Pairs without an update continue: beta = |r|^2 / rho, rho = |r|^2.
__global__ __launch_bounds__(kLat) void batch_beta_kernel(const LatDesc* __restrict__ lats, int R,
                                                          BatchPair* __restrict__ pairs,
                                                          const double* __restrict__ part)
{
    const LatDesc& L = lats[blockIdx.x];
    if (!lattice_busy(pairs, L.pair0, R, false)) return;
    __shared__ double rn[4];
    lattice_sums(L, part, R, rn);
    if (threadIdx.x >= 64) return;   // lane r of the first wave takes pair r
    const int r = threadIdx.x;
    BatchPair* q = r < R ? &pairs[L.pair0 + r] : nullptr;
    bool live = q && !q->done;
    if (live) {
        q->iter += 1;
        q->rn = rn[r];
        if (!isfinite(q->rn)) {
            q->status = KS_ERR_NONFINITE;
            q->done = 1;
            q->t_done = wall_clock64();
            live = false;
        } else if (q->rn <= q->stop2 || q->iter >= q->max_iter) {
            q->ru_now = 1;
        } else if (sqrt(q->rn) < q->delta * q->maxr) {
            q->ru_now = 2;
        }
    }
    const bool drop = __any(live && q->ru_now == 2);
    if (!live) return;
    if (drop && q->ru_now == 0) q->ru_now = 1;
    if (q->ru_now) return;
    q->beta = q->rn / q->rho;
    q->rho = q->rn;
    q->maxr = fmax(q->maxr, sqrt(q->rn));
}

// After r = b - A x in FP64 for the lattices with an update due: each such pair either
// finishes or continues with beta = |r|^2 / rho (thread r of the lattice's block, pair r)
__global__ __launch_bounds__(kLat) void batch_reliable_kernel(const LatDesc* __restrict__ lats, int R,
                                                              BatchPair* __restrict__ pairs,
                                                              const double* __restrict__ part,
                                                              int initial)
{
    const LatDesc& L = lats[blockIdx.x];
    if (!lattice_busy(pairs, L.pair0, R, true)) return;
    __shared__ double tot[4];
    lattice_sums(L, part, R, tot);
    if (threadIdx.x >= R) return;
    BatchPair& q = pairs[L.pair0 + threadIdx.x];
    if (!q.ru_now || q.done) return;
    const double r2 = tot[threadIdx.x];
    q.true_r2 = r2;
    if (!initial) q.ru += 1;
    if (!isfinite(r2)) {
        q.status = KS_ERR_NONFINITE;
        q.done = 1;
    } else if (r2 <= q.stop2) {
        q.done = 1;
    } else if (q.iter >= q.max_iter) {
        q.status = KS_ERR_NOT_CONVERGED;
        q.done = 1;
    }
    if (q.done) {
        q.t_done = wall_clock64();
        q.ru_now = 0;
        return;
    }
    q.beta = initial ? 0.0 : r2 / q.rho;
    q.rho = r2;
    q.maxr = sqrt(r2);
}

__global__ void batch_census_kernel(const BatchPair* __restrict__ pairs, int n, int* __restrict__ out)
{
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int c = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) c += pairs[i].done ? 1 : 0;
    atomicAdd(&cnt, c);
    __syncthreads();
    if (threadIdx.x == 0) *out = cnt;
}

__global__ void batch_clock_kernel(unsigned long long* out) { *out = wall_clock64(); }

// Per tile: partial sums of |b_r|^2 over its sites, for every RHS r (FP64 arena).
template <int R, int NT>
__global__ __launch_bounds__(NT) void batch_b2_kernel(const LatDesc* __restrict__ lats,
                                                     const int2* __restrict__ tiles,
                                                     const char* __restrict__ b64,
                                                     double* __restrict__ partials)
{
    const int t = blockIdx.x;
    const int2 tl = tiles[t];
    const LatDesc& L = lats[tl.x];
    const int vh = L.g.Vh;
    const int h = tl.y + threadIdx.x;
    double nrm[R];
#pragma unroll
    for (int k = 0; k < R; ++k) nrm[k] = 0.0;
    if (h < vh) {
        cx<double> v[3][R];
        MVec<KS_F64, R>::load(b64, L.vec_off, vh, h, v);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < R; ++k) nrm[k] += v[c][k].r * v[c][k].r + v[c][k].i * v[c][k].i;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const double s = block_sum<NT>(nrm[k]);
        if (threadIdx.x == 0) partials[(size_t)t * R + k] = s;
        __syncthreads();
    }
}

// Per pair: |b|^2 (the tile partials in tile order) and the initial scalars (one block per pair).
__global__ __launch_bounds__(kFin) void batch_init_pairs_kernel(const LatDesc* __restrict__ lats,
                                                                int R, BatchPair* __restrict__ pairs,
                                                                const double* __restrict__ part,
                                                                const double* __restrict__ param,
                                                                int npairs, double delta,
                                                                int max_iter,
                                                                double* __restrict__ b2_out)
{
    const int pi = blockIdx.x;
    const LatDesc& L = lats[pi / R];
    const double s = pair_sum(L, part, R, pi % R);
    if (threadIdx.x != 0) return;
    BatchPair q{};
    q.sigma = param[pi];
    const double tol = param[npairs + pi];
    q.stop2 = tol * tol * s;
    q.delta = delta;
    q.max_iter = max_iter;
    q.ru_now = (s > 0.0) ? 1 : 0;   // the initial residual is one FP64 reliable update
    q.done = (s > 0.0) ? 0 : 1;
    pairs[pi] = q;
    b2_out[pi] = s;
}

// Caller vectors (complex128 [Vh][3], one device pointer per pair) <-> arena slots.
template <int R>
__global__ void batch_io_kernel(const LatDesc* __restrict__ lats, char* __restrict__ arena,
                                void* const* __restrict__ ptrs, int to_arena)
{
    const int pi = blockIdx.y;
    const LatDesc& L = lats[pi / R];
    const int r = pi % R;
    const int vh = L.g.Vh;
    double2* u = static_cast<double2*>(ptrs[pi]);
    for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < vh; h += gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double2* a = reinterpret_cast<double2*>(arena) + ((L.vec_off * 3 + (size_t)k * vh + h) * R + r);
            if (to_arena) *a = u[(size_t)h * 3 + k];
            else u[(size_t)h * 3 + k] = *a;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers

template <int R, int NT>
struct BatchLaunch {
    static void dslash(BatchCtx& c, int prec, bool xpay, int par, const char* in, char* out,
                       const char* x, hipStream_t s)
    {
        const int nt = c.ntiles[c.tile_idx];
        const int2* tl = c.tiles[c.tile_idx];
        const int grid = c.grid(nt);
        double* part = c.partials;
#define KS_BD(P, X)                                                                            \
    batch_dslash_kernel<P, R, X, NT><<<grid, NT, 0, s>>>(c.lats_dev, tl, nt, par, in, out, x,   \
                                                       c.pairs, part)
        if (prec == KS_F64) {
            if (xpay) KS_BD(KS_F64, true);
            else KS_BD(KS_F64, false);
        } else {
            if (xpay) KS_BD(KS_F32, true);
            else KS_BD(KS_F32, false);
        }
#undef KS_BD
        KS_HIP(hipGetLastError());
    }
    static void step(BatchCtx& c, hipStream_t s)
    {
        const int nt = c.ntiles[c.tile_idx];
        const int2* tl = c.tiles[c.tile_idx];
        const int grid = nt;   // streaming vector kernels: one block per tile (the tuned
                                // persistent schedule is for the hopping terms)
        const int P = c.prec;
        // inner A-apply
        dslash(c, P, false, 1, c.ps, c.ts, nullptr, s);
        dslash(c, P, true, 0, c.ts, c.qs, c.ps, s);
        const int nlat = (int)c.lats_host.size();
        batch_alpha_kernel<<<nlat, kLat, 0, s>>>(c.lats_dev, R, c.pairs, c.partials);
        if (P == KS_F64)
            batch_update_kernel<KS_F64, R, NT><<<grid, NT, 0, s>>>(c.lats_dev, tl, nt, c.x64, c.ps, c.qs, c.rs, c.pairs, c.partials);
        else
            batch_update_kernel<KS_F32, R, NT><<<grid, NT, 0, s>>>(c.lats_dev, tl, nt, c.dx32, c.ps, c.qs, c.rs, c.pairs, c.partials);
        batch_beta_kernel<<<nlat, kLat, 0, s>>>(c.lats_dev, R, c.pairs, c.partials);
        reliable(c, 0, s);
        if (P == KS_F64)
            batch_xpay_kernel<KS_F64, R, NT><<<grid, NT, 0, s>>>(c.lats_dev, tl, nt, c.rs, c.ps, c.pairs, 0);
        else
            batch_xpay_kernel<KS_F32, R, NT><<<grid, NT, 0, s>>>(c.lats_dev, tl, nt, c.rs, c.ps, c.pairs, 0);
        KS_HIP(hipGetLastError());
    }
    // FP64 r = b - A x for the pairs flagged ru_now, then the per-pair decision
    static void reliable(BatchCtx& c, int initial, hipStream_t s)
    {
        const int nt = c.ntiles[c.tile_idx];
        const int2* tl = c.tiles[c.tile_idx];
        const int grid = nt;   // streaming vector kernels: one block per tile (the tuned
                                // persistent schedule is for the hopping terms)
        const int nlat = (int)c.lats_host.size();
        if (c.prec == KS_F32) flush(c, 0, s);
        batch_dslash_ru_kernel<R, false><<<kRuGrid, 256, 0, s>>>(c.lats_dev, nlat, 1, c.x64, c.t64,
                                                                 nullptr, c.pairs);
        batch_dslash_ru_kernel<R, true><<<kRuGrid, 256, 0, s>>>(c.lats_dev, nlat, 0, c.t64, c.ax64,
                                                                c.x64, c.pairs);
        batch_resid_kernel<R, NT><<<grid, NT, 0, s>>>(c.lats_dev, tl, nt, c.b64, c.ax64, c.r64, c.pairs, c.partials);
        batch_reliable_kernel<<<(int)c.lats_host.size(), kLat, 0, s>>>(c.lats_dev, R, c.pairs, c.partials,
                                                                      initial);
        if (c.prec == KS_F64)
            batch_load_r_kernel<KS_F64, R, NT><<<grid, NT, 0, s>>>(c.lats_dev, tl, nt, c.r64, c.rs, c.pairs);
        else
            batch_load_r_kernel<KS_F32, R, NT><<<grid, NT, 0, s>>>(c.lats_dev, tl, nt, c.r64, c.rs, c.pairs);
        KS_HIP(hipGetLastError());
    }
    static void flush(BatchCtx& c, int all, hipStream_t s)
    {
        const int nt = c.ntiles[c.tile_idx];
        batch_flush_kernel<R, NT><<<nt, NT, 0, s>>>(c.lats_dev, c.tiles[c.tile_idx], nt, c.x64,
                                                    c.dx32, c.pairs, all);
        KS_HIP(hipGetLastError());
    }
    static void b2(BatchCtx& c, hipStream_t s)
    {
        const int nt = c.ntiles[c.tile_idx];
        batch_b2_kernel<R, NT><<<nt, NT, 0, s>>>(c.lats_dev, c.tiles[c.tile_idx], c.b64, c.partials);
        KS_HIP(hipGetLastError());
    }
    static void start(BatchCtx& c, hipStream_t s)
    {
        const int nt = c.ntiles[c.tile_idx];
        const int2* tl = c.tiles[c.tile_idx];
        const int grid = nt;   // streaming vector kernels: one block per tile (the tuned
                                // persistent schedule is for the hopping terms)
        reliable(c, 1, s);
        if (c.prec == KS_F64)
            batch_xpay_kernel<KS_F64, R, NT><<<grid, NT, 0, s>>>(c.lats_dev, tl, nt, c.rs, c.ps, c.pairs, 1);
        else
            batch_xpay_kernel<KS_F32, R, NT><<<grid, NT, 0, s>>>(c.lats_dev, tl, nt, c.rs, c.ps, c.pairs, 1);
        KS_HIP(hipGetLastError());
    }
};

static const int kTileSizes[3] = {64, 128, 256};

template <int R>
static void dispatch(BatchCtx& c, int what, hipStream_t s, int xpay_or_init = 0)
{
    const int nt = kTileSizes[c.tile_idx];
#define KS_DISP(NTV)                                                                    \
    if (nt == NTV) {                                                                    \
        if (what == 0) BatchLaunch<R, NTV>::step(c, s);                                 \
        else if (what == 1) BatchLaunch<R, NTV>::start(c, s);                           \
        else if (what == 3) BatchLaunch<R, NTV>::b2(c, s);                              \
        else if (what == 4) BatchLaunch<R, NTV>::flush(c, 1, s);                        \
        else BatchLaunch<R, NTV>::dslash(c, c.prec, xpay_or_init != 0, 1, c.ps, c.ts, nullptr, s); \
        return;                                                                         \
    }
    KS_DISP(64)
    KS_DISP(128)
    KS_DISP(256)
#undef KS_DISP
}

static void run(BatchCtx& c, int what, hipStream_t s)
{
    switch (c.nrhs) {
    case 1: dispatch<1>(c, what, s); break;
    case 2: dispatch<2>(c, what, s); break;
    case 4: dispatch<4>(c, what, s); break;
    default: KS_REQUIRE(false, KS_ERR_ARG, "batch: nrhs must be 1, 2 or 4");
    }
}

int BatchCtx::grid(int ntiles_now) const
{
    return persistent > 0 ? std::min(ntiles_now, persistent) : ntiles_now;
}

void batch_free(BatchCtx* c)
{
    if (!c) return;
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->owns_gauges)
        for (ks_gauge_t g : c->gauges) {
            gauge_release(g);
            delete g;
        }
    device_free(c->lats_dev);
    for (int k = 0; k < 3; ++k) device_free(c->tiles[k]);
    device_free(c->partials);
    device_free(c->pairs);
    device_free(c->clock);
    device_free(c->census);
    device_free(c->b2);
    device_free(c->pair_param);
    device_free(c->io_ptrs);
    for (char* v : {c->ps, c->qs, c->ts, c->rs, c->x64, c->b64, c->r64, c->t64, c->ax64, c->dx32})
        device_free(v);
    if (c->pairs_host) (void)hipHostFree(c->pairs_host);
    if (c->census_host) (void)hipHostFree(c->census_host);
    if (c->order) (void)hipEventDestroy(c->order);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

// Lattice descriptors, tile tables, pair state and vector arenas for the gauges of c.
static void batch_setup(BatchCtx* c, hipStream_t s)
{
    const int nlat = (int)c->gauges.size();
    const int nrhs = c->nrhs;
    const ks_prec_t inner = c->prec;
    size_t vec_off = 0;
    std::vector<LatDesc> lats(nlat);
    for (int l = 0; l < nlat; ++l) {
        ks_gauge_t g = c->gauges[l];
        if (inner != KS_F64) gauge_prepare(g, inner, KS_RECON_18, s);
        LatDesc& L = lats[l];
        L.g = g->geom;
        for (int par = 0; par < 2; ++par) {
            L.fat64[par] = g->store[KS_F64][0].fat[par];
            L.naik64[par] = g->store[KS_F64][0].naik[par];
            L.fat32[par] = g->store[inner][0].fat[par];
            L.naik32[par] = g->store[inner][0].naik[par];
        }
        L.vec_off = vec_off;
        L.pair0 = l * nrhs;
        vec_off += (size_t)g->geom.Vh;
    }
    c->total_vh = vec_off;
    // tile tables for 64, 128 and 256 sites per tile
    size_t max_tiles = 0;
    for (int k = 0; k < 3; ++k) {
        std::vector<int2> tt;
        for (int l = 0; l < nlat; ++l) {
            if (k == 0) lats[l].tile_begin = (int)tt.size();
            for (int h0 = 0; h0 < lats[l].g.Vh; h0 += kTileSizes[k]) tt.push_back(make_int2(l, h0));
        }
        c->ntiles[k] = (int)tt.size();
        c->tiles[k] = static_cast<int2*>(device_alloc(sizeof(int2) * tt.size()));
        KS_HIP(hipMemcpyAsync(c->tiles[k], tt.data(), sizeof(int2) * tt.size(),
                              hipMemcpyHostToDevice, s));
        max_tiles = std::max(max_tiles, tt.size());
        c->tile_tables[k] = tt;
    }
    c->lats_host = lats;
    c->lats_dev = static_cast<LatDesc*>(device_alloc(sizeof(LatDesc) * nlat));
    c->set_tiles(0, s);
    c->partials = static_cast<double*>(device_alloc(sizeof(double) * max_tiles * nrhs));
    c->pairs = static_cast<BatchPair*>(device_alloc(sizeof(BatchPair) * c->npairs));
    KS_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->pairs_host), sizeof(BatchPair) * c->npairs));
    c->clock = static_cast<unsigned long long*>(device_alloc(sizeof(unsigned long long)));
    c->census = static_cast<int*>(device_alloc(sizeof(int)));
    c->b2 = static_cast<double*>(device_alloc(sizeof(double) * c->npairs));
    c->pair_param = static_cast<double*>(device_alloc(sizeof(double) * 2 * c->npairs));
    c->io_ptrs = static_cast<void**>(device_alloc(sizeof(void*) * c->npairs));
    KS_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->census_host), sizeof(int)));
    const size_t cs = inner == KS_F64 ? 16 : 8;
    const size_t nrec = vec_off * 3 * nrhs;
    c->ps = static_cast<char*>(device_alloc(nrec * cs));
    c->qs = static_cast<char*>(device_alloc(nrec * cs));
    c->ts = static_cast<char*>(device_alloc(nrec * cs));
    c->rs = static_cast<char*>(device_alloc(nrec * cs));
    c->x64 = static_cast<char*>(device_alloc(nrec * 16));
    c->b64 = static_cast<char*>(device_alloc(nrec * 16));
    c->r64 = static_cast<char*>(device_alloc(nrec * 16));
    c->t64 = static_cast<char*>(device_alloc(nrec * 16));
    c->ax64 = static_cast<char*>(device_alloc(nrec * 16));
    if (inner == KS_F32) {
        c->dx32_bytes = nrec * 8;
        c->dx32 = static_cast<char*>(device_alloc(c->dx32_bytes));
    }
    // finished pairs leave their slots of p, q, t untouched: start every arena finite
    for (char* a : {c->ps, c->qs, c->ts, c->rs})
        KS_HIP(hipMemsetAsync(a, 0, nrec * cs, s));
    for (char* a : {c->x64, c->b64, c->r64, c->t64, c->ax64})
        KS_HIP(hipMemsetAsync(a, 0, nrec * 16, s));
    KS_HIP(hipStreamSynchronize(s));
}

static BatchCtx* batch_new(int nrhs, ks_prec_t inner)
{
    KS_REQUIRE(nrhs == 1 || nrhs == 2 || nrhs == 4, KS_ERR_ARG, "batch: nrhs must be 1, 2 or 4");
    KS_REQUIRE(inner == KS_F64 || inner == KS_F32, KS_ERR_ARG, "batch: inner precision F64 or F32");
    BatchCtx* c = new BatchCtx();
    c->nrhs = nrhs;
    c->prec = inner;
    try {
        KS_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        KS_HIP(hipEventCreateWithFlags(&c->order, hipEventDisableTiming));
    } catch (...) {
        batch_free(c);
        throw;
    }
    return c;
}

BatchCtx* batch_create(int nlat, const int* dims, const double* const* fat,
                       const double* const* naik, int on_device, int nrhs, ks_prec_t inner,
                       hipStream_t s)
{
    KS_REQUIRE(nlat >= 1, KS_ERR_ARG, "batch: no lattices");
    BatchCtx* c = batch_new(nrhs, inner);
    try {
        c->npairs = nlat * nrhs;
        for (int l = 0; l < nlat; ++l) {
            const int* d = dims + 4 * l;
            long v = 1;
            for (int mu = 0; mu < 4; ++mu) {
                KS_REQUIRE(d[mu] >= 4 && d[mu] % 2 == 0, KS_ERR_ARG,
                           "batch lattice %d: extent %d of direction %d must be even and >= 4", l,
                           d[mu], mu);
                v *= d[mu];
            }
            KS_REQUIRE(v <= (1L << 29), KS_ERR_ARG, "batch lattice %d: volume too large", l);
            KS_REQUIRE(fat[l] && naik[l], KS_ERR_ARG, "batch lattice %d: null links", l);
            ks_gauge_s* g = new ks_gauge_s();
            c->gauges.push_back(g);
            g->geom = make_geom(d);
            const size_t bytes = (size_t)4 * v * 9 * 16;
            const double* df = fat[l];
            const double* dn = naik[l];
            double* tf = nullptr;
            double* tn = nullptr;
            if (!on_device) {
                tf = static_cast<double*>(device_alloc(bytes));
                tn = static_cast<double*>(device_alloc(bytes));
                KS_HIP(hipMemcpyAsync(tf, fat[l], bytes, hipMemcpyHostToDevice, s));
                KS_HIP(hipMemcpyAsync(tn, naik[l], bytes, hipMemcpyHostToDevice, s));
                df = tf;
                dn = tn;
            }
            gauge_build_f64(g, df, dn, s);
            device_free(tf);
            device_free(tn);
        }
        batch_setup(c, s);
    } catch (...) {
        batch_free(c);
        throw;
    }
    return c;
}

BatchCtx* batch_create_on(ks_gauge_t g, int nrhs, ks_prec_t inner, hipStream_t s)
{
    BatchCtx* c = batch_new(nrhs, inner);
    try {
        c->owns_gauges = false;
        c->npairs = nrhs;
        c->gauges.push_back(g);
        batch_setup(c, s);
    } catch (...) {
        batch_free(c);
        throw;
    }
    return c;
}

void BatchCtx::set_tiles(int k, hipStream_t s)
{
    tile_idx = k;
    std::vector<LatDesc> l = lats_host;
    const std::vector<int2>& tt = tile_tables[k];
    for (size_t i = 0; i < l.size(); ++i) {
        l[i].tile_begin = -1;
        l[i].tile_end = -1;
    }
    for (size_t t = 0; t < tt.size(); ++t) {
        LatDesc& L = l[tt[t].x];
        if (L.tile_begin < 0) L.tile_begin = (int)t;
        L.tile_end = (int)t + 1;
    }
    lats_host = l;
    KS_HIP(hipMemcpyAsync(lats_dev, l.data(), sizeof(LatDesc) * l.size(), hipMemcpyHostToDevice, s));
    KS_HIP(hipStreamSynchronize(s));
    if (graph_exec) {
        (void)hipGraphExecDestroy(graph_exec);
        graph_exec = nullptr;
    }
}

// Caller vectors <-> arena: one launch for every pair through a device pointer table.
static void batch_io(BatchCtx& c, char* arena, const void* const* host_ptrs, int to_arena,
                     hipStream_t s)
{
    KS_HIP(hipMemcpyAsync(c.io_ptrs, host_ptrs, sizeof(void*) * c.npairs, hipMemcpyHostToDevice, s));
    int maxvh = 0;
    for (const LatDesc& L : c.lats_host) maxvh = std::max(maxvh, L.g.Vh);
    const dim3 grid(std::min(blocks_for(maxvh), 64), c.npairs);
    if (c.nrhs == 1) batch_io_kernel<1><<<grid, kBlock, 0, s>>>(c.lats_dev, arena, c.io_ptrs, to_arena);
    else if (c.nrhs == 2) batch_io_kernel<2><<<grid, kBlock, 0, s>>>(c.lats_dev, arena, c.io_ptrs, to_arena);
    else batch_io_kernel<4><<<grid, kBlock, 0, s>>>(c.lats_dev, arena, c.io_ptrs, to_arena);
    KS_HIP(hipGetLastError());
    // the pointer table is read by the kernel: keep it until the copy has been consumed
    KS_HIP(hipStreamSynchronize(s));
}

// The batch runs on its own stream (graphs cannot be captured on the legacy default stream),
// ordered after the caller's stream.
static hipStream_t enter_stream(BatchCtx& c, hipStream_t caller)
{
    KS_HIP(hipEventRecord(c.order, caller));
    KS_HIP(hipStreamWaitEvent(c.stream, c.order, 0));
    return c.stream;
}

ks_status_t batch_solve(BatchCtx& c, const double* masses, const double* const* b,
                        double* const* x, const ks_solver_params& prm, ks_batch_stats* stats,
                        hipStream_t caller)
{
    const int nlat = (int)c.lats_host.size();
    std::vector<double> sigma(c.npairs), tol(c.npairs, prm.tol);
    for (int l = 0; l < nlat; ++l) {
        KS_REQUIRE(std::isfinite(masses[l]), KS_ERR_ARG, "batch: mass %d is not finite", l);
        for (int r = 0; r < c.nrhs; ++r) sigma[l * c.nrhs + r] = 4.0 * masses[l] * masses[l];
    }
    return batch_solve_pairs(c, sigma.data(), tol.data(), b, x, prm, stats, caller);
}

ks_status_t batch_solve_pairs(BatchCtx& c, const double* sigma, const double* tol,
                              const double* const* b, double* const* x,
                              const ks_solver_params& prm, ks_batch_stats* stats,
                              hipStream_t caller)
{
    const auto t0 = std::chrono::steady_clock::now();
    const hipStream_t s = enter_stream(c, caller);
    std::vector<double> param(2 * (size_t)c.npairs);
    for (int p = 0; p < c.npairs; ++p) {
        KS_REQUIRE(b[p] && x[p] && b[p] != x[p], KS_ERR_ARG, "batch: bad vectors for pair %d", p);
        KS_REQUIRE(std::isfinite(sigma[p]) && sigma[p] >= 0.0 && tol[p] > 0.0, KS_ERR_ARG,
                   "batch: bad shift or tolerance for pair %d", p);
        param[p] = sigma[p];
        param[c.npairs + p] = tol[p];
    }
    KS_HIP(hipMemcpyAsync(c.pair_param, param.data(), sizeof(double) * param.size(),
                          hipMemcpyHostToDevice, s));
    batch_io(c, c.b64, reinterpret_cast<const void* const*>(b), 1, s);
    batch_io(c, c.x64, reinterpret_cast<const void* const*>(x), 1, s);
    if (c.dx32) KS_HIP(hipMemsetAsync(c.dx32, 0, c.dx32_bytes, s));   // outside any graph
    batch_clock_kernel<<<1, 1, 0, s>>>(c.clock);
    run(c, 3, s);   // |b|^2 tile partials
    batch_init_pairs_kernel<<<c.npairs, kFin, 0, s>>>(c.lats_dev, c.nrhs, c.pairs, c.partials,
                                                      c.pair_param, c.npairs,
                                                      c.prec == KS_F64 ? 0.0 : prm.delta,
                                                      prm.max_iter, c.b2);
    KS_HIP(hipGetLastError());
    run(c, 1, s);

    // the step sequence, captured once per configuration into a graph of `chunk` steps
    const int chunk = std::max(1, prm.check_every);
    if (!c.graph_exec || c.graph_chunk != chunk) {
        if (c.graph_exec) (void)hipGraphExecDestroy(c.graph_exec);
        c.graph_exec = nullptr;
        hipGraph_t graph;
        KS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            for (int k = 0; k < chunk; ++k) run(c, 0, s);
            batch_census_kernel<<<1, 256, 0, s>>>(c.pairs, c.npairs, c.census);
        } catch (...) {
            hipGraph_t g2;
            (void)hipStreamEndCapture(s, &g2);
            throw;
        }
        KS_HIP(hipStreamEndCapture(s, &graph));
        const hipError_t e = hipGraphInstantiate(&c.graph_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        KS_HIP(e);
        c.graph_chunk = chunk;
    }
    int max_chunks = prm.max_iter / chunk + 4;
    for (int it = 0; it < max_chunks; ++it) {
        KS_HIP(hipGraphLaunch(c.graph_exec, s));
        KS_HIP(hipMemcpyAsync(c.census_host, c.census, sizeof(int), hipMemcpyDeviceToHost, s));
        KS_HIP(hipStreamSynchronize(s));
        if (*c.census_host >= c.npairs) break;
    }
    KS_HIP(hipMemcpyAsync(c.pairs_host, c.pairs, sizeof(BatchPair) * c.npairs, hipMemcpyDeviceToHost, s));
    unsigned long long start = 0;
    KS_HIP(hipMemcpyAsync(&start, c.clock, sizeof(start), hipMemcpyDeviceToHost, s));
    std::vector<double> b2(c.npairs);
    KS_HIP(hipMemcpyAsync(b2.data(), c.b2, sizeof(double) * c.npairs, hipMemcpyDeviceToHost, s));
    if (c.dx32) run(c, 4, s);   // every pair's remaining FP32 increments into x
    batch_io(c, c.x64, reinterpret_cast<const void* const*>(x), 0, s);
    int dev = 0, khz = 100000;
    KS_HIP(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        khz = 100000;
    ks_status_t result = KS_SUCCESS;
    for (int p = 0; p < c.npairs; ++p) {
        const BatchPair& q = c.pairs_host[p];
        ks_batch_stats& o = stats[p];
        o.iters = q.iter;
        o.reliable_updates = q.ru;
        o.true_rel_resid = b2[p] > 0 ? std::sqrt(q.true_r2 / b2[p]) : 0.0;
        o.seconds = (q.done && q.t_done >= start) ? (double)(q.t_done - start) / (khz * 1e3) : -1.0;
        o.status = q.done ? q.status : KS_ERR_NOT_CONVERGED;
        if (o.status != KS_SUCCESS && result == KS_SUCCESS) result = (ks_status_t)o.status;
    }
    c.last_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (result != KS_SUCCESS) set_error("batch: at least one pair failed (first code %d)", (int)result);
    return result;
}

// Autotuner: tile size (64 / 128 / 256 sites per block) and schedule (one block per tile, or
// a persistent grid of k blocks per CU that strides over the tile table), timed on the
// inner-precision multi-RHS Dslash of this batch.
void batch_tune(BatchCtx& c, hipStream_t caller)
{
    const hipStream_t s = enter_stream(c, caller);
    int dev = 0;
    KS_HIP(hipGetDevice(&dev));
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    // every pair active for timing
    for (int p = 0; p < c.npairs; ++p) {
        BatchPair q{};
        c.pairs_host[p] = q;
    }
    KS_HIP(hipMemcpyAsync(c.pairs, c.pairs_host, sizeof(BatchPair) * c.npairs, hipMemcpyHostToDevice, s));
    const size_t cs = c.prec == KS_F64 ? 16 : 8;
    KS_HIP(hipMemsetAsync(c.ps, 0x3f, c.total_vh * 3 * c.nrhs * cs, s));
    hipEvent_t e0, e1;
    KS_HIP(hipEventCreate(&e0));
    KS_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int best_k = 0, best_pers = 0;
    for (int k = 0; k < 3; ++k) {
        c.set_tiles(k, s);
        for (int pers : {0, 1, 2, 4, 8}) {
            c.persistent = pers * cus;
            for (int w = 0; w < 2; ++w) run(c, 2, s);
            KS_HIP(hipEventRecord(e0, s));
            for (int w = 0; w < 5; ++w) run(c, 2, s);
            KS_HIP(hipEventRecord(e1, s));
            KS_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            KS_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                best_k = k;
                best_pers = c.persistent;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c.set_tiles(best_k, s);
    c.persistent = best_pers;
    c.tuned_us = best * 1e3f / 5;
}

}  // namespace ks
