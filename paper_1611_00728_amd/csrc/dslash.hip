// Improved-staggered hopping term on one parity (the staggered dslash of Sec. 3):
//   (D psi)(x) = sum_mu [ V_mu(x) psi(x+mu) - V_mu(x-mu)^+ psi(x-mu)
//                       + W_mu(x) psi(x+3mu) - W_mu(x-3mu)^+ psi(x-3mu) ]
// One thread per output site, looping over the site's 16 matrices, 1, 2 or 4 of them loaded
// per pass (a tuning choice: fewer keeps the register count low and the waves per SIMD high,
// more keeps more loads in flight per wave).  Links
// stream from packed site-major planes (16-byte coalesced loads, read once: the bulk of the
// bytes); the 16 neighbour vectors are gathers that the XCD-aware tile order keeps inside
// one XCD's L2 for most hops.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <string>
#include <unistd.h>
#include <utility>
#include <vector>

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

// acc += m^+ v
template <class R>
__device__ __forceinline__ void matvec_adj_acc(cx<R> acc[3], const cx<R> m[9], const cx<R> v[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const cx<R> e = m[b * 3 + a];
            acc[a].r = fma(e.r, v[b].r, fma(e.i, v[b].i, acc[a].r));
            acc[a].i = fma(e.r, v[b].i, fma(-e.i, v[b].r, acc[a].i));
        }
}

// rows 0, 1 stored; row 2 = conj(row0 x row1)
template <class R>
__device__ __forceinline__ void reconstruct_row2(cx<R> m[9])
{
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

// Bytes of one colour vector of precision P and the LDS halo (in checkerboard sites) around a
// block's sites that covers every x and y neighbour: x hops move the checkerboard index by at
// most 2, y hops by 1 or 3 rows of Nx/2 (hops that wrap around the lattice fall outside and
// are read from memory).
__host__ __device__ constexpr int spinor_bytes_of(int P) { return P == KS_F64 ? 48 : P == KS_F32 ? 24 : 16; }
__host__ __device__ inline int staged_halo(int nx) { return 3 * (nx / 2) + 2; }

// Copies sites [lo, lo + len) of a colour-vector field into LDS with the field's own plane
// structure (plane length len), so that Spinor<P>::load(lds, len, h - lo, v) reads site h.
template <int P, int NT>
__device__ __forceinline__ void stage_spinor(const void* __restrict__ in, int vh, int lo, int len,
                                             void* lds)
{
    if constexpr (P == KS_F64) {
        const double2* src = static_cast<const double2*>(in);
        double2* dst = static_cast<double2*>(lds);
        for (int k = 0; k < 3; ++k)
            for (int j = threadIdx.x; j < len; j += NT) dst[k * len + j] = src[(size_t)k * vh + lo + j];
    } else if constexpr (P == KS_F32) {
        const float4* a = static_cast<const float4*>(in);
        const float2* b = reinterpret_cast<const float2*>(a + vh);
        float4* da = static_cast<float4*>(lds);
        float2* db = reinterpret_cast<float2*>(da + len);
        for (int j = threadIdx.x; j < len; j += NT) {
            da[j] = a[lo + j];
            db[j] = b[lo + j];
        }
    } else {
        const uint4* src = static_cast<const uint4*>(in);
        uint4* dst = static_cast<uint4*>(lds);
        for (int j = threadIdx.x; j < len; j += NT) dst[j] = src[lo + j];
    }
}

// W4: 4-way link access.  The backward matrices -V_mu(x-mu)^+ and -W_mu(x-3mu)^+ are formed
// from the forward links of the neighbour sites (slots 0-3 of the other parity's store, read
// at the neighbour's index) instead of the site's own backward slots 4-7, so only the forward
// half of each store is read.
// LG: the input sites of the block's x and y neighbourhood are first staged in LDS (one
// coalesced read of the range) and those gathers read LDS; z and t gathers, and wrapped
// hops, read memory through the caches.
template <int P, int RECON, bool XPAY, int NT, int U, bool W4, bool LG>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void dslash_kernel(Geom g, int par, const void* __restrict__ fat,
                                                        const void* __restrict__ naik,
                                                        const void* __restrict__ fat_o,
                                                        const void* __restrict__ naik_o,
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
    const int h = tile * NT + threadIdx.x;
    const int vh = g.Vh;
    double dot = 0.0;
    extern __shared__ __align__(16) char staged[];
    int lo = 0, len = 0;
    if constexpr (LG) {
        const int halo = staged_halo(g.n[0]);
        lo = max(0, tile * NT - halo);
        len = min(vh, tile * NT + NT + halo) - lo;
        stage_spinor<P, NT>(in, vh, lo, len, staged);
        __syncthreads();
    }
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
        // U matrices per pass: their loads are issued together, then consumed in order.  U
        // divides 8, so a pass holds only fat or only Naik links.
#pragma unroll 1
        for (int s0 = 0; s0 < 16; s0 += U) {
            cx<R> m[U][9], v[U][3];
            const bool bwd4 = W4 && (s0 & 7) >= 4;   // U divides 4: a pass is all one kind
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int s = s0 + u;
                if (bwd4) {
                    if (s0 < 8) load_link<P, 9>(fat_o, s - 4, g.lp, nb[s], m[u]);
                    else if (RECON == 12) load_link<P, 6>(naik_o, s - 12, g.lp, nb[s], m[u]);
                    else load_link<P, 9>(naik_o, s - 12, g.lp, nb[s], m[u]);
                } else {
                    if (s0 < 8) load_link<P, 9>(fat, s, g.lp, h, m[u]);
                    else if (RECON == 12) load_link<P, 6>(naik, s - 8, g.lp, h, m[u]);
                    else load_link<P, 9>(naik, s - 8, g.lp, h, m[u]);
                }
                const int j = nb[s] - lo;
                if (LG && (s & 3) < 2 && j >= 0 && j < len) Spinor<P>::load(staged, len, j, v[u]);
                else Spinor<P>::load(in, vh, nb[s], v[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                R sc;
                if (s0 < 8) {
                    sc = (R)(bwd4 ? -fat_scale : fat_scale);
                } else if (RECON == 12) {
                    // the sign of the 8-way slot covers the backward minus and adjoint
                    reconstruct_row2(m[u]);
                    sc = (R)(naik_c0 * naik_sign(c, s0 + u - 8, g.n[3]));
                } else {
                    sc = (R)(bwd4 ? -naik_scale : naik_scale);
                }
                cx<R> t[3] = {{0, 0}, {0, 0}, {0, 0}};
                if (bwd4) matvec_adj_acc(t, m[u], v[u]);
                else matvec_acc(t, m[u], v[u]);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    res[k].r = fma(sc, t[k].r, res[k].r);
                    res[k].i = fma(sc, t[k].i, res[k].i);
                }
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
        const double s = block_sum<NT>(dot);
        if (threadIdx.x == 0) partials[tile] = s;
    }
}

// dynamic LDS of the staged form: the block's sites and the x/y halo on both sides
int staged_lds_bytes(int P, int NT, const Geom& G)
{
    const int halo = staged_halo(G.n[0]);
    const int sites = std::min(G.Vh, NT + 2 * halo);
    return ((sites * spinor_bytes_of(P) + 255) / 256) * 256;
}

// Forms that are built: more link matrices per pass would exceed the 128-VGPR budget of 4
// waves per SIMD and spill (FP64 holds two passes' matrices only with its own backward slots
// and cache-read neighbours).
constexpr bool form_built(int P, int RECON, int U, bool W4, bool LG)
{
    return U == 1 || (U == 2 && P != KS_F64) || (U == 2 && RECON == 18 && !W4 && !LG) ||
           (U == 4 && P != KS_F64 && RECON == 18);
}

template <int P, int RECON, int NT, int U, bool W4, bool LG>
void launch_g(const LinkStore& st, const Geom& G, double c0, const DslashArgs& a, int lds,
              hipStream_t s)
{
    if constexpr (!form_built(P, RECON, U, W4, LG)) {
        KS_REQUIRE(false, KS_ERR_ARG, "Dslash: this launch form is not built");
    } else {
    const int nb = blocks_for(G.Vh, NT);
    const int p = a.out_parity;
    if (LG) lds = std::max(lds, staged_lds_bytes(P, NT, G));
    if (a.x)
        dslash_kernel<P, RECON, true, NT, U, W4, LG><<<nb, NT, lds, s>>>(
            G, p, st.fat[p], st.naik[p], st.fat[1 - p], st.naik[1 - p], a.in, a.out, a.x, a.a,
            a.dot_partials, a.gate, st.fat_scale, st.naik_scale, c0);
    else
        dslash_kernel<P, RECON, false, NT, U, W4, LG><<<nb, NT, lds, s>>>(
            G, p, st.fat[p], st.naik[p], st.fat[1 - p], st.naik[1 - p], a.in, a.out, nullptr,
            0.0, nullptr, a.gate, st.fat_scale, st.naik_scale, c0);
    KS_HIP(hipGetLastError());
    }
}

template <int P, int RECON, int NT, int U>
void launch_u(const LinkStore& st, const Geom& G, double c0, const DslashArgs& a,
              const TuneEntry& t, hipStream_t s)
{
    if (t.way == 4) {
        if (t.staged) launch_g<P, RECON, NT, U, true, true>(st, G, c0, a, t.lds, s);
        else launch_g<P, RECON, NT, U, true, false>(st, G, c0, a, t.lds, s);
    } else {
        if (t.staged) launch_g<P, RECON, NT, U, false, true>(st, G, c0, a, t.lds, s);
        else launch_g<P, RECON, NT, U, false, false>(st, G, c0, a, t.lds, s);
    }
}

template <int P, int RECON, int NT>
void launch_nt(const LinkStore& st, const Geom& G, double c0, const DslashArgs& a,
               const TuneEntry& t, hipStream_t s)
{
    if (t.group == 2) launch_u<P, RECON, NT, 2>(st, G, c0, a, t, s);
    else if (t.group == 4) launch_u<P, RECON, NT, 4>(st, G, c0, a, t, s);
    else launch_u<P, RECON, NT, 1>(st, G, c0, a, t, s);
}

template <int P, int RECON>
void launch_p(const LinkStore& st, const Geom& G, double c0, const DslashArgs& a,
              const TuneEntry& t, hipStream_t s)
{
    if (t.nt == 64) launch_nt<P, RECON, 64>(st, G, c0, a, t, s);
    else if (t.nt == 128) launch_nt<P, RECON, 128>(st, G, c0, a, t, s);
    else launch_nt<P, RECON, 256>(st, G, c0, a, t, s);
}

void launch(ks_gauge_t g, ks_prec_t prec, int ri, const DslashArgs& a, const TuneEntry& t,
            hipStream_t s)
{
    const LinkStore& st = g->store[prec][ri];
    const Geom& G = g->geom;
    const double c0 = g->naik_c0;
    if (prec == KS_F64)
        ri ? launch_p<KS_F64, 12>(st, G, c0, a, t, s) : launch_p<KS_F64, 18>(st, G, c0, a, t, s);
    else if (prec == KS_F32)
        ri ? launch_p<KS_F32, 12>(st, G, c0, a, t, s) : launch_p<KS_F32, 18>(st, G, c0, a, t, s);
    else
        ri ? launch_p<KS_F16, 12>(st, G, c0, a, t, s) : launch_p<KS_F16, 18>(st, G, c0, a, t, s);
}

}  // namespace

int dslash_blocks(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon)
{
    return blocks_for(g->geom.Vh, g->tune[prec][recon_index(recon)].nt);
}

bool dslash_form_built(ks_prec_t prec, ks_recon_t recon, int links_per_pass, int link_access,
                       int staged)
{
    return (links_per_pass == 1 || links_per_pass == 2 || links_per_pass == 4) &&
           form_built((int)prec, (int)recon, links_per_pass, link_access == 4, staged != 0);
}

int dslash_max_blocks(const Geom& g) { return blocks_for(g.Vh, 64); }

void dslash(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon, const DslashArgs& a, hipStream_t s)
{
    const int ri = recon_index(recon);
    if (!g->store[prec][ri].ready) gauge_prepare(g, prec, recon, s);
    launch(g, prec, ri, a, g->tune[prec][ri], s);
}

// mean time of one launch over `reps` launches of one candidate (HIP events)
static float time_launches(ks_gauge_t g, ks_prec_t prec, int ri, const DslashArgs& a,
                           const TuneEntry& t, int reps, hipEvent_t e0, hipEvent_t e1,
                           hipStream_t s)
{
    KS_HIP(hipEventRecord(e0, s));
    for (int k = 0; k < reps; ++k) launch(g, prec, ri, a, t, s);
    KS_HIP(hipEventRecord(e1, s));
    KS_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    KS_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ms * 1e3f / reps;
}

// Candidates: neighbours through the caches or x/y neighbours staged in LDS, 8-way or 4-way
// link access, 1, 2 or 4 matrices loaded per pass (2 at most in
// FP64), 64, 128 or 256 threads per block, each with the number of resident blocks per CU capped through the dynamic LDS
// request (how many waves share a SIMD also decides how
// evenly the last round of waves fills the chip).  Each candidate is timed over a few
// launches with HIP events on this lattice; the four fastest are then timed again over 20
// launches each, twice in alternation, and the one with the best mean is kept for the handle
// (a single short timing picks a lucky candidate too often).
// ---------------------------------------------------------------- tuning cache
// With the environment variable KS_TUNE_CACHE naming a file, a variant's configuration is
// looked up there before any timing and recorded there after tuning.  One JSON object per
// line, keyed by the device (architecture name, compute units), the lattice extents, the
// precision and the Naik storage; lines the library cannot read are kept as they are.
namespace {

std::mutex g_cache_mu;

struct CacheKey {
    std::string arch;
    int cus;
    int dims[4];
    int prec;
    int naik;
};

std::string cache_line(const CacheKey& k, const TuneEntry& t)
{
    char b[512];
    std::snprintf(b, sizeof(b),
                  "{\"arch\": \"%s\", \"cus\": %d, \"dims\": [%d, %d, %d, %d], \"prec\": %d, "
                  "\"naik\": %d, \"threads\": %d, \"lds_bytes\": %d, \"links_per_pass\": %d, "
                  "\"link_access\": %d, \"staged\": %d, \"us\": %.2f}",
                  k.arch.c_str(), k.cus, k.dims[0], k.dims[1], k.dims[2], k.dims[3], k.prec, k.naik,
                  t.nt, t.lds, t.group, t.way, t.staged, (double)t.us);
    return b;
}

bool parse_line(const std::string& line, CacheKey& k, TuneEntry& t)
{
    char arch[64];
    float us = 0.f;
    const int n = std::sscanf(
        line.c_str(),
        "{\"arch\": \"%63[^\"]\", \"cus\": %d, \"dims\": [%d, %d, %d, %d], \"prec\": %d, "
        "\"naik\": %d, \"threads\": %d, \"lds_bytes\": %d, \"links_per_pass\": %d, "
        "\"link_access\": %d, \"staged\": %d, \"us\": %f}",
        arch, &k.cus, &k.dims[0], &k.dims[1], &k.dims[2], &k.dims[3], &k.prec, &k.naik, &t.nt,
        &t.lds, &t.group, &t.way, &t.staged, &us);
    if (n != 14) return false;
    k.arch = arch;
    t.us = us;
    return true;
}

bool same_key(const CacheKey& a, const CacheKey& b)
{
    return a.arch == b.arch && a.cus == b.cus && a.dims[0] == b.dims[0] && a.dims[1] == b.dims[1] &&
           a.dims[2] == b.dims[2] && a.dims[3] == b.dims[3] && a.prec == b.prec &&
           a.naik == b.naik;
}

std::vector<std::string> cache_lines(const char* path)
{
    std::vector<std::string> out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line))
        if (!line.empty()) out.push_back(line);
    return out;
}

bool cache_lookup(const char* path, const CacheKey& key, TuneEntry& t)
{
    std::lock_guard<std::mutex> lock(g_cache_mu);
    bool found = false;
    for (const std::string& line : cache_lines(path)) {
        CacheKey k;
        TuneEntry e;
        if (parse_line(line, k, e) && same_key(k, key)) {
            t = e;
            found = true;   // the last entry of a key wins
        }
    }
    return found;
}

// Replaces the key's entry (or appends it) through a temporary file renamed over the cache,
// so that a reader never sees a half-written file.  Failures are reported, not fatal.
void cache_store(const char* path, const CacheKey& key, const TuneEntry& t)
{
    std::lock_guard<std::mutex> lock(g_cache_mu);
    std::vector<std::string> keep;
    for (const std::string& line : cache_lines(path)) {
        CacheKey k;
        TuneEntry e;
        if (!(parse_line(line, k, e) && same_key(k, key))) keep.push_back(line);
    }
    keep.push_back(cache_line(key, t));
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    {
        std::ofstream f(tmp, std::ios::trunc);
        for (const std::string& line : keep) f << line << '\n';
        if (!f) {
            log_msg(1, "tuning cache %s: cannot write %s", path, tmp.c_str());
            return;
        }
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        log_msg(1, "tuning cache %s: cannot replace it", path);
        std::remove(tmp.c_str());
    }
}

}  // namespace

void dslash_tune(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon, hipStream_t s)
{
    const int ri = recon_index(recon);
    gauge_prepare(g, prec, recon, s);
    int dev = 0;
    KS_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    KS_HIP(hipGetDeviceProperties(&prop, dev));
    const long lds_cu = prop.maxSharedMemoryPerMultiProcessor > 0
                            ? (long)prop.maxSharedMemoryPerMultiProcessor
                            : 65536L;
    const long lds_blk = (long)prop.sharedMemPerBlock;
    const Geom& G = g->geom;
    const int naik = ri ? 12 : 18;
    const char* cache = std::getenv("KS_TUNE_CACHE");
    const CacheKey key{prop.gcnArchName, prop.multiProcessorCount,
                       {G.n[0], G.n[1], G.n[2], G.n[3]}, (int)prec, naik};
    if (cache && *cache) {
        TuneEntry t;
        const bool hit = cache_lookup(cache, key, t);
        const bool usable = hit && (t.nt == 64 || t.nt == 128 || t.nt == 256) &&
                            (t.way == 4 || t.way == 8) && (t.staged == 0 || t.staged == 1) &&
                            t.lds >= 0 && t.lds <= lds_blk &&
                            form_built((int)prec, naik, t.group, t.way == 4, t.staged != 0);
        log_msg(2, "tuning cache %s: %s for %s %d-real %dx%dx%dx%d", cache,
                usable ? "hit" : hit ? "unusable entry" : "miss",
                prec == KS_F64 ? "FP64" : prec == KS_F32 ? "FP32" : "FP16", naik, G.n[0], G.n[1],
                G.n[2], G.n[3]);
        if (usable) {
            t.tuned = true;
            g->tune[prec][ri] = t;
            return;
        }
    }
    const size_t fb = field_bytes(G, prec);
    void* in = device_alloc(fb);
    void* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TuneEntry best;
    float best_us = 1e30f;
    std::vector<std::pair<float, TuneEntry>> timed;
    try {
        out = device_alloc(fb);
        KS_HIP(hipMemsetAsync(in, 0x3f, fb, s));
        KS_HIP(hipEventCreate(&e0));
        KS_HIP(hipEventCreate(&e1));
        DslashArgs a;
        a.out_parity = 0;
        a.in = in;
        a.out = out;
        for (int staged : {0, 1}) {
        for (int way : {8, 4}) {
        for (int group : {1, 2, 4}) {
        if (!form_built((int)prec, naik, group, way == 4, staged != 0)) continue;
        for (int nt : {64, 128, 256}) {
            for (int blocks_cu : {0, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32}) {
                TuneEntry t;
                t.nt = nt;
                t.group = group;
                t.way = way;
                t.staged = staged;
                if (blocks_cu > 0) {
                    long l = lds_cu / blocks_cu - 256;
                    l -= l % 256;
                    if (l <= 0 || l > lds_blk) continue;
                    t.lds = (int)l;
                }
                for (int k = 0; k < 2; ++k) launch(g, prec, ri, a, t, s);
                timed.push_back({time_launches(g, prec, ri, a, t, 5, e0, e1, s), t});
            }
        }
        }
        }
        }
        std::stable_sort(timed.begin(), timed.end(),
                         [](const std::pair<float, TuneEntry>& x,
                            const std::pair<float, TuneEntry>& y) { return x.first < y.first; });
        const size_t nfin = std::min<size_t>(4, timed.size());
        std::vector<float> sum(nfin, 0.f);
        for (int round = 0; round < 2; ++round)
            for (size_t i = 0; i < nfin; ++i) {
                launch(g, prec, ri, a, timed[i].second, s);
                sum[i] += time_launches(g, prec, ri, a, timed[i].second, 20, e0, e1, s);
            }
        for (size_t i = 0; i < nfin; ++i)
            if (sum[i] / 2 < best_us) {
                best_us = sum[i] / 2;
                best = timed[i].second;
            }
    } catch (...) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        device_free(in);
        device_free(out);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    device_free(in);
    device_free(out);
    best.us = best_us;
    best.tuned = true;
    g->tune[prec][ri] = best;
    log_msg(1, "tuned %s %d-real Dslash at %dx%dx%dx%d: %d threads, %d links per pass, %d-way, "
               "%s gathers, %d B LDS, %.1f us",
            prec == KS_F64 ? "FP64" : prec == KS_F32 ? "FP32" : "FP16", naik, G.n[0], G.n[1],
            G.n[2], G.n[3], best.nt, best.group, best.way, best.staged ? "staged" : "cached",
            best.lds, (double)best_us);
    if (cache && *cache) cache_store(cache, key, best);
}

}  // namespace ks
