// Inference form of the network N = L^+ L (four layers 1 -> 8 -> 8 -> 8 -> 1) with the channel
// mixing on the matrix cores and binary16 activations.
//
// A layer is y_c(x) = sum_p sum_c' w[c][c'][p] (T_p phi_c')(x), p = 0 the identity, 1 + mu the
// forward hop V_mu(x) phi(x + mu), 5 + mu the backward hop V_mu(x - mu)^+ phi(x - mu).  For a
// group of 16 sites it is a sum of real GEMM steps D[16 x 48] += A[16 x 16] B[16 x 48] on
// v_mfma_f32_16x16x16_f16: rows of D are (re, im) x 8 output channels, columns (colour, site).
//
// Lane (n, g) of a wave (n = lane % 16 the site, g = lane / 16) owns the two hops along
// direction mu = g: it loads its site's two stored links for that direction and the neighbours'
// eight input channels, and transports all eight channels (dot2 of binary16 pairs, FP32
// accumulation).  A B fragment row block 4g..4g+3 is then two channels of lane group g's own
// path, so one MFMA mixes four paths at once: K = 16 covers (path of group g) x (channel pair
// cp) x (re, im), and the A fragment of (hop j, pair cp) holds w[c][2cp + i/2][path of g] in
// the rows of group g.  Every link and every neighbour index is loaded or computed once per
// site; nine MFMA blocks per colour (the identity and two hops times four channel pairs)
// accumulate in registers.
//
// The stored links are binary16 scaled by 1/fat_scale, and the backward slots hold
// -V_mu(x - mu)^+: both factors are folded into the A fragments.
//
// Activations between layers: [parity][plane a*2 + q][Vh] records of 16 bytes, plane (a, q)
// holding channels 4q..4q+3 of colour a as binary16 (re, im) pairs.  The first layer reads the
// solver's vector (even sites; the odd sites of the input are zero, so even outputs take only
// the identity path and odd outputs only the hops), the last layer computes even sites only
// and writes the solver's vector.
#include <type_traits>

#include "ks_device.h"
#include "ks_net.h"

namespace ks {

namespace {

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float2_t __attribute__((ext_vector_type(2)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kWaveSites = 16;     // sites per wave
constexpr int kBlockSites = 64;    // four waves per block
constexpr int kFrags = 9;          // A fragments per layer: identity, then (hop j, pair cp)

// complex128 site-major vectors [Vh][3] (the network's own entry point)
struct SpinorAos {
    using R = double;
    __device__ static __forceinline__ void load(const void* b, int, int h, cx<R> v[3])
    {
        const double2* p = static_cast<const double2*>(b) + (size_t)3 * h;
#pragma unroll
        for (int k = 0; k < 3; ++k) v[k] = {p[k].x, p[k].y};
    }
    __device__ static __forceinline__ void store(void* b, int, int h, const cx<R> v[3])
    {
        double2* p = static_cast<double2*>(b) + (size_t)3 * h;
#pragma unroll
        for (int k = 0; k < 3; ++k) p[k] = make_double2(v[k].r, v[k].i);
    }
};

__device__ __forceinline__ half2_t as_h2(unsigned u)
{
    half2_t h;
    __builtin_memcpy(&h, &u, 4);
    return h;
}

__device__ __forceinline__ unsigned as_u(half2_t h)
{
    unsigned u;
    __builtin_memcpy(&u, &h, 4);
    return u;
}

__device__ __forceinline__ half2_t to_h2(float re, float im)
{
    const float2_t f = {re, im};
    return __builtin_convertvector(f, half2_t);
}

__device__ __forceinline__ half4_t cat(half2_t a, half2_t b)
{
    return {a[0], a[1], b[0], b[1]};
}

// A fragments: lane l holds A[m][k], m = l % 16, k = 4 (l / 16) + i, i = 0..3; row m is output
// channel m % 8, real part for m < 8 and imaginary part otherwise; k = 4 g + i is input channel
// c' and (i odd) its imaginary part:
//   fragment 0 (identity): c' = 2 g + i / 2, path 0;
//   fragment 1 + 4 j + cp:  c' = 2 cp + i / 2, path 1 + g (j = 0) or 5 + g (j = 1), weight
//                           times the link scale, negated for j = 1 (stored -V^+).
__global__ void net_frag_kernel(const float2* __restrict__ w, int cin, int cout, float link_scale,
                                half4_t* __restrict__ frag)
{
    const int f = blockIdx.x;      // 0..8
    const int l = threadIdx.x;     // 0..63
    const int m = l % 16, g = l / 16;
    const int c = m % 8;
    half4_t v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int ci, p;
        float sc;
        if (f == 0) {
            ci = 2 * g + i / 2;
            p = 0;
            sc = 1.f;
        } else {
            const int j = (f - 1) / 4, cp = (f - 1) % 4;
            ci = 2 * cp + i / 2;
            p = j ? 5 + g : 1 + g;
            sc = j ? -link_scale : link_scale;
        }
        const bool imag_in = (i & 1) != 0;
        float2 wc = make_float2(0.f, 0.f);
        if (c < cout && ci < cin) {
            wc = w[(c * cin + ci) * 9 + p];
            wc = make_float2(sc * wc.x, sc * wc.y);
        }
        float a;
        if (m < 8) a = imag_in ? -wc.y : wc.x;      // Re y = Re w Re u - Im w Im u
        else a = imag_in ? wc.x : wc.y;             // Im y = Im w Re u + Re w Im u
        v[i] = (_Float16)a;
    }
    frag[f * 64 + l] = v;
}

// Checkerboard row of the site k steps along mu = g (lane-dependent) from site i.  The extents
// and strides pass through readfirstlane (they are uniform) so that the per-lane choice stays a
// select between registers, not an indexed read of the kernel argument from scratch memory.
__device__ __forceinline__ int lane_hop(const Geom& geo, int i, const int c[4], int g, int k)
{
    int ext[4], str[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        ext[d] = __builtin_amdgcn_readfirstlane(geo.n[d]);
        str[d] = __builtin_amdgcn_readfirstlane(geo.stride[d]);
    }
    const int cm = (g == 0 ? c[0] : g == 1 ? c[1] : g == 2 ? c[2] : c[3]) + k;
    const int n = g == 0 ? ext[0] : g == 1 ? ext[1] : g == 2 ? ext[2] : ext[3];
    const int st = g == 0 ? str[0] : g == 1 ? str[1] : g == 2 ? str[2] : str[3];
    int j = i + k * st;
    if (cm >= n) j -= n * st;
    else if (cm < 0) j += n * st;
    return j >> 1;
}

// The nine entries of stored link slot s at checkerboard row h (binary16 (re, im) pairs, planes
// of lp sites), returned as the two operand forms of a complex product by dot2:
// lr = (re, -im) gives Re(m v) = dot2(lr, v), li = (im, re) gives Im(m v) = dot2(li, v).
__device__ __forceinline__ void link_pairs(const void* fat, int s, int lp, int h, half2_t lr[9],
                                           half2_t li[9])
{
    using LP = LinkPack<KS_F16, 9>;
    static_assert(LP::NF == 2 && LP::NR == 1, "binary16 link packing");
    const char* sb = static_cast<const char*>(fat) + (size_t)s * 9 * LP::ES * lp;
    unsigned u[9];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        // streamed once per layer: non-temporal, so that they do not evict the activations,
        // which the neighbours read again
        const uvec4 q =
            __builtin_nontemporal_load(reinterpret_cast<const uvec4*>(sb + (size_t)j * 16 * lp) + h);
        u[4 * j] = q.x;
        u[4 * j + 1] = q.y;
        u[4 * j + 2] = q.z;
        u[4 * j + 3] = q.w;
    }
    u[8] = __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(sb + (size_t)2 * 16 * lp) + h);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        lr[e] = as_h2(u[e] ^ 0x80000000u);
        li[e] = as_h2(__builtin_amdgcn_alignbit(u[e], u[e], 16));
    }
}

template <int CIN>
struct Gathered {
    // v[ch][b]: input channel ch, colour b, binary16 (re, im)
    half2_t v[CIN][3];
};

// the eight channels of activation record (par, h): plane (a, q) holds channels 4q..4q+3
__device__ __forceinline__ void load_act(const uvec4* act, int par, int vh, int h, Gathered<8>& x)
{
    const uvec4* base = act + (size_t)par * 6 * vh;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const uvec4 r = base[(size_t)(a * 2 + q) * vh + h];
            x.v[4 * q][a] = as_h2(r.x);
            x.v[4 * q + 1][a] = as_h2(r.y);
            x.v[4 * q + 2][a] = as_h2(r.z);
            x.v[4 * q + 3][a] = as_h2(r.w);
        }
}

// dot2 of two binary16 pairs into FP32 with a zero accumulator, in the three-operand form (the
// builtin with a constant zero becomes a move of zero plus the accumulating two-operand form)
__device__ __forceinline__ float dot2_new(half2_t a, half2_t b)
{
    float r;
    asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Re and Im of row a of the link times input channel ch (FP32)
template <int CIN>
__device__ __forceinline__ float2_t transport(const half2_t lr[9], const half2_t li[9],
                                              const Gathered<CIN>& x, int ch, int a)
{
    float re = dot2_new(lr[a * 3], x.v[ch][0]);
    float im = dot2_new(li[a * 3], x.v[ch][0]);
#pragma unroll
    for (int b = 1; b < 3; ++b) {
        re = __builtin_amdgcn_fdot2(lr[a * 3 + b], x.v[ch][b], re, false);
        im = __builtin_amdgcn_fdot2(li[a * 3 + b], x.v[ch][b], im, false);
    }
    return {re, im};
}

// IN: the first layer reads an inner-precision vector IN (even sites, times *scale); otherwise
// (IN = void) the binary16 activations.  OUT: the last layer writes OUT (even sites, divided by
// *scale); otherwise binary16 activations of both parities.
// At least five waves per SIMD (the 8 -> 8 layer from 99 to 88 registers, no spills): more
// gathers in flight per CU (32^4 application 408 -> 397 us).
template <int CIN, int COUT, class IN, class OUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void net_mfma_layer_kernel(
    Geom geo, const void* __restrict__ in, void* __restrict__ out, const void* __restrict__ fat_e,
    const void* __restrict__ fat_o, const half4_t* __restrict__ frag,
    const double* __restrict__ scale, const int* __restrict__ gate, int slab)
{
    constexpr bool kFirst = CIN == 1;
    constexpr bool kLast = COUT == 1;
    static_assert(kFirst != std::is_same<IN, void>::value, "the first layer reads a vector");
    static_assert(kLast != std::is_same<OUT, void>::value, "the last layer writes a vector");
    if (gate && *gate) return;
    const int vh = geo.Vh;
    const int nsites = kLast ? vh : 2 * vh;
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, grp = lane >> 4;
    bool live;
    int par, h;
    if (slab) {
        // workgroups are dealt to the 8 XCDs in turn; XCD k takes the z-planes
        // [k Nz / 8, (k + 1) Nz / 8) of every t, t after t, both parities of a (z, t) plane
        // together.  A block's x, y, z and t neighbours are then loaded by its own XCD's
        // blocks shortly before or after it, while they are still in that XCD's L2; only
        // the two z-planes next to the slab come from another XCD's share (32^4 application
        // 428 -> 408 us against contiguous site ranges per XCD).
        constexpr int npar = kLast ? 1 : 2;
        const int plane = geo.n[0] * geo.n[1] / 2;          // rows of one (z, t) plane
        const int tpp = plane / kBlockSites;
        const int zs = geo.n[2] >> 3;
        int q = blockIdx.x >> 3;
        const int yb = q % tpp;
        q /= tpp;
        par = npar == 1 ? 0 : q & 1;
        q /= npar;
        const int z = (blockIdx.x & 7) * zs + q % zs;
        const int tt = q / zs;
        h = (tt * geo.n[2] + z) * plane + yb * kBlockSites + (threadIdx.x >> 6) * kWaveSites + n;
        live = true;
    } else {
        const int t = xcd_tile(blockIdx.x, gridDim.x) * kBlockSites + (threadIdx.x >> 6) * kWaveSites + n;
        live = t < nsites;
        par = (live && t >= vh) ? 1 : 0;
        h = live ? t - par * vh : 0;
    }
    const void* fat = par ? fat_o : fat_e;
    float sc = 1.f;
    if (kFirst || kLast) sc = scale ? (float)*scale : 1.f;

    half4_t af[kFrags];
#pragma unroll
    for (int f = 0; f < kFrags; ++f) af[f] = frag[f * 64 + lane];

    float4_t acc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a] = {0.f, 0.f, 0.f, 0.f};

    // A lane past the end works on site 0 of the even parity: its values reach only its own
    // column of D, which is never stored.  The middle layers therefore load without branches;
    // the first layer's branches follow the parity, which is uniform across a wave except at
    // the one wave that straddles the two halves.
    const half2_t z = {(_Float16)0.f, (_Float16)0.f};

    // identity path: lane (n, g) supplies channels 2g, 2g+1 of its own site
    {
        half2_t lo[3], hi[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) lo[a] = hi[a] = z;
        if constexpr (kFirst) {
            if (par == 0 && grp == 0) {   // odd input sites are zero; groups g > 0 meet zero weights
                cx<typename IN::R> v[3];
                IN::load(in, vh, h, v);
#pragma unroll
                for (int a = 0; a < 3; ++a) lo[a] = to_h2(sc * (float)v[a].r, sc * (float)v[a].i);
            }
        } else {
            const uvec2* base = static_cast<const uvec2*>(in) + (size_t)par * 6 * 2 * vh;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const uvec2 r = base[(size_t)(a * 2 + (grp >> 1)) * 2 * vh + 2 * h + (grp & 1)];
                lo[a] = as_h2(r.x);
                hi[a] = as_h2(r.y);
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
            acc[a] = __builtin_amdgcn_mfma_f32_16x16x16f16(af[0], cat(lo[a], hi[a]), acc[a], 0, 0, 0);
    }

    // the two hops along mu = grp; the first layer's even outputs have none (odd input is zero)
    int c[4];
    cb_coords(geo, h, par, c);
    const int i = site_index(geo, c);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        half2_t lr[9], li[9];
        Gathered<CIN> x;
        if (!kFirst || par == 1) {
            const int nbh = lane_hop(geo, i, c, grp, j ? -1 : +1);
            link_pairs(fat, j * 4 + grp, geo.lp, h, lr, li);
            if constexpr (kFirst) {
                cx<typename IN::R> v[3];
                IN::load(in, vh, nbh, v);
#pragma unroll
                for (int b = 0; b < 3; ++b) x.v[0][b] = to_h2(sc * (float)v[b].r, sc * (float)v[b].i);
            } else {
                load_act(static_cast<const uvec4*>(in), 1 - par, vh, nbh, x);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 9; ++e) lr[e] = li[e] = z;
#pragma unroll
            for (int b = 0; b < 3; ++b) x.v[0][b] = z;
        }
        constexpr int NCP = CIN == 1 ? 1 : 4;
#pragma unroll
        for (int cp = 0; cp < NCP; ++cp) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const float2_t u0 = transport<CIN>(lr, li, x, 2 * cp, a);
                half2_t h1 = z;
                if constexpr (CIN > 1) {
                    const float2_t u1 = transport<CIN>(lr, li, x, 2 * cp + 1, a);
                    h1 = to_h2(u1[0], u1[1]);
                }
                acc[a] = __builtin_amdgcn_mfma_f32_16x16x16f16(
                    af[1 + 4 * j + cp], cat(to_h2(u0[0], u0[1]), h1), acc[a], 0, 0, 0);
            }
        }
    }

    // lane (n, g) holds D[4 g + r][n] for colour a: g = 0, 1 the real parts of channels
    // 4 g .. 4 g + 3, g = 2, 3 the imaginary parts of channels 4 (g - 2) .. 4 (g - 2) + 3
    float4_t other[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) other[a][r] = __shfl_xor(acc[a][r], 32, 64);
    if (!live) return;
    if constexpr (kLast) {
        if (grp == 0) {
            const double inv = 1.0 / (scale ? *scale : 1.0);
            cx<typename OUT::R> v[3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                v[a] = {(typename OUT::R)(inv * acc[a][0]), (typename OUT::R)(inv * other[a][0])};
            OUT::store(out, vh, h, v);
        }
    } else {
        // lanes g < 2 write colours 0 and 1 of channel block q = g, lanes g >= 2 colour 2 of
        // block q = g - 2
        uvec4* base = static_cast<uvec4*>(out) + (size_t)par * 6 * vh;
        const int q = grp & 1;
        const bool re_own = grp < 2;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if ((a < 2) != re_own) continue;
            const float4_t re = re_own ? acc[a] : other[a];
            const float4_t im = re_own ? other[a] : acc[a];
            uvec4 rec;
            rec.x = as_u(to_h2(re[0], im[0]));
            rec.y = as_u(to_h2(re[1], im[1]));
            rec.z = as_u(to_h2(re[2], im[2]));
            rec.w = as_u(to_h2(re[3], im[3]));
            base[(size_t)(a * 2 + q) * vh + h] = rec;
        }
    }
}

template <int CIN, int COUT, class IN, class OUT>
void launch_layer(ks_gauge_t g, const void* in, void* out, const half4_t* frag,
                  const double* scale, const int* gate, hipStream_t s)
{
    const LinkStore& st = g->store[KS_F16][0];
    const Geom& G = g->geom;
    const long nsites = COUT == 1 ? G.Vh : 2L * G.Vh;
    // the z-slab order needs 8 | Nz and whole blocks per (z, t) plane; it then tiles the
    // sites exactly
    const int slab = (G.n[2] % 8 == 0 && (G.n[0] * G.n[1] / 2) % kBlockSites == 0) ? 1 : 0;
    net_mfma_layer_kernel<CIN, COUT, IN, OUT><<<blocks_for(nsites, kBlockSites), 256, 0, s>>>(
        G, in, out, st.fat[0], st.fat[1], frag, scale, gate, slab);
    KS_HIP(hipGetLastError());
}

template <class V>
void apply_layers(NetCtx& n, ks_gauge_t g, const void* r, void* z, const double* scale,
                  const int* gate, hipStream_t s)
{
    NetBuffers& B = net_buffers(n, g->geom);
    if (!B.act16[1]) {
        const size_t bytes = (size_t)2 * 6 * 16 * g->geom.Vh;
        for (int l = 1; l <= 3; ++l) B.act16[l] = static_cast<__half*>(device_alloc(bytes));
    }
    const half4_t* fr = reinterpret_cast<const half4_t*>(n.wmma);
    constexpr int F = kFrags * 64;
    launch_layer<1, 8, V, void>(g, r, B.act16[1], fr, scale, gate, s);
    launch_layer<8, 8, void, void>(g, B.act16[1], B.act16[2], fr + F, scale, gate, s);
    launch_layer<8, 8, void, void>(g, B.act16[2], B.act16[3], fr + 2 * F, scale, gate, s);
    launch_layer<8, 1, void, V>(g, B.act16[3], z, fr + 3 * F, scale, gate, s);
}

}  // namespace

void net_mfma_prepare(NetCtx& n, ks_gauge_t g, hipStream_t s)
{
    gauge_prepare(g, KS_F16, KS_RECON_18, s);
    const float link_scale = g->store[KS_F16][0].fat_scale;
    if (n.wmma_version == n.version && n.wmma_scale == link_scale) return;
    if (!n.wmma) n.wmma = static_cast<__half*>(device_alloc(sizeof(half4_t) * kFrags * 64 * 4));
    half4_t* fr = reinterpret_cast<half4_t*>(n.wmma);
    const float2* w = reinterpret_cast<const float2*>(n.w32);
    for (int l = 0; l < 4; ++l)
        net_frag_kernel<<<kFrags, 64, 0, s>>>(w + layer_weight_offset(l), kLayerIn[l],
                                              kLayerOut[l], link_scale, fr + l * kFrags * 64);
    KS_HIP(hipGetLastError());
    n.wmma_version = n.version;
    n.wmma_scale = link_scale;
}

void net_apply_mfma_spinor(NetCtx& n, ks_gauge_t g, ks_prec_t prec, const void* r, void* z,
                           const double* in_scale, const int* gate, hipStream_t s)
{
    net_mfma_prepare(n, g, s);
    if (prec == KS_F64) apply_layers<Spinor<KS_F64>>(n, g, r, z, in_scale, gate, s);
    else apply_layers<Spinor<KS_F32>>(n, g, r, z, in_scale, gate, s);
}

void net_apply_mfma(NetCtx& n, ks_gauge_t g, const double* in, double* out, hipStream_t s)
{
    net_mfma_prepare(n, g, s);
    apply_layers<SpinorAos>(n, g, in, out, nullptr, nullptr, s);
}

double net_mfma_model_bytes_per_site(int vec_bytes)
{
    // per site of the full lattice: the first layer reads the even sites' input vector and the
    // odd sites' eight binary16 links and writes both parities' activations; the middle layers
    // read all activations and links and write all activations; the last layer reads all
    // activations and the even sites' links and writes the even sites' output vector
    const double links = 8 * 36.0, act = 96.0;
    const double first = 0.5 * vec_bytes + 0.5 * links + act;
    const double middle = act + links + act;
    const double last = act + 0.5 * links + 0.5 * vec_bytes;
    return first + 2 * middle + last;
}

}  // namespace ks
