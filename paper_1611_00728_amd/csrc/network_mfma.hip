// Inference form of the 8 -> 8 and 8 -> 1 network layers with the channel mixing on the matrix
// cores (for 8 -> 1 only rows 0 and 8 of the weight operand are nonzero).
//
// For a group of 16 sites the layer is nine accumulated real GEMM steps, one per path p:
//     D[16 x 48] += A_p[16 x 16] B_p[16 x 48],
// rows of D: (re, im) x 8 output channels; columns: (colour, site); rows of B_p: the 8 input
// channels' transported values (T_p phi_c')(x)_a as (re, im) pairs; A_p the real embedding
// of the complex weights w[c][c'][p], [[Re w, -Im w], [Im w, Re w]] interleaved to match.
// Lane (n, g) of a wave (n = lane % 16 the site, g = lane / 16) transports the input channels
// 2g and 2g+1 of its site along p in FP32 on the vector ALUs (links read from the binary16
// store, which halves their bytes; the products are rounded to binary16 for the matrix cores
// anyway), which is exactly its part of
// the B_p operand of v_mfma_f32_16x16x16_f16 for each of the three colour tiles: no staging
// through LDS.  The accumulators stay in registers over the nine paths.
#include "ks_device.h"
#include "ks_net.h"

namespace ks {

namespace {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kWaveSites = 16;     // sites per wave
constexpr int kBlockSites = 64;    // four waves per block

template <int C>
__device__ __forceinline__ const float2* aptr(const float2* a, int par, int c, int k, int vh)
{
    return a + ((size_t)(par * C + c) * 3 + k) * vh;
}

// A fragments: lane l of path p holds A_p[m][k], m = l % 16, k = 4 (l / 16) + i, i = 0..3;
// k = 2 c' + (0 for the real part of the input, 1 for the imaginary part).
// Rows of output channels c >= cout are zero.
__global__ void net_mfma_weights_kernel(const float2* __restrict__ w, int cout,
                                        half4_t* __restrict__ frag)
{
    const int p = blockIdx.x;      // 0..8
    const int l = threadIdx.x;     // 0..63
    const int m = l % 16;
    const int c = m % 8;
    half4_t v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = 4 * (l / 16) + i;
        const int ci = k / 2;
        const bool imag_in = (k & 1) != 0;
        const float2 wc = c < cout ? w[(c * 8 + ci) * 9 + p] : make_float2(0.f, 0.f);
        float a;
        if (m < 8) a = imag_in ? -wc.y : wc.x;      // Re y = Re w Re u - Im w Im u
        else a = imag_in ? wc.x : wc.y;             // Im y = Im w Re u + Re w Im u
        v[i] = (_Float16)a;
    }
    frag[p * 64 + l] = v;
}

// LP: storage of the fat links that transport (FP32, or FP16 times link_scale)
template <int COUT, int LP>
__global__ __launch_bounds__(256) void net_layer_mfma_kernel(Geom g, const float2* __restrict__ in,
                                                             float2* __restrict__ out,
                                                             const void* __restrict__ fat_e,
                                                             const void* __restrict__ fat_o,
                                                             const half4_t* __restrict__ frag,
                                                             float link_scale,
                                                             const int* __restrict__ gate)
{
    if (gate && *gate) return;
    const int vh = g.Vh;
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, grp = lane >> 4;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int t = tile * kBlockSites + (threadIdx.x >> 6) * kWaveSites + n;
    const bool live = t < 2 * vh;
    const int par = (live && t >= vh) ? 1 : 0;
    const int h = live ? t - par * vh : 0;
    const void* fat = par ? fat_o : fat_e;
    int c[4];
    cb_coords(g, h, par, c);
    const int i = site_index(g, c);
    float4_t acc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int p = 0; p < 9; ++p) {
        const half4_t af = frag[p * 64 + lane];
        cx<float> u[2][3];
        int nbh = h, spar = par;
        cx<float> m[9];
        if (p > 0) {
            const int s = p - 1;
            nbh = hop_cb(g, i, c, s & 3, s >= 4 ? -1 : +1);
            spar = 1 - par;
            load_link<LP, 9>(fat, s, vh, h, m);
            // the store holds -V(x-mu)^+ for the backward slots
            const float sc = s >= 4 ? -link_scale : link_scale;
#pragma unroll
            for (int e = 0; e < 9; ++e) m[e] = {sc * m[e].r, sc * m[e].i};
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            cx<float> v[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float2 x = live ? aptr<8>(in, spar, 2 * grp + q, k, vh)[nbh]
                                      : make_float2(0.f, 0.f);
                v[k] = {x.x, x.y};
            }
            if (p == 0) {
#pragma unroll
                for (int k = 0; k < 3; ++k) u[q][k] = v[k];
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    u[q][a] = {0.f, 0.f};
#pragma unroll
                    for (int b = 0; b < 3; ++b) cfma(u[q][a], m[a * 3 + b], v[b]);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            half4_t bv;
            bv[0] = (_Float16)u[0][a].r;
            bv[1] = (_Float16)u[0][a].i;
            bv[2] = (_Float16)u[1][a].r;
            bv[3] = (_Float16)u[1][a].i;
            acc[a] = __builtin_amdgcn_mfma_f32_16x16x16f16(af, bv, acc[a], 0, 0, 0);
        }
    }
    // lane (n, g) holds D[4 g + j][n]: g = 0, 1 real parts of channels 4 g + j, g = 2, 3 the
    // imaginary parts of channels 4 (g - 2) + j
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float4_t im;
#pragma unroll
        for (int j = 0; j < 4; ++j) im[j] = __shfl_xor(acc[a][j], 32, 64);
        if (grp < 2 && live) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ch = 4 * grp + j;
                if (ch < COUT) {
                    float2* dst = const_cast<float2*>(aptr<COUT>(out, par, ch, a, vh));
                    dst[h] = make_float2(acc[a][j], im[j]);
                }
            }
        }
    }
}

}  // namespace

void net_mfma_prepare(NetCtx& n, hipStream_t s)
{
    if (n.wmma_version == n.version) return;
    if (!n.wmma) n.wmma = static_cast<__half*>(device_alloc(sizeof(half4_t) * 9 * 64 * 3));
    half4_t* fr = reinterpret_cast<half4_t*>(n.wmma);
    const float2* w = reinterpret_cast<const float2*>(n.w32);
    for (int l = 1; l <= 3; ++l)
        net_mfma_weights_kernel<<<9, 64, 0, s>>>(w + layer_weight_offset(l), kLayerOut[l],
                                                 fr + (l - 1) * 9 * 64);
    KS_HIP(hipGetLastError());
    n.wmma_version = n.version;
}

void net_layer_mfma(NetCtx& n, ks_gauge_t g, const float2* in, float2* out, int which,
                    const int* gate, hipStream_t s)
{
    const LinkStore& st = g->store[KS_F16][0];
    const half4_t* fr = reinterpret_cast<const half4_t*>(n.wmma) + (which - 1) * 9 * 64;
    const int nb = blocks_for(2L * g->geom.Vh, kBlockSites);
    if (kLayerOut[which] == 8)
        net_layer_mfma_kernel<8, KS_F16><<<nb, 256, 0, s>>>(g->geom, in, out, st.fat[0], st.fat[1],
                                                             fr, st.fat_scale, gate);
    else
        net_layer_mfma_kernel<1, KS_F16><<<nb, 256, 0, s>>>(g->geom, in, out, st.fat[0], st.fat[1],
                                                             fr, st.fat_scale, gate);
    KS_HIP(hipGetLastError());
}

}  // namespace ks
