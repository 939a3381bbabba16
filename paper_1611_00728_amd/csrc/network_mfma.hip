// Inference form of the 8 -> 8 network layer with the channel mixing on the matrix cores.
//
// Per tile of 64 sites the layer is a real GEMM  D[16 x 192] = A[16 x 144] B[144 x 192]:
// rows of D are (re, im) x 8 output channels, columns (site, colour); B holds the transported
// activations (T_p phi_c')(x)_a for the 72 (path, channel) pairs, real parts in rows 0..71 and
// imaginary parts in rows 72..143; A is the real embedding of the complex weights,
// [[Re w, -Im w], [Im w, Re w]].  The transports run on the vector ALUs in FP32 and are
// written to LDS in binary16; v_mfma_f32_16x16x16_f16 (FP16 inputs, FP32 accumulation) does
// the mixing: 9 K-steps x 12 column tiles per block, three column tiles per wave.
#include "ks_device.h"
#include "ks_net.h"

namespace ks {

namespace {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;          // sites per block
constexpr int kK = 144;            // GEMM depth (2 x 9 paths x 8 channels)
constexpr int kRow = kK + 8;       // LDS row pitch in halves (padding against bank conflicts)

template <int C>
__device__ __forceinline__ const float2* aptr(const float2* a, int par, int c, int k, int vh)
{
    return a + ((size_t)(par * C + c) * 3 + k) * vh;
}

// A fragments: lane l of K-step kb holds A[l % 16][16 kb + 4 (l / 16) + i], i = 0..3.
__global__ void net_mfma_weights_kernel(const float2* __restrict__ w, half4_t* __restrict__ frag)
{
    const int kb = blockIdx.x;     // 0..8
    const int l = threadIdx.x;     // 0..63
    const int m = l % 16;
    half4_t v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = 16 * kb + 4 * (l / 16) + i;
        const int kk = k % 72;               // (path, channel) pair
        const bool imag_col = k >= 72;
        const int p = kk / 8, ci = kk % 8;
        const int c = m % 8;
        const float2 wc = w[(c * 8 + ci) * 9 + p];
        float a;
        if (m < 8) a = imag_col ? -wc.y : wc.x;     // Re y = Re w Re u - Im w Im u
        else a = imag_col ? wc.x : wc.y;            // Im y = Im w Re u + Re w Im u
        v[i] = (_Float16)a;
    }
    frag[kb * 64 + l] = v;
}

__global__ __launch_bounds__(256) void net_layer_mfma_kernel(Geom g, const float2* __restrict__ in,
                                                             float2* __restrict__ out,
                                                             const void* __restrict__ fat_e,
                                                             const void* __restrict__ fat_o,
                                                             const half4_t* __restrict__ frag)
{
    __shared__ _Float16 bt[kTile * 3][kRow];
    const int vh = g.Vh;
    const int tid = threadIdx.x;
    // ---- phase 1: transports of 64 sites, four threads per site
    {
        const int sl = tid >> 2, sub = tid & 3;
        const int t = blockIdx.x * kTile + sl;
        const bool live = t < 2 * vh;
        const int par = (live && t >= vh) ? 1 : 0;
        const int h = live ? t - par * vh : 0;
        const void* fat = par ? fat_o : fat_e;
        int c[4];
        cb_coords(g, h, par, c);
        const int i = site_index(g, c);
        const int p_lo = sub == 0 ? 0 : 1 + 2 * sub;      // {0,1,2} {3,4} {5,6} {7,8}
        const int p_hi = sub == 0 ? 3 : 3 + 2 * sub;
        for (int p = p_lo; p < p_hi; ++p) {
            cx<float> m[9];
            int nbh = h, spar = par;
            if (p > 0) {
                const int s = p - 1;
                const int mu = s & 3;
                const bool bwd = s >= 4;
                nbh = hop_cb(g, i, c, mu, bwd ? -1 : +1);
                spar = 1 - par;
                load_link<KS_F32, 9>(fat, s, vh, h, m);
                if (bwd)
#pragma unroll
                    for (int e = 0; e < 9; ++e) m[e] = {-m[e].r, -m[e].i};
            }
#pragma unroll 2
            for (int ci = 0; ci < 8; ++ci) {
                cx<float> v[3], tv[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const float2 q = live ? aptr<8>(in, spar, ci, k, vh)[nbh] : make_float2(0.f, 0.f);
                    v[k] = {q.x, q.y};
                }
                if (p == 0) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) tv[k] = v[k];
                } else {
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        tv[a] = {0.f, 0.f};
#pragma unroll
                        for (int b = 0; b < 3; ++b) cfma(tv[a], m[a * 3 + b], v[b]);
                    }
                }
                const int kk = p * 8 + ci;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    bt[sl * 3 + a][kk] = (_Float16)tv[a].r;
                    bt[sl * 3 + a][72 + kk] = (_Float16)tv[a].i;
                }
            }
        }
    }
    __syncthreads();
    // ---- phase 2: D = A B on the matrix cores, three 16-column tiles per wave
    const int lane = tid & 63, wv = tid >> 6;
    half4_t af[9];
#pragma unroll
    for (int kb = 0; kb < 9; ++kb) af[kb] = frag[kb * 64 + lane];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int nb = wv * 3 + j;
        const int col = nb * 16 + (lane & 15);
        float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 9; ++kb) {
            const _Float16* src = &bt[col][16 * kb + 4 * (lane >> 4)];
            half4_t bv;
            bv[0] = src[0];
            bv[1] = src[1];
            bv[2] = src[2];
            bv[3] = src[3];
            acc = __builtin_amdgcn_mfma_f32_16x16x16f16(af[kb], bv, acc, 0, 0, 0);
        }
        // lane holds D[4 (lane / 16) + i][col]: rows 0..7 real parts, 8..15 imaginary parts
        float4_t im;
#pragma unroll
        for (int q = 0; q < 4; ++q) im[q] = __shfl_xor(acc[q], 32, 64);
        if ((lane >> 4) < 2) {
            const int sl = col / 3, a = col % 3;
            const int t = blockIdx.x * kTile + sl;
            if (t < 2 * vh) {
                const int par = t >= vh ? 1 : 0;
                const int h = t - par * vh;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int ch = 4 * (lane >> 4) + q;
                    float2* dst = const_cast<float2*>(aptr<8>(out, par, ch, a, vh));
                    dst[h] = make_float2(acc[q], im[q]);
                }
            }
        }
    }
}

}  // namespace

void net_mfma_prepare(NetCtx& n, hipStream_t s)
{
    if (n.wmma_version == n.version) return;
    if (!n.wmma) n.wmma = static_cast<__half*>(device_alloc(sizeof(half4_t) * 9 * 64 * 2));
    half4_t* fr = reinterpret_cast<half4_t*>(n.wmma);
    const float2* w = reinterpret_cast<const float2*>(n.w32);
    for (int l = 1; l <= 2; ++l)
        net_mfma_weights_kernel<<<9, 64, 0, s>>>(w + layer_weight_offset(l), fr + (l - 1) * 9 * 64);
    KS_HIP(hipGetLastError());
    n.wmma_version = n.version;
}

void net_layer_mfma(NetCtx& n, ks_gauge_t g, const float2* in, float2* out, int which,
                    hipStream_t s)
{
    const LinkStore& st = g->store[KS_F32][0];
    const half4_t* fr = reinterpret_cast<const half4_t*>(n.wmma) + (which - 1) * 9 * 64;
    net_layer_mfma_kernel<<<blocks_for(2L * g->geom.Vh, kTile), 256, 0, s>>>(
        g->geom, in, out, st.fat[0], st.fat[1], fr);
    KS_HIP(hipGetLastError());
}

}  // namespace ks
