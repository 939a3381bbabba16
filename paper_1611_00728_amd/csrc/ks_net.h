// Preconditioner network: internal state.
#pragma once

#include <map>

#include "ks_common.h"

namespace ks {

// N = L^+ L: the free weights are those of L's two layers (1 -> 8, 8 -> 8); the network
// applies four layers (1 -> 8 -> 8 -> 8 -> 1), the last two the adjoints of the first two.
constexpr int kNetWeights = 1 * 8 * 9 + 8 * 8 * 9;                             // free, complex
constexpr int kNetLayerWeights = kNetWeights + 8 * 8 * 9 + 8 * 1 * 9;          // applied, complex
constexpr int kWgradBlocks = 512;

extern const int kLayerIn[4];
extern const int kLayerOut[4];
size_t layer_weight_offset(int l);   // complex offset of layer l's weights

// Activation and gradient buffers of one lattice size: levels 0..4 (channels 1, 8, 8, 8, 1),
// each [parity][channel][colour][Vh] complex FP32.
struct NetBuffers {
    int vh = 0;
    float2* act[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    float2* grad[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    // matrix-core path: levels 1..3 as binary16 records [parity][6][Vh] x 16 bytes
    __half* act16[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int npart = 0;
    double* part = nullptr;
    double* wpart = nullptr;
};

struct NetCtx {
    double* w64 = nullptr;      // master free weights, complex as (re, im) pairs, layer by layer
    float* w32 = nullptr;       // FP32 weights of the four applied layers
    float* wadj = nullptr;      // adjoint-layer weights of the applied layers (backward)
    double* adam_m = nullptr;
    double* adam_v = nullptr;
    double* grad = nullptr;     // gradient of the free weights
    double* grad4 = nullptr;    // gradient of the four applied layers' weights
    double* scal = nullptr;
    double* host = nullptr;     // pinned
    int step = 0;               // Adam steps taken
    unsigned version = 0;       // bumps whenever the weights change
    std::map<int, NetBuffers> bufs;
    // MFMA operand cache
    __half* wmma = nullptr;
    unsigned wmma_version = ~0u;
    float wmma_scale = 0.f;     // binary16 link scale folded into the operands
};

NetCtx* net_create(const double* w_host);
void net_free(NetCtx* n);
void net_set_weights(NetCtx& n, const double* w_host, hipStream_t s);
void net_get_weights(NetCtx& n, double* w_host, hipStream_t s);
// the free weights, Adam's moments and step count (host arrays of 2 * kNetWeights reals each)
void net_get_state(NetCtx& n, double* w, double* m, double* v, int* step, hipStream_t s);
void net_set_state(NetCtx& n, const double* w, const double* m, const double* v, int step,
                   hipStream_t s);
NetBuffers& net_buffers(NetCtx& n, const Geom& g);
void net_forward(NetCtx& n, NetBuffers& B, ks_gauge_t g, hipStream_t s);
void net_apply_f32(NetCtx& n, ks_gauge_t g, const double* in, double* out, double in_scale,
                   hipStream_t s);
// complex128 [Vh][3] even-site vectors, on the matrix-core path
void net_apply_mfma(NetCtx& n, ks_gauge_t g, const double* in, double* out, hipStream_t s);
// matrix-core operands of the four layers for the current weights and g's binary16 link scale
void net_mfma_prepare(NetCtx& n, ks_gauge_t g, hipStream_t s);
void net_apply_mfma_spinor(NetCtx& n, ks_gauge_t g, ks_prec_t prec, const void* r, void* z,
                           const double* in_scale, const int* gate, hipStream_t s);
// algorithmic bytes of one application per even site, the solver's vector taking vec_bytes
// per even site (matrix-core path: per full-lattice site as net_mfma_model_bytes_per_site)
double net_model_bytes(int use_mfma, double vec_bytes);
double net_mfma_model_bytes_per_site(int vec_bytes);
// N applied to an inner-precision field r (Spinor<prec> layout) into z, for the solver: the
// input is multiplied by *in_scale (device) and the output divided by it; every launch does
// nothing while *gate != 0.
void net_apply_spinor(NetCtx& n, ks_gauge_t g, ks_prec_t prec, const void* r, void* z,
                      const double* in_scale, const int* gate, int use_mfma, hipStream_t s);
double net_loss_grad(NetCtx& n, int npairs, const ks_gauge_t* gauges, const double* sigma,
                     const double* const* b, const double* const* x, hipStream_t s);
void net_adam(NetCtx& n, double lr, hipStream_t s);

ks_status_t fcg_core(ks_gauge_t g, NetCtx& net, double sigma, const double* b, double* x,
                     const ks_solver_params& prm, int use_mfma, ks_solver_stats& stats,
                     hipStream_t s);
void fcg_release(ks_gauge_t g);

}  // namespace ks

struct ks_net_s {
    ks::NetCtx* ctx;
};
