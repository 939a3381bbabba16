// Internal declarations of libks: handles, device helpers, launch helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/ks.h"

namespace ks {

// ------------------------------------------------------------------ errors

void set_error(const char* fmt, ...);

// Diagnostics on stderr, one line each prefixed "[ks]", when the environment variable KS_LOG
// holds a level >= `level` (read once per process; unset or 0: silent).  1: every solve's
// summary, tuning results and returned errors; 2: also the tuner's cache decisions.
int log_level();
void log_msg(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

struct Failure {
    ks_status_t code;
};

#define KS_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ::ks::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),      \
                            __FILE__, __LINE__);                                        \
            throw ::ks::Failure{KS_ERR_HIP};                                            \
        }                                                                               \
    } while (0)

#define KS_REQUIRE(cond, code, ...)                                                     \
    do {                                                                                \
        if (!(cond)) {                                                                  \
            ::ks::set_error(__VA_ARGS__);                                               \
            throw ::ks::Failure{code};                                                  \
        }                                                                               \
    } while (0)

void* device_alloc(size_t bytes);
// device_alloc, then the memory cleared on stream s (link stores: their padding rows are zero)
void* device_alloc_zero(size_t bytes, hipStream_t s);
void device_free(void* p);

// ------------------------------------------------------------------ geometry

struct Geom {
    int n[4];
    int stride[4];     // lexicographic strides 1, Nx, Nx Ny, Nx Ny Nz
    int V, Vh;
    int lp;            // sites per link plane (link_pitch(Vh) >= Vh)
};

// Sites per plane of a link store: Vh rounded up to a multiple of 512, plus 256.  A hopping
// term streams 144 link planes at the same site offset; with a power-of-two pitch (Vh = 2^19
// at 32^4) those streams meet the same HBM channels, and a pitch of 256 (mod 512) sites
// spreads them (144 planes of 16-byte entries read at 32^4: 5.5 TB/s at pitch Vh, 6.8 TB/s at
// Vh + 256; 1024 and 4096 extra sites are as slow as none).
inline int link_pitch(int vh) { return ((vh + 511) / 512) * 512 + 256; }

Geom make_geom(const int dims[4]);

// ------------------------------------------------------------------ link stores

// Per precision, per output parity: fat planes [8 slots][9 entries][lp] and Naik planes
// [8 slots][9 or 6 entries][lp] of complex numbers (double2 / float2 / __half2), lp the link
// pitch of the geometry (rows Vh .. lp - 1 of a plane are zero and never read).
// Slot s < 4: forward link of direction s at the site; s >= 4: minus the adjoint of the
// backward link of direction s - 4 (one hop for fat, three hops for Naik).
struct LinkStore {
    bool ready = false;
    void* fat[2] = {nullptr, nullptr};
    void* naik[2] = {nullptr, nullptr};
    float fat_scale = 1.f;     // value = stored * scale (FP16 power-of-two scales; else 1)
    float naik_scale = 1.f;
    size_t bytes = 0;
};

struct Workspace;   // solver buffers, solvers.hip

// Launch configuration of one Dslash variant: threads per block and dynamic LDS bytes per
// block (LDS only limits how many blocks share a CU; the kernel does not use it).
struct TuneEntry {
    int nt = 256;
    int group = 1;      // link matrices loaded per pass of the Dslash site loop
    int way = 8;        // 8: a site's own backward slots; 4: neighbours' forward slots
    int staged = 0;     // 1: x/y neighbour vectors staged in LDS
    int lds = 0;
    float us = 0.f;     // measured time per launch when tuned
    bool tuned = false;
};

}  // namespace ks

struct ks_gauge_s {
    ks::Geom geom;
    // [prec][recon: 0 = 18, 1 = 12]
    ks::LinkStore store[3][2];
    double naik_c0 = 0.0;       // real Naik scale c for 12-real storage
    ks::TuneEntry tune[3][2];   // Dslash launch configuration per [prec][recon]
    ks::Workspace* ws = nullptr;
    size_t extra_bytes = 0;
};

struct ks_field_s {
    ks_gauge_t g;
    int parity;
    ks_prec_t prec;
    void* data;
    size_t bytes;
};

namespace ks {

size_t field_bytes(const Geom& g, ks_prec_t prec);
size_t entry_bytes(ks_prec_t prec);   // one complex number of a link
int recon_index(ks_recon_t r);

// ------------------------------------------------------------------ device helpers

constexpr int kBlock = 256;

// Bijective workgroup -> tile map that hands each of the 8 XCDs (workgroups are dealt to
// them round-robin) one contiguous range of tiles, so that neighbouring sites share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks)
{
    const int q = nblocks >> 3, r = nblocks & 7;
    const int xcd = bid & 7;
    return xcd * q + (xcd < r ? xcd : r) + (bid >> 3);
}

// Site coordinates of checkerboard row h of parity `par`.
__device__ __forceinline__ void cb_coords(const Geom& g, int h, int par, int c[4])
{
    const unsigned i0 = 2u * (unsigned)h;
    const unsigned x0 = i0 % (unsigned)g.n[0];
    unsigned r = i0 / (unsigned)g.n[0];
    c[1] = (int)(r % (unsigned)g.n[1]);
    r /= (unsigned)g.n[1];
    c[2] = (int)(r % (unsigned)g.n[2]);
    c[3] = (int)(r / (unsigned)g.n[2]);
    c[0] = (int)x0 + ((c[1] + c[2] + c[3] + par) & 1);
}

// Checkerboard row of the site k steps (|k| <= 3 < extent) along mu from site i.
__device__ __forceinline__ int hop_cb(const Geom& g, int i, const int c[4], int mu, int k)
{
    int cm = c[mu] + k;
    int j = i + k * g.stride[mu];
    if (cm >= g.n[mu]) j -= g.n[mu] * g.stride[mu];
    else if (cm < 0) j += g.n[mu] * g.stride[mu];
    return j >> 1;
}

__device__ __forceinline__ int site_index(const Geom& g, const int c[4])
{
    return c[0] + g.stride[1] * c[1] + g.stride[2] * c[2] + g.stride[3] * c[3];
}

// Wave + block sum of a double into one value per block (thread 0 holds it).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double red[NT / 64];
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NT / 64; ++k) s += red[k];
    }
    return s;
}

template <int NT>
__device__ __forceinline__ double block_max(double v)
{
    __shared__ double red[NT / 64];
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NT / 64; ++k) s = fmax(s, red[k]);
    }
    return s;
}

inline int blocks_for(long n, int nt = kBlock) { return (int)((n + nt - 1) / nt); }

// ------------------------------------------------------------------ reductions (blas.hip)

// Deterministic sum of `n` doubles (fixed order), result written to *out (device).
void reduce_sum(const double* partials, int n, double* out, hipStream_t s);
void reduce_max(const double* partials, int n, double* out, hipStream_t s);

// ------------------------------------------------------------------ launchers

void gauge_build_f64(ks_gauge_t g, const double* fat_dev, const double* naik_dev,
                     hipStream_t s);
void gauge_prepare(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon, hipStream_t s);
void gauge_release(ks_gauge_t g);

// out = D in (out parity p, in parity 1-p).  With xpay: out = a * x - D in, and when
// dot_partials is set, per-block partial sums of Re<x, out> are written there.
struct DslashArgs {
    int out_parity;
    const void* in;
    void* out;
    const void* x = nullptr;       // xpay operand (same parity as out)
    double a = 0.0;
    double* dot_partials = nullptr;
    const int* gate = nullptr;     // when set and *gate != 0 the launch does nothing
};
void dslash(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon, const DslashArgs& a,
            hipStream_t s);
// number of per-block partial sums a Dslash launch of this variant writes
int dslash_blocks(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon);
// upper bound of dslash_blocks over every launch configuration
int dslash_max_blocks(const Geom& g);
// fat and Naik links from thin links by two smearing levels with a U(3) projection between
extern const double kHisqLevel1[5];
extern const double kHisqLevel2[5];
extern const double kHisqNaik;
void hisq_links(const Geom& G, const double* thin, double* fat, double* naik,
                const double* level1, const double* level2, double c_naik, hipStream_t st);
// frees the link construction's scratch on every device
void hisq_release();
// whether the kernel of this launch form exists for the variant
bool dslash_form_built(ks_prec_t prec, ks_recon_t recon, int links_per_pass, int link_access,
                       int staged);
// times the candidate launch configurations on this lattice and keeps the fastest
void dslash_tune(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon, hipStream_t s);

// Field conversions between complex128 [Vh][3] (AoS) and the internal layouts.
void import_field(const Geom& g, ks_prec_t prec, const double* src, void* dst, hipStream_t s);
void export_field(const Geom& g, ks_prec_t prec, const void* src, double* dst, hipStream_t s);

}  // namespace ks
