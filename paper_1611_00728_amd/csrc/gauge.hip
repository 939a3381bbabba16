// Gauge-field layout: canonical complex128 [4][V][3][3] links -> per-parity, per-precision
// site-major planes of the 16 matrices every site needs (8-way storage: forward links and
// minus the adjoints of the backward links, Sec. 3), and the 12-real Naik storage.
#include <cmath>
#include <complex>
#include <vector>

#include "ks_device.h"
#include "ks_naik.h"

namespace ks {

namespace {

// One thread per output site h of parity `par`: writes the 8 fat and 8 Naik matrices.
__global__ __launch_bounds__(kBlock) void layout_f64_kernel(Geom g, int par,
                                                            const double2* __restrict__ fat,
                                                            const double2* __restrict__ naik,
                                                            double2* __restrict__ fat_out,
                                                            double2* __restrict__ naik_out)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= g.Vh) return;
    int c[4];
    cb_coords(g, h, par, c);
    const int i = site_index(g, c);
    const size_t V = (size_t)g.V;
    for (int s = 0; s < 8; ++s) {
        const int mu = s & 3;
        const bool bwd = s >= 4;
        for (int which = 0; which < 2; ++which) {
            const int hops = which ? 3 : 1;
            const double2* src = which ? naik : fat;
            double2* dst = which ? naik_out : fat_out;
            int j = i;
            if (bwd) {
                int cm = c[mu] - hops;
                j = i - hops * g.stride[mu];
                if (cm < 0) j += g.n[mu] * g.stride[mu];
            }
            const double2* L = src + ((size_t)mu * V + (size_t)j) * 9;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double2 v;
                    if (!bwd) {
                        v = L[a * 3 + b];
                    } else {
                        const double2 t = L[b * 3 + a];
                        v = make_double2(-t.x, t.y);   // -(conj of the transpose)
                    }
                    dst[(size_t)(s * 9 + a * 3 + b) * g.lp + h] = v;
                }
        }
    }
}

// FP64 planes [8 slots][N][lp] -> packed planes of precision P (value * scale), pitch lp.
template <int P, int N>
__global__ __launch_bounds__(kBlock) void pack_kernel(const double2* __restrict__ src,
                                                      char* __restrict__ dst, int vh, int lp,
                                                      double scale)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= vh) return;
    using LP = LinkPack<P, N>;
    for (int slot = 0; slot < 8; ++slot)
        for (int e = 0; e < N; ++e) {
            const double2 v = src[(size_t)(slot * N + e) * lp + h];
            char* d = dst + LP::offset(slot, e, lp, h);
            if constexpr (P == KS_F64)
                *reinterpret_cast<double2*>(d) = make_double2(v.x * scale, v.y * scale);
            else if constexpr (P == KS_F32)
                *reinterpret_cast<float2*>(d) = make_float2((float)(v.x * scale), (float)(v.y * scale));
            else
                *reinterpret_cast<unsigned*>(d) = pack_half2_from_double(v.x * scale, v.y * scale);
        }
}

template <int N>
void pack(ks_prec_t p, const double2* src, void* dst, const Geom& g, double scale, hipStream_t s)
{
    const int nb = blocks_for(g.Vh);
    char* d = static_cast<char*>(dst);
    if (p == KS_F64) pack_kernel<KS_F64, N><<<nb, kBlock, 0, s>>>(src, d, g.Vh, g.lp, scale);
    else if (p == KS_F32) pack_kernel<KS_F32, N><<<nb, kBlock, 0, s>>>(src, d, g.Vh, g.lp, scale);
    else pack_kernel<KS_F16, N><<<nb, kBlock, 0, s>>>(src, d, g.Vh, g.lp, scale);
    KS_HIP(hipGetLastError());
}

__global__ __launch_bounds__(kBlock) void absmax_kernel(const double* __restrict__ in, size_t n,
                                                        double* __restrict__ partials)
{
    double m = 0.0;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
         k += (size_t)gridDim.x * blockDim.x)
        m = fmax(m, fabs(in[k]));
    m = block_max<kBlock>(m);
    if (threadIdx.x == 0) partials[blockIdx.x] = m;
}

// Minimal complex arithmetic for the 12-real builder.
struct zd {
    double r, i;
};
__device__ __forceinline__ zd zmul(zd a, zd b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ zd zsub(zd a, zd b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ zd zadd(zd a, zd b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ zd zconj(zd a) { return {a.r, -a.i}; }
__device__ __forceinline__ double zabs(zd a) { return sqrt(a.r * a.r + a.i * a.i); }

// 12-real Naik store from the FP64 Naik planes: rows 0 and 1 of U = L / s, s the scale of
// the slot at the site; per-block maximum of the SU(3) defect |U U^+ - 1|, |det U - 1|.
__global__ __launch_bounds__(kBlock) void recon12_kernel(Geom g, int par,
                                                         const double2* __restrict__ naik,
                                                         double2* __restrict__ out, double c0,
                                                         double* __restrict__ partials)
{
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    double defect = 0.0;
    if (h < g.Vh) {
        int c[4];
        cb_coords(g, h, par, c);
        for (int s = 0; s < 8; ++s) {
            const double sc = c0 * naik_sign(c, s, g.n[3]);
            zd u[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    const double2 v = naik[(size_t)(s * 9 + a * 3 + b) * g.lp + h];
                    u[a][b] = {v.x / sc, v.y / sc};
                }
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    zd d = {(a == b) ? -1.0 : 0.0, 0.0};
                    for (int k = 0; k < 3; ++k) d = zadd(d, zmul(u[a][k], zconj(u[b][k])));
                    defect = fmax(defect, zabs(d));
                }
            const zd det = zadd(zsub(zmul(u[0][0], zsub(zmul(u[1][1], u[2][2]), zmul(u[1][2], u[2][1]))),
                                     zmul(u[0][1], zsub(zmul(u[1][0], u[2][2]), zmul(u[1][2], u[2][0])))),
                                zmul(u[0][2], zsub(zmul(u[1][0], u[2][1]), zmul(u[1][1], u[2][0]))));
            defect = fmax(defect, zabs(zsub(det, zd{1.0, 0.0})));
            for (int e = 0; e < 6; ++e) {
                const zd v = u[e / 3][e % 3];
                out[(size_t)(s * 6 + e) * g.lp + h] = make_double2(v.r, v.i);
            }
        }
    }
    defect = block_max<kBlock>(defect);
    if (threadIdx.x == 0) partials[blockIdx.x] = defect;
}

double device_absmax(const double* data, size_t n, hipStream_t s)
{
    const int nb = 4096;
    double* part = static_cast<double*>(device_alloc(sizeof(double) * (nb + 1)));
    double host = 0.0;
    try {
        absmax_kernel<<<nb, kBlock, 0, s>>>(data, n, part);
        KS_HIP(hipGetLastError());
        reduce_max(part, nb, part + nb, s);
        KS_HIP(hipMemcpyAsync(&host, part + nb, sizeof(double), hipMemcpyDeviceToHost, s));
        KS_HIP(hipStreamSynchronize(s));
    } catch (...) {
        device_free(part);
        throw;
    }
    device_free(part);
    return host;
}

}  // namespace

size_t entry_bytes(ks_prec_t prec)
{
    return prec == KS_F64 ? 16 : prec == KS_F32 ? 8 : 4;
}

int recon_index(ks_recon_t r) { return r == KS_RECON_12 ? 1 : 0; }

void gauge_build_f64(ks_gauge_t g, const double* fat_dev, const double* naik_dev, hipStream_t s)
{
    LinkStore& st = g->store[KS_F64][0];
    const size_t plane = (size_t)72 * g->geom.lp * 16;   // 8 slots x 9 entries x lp x 16 B
    for (int par = 0; par < 2; ++par) {
        st.fat[par] = device_alloc_zero(plane, s);
        st.naik[par] = device_alloc_zero(plane, s);
        st.bytes += 2 * plane;
    }
    for (int par = 0; par < 2; ++par) {
        layout_f64_kernel<<<blocks_for(g->geom.Vh), kBlock, 0, s>>>(
            g->geom, par, reinterpret_cast<const double2*>(fat_dev),
            reinterpret_cast<const double2*>(naik_dev), static_cast<double2*>(st.fat[par]),
            static_cast<double2*>(st.naik[par]));
        KS_HIP(hipGetLastError());
    }
    KS_HIP(hipStreamSynchronize(s));
    st.ready = true;
}

static double frexp_scale(double m)
{
    if (m <= 0.0) return 1.0;
    int e = 0;
    std::frexp(m, &e);
    return std::ldexp(1.0, -e);
}

void gauge_prepare(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon, hipStream_t s)
{
    KS_REQUIRE(prec == KS_F64 || prec == KS_F32 || prec == KS_F16, KS_ERR_ARG, "bad precision %d",
               (int)prec);
    KS_REQUIRE(recon == KS_RECON_18 || recon == KS_RECON_12, KS_ERR_ARG, "bad recon %d",
               (int)recon);
    const int ri = recon_index(recon);
    LinkStore& st = g->store[prec][ri];
    if (st.ready) return;
    const LinkStore& m = g->store[KS_F64][0];
    const Geom& G = g->geom;
    const size_t n18 = (size_t)72 * G.lp;   // complex entries per parity and class

    // fat planes: shared between the 18- and 12-real stores of one precision
    LinkStore& base = g->store[prec][0];
    if (!base.fat[0]) {
        double fs = 1.0;
        if (prec == KS_F16) {
            double mx = 0.0;
            for (int par = 0; par < 2; ++par)
                mx = fmax(mx, device_absmax(static_cast<const double*>(m.fat[par]), 2 * n18, s));
            fs = frexp_scale(mx);
        }
        for (int par = 0; par < 2; ++par) {
            base.fat[par] = device_alloc_zero(n18 * entry_bytes(prec), s);
            base.bytes += n18 * entry_bytes(prec);
            pack<9>(prec, static_cast<const double2*>(m.fat[par]), base.fat[par], G, fs, s);
        }
        base.fat_scale = (float)(1.0 / fs);
    }
    if (ri == 1) {
        st.fat[0] = base.fat[0];
        st.fat[1] = base.fat[1];
        st.fat_scale = base.fat_scale;
    }

    if (ri == 0) {
        double ns = 1.0;
        if (prec == KS_F16) {
            double mx = 0.0;
            for (int par = 0; par < 2; ++par)
                mx = fmax(mx, device_absmax(static_cast<const double*>(m.naik[par]), 2 * n18, s));
            ns = frexp_scale(mx);
        }
        for (int par = 0; par < 2; ++par) {
            if (prec == KS_F64) {
                st.naik[par] = m.naik[par];
                continue;
            }
            st.naik[par] = device_alloc_zero(n18 * entry_bytes(prec), s);
            st.bytes += n18 * entry_bytes(prec);
            pack<9>(prec, static_cast<const double2*>(m.naik[par]), st.naik[par], G, ns, s);
        }
        st.naik_scale = (float)(1.0 / ns);
    } else {
        // the real scale c: cube root of det W_0 at the origin (phase +1 there)
        if (g->naik_c0 == 0.0) {
            double2 w[9];
            for (int k = 0; k < 9; ++k)
                KS_HIP(hipMemcpyAsync(&w[k], static_cast<const double2*>(m.naik[0]) + (size_t)k * G.lp,
                                      sizeof(double2), hipMemcpyDeviceToHost, s));
            KS_HIP(hipStreamSynchronize(s));
            std::complex<double> u[3][3];
            for (int k = 0; k < 9; ++k) u[k / 3][k % 3] = std::complex<double>(w[k].x, w[k].y);
            const std::complex<double> det =
                u[0][0] * (u[1][1] * u[2][2] - u[1][2] * u[2][1]) -
                u[0][1] * (u[1][0] * u[2][2] - u[1][2] * u[2][0]) +
                u[0][2] * (u[1][0] * u[2][1] - u[1][1] * u[2][0]);
            KS_REQUIRE(std::abs(det.imag()) <= 1e-10 * std::abs(det) && det.real() != 0.0,
                       KS_ERR_NOT_SU3, "12-real Naik storage: det W at the origin is not real");
            g->naik_c0 = std::cbrt(det.real());
        }
        const size_t n12 = (size_t)48 * G.lp;
        const int nb = blocks_for(G.Vh);
        double* part = static_cast<double*>(device_alloc(sizeof(double) * (nb + 1)));
        double defect[2] = {0, 0};
        void* outs[2] = {nullptr, nullptr};
        double2* tmp = nullptr;
        try {
            if (prec != KS_F64) tmp = static_cast<double2*>(device_alloc_zero(n12 * 16, s));
            for (int par = 0; par < 2; ++par) {
                outs[par] = device_alloc_zero(n12 * entry_bytes(prec), s);
                const double2* src = static_cast<const double2*>(m.naik[par]);
                double2* u = (prec == KS_F64) ? static_cast<double2*>(outs[par]) : tmp;
                recon12_kernel<<<nb, kBlock, 0, s>>>(G, par, src, u, g->naik_c0, part);
                KS_HIP(hipGetLastError());
                if (prec != KS_F64) pack<6>(prec, tmp, outs[par], G, 1.0, s);
                reduce_max(part, nb, part + nb, s);
                KS_HIP(hipMemcpyAsync(&defect[par], part + nb, sizeof(double),
                                      hipMemcpyDeviceToHost, s));
                KS_HIP(hipStreamSynchronize(s));
            }
        } catch (...) {
            device_free(part);
            device_free(tmp);
            device_free(outs[0]);
            device_free(outs[1]);
            throw;
        }
        device_free(part);
        device_free(tmp);
        if (!(defect[0] <= 1e-10 && defect[1] <= 1e-10)) {
            device_free(outs[0]);
            device_free(outs[1]);
            KS_REQUIRE(false, KS_ERR_NOT_SU3,
                       "12-real Naik storage: links are not c * phase * SU(3) (defect %.3g)",
                       fmax(defect[0], defect[1]));
        }
        st.naik[0] = outs[0];
        st.naik[1] = outs[1];
        st.bytes += 2 * n12 * entry_bytes(prec);
        st.naik_scale = 1.f;
    }
    KS_HIP(hipStreamSynchronize(s));
    st.ready = true;
}

void gauge_release(ks_gauge_t g)
{
    // fat planes of a 12-real store alias the 18-real store's; the FP64 18-real Naik
    // planes are shared between [F64][0] and the master
    for (int p = 0; p < 3; ++p) {
        LinkStore& s18 = g->store[p][0];
        LinkStore& s12 = g->store[p][1];
        for (int par = 0; par < 2; ++par) {
            device_free(s12.naik[par]);
            device_free(s18.fat[par]);
            device_free(s18.naik[par]);
        }
        s18 = LinkStore();
        s12 = LinkStore();
    }
}

}  // namespace ks
