// Fat and Naik links built from thin links on the device: a two-level smearing with a unitary
// projection in between (the HISQ construction that produces the links the solver of Sec. 3
// reads).  All fields are FP64 in the link layout of ks_gauge_load, [4][V][3][3] complex with
// lexicographic sites.
//
// Staple of a field M on mu-links in the signed transverse direction (nu, s):
//     S[M](x) = L(x) M(x + s nu) L(x + mu)^+,   L(y) = U_nu(y) (s = +1), U_nu(y - nu)^+ (s = -1).
// A smearing with coefficients (c1, c3, c5, c7, cL) is
//     F_mu = c1 U + cL sum_a S_a[S_a[U]] + sum_a S_a[ c3 U + sum_b S_b[ c5 U + c7 sum_c S_c[U] ] ]
// over signed transverse directions on distinct axes (6 three-link, 24 five-link, 48
// seven-link staples, 6 double-width Lepage staples; the nesting follows from linearity of the
// staple in M).  Per mu: the six three-link staples S_c[U] by `staple_kernel`, then one
// `fat_term_kernel` pass per outer direction a that builds the whole middle field of S_a at
// x + s_a a in registers (its four five-link staples with their seven-link middles, and the
// Lepage term, which shares the outer links).
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "ks_device.h"

namespace ks {

namespace {

using cxd = cx<double>;

struct Mat {
    cxd e[9];
};

__device__ __forceinline__ Mat load_mat(const double2* f, long site)
{
    Mat m;
    const double2* p = f + site * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) m.e[k] = {p[k].x, p[k].y};
    return m;
}

__device__ __forceinline__ void store_mat(double2* f, long site, const Mat& m)
{
    double2* p = f + site * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) p[k] = make_double2(m.e[k].r, m.e[k].i);
}

__device__ __forceinline__ Mat mul(const Mat& a, const Mat& b)
{
    Mat c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cxd s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cfma(s, a.e[i * 3 + k], b.e[k * 3 + j]);
            c.e[i * 3 + j] = s;
        }
    return c;
}

// a b^+
__device__ __forceinline__ Mat mul_adj(const Mat& a, const Mat& b)
{
    Mat c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cxd s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const cxd x = a.e[i * 3 + k], y = b.e[j * 3 + k];
                s.r = fma(x.r, y.r, fma(x.i, y.i, s.r));
                s.i = fma(x.i, y.r, fma(-x.r, y.i, s.i));
            }
            c.e[i * 3 + j] = s;
        }
    return c;
}

__device__ __forceinline__ Mat adj(const Mat& a)
{
    Mat c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) c.e[i * 3 + j] = {a.e[j * 3 + i].r, -a.e[j * 3 + i].i};
    return c;
}

__device__ __forceinline__ void site_coords(const Geom& g, long x, int c[4])
{
    long r = x;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c[d] = (int)(r % g.n[d]);
        r /= g.n[d];
    }
    c[3] = (int)r;
}

// lexicographic index of x + k mu (|k| < n[mu], one wrap at most)
__device__ __forceinline__ long hop_lex(const Geom& g, long x, const int c[4], int mu, int k)
{
    int cm = c[mu] + k;
    long j = x + (long)k * g.stride[mu];
    if (cm >= g.n[mu]) j -= (long)g.n[mu] * g.stride[mu];
    else if (cm < 0) j += (long)g.n[mu] * g.stride[mu];
    return j;
}

struct Middle {
    const double2* f[3];
    double w[3];
    int n;
};

// out(x) = (acc ? out(x) : 0) + coef L(x) M(x + s nu) L(x + mu)^+, M = sum_k w_k f_k
__global__ __launch_bounds__(kBlock) void staple_kernel(Geom g, const double2* __restrict__ U,
                                                        int mu, int nu, int s, Middle mid,
                                                        double coef, int acc,
                                                        double2* __restrict__ out)
{
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.V) return;
    int c[4];
    site_coords(g, x, c);
    const long vol = g.V;
    const double2* Unu = U + (long)nu * vol * 9;
    const long xn = hop_lex(g, x, c, nu, s);          // x + s nu
    const long xm = hop_lex(g, x, c, mu, 1);          // x + mu
    Mat L0, L1;
    if (s > 0) {
        L0 = load_mat(Unu, x);
        L1 = load_mat(Unu, xm);
    } else {
        int cm[4] = {c[0], c[1], c[2], c[3]};
        cm[mu] = (c[mu] + 1) % g.n[mu];
        L0 = adj(load_mat(Unu, xn));
        L1 = adj(load_mat(Unu, hop_lex(g, xm, cm, nu, -1)));
    }
    Mat M;
#pragma unroll
    for (int k = 0; k < 9; ++k) M.e[k] = {0.0, 0.0};
    for (int q = 0; q < mid.n; ++q) {
        const Mat f = load_mat(mid.f[q], xn);
        const double w = mid.w[q];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            M.e[k].r = fma(w, f.e[k].r, M.e[k].r);
            M.e[k].i = fma(w, f.e[k].i, M.e[k].i);
        }
    }
    const Mat r = mul_adj(mul(L0, M), L1);
    Mat o;
    if (acc) o = load_mat(out, x);
    else
#pragma unroll
        for (int k = 0; k < 9; ++k) o.e[k] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        o.e[k].r = fma(coef, r.e[k].r, o.e[k].r);
        o.e[k].i = fma(coef, r.e[k].i, o.e[k].i);
    }
    store_mat(out, x, o);
}

// One outer term of the smearing for every x, all its inner terms fused:
//   F(x) (+)= S_a[ c3 U + cL S_a[U] + sum_b S_b[ c5 U + c7 sum_c S_c[U] ] ](x)
// (F(x) = c1 U(x) + ... when `first`).  The outer staple reads its middle field at
// y = x + s_a a only, so each x builds that field at y in registers: the inner sum is never
// stored, and the Lepage term shares the outer staple's links.  b runs over the four signed
// directions off mu and a's axis, c over the two on the remaining axis (precomputed
// three-link staples S_c[U], in s1).
struct FatTerm {
    const double2* s1[6];   // S_d[U_mu] for the six signed directions off mu
    int mu, anu, as, aidx;
    int bnu[4], bs[4], cidx[4][2];
    double c1, c3, c5, c7, cl;
    int first;
};

__device__ __forceinline__ void axpy_mat(Mat& acc, double w, const Mat& m)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        acc.e[k].r = fma(w, m.e[k].r, acc.e[k].r);
        acc.e[k].i = fma(w, m.e[k].i, acc.e[k].i);
    }
}

__global__ __launch_bounds__(kBlock) void fat_term_kernel(Geom g, const double2* __restrict__ U,
                                                          FatTerm t, double2* __restrict__ F)
{
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.V) return;
    const long vol = g.V;
    const int mu = t.mu;
    const double2* Umu = U + (long)mu * vol * 9;
    int c[4];
    site_coords(g, x, c);
    // y = x + s_a a and its coordinates; y + mu
    const long y = hop_lex(g, x, c, t.anu, t.as);
    int cy[4] = {c[0], c[1], c[2], c[3]};
    cy[t.anu] = (c[t.anu] + t.as + g.n[t.anu]) % g.n[t.anu];
    const long ym = hop_lex(g, y, cy, mu, 1);
    int cym[4] = {cy[0], cy[1], cy[2], cy[3]};
    cym[mu] = (cy[mu] + 1) % g.n[mu];
    Mat inner;
#pragma unroll
    for (int k = 0; k < 9; ++k) inner.e[k] = {0.0, 0.0};
    axpy_mat(inner, t.c3, load_mat(Umu, y));
    if (t.cl != 0.0) axpy_mat(inner, t.cl, load_mat(t.s1[t.aidx], y));
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
        const int bn = t.bnu[k], bsg = t.bs[k];
        const double2* Ub = U + (long)bn * vol * 9;
        const long z = hop_lex(g, y, cy, bn, bsg);   // y + s_b b
        Mat M;
#pragma unroll
        for (int e = 0; e < 9; ++e) M.e[e] = {0.0, 0.0};
        axpy_mat(M, t.c5, load_mat(Umu, z));
        if (t.c7 != 0.0) {
            axpy_mat(M, t.c7, load_mat(t.s1[t.cidx[k][0]], z));
            axpy_mat(M, t.c7, load_mat(t.s1[t.cidx[k][1]], z));
        }
        Mat B0, B1;
        if (bsg > 0) {
            B0 = load_mat(Ub, y);
            B1 = load_mat(Ub, ym);
        } else {
            B0 = adj(load_mat(Ub, z));
            B1 = adj(load_mat(Ub, hop_lex(g, ym, cym, bn, -1)));
        }
        const Mat r = mul_adj(mul(B0, M), B1);
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            inner.e[e].r += r.e[e].r;
            inner.e[e].i += r.e[e].i;
        }
    }
    // outer staple at x in direction a
    const double2* Ua = U + (long)t.anu * vol * 9;
    const long xm = hop_lex(g, x, c, mu, 1);
    Mat L0, L1;
    if (t.as > 0) {
        L0 = load_mat(Ua, x);
        L1 = load_mat(Ua, xm);
    } else {
        int cm[4] = {c[0], c[1], c[2], c[3]};
        cm[mu] = (c[mu] + 1) % g.n[mu];
        L0 = adj(load_mat(Ua, y));
        L1 = adj(load_mat(Ua, hop_lex(g, xm, cm, t.anu, -1)));
    }
    const Mat r = mul_adj(mul(L0, inner), L1);
    Mat o;
    if (t.first) {
#pragma unroll
        for (int e = 0; e < 9; ++e) o.e[e] = {0.0, 0.0};
        axpy_mat(o, t.c1, load_mat(Umu, x));
    } else {
        o = load_mat(F, x);
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        o.e[e].r += r.e[e].r;
        o.e[e].i += r.e[e].i;
    }
    store_mat(F, x, o);
}

// W = V (V^+ V)^(-1/2) by the scaled Newton iteration for the polar factor,
// X <- (g X + (g X)^-+ ) / 2 with g = |det X|^(-1/3), at most kPolarIters steps; a singular or
// non-finite V sets *bad.
constexpr int kPolarIters = 40;

__device__ __forceinline__ cxd cdiv(cxd a, cxd b)
{
    const double d = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}

__global__ __launch_bounds__(kBlock) void u3_project_kernel(long n, const double2* __restrict__ V,
                                                            double2* __restrict__ W,
                                                            int* __restrict__ bad)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Mat X = load_mat(V, i);
    bool ok = true;
    for (int it = 0; it < kPolarIters; ++it) {
        // cofactors: (X^-1)^+ = conj(cof(X)) / conj(det X), cof the cofactor matrix
        Mat cf;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int a1 = (a + 1) % 3, a2 = (a + 2) % 3, b1 = (b + 1) % 3, b2 = (b + 2) % 3;
                cxd t = cmul(X.e[a1 * 3 + b1], X.e[a2 * 3 + b2]);
                const cxd u = cmul(X.e[a1 * 3 + b2], X.e[a2 * 3 + b1]);
                cf.e[a * 3 + b] = {t.r - u.r, t.i - u.i};
            }
        cxd det = {0.0, 0.0};
#pragma unroll
        for (int b = 0; b < 3; ++b) cfma(det, X.e[b], cf.e[b]);
        const double ad = sqrt(det.r * det.r + det.i * det.i);
        if (!(ad > 0.0) || !isfinite(ad)) {
            ok = false;
            break;
        }
        const double gam = it < 6 ? cbrt(1.0 / ad) : 1.0;
        const cxd dc = {det.r, -det.i};
        double diff = 0.0, nrm = 0.0;
        Mat Y;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            // (X^-1)^+ entry (a, b) = conj(cof(a, b)) / conj(det)
            const cxd inv = cdiv({cf.e[k].r, -cf.e[k].i}, dc);
            Y.e[k] = {0.5 * (gam * X.e[k].r + inv.r / gam), 0.5 * (gam * X.e[k].i + inv.i / gam)};
            const double dr = Y.e[k].r - X.e[k].r, di = Y.e[k].i - X.e[k].i;
            diff += dr * dr + di * di;
            nrm += Y.e[k].r * Y.e[k].r + Y.e[k].i * Y.e[k].i;
        }
        X = Y;
        if (it >= 6 && diff <= 1e-30 * nrm) break;
    }
    if (!ok) {
        *bad = 1;
#pragma unroll
        for (int k = 0; k < 9; ++k) X.e[k] = {0.0, 0.0};
    }
    store_mat(W, i, X);
}

// N_mu(x) = c W_mu(x) W_mu(x + mu) W_mu(x + 2 mu), all four directions
__global__ __launch_bounds__(kBlock) void naik_kernel(Geom g, const double2* __restrict__ W,
                                                      double c, double2* __restrict__ N)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4L * g.V) return;
    const int mu = (int)(t / g.V);
    const long x = t - (long)mu * g.V;
    int cc[4];
    site_coords(g, x, cc);
    const double2* Wm = W + (long)mu * g.V * 9;
    const long x1 = hop_lex(g, x, cc, mu, 1), x2 = hop_lex(g, x, cc, mu, 2);
    Mat r = mul(mul(load_mat(Wm, x), load_mat(Wm, x1)), load_mat(Wm, x2));
#pragma unroll
    for (int k = 0; k < 9; ++k) r.e[k] = {c * r.e[k].r, c * r.e[k].i};
    store_mat(N, t, r);
}

// staggered phases eta_mu(x) and the antiperiodic time sign (one-link: t = Nt-1; three-link:
// t >= Nt-3) multiplied into the fat and Naik links
__global__ __launch_bounds__(kBlock) void fold_signs_kernel(Geom g, double2* __restrict__ fat,
                                                            double2* __restrict__ naik)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4L * g.V) return;
    const int mu = (int)(t / g.V);
    const long x = t - (long)mu * g.V;
    int c[4];
    site_coords(g, x, c);
    int e = 0;
    if (mu >= 1) e += c[0];
    if (mu >= 2) e += c[1];
    if (mu >= 3) e += c[2];
    const double eta = (e & 1) ? -1.0 : 1.0;
    const double s1 = (mu == 3 && c[3] == g.n[3] - 1) ? -eta : eta;
    const double s3 = (mu == 3 && c[3] >= g.n[3] - 3) ? -eta : eta;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double2 a = fat[t * 9 + k], b = naik[t * 9 + k];
        fat[t * 9 + k] = make_double2(s1 * a.x, s1 * a.y);
        naik[t * 9 + k] = make_double2(s3 * b.x, s3 * b.y);
    }
}

struct Dir {
    int nu, s;
};

void staple(const Geom& G, const double2* U, int mu, Dir d, const Middle& m, double coef,
            bool acc, double2* out, hipStream_t st)
{
    staple_kernel<<<blocks_for(G.V), kBlock, 0, st>>>(G, U, mu, d.nu, d.s, m, coef, acc ? 1 : 0,
                                                       out);
    KS_HIP(hipGetLastError());
}

Middle one(const double2* f, double w)
{
    Middle m{};
    m.f[0] = f;
    m.w[0] = w;
    m.n = 1;
    return m;
}

// out[4][V] = F(U; c): per mu, the six three-link staples S_d[U_mu] into s1, then one fused
// launch per outer direction a (its inner five- and seven-link and Lepage terms included)
void smear(const Geom& G, const double2* U, const double* c, double2* out, double2* const* s1,
           hipStream_t st)
{
    const long vol = G.V;
    for (int mu = 0; mu < 4; ++mu) {
        const double2* Umu = U + (long)mu * vol * 9;
        double2* F = out + (long)mu * vol * 9;
        std::vector<Dir> dirs;
        for (int nu = 0; nu < 4; ++nu)
            if (nu != mu) {
                dirs.push_back({nu, +1});
                dirs.push_back({nu, -1});
            }
        for (int a = 0; a < 6; ++a) staple(G, U, mu, dirs[a], one(Umu, 1.0), 1.0, false, s1[a], st);
        for (int a = 0; a < 6; ++a) {
            FatTerm t{};
            for (int q = 0; q < 6; ++q) t.s1[q] = s1[q];
            t.mu = mu;
            t.anu = dirs[a].nu;
            t.as = dirs[a].s;
            t.aidx = a;
            int k = 0;
            for (int b = 0; b < 6; ++b) {
                if (dirs[b].nu == dirs[a].nu) continue;
                t.bnu[k] = dirs[b].nu;
                t.bs[k] = dirs[b].s;
                int n = 0;
                for (int q = 0; q < 6; ++q)
                    if (dirs[q].nu != dirs[a].nu && dirs[q].nu != dirs[b].nu) t.cidx[k][n++] = q;
                ++k;
            }
            t.c1 = c[0];
            t.c3 = c[1];
            t.c5 = c[2];
            t.c7 = c[3];
            t.cl = c[4];
            t.first = a == 0 ? 1 : 0;
            fat_term_kernel<<<blocks_for(vol), kBlock, 0, st>>>(G, U, t, F);
            KS_HIP(hipGetLastError());
        }
    }
}

}  // namespace

const double kHisqLevel1[5] = {1.0 / 8, 1.0 / 16, 1.0 / 64, 1.0 / 384, 0.0};
const double kHisqLevel2[5] = {1.0, 1.0 / 16, 1.0 / 64, 1.0 / 384, -1.0 / 8};
const double kHisqNaik = -1.0 / 24;

namespace {

// Scratch of the link construction (six staple fields, the level-1 links and their U(3)
// projection: 14 link fields), kept per device between calls and grown when a larger lattice
// comes, so that repeated calls allocate nothing.
struct HisqScratch {
    void* ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_hisq_mu;
std::map<int, HisqScratch> g_hisq;

char* hisq_scratch(size_t bytes)
{
    int dev = 0;
    KS_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_hisq_mu);
    HisqScratch& h = g_hisq[dev];
    if (h.bytes < bytes) {
        device_free(h.ptr);
        h.ptr = nullptr;
        h.bytes = 0;
        h.ptr = device_alloc(bytes);
        h.bytes = bytes;
    }
    return static_cast<char*>(h.ptr);
}

}  // namespace

void hisq_release()
{
    std::lock_guard<std::mutex> lk(g_hisq_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_hisq) {
        (void)hipSetDevice(kv.first);
        (void)hipDeviceSynchronize();
        device_free(kv.second.ptr);
    }
    (void)hipSetDevice(cur);
    g_hisq.clear();
}

void hisq_links(const Geom& G, const double* thin, double* fat, double* naik,
                const double* level1, const double* level2, double c_naik, hipStream_t st)
{
    const long vol = G.V;
    const size_t mat = (size_t)vol * 9 * sizeof(double2);
    char* base = hisq_scratch(14 * mat + 256);
    size_t used = 0;
    auto get = [&](size_t bytes) {
        double2* p = reinterpret_cast<double2*>(base + used);
        used += (bytes + 255) / 256 * 256;
        return p;
    };
    {
        double2* s1[6];
        for (auto& p : s1) p = get(mat);
        double2* V1 = get(4 * mat);
        double2* W = get(4 * mat);
        int* bad = reinterpret_cast<int*>(get(sizeof(double2)));
        const double2* U = reinterpret_cast<const double2*>(thin);
        smear(G, U, level1, V1, s1, st);
        KS_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
        u3_project_kernel<<<blocks_for(4 * vol), kBlock, 0, st>>>(4 * vol, V1, W, bad);
        KS_HIP(hipGetLastError());
        smear(G, W, level2, reinterpret_cast<double2*>(fat), s1, st);
        naik_kernel<<<blocks_for(4 * vol), kBlock, 0, st>>>(G, W, c_naik,
                                                             reinterpret_cast<double2*>(naik));
        KS_HIP(hipGetLastError());
        fold_signs_kernel<<<blocks_for(4 * vol), kBlock, 0, st>>>(
            G, reinterpret_cast<double2*>(fat), reinterpret_cast<double2*>(naik));
        KS_HIP(hipGetLastError());
        int hbad = 0;
        KS_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
        KS_HIP(hipStreamSynchronize(st));
        KS_REQUIRE(!hbad, KS_ERR_NONFINITE,
                   "link construction: a level-1 smeared link is singular or not finite");
    }
}

}  // namespace ks
