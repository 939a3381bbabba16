// C ABI of libks (declared in include/ks.h): argument checks, handle management, error
// reporting.  Every entry point catches the library's internal failures and returns a code.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "ks_common.h"
#include "ks_batch.h"
#include "ks_net.h"
#include "ks_solvers.h"

namespace ks {

namespace {
thread_local char g_err[512] = "";
}

const char* error_text() { return g_err; }

int log_level()
{
    static const int level = [] {
        const char* e = std::getenv("KS_LOG");
        return e ? std::atoi(e) : 0;
    }();
    return level;
}

void log_msg(int level, const char* fmt, ...)
{
    if (log_level() < level) return;
    char line[640];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(line, sizeof(line), fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[ks] %s\n", line);
}

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void* device_alloc(size_t bytes)
{
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, bytes ? bytes : 1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        throw Failure{KS_ERR_NOMEM};
    }
    return p;
}

void* device_alloc_zero(size_t bytes, hipStream_t s)
{
    void* p = device_alloc(bytes);
    const hipError_t e = hipMemsetAsync(p, 0, bytes ? bytes : 1, s);
    if (e != hipSuccess) {
        (void)hipFree(p);
        set_error("hipMemsetAsync of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        throw Failure{KS_ERR_HIP};
    }
    return p;
}

void device_free(void* p)
{
    if (p) (void)hipFree(p);
}

Geom make_geom(const int dims[4])
{
    Geom g;
    long v = 1;
    for (int mu = 0; mu < 4; ++mu) {
        g.n[mu] = dims[mu];
        g.stride[mu] = (int)v;
        v *= dims[mu];
    }
    g.V = (int)v;
    g.Vh = (int)(v / 2);
    g.lp = link_pitch(g.Vh);
    return g;
}

size_t field_bytes(const Geom& g, ks_prec_t prec)
{
    return (size_t)g.Vh * (prec == KS_F64 ? 48 : prec == KS_F32 ? 24 : 16);
}

}  // namespace ks

using namespace ks;

#define KS_API_BEGIN try {
#define KS_API_END                                                                      \
    }                                                                                   \
    catch (const Failure& f) {                                                          \
        log_msg(1, "%s: error %d: %s", __func__, (int)f.code, error_text());             \
        return f.code;                                                                  \
    }                                                                                   \
    catch (const std::bad_alloc&) {                                                     \
        set_error("host memory exhausted");                                             \
        return KS_ERR_NOMEM;                                                            \
    }                                                                                   \
    catch (...) {                                                                       \
        set_error("unexpected C++ exception");                                          \
        return KS_ERR_HIP;                                                              \
    }

static_assert(kNetWeights == KS_NET_WEIGHTS, "network weight count of the ABI");

static void log_solve(const char* what, ks_status_t rc, const ks_solver_stats& s)
{
    log_msg(1, "%s: status %d, %d steps, %d reliable updates, true residual %.3g, %.4f s, "
               "%.1f GB/s model", what, (int)rc, s.iters, s.reliable_updates, s.true_rel_resid,
            s.seconds, s.seconds > 0 ? s.model_bytes / s.seconds / 1e9 : 0.0);
}

static bool prec_ok(int p) { return p == KS_F64 || p == KS_F32 || p == KS_F16; }
static bool recon_ok(int r) { return r == KS_RECON_18 || r == KS_RECON_12; }

extern "C" {

void ks_default_params(ks_solver_params* p)
{
    if (!p) return;
    p->tol = 1e-10;
    p->max_iter = 100000;
    p->inner = KS_F64;
    p->recon = KS_RECON_18;
    p->delta = 0.1;
    p->check_every = 16;
    p->max_restarts = 5;
}

const char* ks_last_error(void) { return error_text(); }

ks_status_t ks_gauge_load(ks_gauge_t* out, const int dims[4], const double* fat,
                          const double* naik, int on_device, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(out && dims && fat && naik, KS_ERR_ARG, "ks_gauge_load: null argument");
    *out = nullptr;
    long v = 1;
    for (int mu = 0; mu < 4; ++mu) {
        KS_REQUIRE(dims[mu] >= 4 && dims[mu] % 2 == 0, KS_ERR_ARG,
                   "ks_gauge_load: extent %d of direction %d must be even and >= 4", dims[mu], mu);
        v *= dims[mu];
    }
    KS_REQUIRE(v <= (1L << 29), KS_ERR_ARG, "ks_gauge_load: volume %ld too large", v);
    ks_gauge_s* g = new ks_gauge_s();
    g->geom = make_geom(dims);
    const size_t bytes = (size_t)4 * v * 9 * 16;
    double* tmp_fat = nullptr;
    double* tmp_naik = nullptr;
    try {
        const double* df = fat;
        const double* dn = naik;
        if (!on_device) {
            tmp_fat = static_cast<double*>(device_alloc(bytes));
            tmp_naik = static_cast<double*>(device_alloc(bytes));
            KS_HIP(hipMemcpyAsync(tmp_fat, fat, bytes, hipMemcpyHostToDevice, stream));
            KS_HIP(hipMemcpyAsync(tmp_naik, naik, bytes, hipMemcpyHostToDevice, stream));
            df = tmp_fat;
            dn = tmp_naik;
        }
        gauge_build_f64(g, df, dn, stream);
    } catch (...) {
        device_free(tmp_fat);
        device_free(tmp_naik);
        gauge_release(g);
        delete g;
        throw;
    }
    device_free(tmp_fat);
    device_free(tmp_naik);
    *out = g;
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_gauge_prepare(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(g, KS_ERR_ARG, "ks_gauge_prepare: null handle");
    KS_REQUIRE(prec_ok(prec) && recon_ok(recon), KS_ERR_ARG, "ks_gauge_prepare: bad precision/recon");
    gauge_prepare(g, prec, recon, stream);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_gauge_free(ks_gauge_t g)
{
    KS_API_BEGIN
    if (!g) return KS_SUCCESS;
    (void)hipDeviceSynchronize();
    fcg_release(g);
    workspace_free(g->ws);
    g->ws = nullptr;
    gauge_release(g);
    delete g;
    return KS_SUCCESS;
    KS_API_END
}

size_t ks_gauge_device_bytes(ks_gauge_t g)
{
    if (!g) return 0;
    size_t b = 0;
    for (int p = 0; p < 3; ++p)
        for (int r = 0; r < 2; ++r) b += g->store[p][r].bytes;
    if (g->ws) b += g->ws->bytes;
    return b;
}

ks_status_t ks_field_create(ks_field_t* f, ks_gauge_t g, ks_parity_t parity, ks_prec_t prec)
{
    KS_API_BEGIN
    KS_REQUIRE(f && g, KS_ERR_ARG, "ks_field_create: null argument");
    KS_REQUIRE(parity == KS_EVEN || parity == KS_ODD, KS_ERR_ARG, "ks_field_create: bad parity");
    KS_REQUIRE(prec_ok(prec), KS_ERR_ARG, "ks_field_create: bad precision");
    *f = nullptr;
    ks_field_s* h = new ks_field_s();
    h->g = g;
    h->parity = parity;
    h->prec = prec;
    h->bytes = field_bytes(g->geom, prec);
    try {
        h->data = device_alloc(h->bytes);
    } catch (...) {
        delete h;
        throw;
    }
    *f = h;
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_field_free(ks_field_t f)
{
    KS_API_BEGIN
    if (!f) return KS_SUCCESS;
    device_free(f->data);
    delete f;
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_field_import(ks_field_t f, const double* src_dev, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(f && src_dev, KS_ERR_ARG, "ks_field_import: null argument");
    import_field(f->g->geom, f->prec, src_dev, f->data, stream);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_field_export(ks_field_t f, double* dst_dev, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(f && dst_dev, KS_ERR_ARG, "ks_field_export: null argument");
    export_field(f->g->geom, f->prec, f->data, dst_dev, stream);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_dslash_eo(ks_gauge_t g, ks_field_t out, ks_field_t in, ks_recon_t recon,
                         hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(g && out && in, KS_ERR_ARG, "ks_dslash_eo: null argument");
    KS_REQUIRE(out != in && out->data != in->data, KS_ERR_ARG, "ks_dslash_eo: out aliases in");
    KS_REQUIRE(out->g == g && in->g == g, KS_ERR_ARG, "ks_dslash_eo: field of another lattice");
    KS_REQUIRE(out->parity != in->parity, KS_ERR_ARG, "ks_dslash_eo: parities must differ");
    KS_REQUIRE(out->prec == in->prec, KS_ERR_ARG, "ks_dslash_eo: precisions differ");
    KS_REQUIRE(recon_ok(recon), KS_ERR_ARG, "ks_dslash_eo: bad recon");
    DslashArgs a;
    a.out_parity = out->parity;
    a.in = in->data;
    a.out = out->data;
    dslash(g, out->prec, recon, a, stream);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_tune_dslash(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(g, KS_ERR_ARG, "ks_tune_dslash: null handle");
    KS_REQUIRE(prec_ok(prec) && recon_ok(recon), KS_ERR_ARG, "ks_tune_dslash: bad precision/recon");
    dslash_tune(g, prec, recon, stream);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_dslash_config(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon,
                             ks_dslash_launch* out)
{
    KS_API_BEGIN
    KS_REQUIRE(g && out, KS_ERR_ARG, "ks_dslash_config: null argument");
    KS_REQUIRE(prec_ok(prec) && recon_ok(recon), KS_ERR_ARG, "ks_dslash_config: bad precision/recon");
    const TuneEntry& t = g->tune[prec][recon_index(recon)];
    out->threads = t.nt;
    out->lds_bytes = t.lds;
    out->links_per_pass = t.group;
    out->link_access = t.way;
    out->staged = t.staged;
    out->tuned_us = t.tuned ? t.us : 0.f;
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_dslash_set_config(ks_gauge_t g, ks_prec_t prec, ks_recon_t recon,
                                 const ks_dslash_launch* cfg)
{
    KS_API_BEGIN
    KS_REQUIRE(g && cfg, KS_ERR_ARG, "ks_dslash_set_config: null argument");
    KS_REQUIRE(prec_ok(prec) && recon_ok(recon), KS_ERR_ARG,
               "ks_dslash_set_config: bad precision/recon");
    KS_REQUIRE(cfg->threads == 64 || cfg->threads == 128 || cfg->threads == 256, KS_ERR_ARG,
               "ks_dslash_set_config: threads must be 64, 128 or 256");
    int dev = 0, lds_max = 0;
    KS_HIP(hipGetDevice(&dev));
    KS_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    KS_REQUIRE(cfg->lds_bytes >= 0 && cfg->lds_bytes <= lds_max, KS_ERR_ARG,
               "ks_dslash_set_config: lds_bytes must lie in [0, %d]", lds_max);
    KS_REQUIRE(cfg->link_access == 8 || cfg->link_access == 4, KS_ERR_ARG,
               "ks_dslash_set_config: link_access must be 8 or 4");
    KS_REQUIRE(cfg->staged == 0 || cfg->staged == 1, KS_ERR_ARG,
               "ks_dslash_set_config: staged must be 0 or 1");
    KS_REQUIRE(dslash_form_built(prec, recon, cfg->links_per_pass, cfg->link_access, cfg->staged),
               KS_ERR_ARG, "ks_dslash_set_config: %d links per pass with %d-way access%s is "
               "not built for this variant", cfg->links_per_pass, cfg->link_access,
               cfg->staged ? " and staged gathers" : "");
    TuneEntry t;
    t.nt = cfg->threads;
    t.lds = cfg->lds_bytes;
    t.group = cfg->links_per_pass;
    t.way = cfg->link_access;
    t.staged = cfg->staged;
    g->tune[prec][recon_index(recon)] = t;
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_apply_A(ks_gauge_t g, double sigma, const double* in_dev, double* out_dev,
                       hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(g && in_dev && out_dev, KS_ERR_ARG, "ks_apply_A: null argument");
    KS_REQUIRE(in_dev != out_dev, KS_ERR_ARG, "ks_apply_A: out aliases in");
    Workspace& w = workspace(g);
    import_field(g->geom, KS_F64, in_dev, w.b64, stream);
    apply_A64(g, sigma, static_cast<const double*>(w.b64), static_cast<double*>(w.ax64), stream,
              nullptr);
    export_field(g->geom, KS_F64, w.ax64, out_dev, stream);
    return KS_SUCCESS;
    KS_API_END
}

static void check_params(const ks_solver_params* p)
{
    KS_REQUIRE(p, KS_ERR_ARG, "solver: null params");
    KS_REQUIRE(p->tol > 0 && p->max_iter >= 1, KS_ERR_ARG, "solver: tol must be > 0, max_iter >= 1");
    KS_REQUIRE(prec_ok(p->inner) && recon_ok(p->recon), KS_ERR_ARG, "solver: bad inner precision/recon");
    KS_REQUIRE(p->delta >= 0 && p->delta < 1, KS_ERR_ARG, "solver: delta must be in [0, 1)");
}

ks_status_t ks_cg_solve(ks_gauge_t g, double mass, const double* b_dev, double* x_dev,
                        const ks_solver_params* p, ks_solver_stats* st, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(g && b_dev && x_dev, KS_ERR_ARG, "ks_cg_solve: null argument");
    KS_REQUIRE(b_dev != x_dev, KS_ERR_ARG, "ks_cg_solve: x aliases b");
    check_params(p);
    Workspace& w = workspace(g);
    import_field(g->geom, KS_F64, b_dev, w.b64, stream);
    import_field(g->geom, KS_F64, x_dev, w.x64, stream);
    ks_solver_stats local;
    const ks_status_t rc = cg_core(g, 4.0 * mass * mass, static_cast<const double*>(w.b64),
                                   static_cast<double*>(w.x64), *p, local, stream);
    export_field(g->geom, KS_F64, w.x64, x_dev, stream);
    KS_HIP(hipStreamSynchronize(stream));
    log_solve("cg", rc, local);
    if (st) *st = local;
    return rc;
    KS_API_END
}

ks_status_t ks_full_solve(ks_gauge_t g, double mass, const double* b_even, const double* b_odd,
                          double* x_even, double* x_odd, const ks_solver_params* p,
                          ks_solver_stats* st, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(g && b_even && b_odd && x_even && x_odd, KS_ERR_ARG, "ks_full_solve: null argument");
    KS_REQUIRE(mass > 0.0 && std::isfinite(mass), KS_ERR_ARG, "ks_full_solve: mass must be > 0");
    const void* ins[2] = {b_even, b_odd};
    const void* outs[2] = {x_even, x_odd};
    for (const void* i : ins)
        for (const void* o : outs)
            KS_REQUIRE(i != o, KS_ERR_ARG, "ks_full_solve: a solution aliases a source");
    KS_REQUIRE(x_even != x_odd && b_even != b_odd, KS_ERR_ARG, "ks_full_solve: aliased vectors");
    check_params(p);
    Workspace& w = workspace(g);
    const size_t fb = field_bytes(g->geom, KS_F64);
    for (double*& v : w.full)
        if (!v) {
            v = static_cast<double*>(device_alloc(fb));
            w.bytes += fb;
        }
    import_field(g->geom, KS_F64, b_even, w.b64, stream);
    import_field(g->geom, KS_F64, b_odd, w.full[3], stream);
    import_field(g->geom, KS_F64, x_even, w.x64, stream);
    ks_solver_stats local;
    const ks_status_t rc = full_solve_core(g, mass, w.b64, w.full[3], w.x64, w.full[4], *p, local,
                                           stream);
    export_field(g->geom, KS_F64, w.x64, x_even, stream);
    export_field(g->geom, KS_F64, w.full[4], x_odd, stream);
    KS_HIP(hipStreamSynchronize(stream));
    log_solve("full solve", rc, local);
    if (st) *st = local;
    return rc;
    KS_API_END
}

ks_status_t ks_force(ks_gauge_t g, int nterm, const double* residues, const double* const* x_even,
                     double* force_fat, double* force_naik, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(g && residues && x_even && force_fat && force_naik, KS_ERR_ARG,
               "ks_force: null argument");
    KS_REQUIRE(nterm >= 1 && nterm <= force_max_terms(), KS_ERR_ARG,
               "ks_force: nterm must lie in [1, %d]", force_max_terms());
    KS_REQUIRE(force_fat != force_naik, KS_ERR_ARG, "ks_force: the two outputs alias");
    for (int i = 0; i < nterm; ++i) {
        KS_REQUIRE(x_even[i], KS_ERR_ARG, "ks_force: null solution %d", i);
        KS_REQUIRE(std::isfinite(residues[i]), KS_ERR_ARG, "ks_force: residue %d not finite", i);
    }
    force_core(g, nterm, residues, x_even, force_fat, force_naik, stream);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_multishift_cg_solve(ks_gauge_t g, int nshift, const double* sigma,
                                   const double* b_dev, double* const* x_dev, const double* tol,
                                   const ks_solver_params* p, ks_solver_stats* st,
                                   hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(g && sigma && b_dev && x_dev && tol && st, KS_ERR_ARG,
               "ks_multishift_cg_solve: null argument");
    KS_REQUIRE(nshift >= 1 && nshift <= 32, KS_ERR_ARG, "ks_multishift_cg_solve: nshift in [1, 32]");
    check_params(p);
    for (int i = 0; i < nshift; ++i)
        KS_REQUIRE(x_dev[i] && x_dev[i] != b_dev, KS_ERR_ARG, "ks_multishift_cg_solve: bad x[%d]", i);
    Workspace& w = workspace(g);
    import_field(g->geom, KS_F64, b_dev, w.b64, stream);
    // solutions are kept in the library's FP64 planes, then exported into the caller's arrays
    std::vector<double*> xs(nshift);
    std::vector<void*>& keep = w.ms_x;
    while ((int)keep.size() < nshift) keep.push_back(device_alloc(field_bytes(g->geom, KS_F64)));
    for (int i = 0; i < nshift; ++i) xs[i] = static_cast<double*>(keep[i]);
    const ks_status_t rc = multishift_core(g, nshift, sigma, static_cast<const double*>(w.b64),
                                           xs.data(), tol, *p, st, stream);
    for (int i = 0; i < nshift; ++i) export_field(g->geom, KS_F64, xs[i], x_dev[i], stream);
    KS_HIP(hipStreamSynchronize(stream));
    for (int i = 0; i < nshift; ++i) log_solve("multishift shift", rc, st[i]);
    return rc;
    KS_API_END
}

ks_status_t ks_batch_create(ks_batch_t* out, int nlat, const int* dims, const double* const* fat,
                            const double* const* naik, int on_device, int nrhs, ks_prec_t inner,
                            hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(out && dims && fat && naik, KS_ERR_ARG, "ks_batch_create: null argument");
    *out = nullptr;
    BatchCtx* c = batch_create(nlat, dims, fat, naik, on_device, nrhs, inner, stream);
    *out = new ks_batch_s{c};
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_batch_solve(ks_batch_t b, const double* masses, const double* const* b_dev,
                           double* const* x_dev, const ks_solver_params* p, ks_batch_stats* st,
                           hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(b && b->ctx && masses && b_dev && x_dev && st, KS_ERR_ARG,
               "ks_batch_solve: null argument");
    check_params(p);
    const ks_status_t rc = batch_solve(*b->ctx, masses, b_dev, x_dev, *p, st, stream);
    if (log_level() >= 1) {
        int it = 0, worst = 0;
        double res = 0.0, sec = 0.0;
        for (int k = 0; k < b->ctx->npairs; ++k) {
            it = std::max(it, st[k].iters);
            res = std::max(res, st[k].true_rel_resid);
            sec = std::max(sec, st[k].seconds);
            if (st[k].status != 0 && worst == 0) worst = st[k].status;
        }
        log_msg(1, "batch: status %d, %d pairs, at most %d steps, largest residual %.3g, %.4f s",
                worst ? worst : (int)rc, b->ctx->npairs, it, res, sec);
    }
    return rc;
    KS_API_END
}

ks_status_t ks_batch_tune(ks_batch_t b, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(b && b->ctx, KS_ERR_ARG, "ks_batch_tune: null handle");
    batch_tune(*b->ctx, stream);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_batch_config(ks_batch_t b, int* tile_sites, int* persistent_blocks,
                            float* tuned_us, double* last_solve_seconds)
{
    KS_API_BEGIN
    KS_REQUIRE(b && b->ctx, KS_ERR_ARG, "ks_batch_config: null handle");
    const BatchCtx& c = *b->ctx;
    if (tile_sites) *tile_sites = 64 << c.tile_idx;
    if (persistent_blocks) *persistent_blocks = c.persistent;
    if (tuned_us) *tuned_us = c.tuned_us;
    if (last_solve_seconds) *last_solve_seconds = c.last_seconds;
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_net_create(ks_net_t* out, const double* weights)
{
    KS_API_BEGIN
    KS_REQUIRE(out && weights, KS_ERR_ARG, "ks_net_create: null argument");
    *out = nullptr;
    NetCtx* n = net_create(weights);
    *out = new ks_net_s{n};
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_net_set_weights(ks_net_t n, const double* weights)
{
    KS_API_BEGIN
    KS_REQUIRE(n && n->ctx && weights, KS_ERR_ARG, "ks_net_set_weights: null argument");
    net_set_weights(*n->ctx, weights, nullptr);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_net_get_weights(ks_net_t n, double* weights)
{
    KS_API_BEGIN
    KS_REQUIRE(n && n->ctx && weights, KS_ERR_ARG, "ks_net_get_weights: null argument");
    net_get_weights(*n->ctx, weights, nullptr);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_net_get_state(ks_net_t n, double* weights, double* adam_m, double* adam_v,
                             int* step)
{
    KS_API_BEGIN
    KS_REQUIRE(n && n->ctx && weights && adam_m && adam_v && step, KS_ERR_ARG,
               "ks_net_get_state: null argument");
    net_get_state(*n->ctx, weights, adam_m, adam_v, step, nullptr);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_net_set_state(ks_net_t n, const double* weights, const double* adam_m,
                             const double* adam_v, int step)
{
    KS_API_BEGIN
    KS_REQUIRE(n && n->ctx && weights && adam_m && adam_v, KS_ERR_ARG,
               "ks_net_set_state: null argument");
    KS_REQUIRE(step >= 0, KS_ERR_ARG, "ks_net_set_state: negative step count %d", step);
    for (int k = 0; k < 2 * KS_NET_WEIGHTS; ++k)
        KS_REQUIRE(std::isfinite(weights[k]) && std::isfinite(adam_m[k]) &&
                       std::isfinite(adam_v[k]) && adam_v[k] >= 0.0,
                   KS_ERR_ARG, "ks_net_set_state: entry %d is not finite (or a negative second moment)", k);
    net_set_state(*n->ctx, weights, adam_m, adam_v, step, nullptr);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_net_free(ks_net_t n)
{
    KS_API_BEGIN
    if (!n) return KS_SUCCESS;
    (void)hipDeviceSynchronize();
    net_free(n->ctx);
    delete n;
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_net_apply(ks_net_t n, ks_gauge_t g, const double* in_dev, double* out_dev,
                         int use_mfma, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(n && n->ctx && g && in_dev && out_dev, KS_ERR_ARG, "ks_net_apply: null argument");
    KS_REQUIRE(in_dev != out_dev, KS_ERR_ARG, "ks_net_apply: out aliases in");
    if (use_mfma) net_apply_mfma(*n->ctx, g, in_dev, out_dev, stream);
    else net_apply_f32(*n->ctx, g, in_dev, out_dev, 1.0, stream);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_net_apply_field(ks_net_t n, ks_field_t out, ks_field_t in, int use_mfma,
                               hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(n && n->ctx && out && in, KS_ERR_ARG, "ks_net_apply_field: null argument");
    KS_REQUIRE(out != in && out->data != in->data, KS_ERR_ARG,
               "ks_net_apply_field: out aliases in");
    KS_REQUIRE(out->g == in->g, KS_ERR_ARG, "ks_net_apply_field: fields of different lattices");
    KS_REQUIRE(out->parity == KS_EVEN && in->parity == KS_EVEN, KS_ERR_ARG,
               "ks_net_apply_field: the network maps even-parity fields");
    KS_REQUIRE(out->prec == in->prec && (in->prec == KS_F64 || in->prec == KS_F32), KS_ERR_ARG,
               "ks_net_apply_field: both fields KS_F64 or both KS_F32");
    net_apply_spinor(*n->ctx, in->g, in->prec, in->data, out->data, nullptr, nullptr, use_mfma,
                     stream);
    return KS_SUCCESS;
    KS_API_END
}

static void check_pairs(int npairs, const ks_gauge_t* gauges, const double* sigma,
                        const double* const* b, const double* const* x)
{
    KS_REQUIRE(npairs >= 1 && gauges && sigma && b && x, KS_ERR_ARG,
               "network: bad training pairs");
    for (int j = 0; j < npairs; ++j) {
        KS_REQUIRE(gauges[j] && b[j] && x[j], KS_ERR_ARG, "network: null entry in pair %d", j);
        KS_REQUIRE(std::isfinite(sigma[j]) && sigma[j] >= 0, KS_ERR_ARG,
                   "network: shift of pair %d must be finite and >= 0", j);
    }
}

ks_status_t ks_net_loss_grad(ks_net_t n, int npairs, const ks_gauge_t* gauges,
                             const double* sigma, const double* const* b_dev,
                             const double* const* x_dev, double* loss, double* grad,
                             hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(n && n->ctx, KS_ERR_ARG, "ks_net_loss_grad: null handle");
    check_pairs(npairs, gauges, sigma, b_dev, x_dev);
    const double l = net_loss_grad(*n->ctx, npairs, gauges, sigma, b_dev, x_dev, stream);
    if (loss) *loss = l;
    if (grad) {
        KS_HIP(hipMemcpyAsync(grad, n->ctx->grad, sizeof(double) * 2 * kNetWeights,
                              hipMemcpyDeviceToHost, stream));
        KS_HIP(hipStreamSynchronize(stream));
    }
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_net_train(ks_net_t n, int npairs, const ks_gauge_t* gauges, const double* sigma,
                         const double* const* b_dev, const double* const* x_dev, int steps,
                         int batch, double lr, double* loss_history, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(n && n->ctx, KS_ERR_ARG, "ks_net_train: null handle");
    check_pairs(npairs, gauges, sigma, b_dev, x_dev);
    KS_REQUIRE(steps >= 0 && batch >= 1 && lr > 0, KS_ERR_ARG, "ks_net_train: bad steps/batch/lr");
    batch = std::min(batch, npairs);
    std::vector<ks_gauge_t> gs(batch);
    std::vector<double> sg(batch);
    std::vector<const double*> bs(batch), xs(batch);
    for (int k = 0; k < steps; ++k) {
        for (int j = 0; j < batch; ++j) {
            const int q = (k * batch + j) % npairs;
            gs[j] = gauges[q];
            sg[j] = sigma[q];
            bs[j] = b_dev[q];
            xs[j] = x_dev[q];
        }
        const double l = net_loss_grad(*n->ctx, batch, gs.data(), sg.data(), bs.data(), xs.data(),
                                       stream);
        if (loss_history) loss_history[k] = l;
        net_adam(*n->ctx, lr, stream);
    }
    KS_HIP(hipStreamSynchronize(stream));
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_fcg_solve(ks_gauge_t g, ks_net_t n, double mass, const double* b_dev,
                         double* x_dev, const ks_solver_params* p, int use_mfma,
                         ks_solver_stats* st, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(g && n && n->ctx && b_dev && x_dev, KS_ERR_ARG, "ks_fcg_solve: null argument");
    KS_REQUIRE(b_dev != x_dev, KS_ERR_ARG, "ks_fcg_solve: x aliases b");
    check_params(p);
    Workspace& w = workspace(g);
    import_field(g->geom, KS_F64, b_dev, w.b64, stream);
    import_field(g->geom, KS_F64, x_dev, w.x64, stream);
    ks_solver_stats local;
    const ks_status_t rc = fcg_core(g, *n->ctx, 4.0 * mass * mass, w.b64, w.x64, *p, use_mfma,
                                    local, stream);
    export_field(g->geom, KS_F64, w.x64, x_dev, stream);
    KS_HIP(hipStreamSynchronize(stream));
    log_solve("fcg", rc, local);
    if (st) *st = local;
    return rc;
    KS_API_END
}

ks_status_t ks_hisq_links(const int dims[4], const double* thin_dev, double* fat_dev,
                          double* naik_dev, const double* level1, const double* level2,
                          double c_naik, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(dims && thin_dev && fat_dev && naik_dev, KS_ERR_ARG, "ks_hisq_links: null argument");
    long v = 1;
    for (int mu = 0; mu < 4; ++mu) {
        KS_REQUIRE(dims[mu] >= 4 && dims[mu] % 2 == 0, KS_ERR_ARG,
                   "ks_hisq_links: extent %d of direction %d must be even and >= 4", dims[mu], mu);
        v *= dims[mu];
    }
    KS_REQUIRE(v <= (1L << 29), KS_ERR_ARG, "ks_hisq_links: volume %ld too large", v);
    KS_REQUIRE(fat_dev != naik_dev && (const double*)fat_dev != thin_dev &&
                   (const double*)naik_dev != thin_dev,
               KS_ERR_ARG, "ks_hisq_links: outputs must not alias each other or the input");
    KS_REQUIRE(std::isfinite(c_naik), KS_ERR_ARG, "ks_hisq_links: Naik coefficient not finite");
    const double* l1 = level1 ? level1 : kHisqLevel1;
    const double* l2 = level2 ? level2 : kHisqLevel2;
    for (int k = 0; k < 5; ++k)
        KS_REQUIRE(std::isfinite(l1[k]) && std::isfinite(l2[k]), KS_ERR_ARG,
                   "ks_hisq_links: smearing coefficient %d not finite", k);
    hisq_links(make_geom(dims), thin_dev, fat_dev, naik_dev, l1, l2, c_naik, stream);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_hisq_release(void)
{
    KS_API_BEGIN
    hisq_release();
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_stream_copy(void* dst_dev, const void* src_dev, size_t bytes, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(bytes == 0 || (dst_dev && src_dev), KS_ERR_ARG, "ks_stream_copy: null pointer");
    KS_REQUIRE(bytes % 16 == 0 && ((uintptr_t)dst_dev | (uintptr_t)src_dev) % 16 == 0, KS_ERR_ARG,
               "ks_stream_copy: bytes and both addresses must be multiples of 16");
    const char* d = static_cast<const char*>(dst_dev);
    const char* sp = static_cast<const char*>(src_dev);
    KS_REQUIRE(bytes == 0 || d + bytes <= sp || sp + bytes <= d, KS_ERR_ARG,
               "ks_stream_copy: buffers overlap");
    stream_copy(dst_dev, src_dev, bytes, stream);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_cg_coefficients(ks_gauge_t g, int n_max, double* alpha, double* beta, int* n)
{
    KS_API_BEGIN
    KS_REQUIRE(g && n && n_max >= 0 && (n_max == 0 || (alpha && beta)), KS_ERR_ARG,
               "ks_cg_coefficients: null argument or n_max < 0");
    cg_coefficients(g, n_max, alpha, beta, n);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_stream_read(const void* src_dev, size_t bytes, hipStream_t stream)
{
    KS_API_BEGIN
    KS_REQUIRE(bytes == 0 || src_dev, KS_ERR_ARG, "ks_stream_read: null pointer");
    KS_REQUIRE(bytes % 16 == 0 && (uintptr_t)src_dev % 16 == 0, KS_ERR_ARG,
               "ks_stream_read: bytes and the address must be multiples of 16");
    stream_read(src_dev, bytes, stream);
    return KS_SUCCESS;
    KS_API_END
}

ks_status_t ks_batch_free(ks_batch_t b)
{
    KS_API_BEGIN
    if (!b) return KS_SUCCESS;
    (void)hipDeviceSynchronize();
    batch_free(b->ctx);
    delete b;
    return KS_SUCCESS;
    KS_API_END
}

}  // extern "C"
