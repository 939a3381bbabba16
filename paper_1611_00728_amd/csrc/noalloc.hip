// Allocation-free form of the normal operator A_sigma = sigma - D_eo D_oe in FP64, for callers
// that cannot allocate device memory (code under graph capture, tight serving loops).
//
// Its temporaries (the odd-parity image D_oe x and the result planes before they are written
// out in the boundary layout) live in one file-scope device array of fixed size; the caller's
// output array doubles as the staging of the input planes.  Every call on one device uses
// that device's copy of the array, so calls that overlap in time on one device race.
#include <array>
#include <mutex>

#include "ks_common.h"

namespace ks {

namespace {

constexpr int kNoAllocMaxVh = 1 << 19;   // even sites: 524288, a 32^4 lattice
constexpr size_t kPlanes = (size_t)48 * kNoAllocMaxVh;   // one FP64 [3][Vh] field
constexpr size_t kScratchBytes = 2 * kPlanes;            // 48 MiB
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::array<void*, kMaxDevices> g_scratch_ptr{};

// The device address of this device's scratch array, looked up once per device.  In host code
// the array's name is only a host-side stand-in; the kernels get this address instead.
void* scratch_address()
{
    int dev = 0;
    KS_HIP(hipGetDevice(&dev));
    KS_REQUIRE(dev >= 0 && dev < kMaxDevices, KS_ERR_ARG, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        KS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        KS_REQUIRE(p != nullptr, KS_ERR_HIP, "no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

}  // namespace ks

using namespace ks;

extern "C" ks_status_t ks_apply_A_noalloc(ks_gauge_t g, double sigma, const double* in_dev,
                                          double* out_dev, hipStream_t stream)
{
    try {
        KS_REQUIRE(g && in_dev && out_dev, KS_ERR_ARG, "ks_apply_A_noalloc: null argument");
        KS_REQUIRE(in_dev != out_dev, KS_ERR_ARG, "ks_apply_A_noalloc: out aliases in");
        const Geom& G = g->geom;
        KS_REQUIRE(G.Vh <= kNoAllocMaxVh, KS_ERR_ARG,
                   "ks_apply_A_noalloc: %d even sites exceed the scratch limit of %d "
                   "(a 32^4 lattice)", G.Vh, kNoAllocMaxVh);
        char* base = static_cast<char*>(scratch_address());
        double* t = reinterpret_cast<double*>(base);              // D_oe x, odd parity
        double* y = reinterpret_cast<double*>(base + kPlanes);    // A x in FP64 planes
        double* x = out_dev;                                      // x as FP64 planes
        import_field(G, KS_F64, in_dev, x, stream);
        DslashArgs a1;
        a1.out_parity = 1;
        a1.in = x;
        a1.out = t;
        dslash(g, KS_F64, KS_RECON_18, a1, stream);
        DslashArgs a2;
        a2.out_parity = 0;
        a2.in = t;
        a2.out = y;
        a2.x = x;
        a2.a = sigma;
        dslash(g, KS_F64, KS_RECON_18, a2, stream);
        export_field(G, KS_F64, y, out_dev, stream);
        return KS_SUCCESS;
    } catch (const Failure& f) {
        return f.code;
    } catch (...) {
        set_error("ks_apply_A_noalloc: unexpected C++ exception");
        return KS_ERR_HIP;
    }
}
