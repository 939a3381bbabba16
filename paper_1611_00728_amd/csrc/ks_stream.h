// Streamed (non-temporal) loads and stores of colour-vector fields in the layouts of Spinor<P>:
// for vectors a solver step touches once (the solution, the shifted directions), so that they
// do not push out of the caches the vector the next hopping term gathers from its neighbours.
// FP16 records go through Spinor's encoding unchanged.
#pragma once

#include "ks_device.h"

namespace ks {

template <int P>
struct Streamed {
    using R = typename St<P>::R;
    __device__ static __forceinline__ void load(const void* b, int vh, int h, cx<R> v[3])
    {
        if constexpr (P == KS_F64) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const dvec2 t =
                    __builtin_nontemporal_load(static_cast<const dvec2*>(b) + (size_t)k * vh + h);
                v[k] = {t.x, t.y};
            }
        } else if constexpr (P == KS_F32) {
            const fvec4 a = __builtin_nontemporal_load(static_cast<const fvec4*>(b) + h);
            const fvec2 c = __builtin_nontemporal_load(
                reinterpret_cast<const fvec2*>(static_cast<const fvec4*>(b) + vh) + h);
            v[0] = {a.x, a.y};
            v[1] = {a.z, a.w};
            v[2] = {c.x, c.y};
        } else {
            Spinor<P>::load(b, vh, h, v);
        }
    }
    __device__ static __forceinline__ void store(void* b, int vh, int h, const cx<R> v[3])
    {
        if constexpr (P == KS_F64) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                __builtin_nontemporal_store(dvec2{v[k].r, v[k].i},
                                            static_cast<dvec2*>(b) + (size_t)k * vh + h);
        } else if constexpr (P == KS_F32) {
            __builtin_nontemporal_store(fvec4{v[0].r, v[0].i, v[1].r, v[1].i},
                                        static_cast<fvec4*>(b) + h);
            __builtin_nontemporal_store(fvec2{v[2].r, v[2].i},
                                        reinterpret_cast<fvec2*>(static_cast<fvec4*>(b) + vh) + h);
        } else {
            Spinor<P>::store(b, vh, h, v);
        }
    }
};

}  // namespace ks
