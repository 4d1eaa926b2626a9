// Work items of the block kernels (device side).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace apx {

// Arguments of launch item `item` of a block kernel: the launch's own (one signal), or in a
// multi-signal launch those of the item's signal, with `item` turned into the index inside it
// (blocks 0..P-1, then block 0's prefix item on the FFT cores).  The kernel's own argument is
// never written: that keeps it in the argument segment instead of a private-memory copy.  The
// signal table is read through the constant address space: no store of the kernel can change
// it, so its fields are read once (scalar loads) instead of again after every output store
// through a pointer the compiler cannot tell apart from the table.
template <bool MANY>
__device__ __forceinline__ const RunArgs& item_args(const RunArgs& a0, int64_t& item) {
    if constexpr (MANY) {
        typedef __attribute__((address_space(4))) const RunArgs CRunArgs;
        typedef __attribute__((address_space(4))) const int32_t CInt;
        const int32_t sig = ((CInt*)a0.many_sig)[item];
        const RunArgs& a = *(const RunArgs*)((CRunArgs*)a0.many + sig);
        item -= a.item0;
        return a;
    } else {
        return a0;
    }
}

// An output sample r_out[.] = v, stored with the non-temporal hint: outputs are written once and
// no kernel of the call reads them, so they stream past the caches instead of filling them.  The
// FFT cores' outputs go out as whole rows of consecutive samples (on the FFT-block workload the
// multi-wave core ran 24.5 -> 22.2 us with the hint).  The integer and time-domain cores store
// 128-byte pieces at unaligned offsets and keep plain stores: there the hint raised the HBM write
// bytes by 8-17% and saved no time.
__device__ __forceinline__ void out_store(float* p, float v) { __builtin_nontemporal_store(v, p); }

}  // namespace apx
