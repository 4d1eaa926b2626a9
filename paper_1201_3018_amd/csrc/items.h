// Work items of the block kernels (device side).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace apx {

// Arguments of launch item `item` of a block kernel: the launch's own (one signal), or in a
// multi-signal launch those of the item's signal, with `item` turned into the index inside it
// (blocks 0..P-1, then block 0's prefix item on the FFT cores).  The kernel's own argument is
// never written: that keeps it in the argument segment instead of a private-memory copy.
template <bool MANY>
__device__ __forceinline__ const RunArgs& item_args(const RunArgs& a0, int64_t& item) {
    if constexpr (MANY) {
        const RunArgs& a = a0.many[a0.many_sig[item]];
        item -= a.item0;
        return a;
    } else {
        return a0;
    }
}

}  // namespace apx
