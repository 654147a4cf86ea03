// Device access to the FP64 near store of a MIXED operator (the store
// itself: near.hip; its layout: NearView in mbem_internal.h).
#pragma once

#include "mbem_internal.h"

namespace mbem {

// Slot of node pair (i, j) in the store, or -1 if the pair is not in its
// pattern: the row's offset, the set bits of the row before j's word and
// those below j in it.
__device__ __forceinline__ int64_t near_slot(const NearView &v, int64_t i, int64_t j) {
    const int64_t w = i * v.nw + (j >> 5);
    const uint32_t word = v.bits[w];
    const uint32_t bit = 1u << (j & 31);
    if (!(word & bit)) return -1;
    return (int64_t)v.rptr[i] + v.wpre[w] + __popc(word & (bit - 1u));
}

// Store value of entry (2 i + al, 2 j + be) of block op, zero outside the
// pattern (and without a store).
__device__ __forceinline__ double2 near_value(const NearView &v, int op, int64_t i, int64_t j, int al, int be) {
    if (!v.bits) return {0.0, 0.0};
    const int64_t s = near_slot(v, i, j);
    return s < 0 ? double2{0.0, 0.0} : v.val[12 * s + 4 * op + 2 * al + be];
}

}  // namespace mbem
