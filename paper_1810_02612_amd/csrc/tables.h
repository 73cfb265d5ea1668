// Nibble tables of a word, built by one wavefront (device code only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbl {

// Value of lane C of each group of four lanes (DPP quad permutation).
template <int C>
__device__ __forceinline__ uint64_t quad_bcast(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, C * 0x55, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), C * 0x55, 0xF, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

// The 16 x 16 nibble tables of one 64-cell word: entry [n][v] is the OR of
// the proposition masks of the cells 4n + b with bit b of v set, so that
// OR over n of entry [n][nibble n of x] is the label of a word value x.
// Lane l holds the mask of cell l; the four lanes of nibble n share their
// masks and lane 4n + j writes the four consecutive entries [n][4j .. 4j+3]
// (32 bytes) to dst[n * 16 + 4j ..].  Every lane of the wavefront must be
// active.
__device__ __forceinline__ void write_tables(uint64_t cell, uint64_t *dst, uint32_t lane)
{
    const uint64_t o0 = quad_bcast<0>(cell), o1 = quad_bcast<1>(cell);
    const uint64_t o2 = quad_bcast<2>(cell), o3 = quad_bcast<3>(cell);
    const uint32_t j = lane & 3u;
    const uint64_t h = ((j & 1u) ? o2 : 0ull) | ((j & 2u) ? o3 : 0ull);  // bits 2, 3 of v = 4j + m
    ulonglong2 *d = reinterpret_cast<ulonglong2 *>(dst + (lane >> 2) * 16 + 4 * j);
    d[0] = make_ulonglong2(h, h | o0);
    d[1] = make_ulonglong2(h | o1, h | o0 | o1);
}

}  // namespace lbl
