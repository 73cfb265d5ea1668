// Nibble tables of a word, built by one wavefront (device code only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbl {

// Nonzero bytes of a 32-bit word -> 4 bits (bit k for byte k).
__device__ __forceinline__ uint32_t nz_bytes(uint32_t x)
{
    const uint32_t y = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;  // high bit of each byte: byte != 0
    const uint32_t h = y & 0x80808080u;
    return ((h >> 7) | (h >> 14) | (h >> 21) | (h >> 28)) & 0xFu;
}

// Four bits -> four bytes 0/1 (bit k to byte k).
__device__ __forceinline__ uint32_t spread_nib(uint32_t x) { return (x * 0x00204081u) & 0x01010101u; }

// Nonzero bytes of 16 bytes -> 16 bits (bit k for byte k).
__device__ __forceinline__ uint32_t nz_bytes16(const uint4 &q)
{
    return nz_bytes(q.x) | (nz_bytes(q.y) << 4) | (nz_bytes(q.z) << 8) | (nz_bytes(q.w) << 12);
}

// Bit p set iff byte p of src[0 .. n) is non-zero, 1 <= n <= 64; 16-, 4- or
// 2-byte loads when n and the address allow.  A group of four loads is
// issued before the first of its results is used (a loop that used each load
// before issuing the next would wait out the memory latency once per load):
// indices past the last piece repeat the last load, which stays in bounds,
// and their bits are dropped by a select rather than a branch, which the
// compiler would turn into a load under a branch again.
__device__ __forceinline__ uint64_t byte_mask(const uint8_t *src, uint32_t n)
{
    uint64_t m = 0;
    const uintptr_t a = reinterpret_cast<uintptr_t>(src);
    if ((n & 15u) == 0 && (a & 15u) == 0) {
        const uint32_t last = n / 16 - 1;  // at most 3
        uint4 q[4];
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) q[k] = reinterpret_cast<const uint4 *>(src)[min(k, last)];
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
            const uint64_t b = (uint64_t)nz_bytes16(q[k]) << (16 * k);
            m |= k <= last ? b : 0ull;
        }
    } else if ((n & 3u) == 0 && (a & 3u) == 0) {
        const uint32_t last = n / 4 - 1;  // at most 15
        for (uint32_t k0 = 0; k0 <= last; k0 += 4) {
            uint32_t d[4];
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k) d[k] = reinterpret_cast<const uint32_t *>(src)[min(k0 + k, last)];
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k) {
                const uint64_t b = (uint64_t)nz_bytes(d[k]) << ((4 * (k0 + k)) & 63u);
                m |= k0 + k <= last ? b : 0ull;
            }
        }
    } else if ((n & 1u) == 0 && (a & 1u) == 0) {
        const uint32_t last = n / 2 - 1;  // at most 31
        for (uint32_t k0 = 0; k0 <= last; k0 += 4) {
            uint32_t h[4];
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k) h[k] = reinterpret_cast<const uint16_t *>(src)[min(k0 + k, last)];
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k) {
                const uint32_t two = ((h[k] & 0xFFu) != 0 ? 1u : 0u) | ((h[k] >> 8) != 0 ? 2u : 0u);
                const uint64_t b = (uint64_t)two << ((2 * (k0 + k)) & 63u);
                m |= k0 + k <= last ? b : 0ull;
            }
        }
    } else {
        for (uint32_t p0 = 0; p0 < n; p0 += 4) {
            uint32_t c[4];
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) c[j] = src[min(p0 + j, n - 1)];
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                const uint64_t b = (uint64_t)(c[j] != 0 ? 1u : 0u) << ((p0 + j) & 63u);
                m |= p0 + j < n ? b : 0ull;
            }
        }
    }
    return m;
}

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

// 32-bit version of quad_bcast.
template <int C>
__device__ __forceinline__ uint32_t quad_bcast32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, C * 0x55, 0xF, 0xF, false);
}

// write_tables for 32-bit proposition masks (frames of at most 32
// propositions): the same 16 x 16 tables with 4-byte entries, lane 4n + j
// writing the 16 bytes of entries [n][4j .. 4j+3] to dst[n * 16 + 4j ..].
__device__ __forceinline__ void write_tables32(uint32_t cell, uint32_t *dst, uint32_t lane)
{
    const uint32_t o0 = quad_bcast32<0>(cell), o1 = quad_bcast32<1>(cell);
    const uint32_t o2 = quad_bcast32<2>(cell), o3 = quad_bcast32<3>(cell);
    const uint32_t j = lane & 3u;
    const uint32_t h = ((j & 1u) ? o2 : 0u) | ((j & 2u) ? o3 : 0u);
    *reinterpret_cast<uint4 *>(dst + (lane >> 2) * 16 + 4 * j) = make_uint4(h, h | o0, h | o1, h | o0 | o1);
}

}  // namespace lbl
