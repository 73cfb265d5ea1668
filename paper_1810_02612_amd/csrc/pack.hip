// Layout kernels: T packing at load time (CSR or dense -> bitpacked rows in
// device cell order, optional int8 copy) and per-frame O packing.
#include "lbl_internal.h"

namespace lbl {

namespace {

__device__ __forceinline__ uint32_t spread3(uint32_t v)
{
    // bits b of v (b < 3) -> position 2b
    return (v & 1u) | ((v & 2u) << 1) | ((v & 4u) << 2);
}

// One workgroup per row: OR every listed cell's bit into the zeroed row.
// A column id outside the grid sets *bad and is skipped.  Ids are row-major,
// or z-order indices when morton (the device position itself).
__global__ void __launch_bounds__(256)
k_pack_csr(uint64_t *__restrict__ T, uint32_t row_stride, const uint64_t *__restrict__ row_ptr,
           uint64_t row_base, uint64_t n_rows, const uint32_t *__restrict__ col_idx, uint64_t col_base,
           const uint32_t *__restrict__ tile_word, uint32_t nx, uint32_t n_cells, uint32_t morton, uint32_t *bad)
{
    const uint64_t r = blockIdx.x;
    if (r >= n_rows) return;
    const uint64_t lo = row_ptr[r] - col_base, hi = row_ptr[r + 1] - col_base;
    uint64_t *Tr = T + (row_base + r) * (uint64_t)row_stride;
    const uint32_t ntx = nx >> 3;
    for (uint64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
        const uint32_t c = col_idx[k];
        if (c >= n_cells) {
            atomicOr(bad, 1u);
            continue;
        }
        uint32_t w, b;
        if (morton) {
            w = c >> 6;
            b = c & 63u;
        } else {
            const uint32_t ix = c % nx, iy = c / nx;
            w = tile_word[(iy >> 3) * ntx + (ix >> 3)];
            b = (spread3(ix & 7u) << 1) | spread3(iy & 7u);
        }
        atomicOr(reinterpret_cast<unsigned long long *>(Tr + w), 1ull << b);
    }
}

// One wavefront per (row, word): lane b tests the byte of the cell at bit b.
__global__ void __launch_bounds__(256)
k_pack_dense(uint64_t *__restrict__ T, uint32_t row_stride, const uint8_t *__restrict__ Td,
             uint64_t n_rows, uint32_t n_cells, const uint32_t *__restrict__ word_cell, uint32_t n_words)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t n_items = n_rows * n_words;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t it = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); it < n_items;
         it += waves) {
        const uint64_t r = it / n_words;
        const uint32_t w = (uint32_t)(it - r * n_words);
        const uint32_t c = word_cell[(uint64_t)w * 64 + lane];
        const uint64_t m = __ballot(Td[r * n_cells + c] != 0);
        if (lane == 0) T[r * row_stride + w] = m;
    }
}

// T8[r][w * 64 + b] = bit b of T[r][w]: one thread per word, 64 bytes out.
__global__ void __launch_bounds__(256)
k_expand_i8(int8_t *__restrict__ T8, const uint64_t *__restrict__ T, uint32_t row_stride,
            uint64_t n_rows, uint32_t n_words)
{
    const uint64_t n_items = n_rows * n_words;
    for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < n_items;
         it += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = it / n_words;
        const uint32_t w = (uint32_t)(it - r * n_words);
        const uint64_t v = T[r * row_stride + w];
        uint4 *dst = reinterpret_cast<uint4 *>(T8 + it * 64);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t x[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const uint32_t nib = (uint32_t)(v >> (16 * q + 4 * h)) & 0xFu;
                x[h] = (nib * 0x00204081u) & 0x01010101u;
            }
            dst[q] = make_uint4(x[0], x[1], x[2], x[3]);
        }
    }
}

__global__ void __launch_bounds__(256)
k_count_words(const uint64_t *__restrict__ T, uint32_t row_stride, uint64_t n_rows, uint32_t n_words,
              unsigned long long *counts)
{
    const uint64_t n_items = n_rows * n_words;
    unsigned long long nz = 0, pop = 0;
    for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < n_items;
         it += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = it / n_words;
        const uint32_t w = (uint32_t)(it - r * n_words);
        const uint64_t v = T[r * row_stride + w];
        nz += v != 0;
        pop += __popcll(v);
    }
    for (int off = 32; off > 0; off >>= 1) {
        nz += __shfl_down(nz, off);
        pop += __shfl_down(pop, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(counts + 0, nz);
        atomicAdd(counts + 1, pop);
    }
}

// One wavefront per word w: lane p gathers the 64 cells' bytes of proposition
// p and assembles Ow[w][p].  Lanes at or above n_props write zero masks.
__global__ void __launch_bounds__(256)
k_pack_O(const uint8_t *__restrict__ O, uint32_t n_props, const uint32_t *__restrict__ word_cell,
         uint32_t n_words, uint64_t *__restrict__ Ow)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= n_words) return;
    const uint32_t *wc = word_cell + (uint64_t)w * 64;
    uint64_t m = 0;
    if (lane < n_props) {
#pragma unroll 16
        for (uint32_t b = 0; b < 64; ++b) {
            const uint8_t v = O[(uint64_t)wc[b] * n_props + lane];
            m |= (uint64_t)(v != 0) << b;
        }
    }
    Ow[(uint64_t)w * 64 + lane] = m;
}

}  // namespace

static unsigned grid_for(uint64_t items, unsigned per_block, unsigned cap = 1u << 20)
{
    uint64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

hipError_t launch_pack_csr(uint64_t *T, uint32_t row_stride, const uint64_t *row_ptr, uint64_t row_base,
                           uint64_t n_rows, const uint32_t *col_idx, uint64_t col_base,
                           const uint32_t *tile_word, uint32_t nx, uint32_t n_cells, bool morton,
                           uint32_t *bad, hipStream_t s)
{
    if (n_rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_csr, dim3((unsigned)n_rows), dim3(256), 0, s, T, row_stride, row_ptr,
                       row_base, n_rows, col_idx, col_base, tile_word, nx, n_cells, (uint32_t)morton, bad);
    return hipGetLastError();
}

hipError_t launch_pack_dense(uint64_t *T, uint32_t row_stride, const uint8_t *Td, uint64_t n_rows,
                             uint32_t n_cells, const uint32_t *word_cell, uint32_t n_words, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_dense, dim3(grid_for(n_rows * n_words, 4)), dim3(256), 0, s, T, row_stride,
                       Td, n_rows, n_cells, word_cell, n_words);
    return hipGetLastError();
}

hipError_t launch_expand_i8(int8_t *T8, const uint64_t *T, uint32_t row_stride, uint64_t n_rows,
                            uint32_t n_words, hipStream_t s)
{
    hipLaunchKernelGGL(k_expand_i8, dim3(grid_for(n_rows * n_words, 256)), dim3(256), 0, s, T8, T,
                       row_stride, n_rows, n_words);
    return hipGetLastError();
}

hipError_t launch_count_words(const uint64_t *T, uint32_t row_stride, uint64_t n_rows, uint32_t n_words,
                              unsigned long long *counts, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_words, dim3(grid_for(n_rows * n_words, 256, 8192)), dim3(256), 0, s, T,
                       row_stride, n_rows, n_words, counts);
    return hipGetLastError();
}

hipError_t launch_pack_O(const lbl_abs *a, const uint8_t *O, uint32_t n_props, uint64_t *Ow, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_O, dim3((a->n_words + 3) / 4), dim3(256), 0, s, O, n_props, a->d_word_cell,
                       a->n_words, Ow);
    return hipGetLastError();
}

}  // namespace lbl
