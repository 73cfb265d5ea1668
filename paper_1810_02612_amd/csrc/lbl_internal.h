// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbl.h"

namespace lbl {

// ---------------------------------------------------------------- errors

void set_error(const std::string &msg);
void clear_error();

#define LBL_HIP_TRY(expr)                                                         \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::lbl::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));  \
            return e_ == hipErrorOutOfMemory ? LBL_ENOMEM : LBL_EDEVICE;          \
        }                                                                         \
    } while (0)

#define LBL_REQUIRE(cond, msg)                \
    do {                                      \
        if (!(cond)) {                        \
            ::lbl::set_error(msg);            \
            return LBL_EINVAL;                \
        }                                     \
    } while (0)

// ---------------------------------------------------------------- layout

// Device cell order: 8x8 tiles, one uint64 word per tile, words ranked by the
// tiles' z-order, bits by the cells' z-order inside the tile (x is the more
// significant bit of each pair).
// word_cell maps a device position to the caller's cell id: the row-major id,
// or, for callers numbering cells in z-order (LBL_MORTON, square grids of
// power-of-two side), the position itself (word * 64 + bit is the z-order
// index there).
struct CellOrder {
    uint32_t nx = 0, ny = 0, ntx = 0, nty = 0, n_words = 0;
    bool morton = false;
    std::vector<uint32_t> tile_word;  // [nty * ntx] -> word index
    std::vector<uint32_t> word_cell;  // [n_words * 64] -> caller's cell id
    void build(uint32_t nx, uint32_t ny, bool morton = false);
};

// Validates a grid (sizes, cell_order) for any entry point.
lbl_status check_grid(const lbl_grid *g);

uint32_t morton2(uint32_t x, uint32_t y);  // x bits at odd positions

// Sparse tiled layout of T (defined with its kernels).
struct SparseLayout;
void free_sparse(SparseLayout *sp);

}  // namespace lbl

// Abstraction: device-resident T in bitpacked (and optionally int8) layout.
struct lbl_abs {
    int device = 0;
    uint32_t nx = 0, ny = 0;
    float cell_m = 0.f;
    uint64_t n_traj = 0;
    uint32_t n_cells = 0;
    uint32_t n_words = 0;     // W
    uint32_t row_stride = 0;  // words per row in T_bits (W rounded up to even)
    uint64_t *T_bits = nullptr;
    int8_t *T_i8 = nullptr;   // [n_traj][n_words * 64] device cell order
    uint32_t *d_tile_word = nullptr;
    uint32_t *d_word_cell = nullptr;
    uint64_t nonzero_words = 0;
    uint64_t set_cells = 0;
    lbl::CellOrder order;
    // sparse tiled layout (null when not built)
    lbl::SparseLayout *sp = nullptr;
};

namespace lbl {

// Per-stream scratch memory, grown on demand (growth synchronizes the stream).
lbl_status workspace(hipStream_t s, size_t bytes, void **out);

// ---------------------------------------------------------------- kernels

// Kernel choices (runtime representation of LBL_KERNEL_*).
enum class Kernel : int { Bits = 0, Mfma = 1, MfmaI8 = 2, Sparse = 3 };

struct BitsTile {
    int unroll = 8;          // 16-byte loads per lane in flight per step
    int waves_per_block = 4; // rows per workgroup
};

// Pack a frame: O (n_cells x n_props bytes, cell-major) -> Ow[w][64] bit masks
// (lane p of word w holds the 64 cells of w for proposition p).
hipError_t launch_pack_O(const lbl_abs *a, const uint8_t *O, uint32_t n_props, uint64_t *Ow,
                         hipStream_t s);

// Bitpacked label kernel for one frame.
hipError_t launch_label_bits(const lbl_abs *a, const uint64_t *Ow, uint32_t n_props, uint8_t *L,
                             const BitsTile &tile, hipStream_t s);

// T packers used at load time.
// Column ids are row-major unless morton (then word = id / 64, bit = id % 64).
hipError_t launch_pack_csr(uint64_t *T, uint32_t row_stride, const uint64_t *row_ptr,
                           uint64_t row_base, uint64_t n_rows, const uint32_t *col_idx,
                           uint64_t col_base, const uint32_t *tile_word, uint32_t nx,
                           uint32_t n_cells, bool morton, uint32_t *bad, hipStream_t s);
hipError_t launch_pack_dense(uint64_t *T, uint32_t row_stride, const uint8_t *Td, uint64_t n_rows,
                             uint32_t n_cells, const uint32_t *word_cell, uint32_t n_words,
                             hipStream_t s);
hipError_t launch_expand_i8(int8_t *T8, const uint64_t *T, uint32_t row_stride, uint64_t n_rows,
                            uint32_t n_words, hipStream_t s);
hipError_t launch_count_words(const uint64_t *T, uint32_t row_stride, uint64_t n_rows,
                              uint32_t n_words, unsigned long long *counts, hipStream_t s);

}  // namespace lbl
