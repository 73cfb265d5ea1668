// Sparse tiled layout of T (built at load time) and its frame kernels.
#pragma once

#include <memory>

#include "lbl_internal.h"

namespace lbl {

// Rows per row block of a tile (local rows fit in 16 bits).
constexpr uint32_t kRowBlock = 4096;
// Consecutive words whose nibble tables a wavefront holds at once.
constexpr uint32_t kWordGroup = 1;
// Wavefronts per tile workgroup.
constexpr uint32_t kTileWaves = 4;

// Build the tiled layout of a from its bitpacked T.
lbl_status build_sparse(lbl_abs *a);

// Workspace bytes for one frame of n_lane_groups 64-column groups
// (cell masks + per-tile partial labels).
size_t swm_workspace_bytes(const lbl_abs *a, uint32_t n_lane_groups = 1);

// Pack O, label through the tiled layout, write L (device pointers).
lbl_status run_swm(const lbl_abs *a, const uint8_t *O, uint32_t n_props, void *ws, uint8_t *L, hipStream_t s);

}  // namespace lbl
