// Kernel plans and the autotuner's shape-class cache.
#pragma once

#include "lbl_internal.h"

namespace lbl {

struct MfmaTile {
    int m_tiles = 2;          // 16-row tiles per wavefront
    int waves_per_block = 4;
};

struct Plan {
    Kernel kernel = Kernel::Bits;
    BitsTile bits;
    MfmaTile mfma;
};

// Plan for labeling n_props propositions on a; kflag is LBL_KERNEL_*.
Plan choose(const lbl_abs *a, uint32_t n_props, uint32_t kflag);
size_t plan_ow_bytes(const lbl_abs *a, uint32_t n_props, const Plan &p);
// Pack O into Ow and run the plan's label kernel, writing L (device pointers).
lbl_status run_plan(const lbl_abs *a, const Plan &p, const uint8_t *O, uint32_t n_props, void *Ow, uint8_t *L,
                    hipStream_t s);
// Drop cached batch graphs that reference a (before a is freed).
void batch_forget(const lbl_abs *a);
std::string plan_name(const Plan &p);

hipError_t launch_label_mfma(const lbl_abs *a, const uint64_t *Ow, uint32_t n_props, uint8_t *L,
                             const MfmaTile &tile, bool from_i8, hipStream_t s);
lbl_status mfma_layout_selftest();

}  // namespace lbl
