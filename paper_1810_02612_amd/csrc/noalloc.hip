// lbl_label_frame_noalloc: one frame labeled with no device allocation.
//
// The per-frame intermediates of lbl_label_frame (the nibble tables and tile
// partials of the sparse path, or the packed proposition masks of the
// bitpacked path) live in the stream's workspace, which the library
// allocates on a stream's first call.  Callers that cannot allocate (code
// under HIP graph capture, serving loops that forbid it) use this variant
// instead: the intermediates go to one fixed device array of kScratchBytes,
// of which every GPU the library runs on holds its own copy until the
// process ends.
#include <mutex>

#include "lbl_internal.h"
#include "sparse.h"

namespace lbl {

namespace {

constexpr size_t kScratchBytes = 96ull << 20;

// The intermediates of the frames labeled through lbl_label_frame_noalloc.
// In host code this name stands for the host-side shadow of the array, not
// its device address: kernels are given the address from scratch_ptr().
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device,
// with that device current).
lbl_status scratch_ptr(int dev, void **out)
{
    LBL_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        LBL_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        LBL_REQUIRE(p != nullptr, "the scratch array has no device address");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return LBL_OK;
}

}  // namespace

}  // namespace lbl

using namespace lbl;

extern "C" {

lbl_status lbl_label_frame_noalloc(lbl_abs_t a, const uint8_t *O, uint32_t n_props, uint8_t *L, void *hip_stream)
{
    clear_error();
    LBL_REQUIRE(a != nullptr, "abstraction is null");
    LBL_REQUIRE(O != nullptr && L != nullptr, "O or L is null");
    LBL_REQUIRE(n_props >= 1 && n_props <= 64, "n_props must be in [1, 64]");
    int dev = 0;
    LBL_HIP_TRY(hipGetDevice(&dev));
    LBL_REQUIRE(dev == a->device, "the current device is not the abstraction's device");
    const bool sparse = a->sp != nullptr;
    LBL_REQUIRE(sparse || a->T_bits != nullptr, "the abstraction holds no layout of T");
    const size_t need = sparse ? swm_frame_workspace_bytes(a, n_props) : (size_t)a->n_words * 64 * sizeof(uint64_t);
    LBL_REQUIRE(need <= kScratchBytes, "the frame needs " + std::to_string(need) +
                                           " bytes of scratch; lbl_label_frame_noalloc holds " +
                                           std::to_string(kScratchBytes) + " (use lbl_label_frame)");
    void *ws = nullptr;
    lbl_status st = scratch_ptr(dev, &ws);
    if (st != LBL_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    // every byte the kernels read from the scratch is written earlier in the
    // same call (tables of every word in use, every partial slot, every
    // packed mask), so nothing is cleared first
    if (sparse) return run_swm(a, O, n_props, ws, L, s, false);
    uint64_t *ow = static_cast<uint64_t *>(ws);
    LBL_HIP_TRY(launch_pack_O(a, O, n_props, ow, s));
    LBL_HIP_TRY(launch_label_bits(a, ow, n_props, L, BitsTile{}, s));
    return LBL_OK;
}

}  // extern "C"
