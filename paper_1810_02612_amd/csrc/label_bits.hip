// Bitpacked AND/OR labeling kernel (Sec. 4.2, Eq. approx on 64-cell words).
//
// One wavefront labels one trajectory row.  The row is streamed from HBM in
// 16-byte pairs of words (coalesced 1 KiB per wavefront load, non-temporal so
// T does not evict the frame's masks from L2).  A ballot finds the pairs
// holding swept cells; only those are visited (rows sweep ~1% of the
// workspace).  For each such word w, lane p ANDs it with Ow[w][p], the
// frame's 64-cell mask of proposition p, so a wavefront evaluates 64
// propositions x 64 cells per step and never splits a proposition across
// lanes.  The row stops early once every proposition has been hit (the early
// termination of Sec. 5.1).  Lane p finally writes L[t][p].
#include "lbl_internal.h"

namespace lbl {

namespace {

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int src)
{
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

template <int UNROLL>
__global__ void __launch_bounds__(1024)
k_label_bits(const uint64_t *__restrict__ T, uint32_t row_stride, uint32_t n_words, uint64_t n_traj,
             const uint64_t *__restrict__ Ow, uint32_t n_props, uint8_t *__restrict__ L)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t row = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= n_traj) return;  // uniform per wavefront
    const u64x2 *Tr = reinterpret_cast<const u64x2 *>(T + row * (uint64_t)row_stride);
    const uint32_t n_pairs = (n_words + 1) >> 1;
    const uint64_t done = n_props >= 64 ? ~0ull : ((1ull << n_props) - 1ull);
    uint32_t hit = 0;
    for (uint32_t base = 0; base < n_pairs; base += 64 * UNROLL) {
        u64x2 v[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint32_t i = base + u * 64 + lane;
            if (i < n_pairs)
                v[u] = __builtin_nontemporal_load(Tr + i);
            else
                v[u] = u64x2{0ull, 0ull};
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            uint64_t nz = __ballot((v[u].x | v[u].y) != 0ull);
            while (nz) {
                const int src = __builtin_ctzll(nz);
                nz &= nz - 1ull;
                const uint64_t w0 = readlane64(v[u].x, src);
                const uint64_t w1 = readlane64(v[u].y, src);
                const uint64_t wi = 2ull * (base + (uint32_t)(u * 64 + src));
                if (w0) hit |= (w0 & Ow[wi * 64 + lane]) != 0ull;
                if (w1) hit |= (w1 & Ow[(wi + 1) * 64 + lane]) != 0ull;
            }
        }
        if ((__ballot(hit != 0) & done) == done) break;
    }
    if (lane < n_props) L[row * n_props + lane] = (uint8_t)hit;
}

template <int U>
hipError_t launch_u(const lbl_abs *a, const uint64_t *Ow, uint32_t n_props, uint8_t *L, int wpb, hipStream_t s)
{
    const uint64_t blocks = (a->n_traj + wpb - 1) / wpb;
    hipLaunchKernelGGL(k_label_bits<U>, dim3((unsigned)blocks), dim3(64 * wpb), 0, s, a->T_bits, a->row_stride,
                       a->n_words, a->n_traj, Ow, n_props, L);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_label_bits(const lbl_abs *a, const uint64_t *Ow, uint32_t n_props, uint8_t *L,
                             const BitsTile &tile, hipStream_t s)
{
    const int wpb = tile.waves_per_block;
    if (wpb < 1 || wpb > 16) return hipErrorInvalidValue;
    switch (tile.unroll) {
    case 2: return launch_u<2>(a, Ow, n_props, L, wpb, s);
    case 4: return launch_u<4>(a, Ow, n_props, L, wpb, s);
    case 8: return launch_u<8>(a, Ow, n_props, L, wpb, s);
    case 16: return launch_u<16>(a, Ow, n_props, L, wpb, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lbl
