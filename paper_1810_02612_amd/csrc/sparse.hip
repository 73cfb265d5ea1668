// Sparse tiled layout of T and its labeling kernels.
//
// Layout.  Every non-zero 64-cell word of T becomes one entry (local row,
// word value).  Entries are grouped into segments (row block rb, word w):
// the rows of block rb (kRowBlock rows) whose swept set meets word w,
// ascending.  Segments are stored in (rb, w) order, so the entries of a tile
// (row block rb, a range of consecutive words) are contiguous, and
// seg[rb * W + w] .. seg[rb * W + w + 1] delimits one segment.  This is the
// compressed-sparse idea of Sec. 4.3 (store only the true entries of M) at
// word granularity, ordered so that the frame data a word needs is prepared
// once per tile and shared by every trajectory of the tile that crosses it.
//
// Per frame:
//   k_pack_cells   O -> Oc[w][b]: 64-bit mask of the propositions that cell
//                  b of word w meets (one lane per cell).
//   k_label_tiles  one workgroup per tile.  Each wavefront takes groups of
//                  kWordGroup consecutive words of the tile, builds in LDS
//                  their 16 x 16 nibble tables (entry [n][v] = OR of Oc over
//                  the cells 4n + b with bit b of v set), and every lane
//                  takes one entry (row t, word value x) and ORs the 16
//                  table entries selected by the nibbles of x: the labels of
//                  that (row, word) pair for up to 64 propositions.  They are
//                  OR-ed into the tile's per-row accumulators with LDS atomics
//                  and written once per row as the tile's partial label.
//   k_combine      OR of a row's partials over the word ranges -> the
//                  caller's L bytes (0/1).
// OR is idempotent and commutative, so neither the order of the LDS atomics
// nor the split into tiles changes the result.  No global atomics are used.
#include <algorithm>

#include "batch.h"
#include "profile.h"
#include "sparse.h"

namespace lbl {

namespace {

// ---------------------------------------------------------------- load time

// One wavefront per word, 8 consecutive words per workgroup.  Counts the rows
// whose word w is non-zero.
__global__ void __launch_bounds__(512)
k_wm_count(const uint64_t *__restrict__ T, uint32_t row_stride, uint64_t n_traj, uint32_t n_words,
           uint64_t *__restrict__ counts)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = blockIdx.x * 8 + (threadIdx.x >> 6);
    if (w >= n_words) return;
    uint64_t n = 0;
    for (uint64_t t0 = 0; t0 < n_traj; t0 += 64 * 4) {
        uint64_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t t = t0 + 64 * u + lane;
            v[u] = t < n_traj ? T[t * row_stride + w] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) n += __popcll(__ballot(v[u] != 0ull));
    }
    if (lane == 0) counts[w] = n;
}

// Same scan; writes each non-zero (row, value) of word w at its position in
// the word-major arrays, rows ascending.
__global__ void __launch_bounds__(512)
k_wm_fill(const uint64_t *__restrict__ T, uint32_t row_stride, uint64_t n_traj, uint32_t n_words,
          const uint64_t *__restrict__ wm_ptr, uint32_t *__restrict__ wm_row, uint64_t *__restrict__ wm_val)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = blockIdx.x * 8 + (threadIdx.x >> 6);
    if (w >= n_words) return;
    uint64_t pos = wm_ptr[w];
    const uint64_t end = wm_ptr[w + 1];
    for (uint64_t t0 = 0; t0 < n_traj; t0 += 64 * 4) {
        uint64_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t t = t0 + 64 * u + lane;
            v[u] = t < n_traj ? T[t * row_stride + w] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t m = __ballot(v[u] != 0ull);
            const uint64_t at = pos + __popcll(m & ((1ull << lane) - 1ull));
            if (v[u] != 0ull && at < end) {
                wm_row[at] = (uint32_t)(t0 + 64 * u + lane);
                wm_val[at] = v[u];
            }
            pos += __popcll(m);
        }
    }
}

// First index in rows[lo, hi) (ascending) that is >= key.
__device__ __forceinline__ uint64_t lower_bound_u32(const uint32_t *rows, uint64_t lo, uint64_t hi, uint64_t key)
{
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if ((uint64_t)rows[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One thread per segment (rb, w): entries of word w with rows in block rb.
__global__ void __launch_bounds__(256)
k_seg_count(const uint64_t *__restrict__ wm_ptr, const uint32_t *__restrict__ wm_row, uint32_t n_words,
            uint32_t n_rb, uint32_t *__restrict__ cnt)
{
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= (uint64_t)n_rb * n_words) return;
    const uint32_t rb = (uint32_t)(s / n_words), w = (uint32_t)(s % n_words);
    const uint64_t lo = lower_bound_u32(wm_row, wm_ptr[w], wm_ptr[w + 1], (uint64_t)rb * kRowBlock);
    const uint64_t hi = lower_bound_u32(wm_row, lo, wm_ptr[w + 1], (uint64_t)(rb + 1) * kRowBlock);
    cnt[s] = (uint32_t)(hi - lo);
}

// Copies segment (rb, w) to its place in the tiled arrays (local rows).
__global__ void __launch_bounds__(256)
k_seg_fill(const uint64_t *__restrict__ wm_ptr, const uint32_t *__restrict__ wm_row,
           const uint64_t *__restrict__ wm_val, uint32_t n_words, uint32_t n_rb, const uint64_t *__restrict__ seg,
           uint16_t *__restrict__ sp_row, uint64_t *__restrict__ sp_val)
{
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= (uint64_t)n_rb * n_words) return;
    const uint32_t rb = (uint32_t)(s / n_words), w = (uint32_t)(s % n_words);
    const uint64_t lo = lower_bound_u32(wm_row, wm_ptr[w], wm_ptr[w + 1], (uint64_t)rb * kRowBlock);
    const uint64_t hi = lower_bound_u32(wm_row, lo, wm_ptr[w + 1], (uint64_t)(rb + 1) * kRowBlock);
    const uint64_t dst = seg[s];
    if (seg[s + 1] - dst != hi - lo) return;  // counts disagree: leave the segment (checked on the host)
    for (uint64_t k = lo; k < hi; ++k) {
        sp_row[dst + (k - lo)] = (uint16_t)(wm_row[k] - (uint64_t)rb * kRowBlock);
        sp_val[dst + (k - lo)] = wm_val[k];
    }
}

// ---------------------------------------------------------------- per frame

// Nonzero bytes of a 32-bit word -> 4 bits (bit k for byte k).
__device__ __forceinline__ uint32_t nz_bytes(uint32_t x)
{
    const uint32_t y = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;  // high bit of each byte: byte != 0
    const uint32_t h = y & 0x80808080u;
    return ((h >> 7) | (h >> 14) | (h >> 21) | (h >> 28)) & 0xFu;
}

// One lane per cell: Oc[w * 64 + b] = propositions met by cell (w, b).
__global__ void __launch_bounds__(256)
k_pack_cells(const uint8_t *__restrict__ O, uint32_t n_props, const uint32_t *__restrict__ word_cell,
             uint32_t n_words, uint64_t *__restrict__ Oc)
{
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;  // w * 64 + b
    if (idx >= (uint64_t)n_words * 64) return;
    const uint8_t *src = O + (uint64_t)word_cell[idx] * n_props;
    uint64_t m = 0;
    if ((n_props & 15u) == 0 && (reinterpret_cast<uintptr_t>(O) & 15u) == 0) {
        for (uint32_t p = 0; p < n_props; p += 16) {
            const uint4 q = *reinterpret_cast<const uint4 *>(src + p);
            const uint64_t bits = nz_bytes(q.x) | (nz_bytes(q.y) << 4) | (nz_bytes(q.z) << 8) | (nz_bytes(q.w) << 12);
            m |= bits << p;
        }
    } else {
        for (uint32_t p = 0; p < n_props; ++p) m |= (uint64_t)(src[p] != 0) << p;
    }
    Oc[idx] = m;
}

// One workgroup per tile (row block rb, word range wr).  Oc_word(w) =
// Oc + w * oc_word_stride holds the 64 cell masks of word w.  Writes the
// tile's partial labels to P[wr * p_stride + row] for its rows.
template <int WAVES, int GROUP>
__device__ __forceinline__ void tile_body(const uint64_t *__restrict__ seg, const uint16_t *__restrict__ sp_row,
                                          const uint64_t *__restrict__ sp_val, const uint64_t *__restrict__ Oc,
                                          uint64_t oc_word_stride, uint32_t n_words, uint32_t rb, uint32_t wr,
                                          uint32_t wr_words, uint64_t n_traj, uint64_t max_entry,
                                          uint64_t *__restrict__ P, uint64_t p_stride, uint64_t *lds)
{
    const uint32_t lane = threadIdx.x & 63;
    // uniform across the wavefront: segment bounds become scalar loads and
    // the per-group branches scalar branches
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint64_t *acc = lds;                                      // kRowBlock accumulators
    uint64_t *tab = lds + kRowBlock + wave * (GROUP * 256);   // this wavefront's tables
    for (uint32_t i = threadIdx.x; i < kRowBlock; i += blockDim.x) acc[i] = 0ull;
    __syncthreads();
    const uint32_t w_lo = wr * wr_words, w_hi = min(w_lo + wr_words, n_words);
    const uint64_t *segb = seg + (uint64_t)rb * n_words;
    const uint32_t nib = lane >> 2, v0 = (lane & 3u) * 4;

    // Everything a word group needs, loaded one group ahead so that the
    // latency of the next group's loads overlaps this group's work.
    struct Group {
        uint64_t lo, hi;           // entry range of the group (uniform)
        uint64_t bound[GROUP];     // end of each word's segment (uniform)
        uint64_t o[GROUP][4];      // this lane's 4 cell masks of each word
        uint64_t x;                // first entry of this lane (valid if lo + lane < hi)
        uint32_t r;
        uint32_t nw;
    };
    // Every load is unconditional at a clamped, in-bounds address (branches
    // around loads would make the compiler wait for all of them); validity
    // is applied when the group is processed.
    const uint64_t last_entry = max_entry;  // last valid index of sp_val / sp_row
    auto fetch = [&](Group &d, uint32_t w0) {
        const uint32_t ws = min(w0, w_hi);  // w0 >= w_hi: an empty group at w_hi
        d.nw = min((uint32_t)GROUP, w_hi - ws);
        d.lo = segb[ws];
        d.hi = segb[ws + d.nw];
#pragma unroll
        for (int j = 0; j < GROUP; ++j) {
            const uint32_t wj = min(ws + (uint32_t)j, w_hi - 1);
            d.bound[j] = segb[min(ws + (uint32_t)j + 1, ws + d.nw)];
            const uint64_t *cell = Oc + (uint64_t)wj * oc_word_stride + 4 * nib;
#pragma unroll
            for (int c = 0; c < 4; ++c) d.o[j][c] = cell[c];
        }
        const uint64_t k = min(d.lo + lane, last_entry);
        d.x = sp_val[k];
        d.r = sp_row[k];
    };

    // Tables and lookups of one group whose loads have arrived.
    auto process = [&](const Group &g) {
        if (g.lo == g.hi) return;  // uniform
        // nibble tables: lane l fills entries [nib][v0 + q] of each word's table
#pragma unroll
        for (int j = 0; j < GROUP; ++j) {
            if ((uint32_t)j >= g.nw) break;
#pragma unroll
            for (uint32_t q = 0; q < 4; ++q) {
                const uint32_t v = v0 + q;
                uint64_t e = (v & 1u) ? g.o[j][0] : 0ull;
                e |= (v & 2u) ? g.o[j][1] : 0ull;
                e |= (v & 4u) ? g.o[j][2] : 0ull;
                e |= (v & 8u) ? g.o[j][3] : 0ull;
                tab[j * 256 + nib * 16 + v] = e;
            }
        }
        // LDS instructions of a wavefront complete in issue order, so the
        // lookups below see the whole table; the barrier only stops the
        // compiler from moving LDS accesses across this point.
        __builtin_amdgcn_wave_barrier();
        auto lookup = [&](uint64_t k, uint64_t x, uint32_t r) {
            uint32_t j = 0;
#pragma unroll
            for (int q = 0; q + 1 < GROUP; ++q) j += k >= g.bound[q] ? 1u : 0u;
            const uint64_t *t = tab + j * 256;
            const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
            uint64_t a = 0;
#pragma unroll
            for (int n = 0; n < 8; ++n) a |= t[n * 16 + ((lo >> (4 * n)) & 0xFu)];
#pragma unroll
            for (int n = 0; n < 8; ++n) a |= t[(n + 8) * 16 + ((hi >> (4 * n)) & 0xFu)];
            if (a) __hip_atomic_fetch_or(acc + r, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        };
        // the first 64 entries were fetched with the group
        if (g.lo + lane < g.hi) lookup(g.lo + lane, g.x, g.r);
        // groups with more entries load the rest here
        for (uint64_t k = g.lo + 64 + lane; k < g.hi; k += 64) lookup(k, sp_val[k], sp_row[k]);
        __builtin_amdgcn_wave_barrier();  // the next group's tables overwrite these
    };

    // ping-pong between two groups so that one group's loads are in flight
    // while the other is processed
    const uint32_t step = WAVES * GROUP;
    Group A, B;
    fetch(A, w_lo + wave * GROUP);
    for (uint32_t w0 = w_lo + wave * GROUP; w0 < w_hi; w0 += 2 * step) {
        fetch(B, w0 + step);
        process(A);
        fetch(A, w0 + 2 * step);
        process(B);
    }
    __syncthreads();
    const uint64_t row0 = (uint64_t)rb * kRowBlock;
    uint64_t *Pw = P + (uint64_t)wr * p_stride + row0;
    for (uint32_t i = threadIdx.x; i < kRowBlock && row0 + i < n_traj; i += blockDim.x) Pw[i] = acc[i];
}

// One workgroup per tile of a single frame: tile = rb * n_wr + wr.
template <int WAVES, int GROUP>
__global__ void __launch_bounds__(64 * WAVES)
k_label_tiles(const uint64_t *__restrict__ seg, const uint16_t *__restrict__ sp_row,
              const uint64_t *__restrict__ sp_val, const uint64_t *__restrict__ Oc, uint64_t oc_word_stride,
              uint32_t n_words, uint32_t n_wr, uint32_t wr_words, uint64_t n_traj, uint64_t max_entry,
              uint64_t *__restrict__ P, uint64_t p_stride)
{
    extern __shared__ uint64_t lds[];
    tile_body<WAVES, GROUP>(seg, sp_row, sp_val, Oc, oc_word_stride, n_words, blockIdx.x / n_wr, blockIdx.x % n_wr,
                            wr_words, n_traj, max_entry, P, p_stride, lds);
}

// One workgroup per (pass, tile, lane group) of a batch.  The pass's cell
// masks are [w][G64][64] (cell-indexed), its partials [G64][n_wr][rows].
template <int WAVES, int GROUP>
__global__ void __launch_bounds__(64 * WAVES)
k_label_tiles_batch(const GroupDesc *__restrict__ groups, const TileItem *__restrict__ items)
{
    extern __shared__ uint64_t lds[];
    const TileItem it = items[blockIdx.x];
    const GroupDesc &g = groups[it.group];
    const uint64_t p_stride = (uint64_t)g.n_rb * kRowBlock;
    tile_body<WAVES, GROUP>(g.sp_seg, g.sp_row, g.sp_val, g.Ow + (uint64_t)it.gi * 64, (uint64_t)g.G64 * 64, g.n_words,
                            it.rb, it.wr, g.wr_words, g.n_traj, g.max_entry,
                            g.P + (uint64_t)it.gi * g.n_wr * p_stride, p_stride, lds);
}

// One wavefront per (pass, lane group, rows [row0, row1)): lane l holds the
// descriptor of column (gi, l); 64 rows at a time, lane j ORs the partials
// of row t0 + j, then every row's bits are broadcast and each lane writes its
// column's byte into its job's L.
__global__ void __launch_bounds__(64)
k_combine_batch(const GroupDesc *__restrict__ groups, const CombineItem *__restrict__ items)
{
    const uint32_t lane = threadIdx.x;
    const CombineItem it = items[blockIdx.x];
    const GroupDesc &g = groups[it.group];
    const LaneDesc d = g.lanes[it.gi * 64 + lane];
    const uint64_t p_stride = (uint64_t)g.n_rb * kRowBlock;
    const uint64_t *Pg = g.P + (uint64_t)it.gi * g.n_wr * p_stride;
    for (uint64_t t0 = it.row0; t0 < it.row1; t0 += 64) {
        const uint64_t t = t0 + lane;
        uint64_t bits = 0;
        if (t < it.row1)
            for (uint32_t r = 0; r < g.n_wr; ++r) bits |= Pg[(uint64_t)r * p_stride + t];
        const uint32_t n = (uint32_t)min<uint64_t>(64, it.row1 - t0);
        for (uint32_t j = 0; j < n; ++j) {
            const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)bits, j);
            const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(bits >> 32), j);
            const uint64_t b = ((uint64_t)hi << 32) | lo;
            if (d.L) d.L[(t0 + j) * d.n_props] = (uint8_t)((b >> lane) & 1ull);
        }
    }
}

__device__ __forceinline__ uint32_t spread_nib(uint32_t x) { return (x * 0x00204081u) & 0x01010101u; }

// One thread per row: OR of the row's partials (coalesced over rows), then
// the row's n_props label bytes.  16-byte stores when a row is whole 16-byte
// units, else 4-byte, else single bytes.
__global__ void __launch_bounds__(256)
k_combine(const uint64_t *__restrict__ P, uint64_t p_stride, uint32_t n_wr, uint64_t n_traj, uint32_t n_props,
          uint8_t *__restrict__ L)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const bool v16 = (n_props & 15u) == 0 && (reinterpret_cast<uintptr_t>(L) & 15u) == 0;
    const bool v4 = (n_props & 3u) == 0 && (reinterpret_cast<uintptr_t>(L) & 3u) == 0;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_traj; t += stride) {
        uint64_t bits = 0;
        uint32_t r = 0;
        for (; r + 4 <= n_wr; r += 4)
            bits |= P[(uint64_t)r * p_stride + t] | P[(uint64_t)(r + 1) * p_stride + t] |
                    P[(uint64_t)(r + 2) * p_stride + t] | P[(uint64_t)(r + 3) * p_stride + t];
        for (; r < n_wr; ++r) bits |= P[(uint64_t)r * p_stride + t];
        uint8_t *dst = L + t * n_props;
        if (v16) {
            for (uint32_t p = 0; p < n_props; p += 16) {
                const uint32_t b = (uint32_t)(bits >> p) & 0xFFFFu;
                *reinterpret_cast<uint4 *>(dst + p) = make_uint4(spread_nib(b & 0xFu), spread_nib((b >> 4) & 0xFu),
                                                                 spread_nib((b >> 8) & 0xFu), spread_nib(b >> 12));
            }
        } else if (v4) {
            for (uint32_t p = 0; p < n_props; p += 4)
                *reinterpret_cast<uint32_t *>(dst + p) = spread_nib((uint32_t)(bits >> p) & 0xFu);
        } else {
            for (uint32_t p = 0; p < n_props; ++p) dst[p] = (uint8_t)((bits >> p) & 1ull);
        }
    }
}

unsigned grid_cap(uint64_t items, unsigned per_block, unsigned cap)
{
    uint64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr size_t kTileLds = (kRowBlock + (size_t)kTileWaves * kWordGroup * 256) * sizeof(uint64_t);

}  // namespace

hipError_t launch_tiles_batch(const GroupDesc *d_groups, const TileItem *d_tiles, uint32_t n_tiles, hipStream_t s)
{
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL((k_label_tiles_batch<kTileWaves, kWordGroup>), dim3(n_tiles), dim3(64 * kTileWaves), kTileLds, s,
                       d_groups, d_tiles);
    return hipGetLastError();
}

hipError_t launch_combine_batch(const GroupDesc *d_groups, const CombineItem *d_items, uint32_t n_items, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(k_combine_batch, dim3(n_items), dim3(64), 0, s, d_groups, d_items);
    return hipGetLastError();
}

lbl_status build_sparse(lbl_abs *a)
{
    if (a->n_traj >= (1ull << 32)) return LBL_OK;  // row ids are 32-bit: keep only the bitpacked layout
    const uint32_t W = a->n_words;
    // 1. word-major entries (temporary)
    uint64_t *d_ptr = nullptr, *d_val = nullptr;
    uint32_t *d_row = nullptr;
    LBL_HIP_TRY(hipMalloc(&d_ptr, (size_t)(W + 1) * sizeof(uint64_t)));
    std::unique_ptr<uint64_t, decltype(&hipFree)> g_ptr(d_ptr, &hipFree);
    hipLaunchKernelGGL(k_wm_count, dim3((W + 7) / 8), dim3(512), 0, nullptr, a->T_bits, a->row_stride, a->n_traj, W,
                       d_ptr);
    LBL_HIP_TRY(hipGetLastError());
    std::vector<uint64_t> ptr(W + 1, 0);
    LBL_HIP_TRY(hipMemcpy(ptr.data(), d_ptr, W * sizeof(uint64_t), hipMemcpyDeviceToHost));
    uint64_t run = 0;
    for (uint32_t w = 0; w < W; ++w) {
        const uint64_t n = ptr[w];
        ptr[w] = run;
        run += n;
    }
    ptr[W] = run;
    LBL_REQUIRE(run == a->nonzero_words, "sparse layout: word counts disagree with the bitpacked T");
    const uint64_t nnz = run;
    LBL_HIP_TRY(hipMemcpy(d_ptr, ptr.data(), (size_t)(W + 1) * sizeof(uint64_t), hipMemcpyHostToDevice));
    LBL_HIP_TRY(hipMalloc(&d_row, std::max<uint64_t>(nnz, 1) * sizeof(uint32_t)));
    std::unique_ptr<uint32_t, decltype(&hipFree)> g_row(d_row, &hipFree);
    LBL_HIP_TRY(hipMalloc(&d_val, std::max<uint64_t>(nnz, 1) * sizeof(uint64_t)));
    std::unique_ptr<uint64_t, decltype(&hipFree)> g_val(d_val, &hipFree);
    hipLaunchKernelGGL(k_wm_fill, dim3((W + 7) / 8), dim3(512), 0, nullptr, a->T_bits, a->row_stride, a->n_traj, W,
                       d_ptr, d_row, d_val);
    LBL_HIP_TRY(hipGetLastError());

    // 2. tile geometry: ~1024 tiles, at least kTileWaves * kWordGroup words per tile
    SparseGeom g;
    g.n_rb = (uint32_t)((a->n_traj + kRowBlock - 1) / kRowBlock);
    const uint32_t min_words = kTileWaves * kWordGroup;
    uint32_t n_wr = std::max<uint32_t>(1, (1024 + g.n_rb - 1) / g.n_rb);
    n_wr = std::min<uint32_t>(n_wr, std::max<uint32_t>(1, W / min_words));
    g.wr_words = (W + n_wr - 1) / n_wr;
    g.n_wr = (W + g.wr_words - 1) / g.wr_words;

    // 3. segment counts -> offsets (host scan) -> tiled copy
    const uint64_t n_seg = (uint64_t)g.n_rb * W;
    uint32_t *d_cnt = nullptr;
    LBL_HIP_TRY(hipMalloc(&d_cnt, n_seg * sizeof(uint32_t)));
    std::unique_ptr<uint32_t, decltype(&hipFree)> g_cnt(d_cnt, &hipFree);
    hipLaunchKernelGGL(k_seg_count, dim3((unsigned)((n_seg + 255) / 256)), dim3(256), 0, nullptr, d_ptr, d_row, W,
                       g.n_rb, d_cnt);
    LBL_HIP_TRY(hipGetLastError());
    std::vector<uint32_t> cnt(n_seg);
    LBL_HIP_TRY(hipMemcpy(cnt.data(), d_cnt, n_seg * sizeof(uint32_t), hipMemcpyDeviceToHost));
    std::vector<uint64_t> seg(n_seg + 1, 0);
    for (uint64_t s = 0; s < n_seg; ++s) seg[s + 1] = seg[s] + cnt[s];
    LBL_REQUIRE(seg[n_seg] == nnz, "sparse layout: segment counts disagree with the word counts");
    LBL_HIP_TRY(hipMalloc(&a->sp_seg, (n_seg + 1) * sizeof(uint64_t)));
    LBL_HIP_TRY(hipMemcpy(a->sp_seg, seg.data(), (n_seg + 1) * sizeof(uint64_t), hipMemcpyHostToDevice));
    LBL_HIP_TRY(hipMalloc(&a->sp_row, std::max<uint64_t>(nnz, 1) * sizeof(uint16_t)));
    LBL_HIP_TRY(hipMalloc(&a->sp_val, std::max<uint64_t>(nnz, 1) * sizeof(uint64_t)));
    hipLaunchKernelGGL(k_seg_fill, dim3((unsigned)((n_seg + 255) / 256)), dim3(256), 0, nullptr, d_ptr, d_row, d_val, W,
                       g.n_rb, a->sp_seg, a->sp_row, a->sp_val);
    LBL_HIP_TRY(hipGetLastError());
    LBL_HIP_TRY(hipDeviceSynchronize());
    a->sp_nnz = nnz;
    a->sp_geom = g;
    return LBL_OK;
}

size_t swm_workspace_bytes(const lbl_abs *a, uint32_t n_lane_groups)
{
    const SparseGeom &g = a->sp_geom;
    return up256((size_t)a->n_words * 64 * n_lane_groups * sizeof(uint64_t)) +
           (size_t)n_lane_groups * g.n_wr * g.n_rb * kRowBlock * sizeof(uint64_t);
}

lbl_status run_swm(const lbl_abs *a, const uint8_t *O, uint32_t n_props, void *ws, uint8_t *L, hipStream_t s)
{
    LBL_REQUIRE(a->sp_seg != nullptr, "the abstraction has no sparse layout");
    const SparseGeom &g = a->sp_geom;
    uint64_t *Oc = static_cast<uint64_t *>(ws);
    uint64_t *P = Oc + up256((size_t)a->n_words * 64 * sizeof(uint64_t)) / sizeof(uint64_t);
    const uint64_t p_stride = (uint64_t)g.n_rb * kRowBlock;
    void *sp = span_begin(s);
    hipLaunchKernelGGL(k_pack_cells, dim3((unsigned)(((uint64_t)a->n_words * 64 + 255) / 256)), dim3(256), 0, s, O,
                       n_props, a->d_word_cell, a->n_words, Oc);
    LBL_HIP_TRY(hipGetLastError());
    span_end(sp, s, 0);
    sp = span_begin(s);
    hipLaunchKernelGGL((k_label_tiles<kTileWaves, kWordGroup>), dim3((unsigned)g.n_tiles()), dim3(64 * kTileWaves),
                       kTileLds, s, a->sp_seg, a->sp_row, a->sp_val, Oc, (uint64_t)64, a->n_words, g.n_wr, g.wr_words,
                       a->n_traj, std::max<uint64_t>(a->sp_nnz, 1) - 1, P, p_stride);
    LBL_HIP_TRY(hipGetLastError());
    span_end(sp, s, 1);
    sp = span_begin(s);
    hipLaunchKernelGGL(k_combine, dim3(grid_cap(a->n_traj, 256, 16384)), dim3(256), 0, s, P, p_stride, g.n_wr,
                       a->n_traj, n_props, L);
    LBL_HIP_TRY(hipGetLastError());
    span_end(sp, s, 3);
    return LBL_OK;
}

}  // namespace lbl
