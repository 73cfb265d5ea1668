// Sparse tiled layout of T and its labeling kernels.
//
// Layout.  Every non-zero 64-cell word of T becomes one entry (local row,
// word value).  Entries are grouped into segments (row block rb, word w):
// the rows of block rb (kRowBlock rows) whose swept set meets word w,
// ascending; only non-empty segments exist, stored in (rb, w) order, so the
// entries of one row block are contiguous.  This is the compressed-sparse
// idea of Sec. 4.3 (store only the true entries of M) at word granularity,
// ordered so that the frame data a word needs is prepared once per row
// block and shared by every trajectory of the block that crosses it.
//
// Tilings (built on the host at load time).  A row block's entries are cut
// into wavefront tasks by the cost of the rounds walked (a round plus a
// charge per table copy), kTileWaves tasks to a tile (one workgroup), each
// task sized to its wavefront's issue share (wave_share).  A task is walked in
// rounds of 64 consecutive entries, one per lane; a round whose entries
// span more than two segments is split so that each round touches at most
// two.  Each round carries which lanes are active, which lanes fall in its
// second segment, and which of its segments' tables must be built first.
//
// Per frame:
//   k_pack_tables  O -> the nibble tables of every word that some entry
//                  holds: entry [n][v] is the OR of the proposition masks of
//                  the cells 4n + b with bit b of v set (16 x 16 uint64 per
//                  word, one wavefront per word).
//   k_label_tiles  one workgroup per tile.  A wavefront keeps two segments'
//                  tables in LDS, copying a segment's tables in when a round
//                  first reaches it (at most one copy per round); every
//                  active lane ORs the 16 entries selected by the nibbles of
//                  its word value (the labels of that (row, word) pair for up
//                  to 64 propositions) into the tile's per-row accumulators
//                  with an LDS atomic.  Two rounds are in flight per
//                  wavefront (loads issued ahead of the round processed).
//                  The accumulators are written once per tile as its partial
//                  labels.
//   k_combine      OR of a row's partials over the tiles of its row block ->
//                  the caller's L bytes (0/1).
// Frames of at most 4 propositions take two other kernels instead:
//   k_pack_masks   O -> NP proposition masks per used word (bit b = cell b);
//                  the grid also zeroes L.
//   k_label_direct one workgroup per tile of equal chunk count: a label bit
//                  is (word value AND mask) != 0, with the masks of the
//                  tile's segments staged in LDS; the tile stores 1 into L's
//                  bytes for the bits its rows' accumulators hold.
// OR is idempotent and commutative, so neither the order of the LDS atomics
// nor the split into tiles changes the result.  No global atomics are used.
#include <algorithm>
#include <cmath>
#include <queue>

#include "batch.h"
#include "profile.h"
#include "sparse.h"
#include "tables.h"

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

// Native vector types: loads and stores of these through address-space
// qualified pointers compile (HIP's vector structs assign only in the
// generic address space).
typedef unsigned long long v2u64 __attribute__((ext_vector_type(2)));
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));


// One wavefront per word, one lane per cell: the mask of the propositions
// cell (w, lane) meets, then the word's nibble tables Tg[w * 256 ..].
// Wavefront i packs word words[i], or word i when words is null (only words
// that some entry of the layout holds need tables), whose first cell is
// first[i] (read once per wavefront, with no load before it): with row-major
// cell ids lane b's cell lies dy rows and dx columns from it, x taking the
// odd bits of b; with z-order ids (morton) it is first + b.
__device__ __forceinline__ uint64_t word_lane_cell(const uint32_t *__restrict__ first, uint32_t i, uint32_t lane,
                                                   uint32_t nx, uint32_t morton)
{
    const uint32_t dx = ((lane >> 1) & 1u) | ((lane >> 2) & 2u) | ((lane >> 3) & 4u);
    const uint32_t dy = (lane & 1u) | ((lane >> 1) & 2u) | ((lane >> 2) & 4u);
    return (uint64_t)first[i] + (morton ? (uint64_t)lane : (uint64_t)dy * nx + dx);
}

// Lane b's mask of the propositions cell b of packed word i meets (cell b as
// word_lane_cell places it).  When n_props is 16, 32 or 64 and O is 16-byte
// aligned, the wavefront reads the word's frame bytes in 16-byte units taken
// in memory order (each row of 8 cells, or with z-order ids the whole word,
// is one contiguous run of O), so that a load instruction covers whole cache
// lines instead of a 16-byte piece of 64 different cells; each unit's 16 bits
// go to their cell's place in the wavefront's 512-byte stage, from which lane
// b then reads cell b.  Otherwise every lane reads its own cell's bytes.
__device__ __forceinline__ uint64_t word_cell_mask(const uint8_t *__restrict__ O, uint32_t n_props,
                                                   const uint32_t *__restrict__ first, uint32_t i, uint32_t lane,
                                                   uint32_t nx, uint32_t morton, uint64_t *stage)
{
    if (!((n_props == 16 || n_props == 32 || n_props == 64) && (reinterpret_cast<uintptr_t>(O) & 15u) == 0))
        return byte_mask(O + word_lane_cell(first, i, lane, nx, morton) * n_props, n_props);
    const uint32_t sh = n_props == 16 ? 0u : n_props == 32 ? 1u : 2u;  // log2 of a cell's units
    const uint32_t last = (1u << sh) - 1u;                               // loads per lane - 1
    const uint64_t c0 = first[i];
    uint4 q[4];
    uint32_t at[4];
    // all loads first (the clamped repeats stay in bounds and are not used)
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t u = lane + 64u * min(j, last);   // unit of the word in memory order
        const uint32_t k = u >> sh, part = u & last;    // its cell in memory order, its part
        const uint32_t x = k & 7u, y = k >> 3;          // the cell's place in the word's 8 x 8 block
        const uint64_t cell = c0 + (morton ? (uint64_t)k : (uint64_t)y * nx + x);
        q[j] = *reinterpret_cast<const uint4 *>(O + cell * n_props + 16u * part);
        const uint32_t b = morton ? k
                                  : (y & 1u) | ((x & 1u) << 1) | ((y & 2u) << 1) | ((x & 2u) << 2) | ((y & 4u) << 2) |
                                        ((x & 4u) << 3);
        at[j] = 4u * b + part;  // 16-bit slot of the unit's bits in the stage
    }
    // LDS accesses of one wavefront complete in issue order: the zeroing
    // precedes the unit stores, which precede the reads (the barriers only
    // keep the compiler from moving accesses across them)
    stage[lane] = 0;
    __builtin_amdgcn_wave_barrier();
    uint16_t *s16 = reinterpret_cast<uint16_t *>(stage);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
        if (j <= last) s16[at[j]] = (uint16_t)nz_bytes16(q[j]);
    __builtin_amdgcn_wave_barrier();
    const uint64_t m = stage[lane];
    __builtin_amdgcn_wave_barrier();
    return m;
}

template <typename M>
__global__ void __launch_bounds__(256)
k_pack_tables(const uint8_t *__restrict__ O, uint32_t n_props, const uint32_t *__restrict__ first, uint32_t nx,
              uint32_t morton, const uint32_t *__restrict__ words, uint32_t n_items, M *__restrict__ Tg)
{
    __shared__ uint64_t stage[4][64];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t i = blockIdx.x * 4 + wave;
    if (i >= n_items) return;  // whole wavefronts
    const uint32_t w = words ? words[i] : i;
    const uint64_t mask = word_cell_mask(O, n_props, first, i, lane, nx, morton, stage[wave]);
    if constexpr (sizeof(M) == 8)
        write_tables(mask, Tg + (uint64_t)w * 256, lane);
    else
        write_tables32((uint32_t)mask, Tg + (uint64_t)w * 256, lane);
}


// Frames of at most NP <= 4 propositions: one wavefront per word, lane b
// holding cell b of packed word i as in k_pack_tables; the word's NP proposition masks
// Tm[w * NP + p] (bit b set iff cell b meets proposition p; zero for
// p >= n_props), lane p writing mask p.  The grid also zeroes the frame's
// n_L label bytes at L, which the label kernel then sets where true.
template <int NP>
__global__ void __launch_bounds__(256)
k_pack_masks(const uint8_t *__restrict__ O, uint32_t n_props, const uint32_t *__restrict__ first, uint32_t nx,
             uint32_t morton, const uint32_t *__restrict__ words, uint32_t n_items, uint64_t *__restrict__ Tm,
             uint8_t *__restrict__ L, uint64_t n_L)
{
    {
        // L in 16-byte units from its first aligned byte, the ends byte by byte
        const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
        const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
        const uint64_t head = min<uint64_t>((16 - (reinterpret_cast<uintptr_t>(L) & 15u)) & 15u, n_L);
        const uint64_t n16 = (n_L - head) / 16;
        const uint64_t tail = head + 16 * n16;
        if (tid < head) L[tid] = 0;
        if (tid < n_L - tail) L[tail + tid] = 0;
        v4u32 *body = reinterpret_cast<v4u32 *>(L + head);
        for (uint64_t i = tid; i < n16; i += stride) body[i] = v4u32{0u, 0u, 0u, 0u};
    }
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i >= n_items) return;  // whole wavefronts
    const uint32_t w = words ? words[i] : i;
    const uint64_t cell = word_lane_cell(first, i, lane, nx, morton);
    const uint64_t mine = byte_mask(O + cell * n_props, n_props);
    uint64_t mp = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const uint64_t b = __ballot((mine >> p) & 1ull);
        mp = lane == (uint32_t)p ? b : mp;
    }
    if (lane < (uint32_t)NP) Tm[(uint64_t)w * NP + lane] = mp;
}

// base + byte K of bytes, in one instruction (the byte is selected as an
// operand, not extracted first).
template <int K>
__device__ __forceinline__ uint32_t add_byte(uint32_t base, uint32_t bytes)
{
    uint32_t r;
    if constexpr (K == 0)
        asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_0 src1_sel:DWORD"
            : "=v"(r) : "v"(bytes), "v"(base));
    else if constexpr (K == 1)
        asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_1 src1_sel:DWORD"
            : "=v"(r) : "v"(bytes), "v"(base));
    else if constexpr (K == 2)
        asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_2 src1_sel:DWORD"
            : "=v"(r) : "v"(bytes), "v"(base));
    else
        asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_3 src1_sel:DWORD"
            : "=v"(r) : "v"(bytes), "v"(base));
    return r;
}

// Lane l gets b where bit l of mask (wavefront-uniform) is set, else a: one
// v_cndmask with the mask read from a scalar register pair.
__device__ __forceinline__ uint32_t select_by_lane(uint64_t mask, uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(mask));
    return r;
}

// Entry (of mask type M) of table row q at LDS byte address
// addr + q * kTabRow * sizeof(M).
template <typename M>
__device__ __forceinline__ M lds_entry(uint32_t addr, int q)
{
    return *reinterpret_cast<__attribute__((address_space(3))) const M *>(
        static_cast<uintptr_t>(addr + q * kTabRow * sizeof(M)));
}

// LDS byte address of p.
__device__ __forceinline__ uint32_t lds_addr(const void *p)
{
    return (uint32_t)reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) const uint8_t *)p);
}

// A raw buffer resource over device memory from p, its base made
// wavefront-uniform (buffer loads take the resource in scalar registers):
// no stride and the largest record count, so that no offset below 4 GiB is
// treated as out of range (gfx9 resource word 3).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(const void *p)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint64_t u = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a) |
                       ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32)) << 32);
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void *>(u), 0, -1, 0x00020000);
}

// Dwords of one word's nibble tables a lane holds while copying them:
// 4 entries of M, 32 bytes (64-bit masks) or 16 (32-bit).
template <typename M>
constexpr uint32_t kTbDwords = sizeof(M);  // 4 entries x sizeof(M) / 4 bytes

// Copy of one word's nibble tables (as written by write_tables) into an LDS
// table slot whose rows are kTabRow entries apart; lane l holds entries
// 4l .. 4l + 3 (row l / 4) in tb.
template <typename M>
__device__ __forceinline__ void copy_tables(const v4u32 (&tb)[kTbDwords<M> / 4], M *t, uint32_t lane)
{
    M *e = t + (lane >> 2) * kTabRow + (lane & 3u) * 4;
    if constexpr (sizeof(M) == 8) {
        e[0] = (uint64_t)tb[0].x | ((uint64_t)tb[0].y << 32);
        e[1] = (uint64_t)tb[0].z | ((uint64_t)tb[0].w << 32);
        e[2] = (uint64_t)tb[1].x | ((uint64_t)tb[1].y << 32);
        e[3] = (uint64_t)tb[1].z | ((uint64_t)tb[1].w << 32);
    } else {
        e[0] = tb[0].x;
        e[1] = tb[0].y;
        e[2] = tb[0].z;
        e[3] = tb[0].w;
    }
}

// One tile: its wavefronts walk their tasks, OR-ing labels into the row
// block's accumulators (M)lds[0 .. kRowBlock), which hold the tile's labels
// when it returns (after a workgroup barrier).  Tg + w * tg_stride holds the
// 256 nibble-table entries of word w.  M is the label mask: uint64_t for up
// to 64 propositions, uint32_t for up to 32 (half the table and accumulator
// bytes, half the LDS bytes per lookup).
template <int WAVES, typename M>
__device__ __forceinline__ void tile_accumulate(const SpTask *__restrict__ wg_tasks,
                                                const SpRound *__restrict__ rounds,
                                                const uint16_t *__restrict__ sp_row,
                                                const uint64_t *__restrict__ sp_val, const M *__restrict__ Tg,
                                                uint64_t tg_stride, void *lds)
{
    const uint32_t lane = threadIdx.x & 63;
    // uniform across the wavefront: task fields and round records become
    // scalars and the per-round branches scalar branches
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    M *acc = static_cast<M *>(lds);                       // kRowBlock accumulators
    M *tab = acc + kRowBlock + wave * (kRing * kTabWords);  // this wavefront's two tables
    // Every array read here is device memory.  The batch path takes these
    // pointers from its descriptors in memory, where the compiler cannot see
    // their address space: without the casts (or the buffer resources below)
    // it would issue flat loads, which count on the LDS wait counter too, so
    // that every wait for the LDS would also wait for them.  The task's
    // fields are moved to scalar registers for the same reason (loads
    // through such pointers land in vector registers).
    typedef __attribute__((address_space(1))) const uint32_t gu32;
    constexpr uint32_t kTbN = kTbDwords<M> / 4;  // 16-byte loads of table data per lane
    const gu32 *task = (const gu32 *)(wg_tasks + wave);
    const uint64_t tk_lo = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)task[0]) |
                           ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)task[1]) << 32);
    const uint32_t n = (uint32_t)__builtin_amdgcn_readfirstlane((int)task[2]);
    const uint32_t round0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)task[3]);
    static_assert(sizeof(SpTask) == 16, "task layout: lo, n_rounds, round0");
    {
        struct Stage {
            uint32_t rec;      // lanes 0-3: the record of the stage's next round
            uint32_t meta;
            uint64_t x;        // this lane's word value
            uint32_t r;        // its local row (zero-extended when loaded)
            v4u32 tb[kTbN];    // this lane's 32 (or 16) bytes of the table the round builds
        };
        // kStages rounds are in flight: round i is fetched (its entries and
        // table data loaded) kStages - 1 rounds before it is processed, and
        // its record (lane l, l < 4, holding word l) kStages rounds before
        // that fetch, so neither wait is on the round's critical path.  A
        // scalar load of the record would instead make every LDS wait also
        // wait for it (the two share one counter).  Every vector load is
        // unconditional and in bounds (the entry arrays carry 64 entries of
        // padding past the last one, and the record index is clamped), since
        // branches around loads would make the compiler wait for all of them;
        // validity is applied when the round is processed.
        // The loads go through raw buffer resources built in scalar registers
        // (a uniform base, a per-lane offset fixed for the walk, and the
        // round's uniform offset added by the load itself): no per-lane
        // address arithmetic in the loop.
        const __amdgpu_buffer_rsrc_t r_rec = uniform_rsrc(rounds + round0);
        const __amdgpu_buffer_rsrc_t r_val = uniform_rsrc(sp_val + tk_lo);
        const __amdgpu_buffer_rsrc_t r_row = uniform_rsrc(sp_row + tk_lo);
        const uint32_t o_rec = (lane & 3u) * 4u, o_val = lane * 8u, o_row = lane * 2u, o_tab = lane * kTbN * 16u;
        auto load_rec = [&](uint32_t i) {
            return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r_rec, (int)o_rec, (int)(min(i, n - 1) * 16u), 0);
        };
        static_assert(sizeof(SpRound) == 16, "a round record is four dwords");
        auto fetch = [&](Stage &st, uint32_t i) {
            // the fields are read before the register is reloaded, so that the
            // reload can take the same register (no copy waiting for it)
            const uint32_t e_off = (uint32_t)__builtin_amdgcn_readlane((int)st.rec, 0);
            const uint32_t tword = (uint32_t)__builtin_amdgcn_readlane((int)st.rec, 1);
            st.meta = (uint32_t)__builtin_amdgcn_readlane((int)st.rec, 3);
            st.rec = load_rec(i + kStages);
            st.x = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r_val, (int)o_val, (int)(e_off * 8u), 0));
            st.r = __builtin_amdgcn_raw_buffer_load_b16(r_row, (int)o_row, (int)(e_off * 2u), 0);
            // a round that builds no table loads one line for the whole
            // wavefront (still unconditionally): the 2 KiB of its last table
            // would mostly come from L2, the 16 wavefronts' last tables
            // filling the CU's L1
            const __amdgpu_buffer_rsrc_t r_tab = uniform_rsrc(Tg + (uint64_t)tword * tg_stride);
            const uint32_t tl = (st.meta & (kMetaBuild0 | kMetaBuild1)) ? o_tab : 0u;
#pragma unroll
            for (uint32_t k = 0; k < kTbN; ++k)
                st.tb[k] = __builtin_amdgcn_raw_buffer_load_b128(r_tab, (int)tl, (int)(16u * k), 0);
        };

        // the two slot addresses live in vector registers for the whole walk
        uint32_t slot_a, slot_b;
        asm("v_mov_b32 %0, %1" : "=v"(slot_a) : "s"(lds_addr(tab)));
        asm("v_mov_b32 %0, %1" : "=v"(slot_b) : "s"(lds_addr(tab) + kTabWords * (uint32_t)sizeof(M)));
        auto process = [&](const Stage &st) {
            const uint32_t meta = st.meta;
            const uint32_t s0 = (meta & kMetaSlot0) ? 1u : 0u;
            if (meta & (kMetaBuild0 | kMetaBuild1))
                copy_tables<M>(st.tb, tab + (s0 ^ ((meta & kMetaBuild1) ? 1u : 0u)) * kTabWords, lane);
            // LDS instructions of a wavefront complete in issue order, so the
            // lookups below see the whole table; the barrier only stops the
            // compiler from moving LDS accesses across this point.
            __builtin_amdgcn_wave_barrier();
            const uint32_t lane_lo = meta & 0xFFu, lane_hi = (meta >> 8) & 0xFFu, cut = (meta >> 16) & 0xFFu;
            // lanes below cut read slot s0, the others slot s0 ^ 1: the lane
            // mask of slot-b readers is formed in scalar registers
            const uint64_t upper = cut >= 64 ? 0ull : (~0ull << cut);
            const uint32_t tb = select_by_lane(s0 ? ~upper : upper, slot_a, slot_b);
            {
                // every lane looks up its word value (an address inside the
                // slot whatever the value); lanes outside [lane_lo, lane_hi)
                // then drop their result, which costs less than a branch.
                // Byte k of ev (od) is sizeof(M) x nibble 2k (2k + 1) of the
                // word value: the byte offset of its entry in the table row
                constexpr uint32_t sh = sizeof(M) == 8 ? 3 : 2;
                const uint64_t m = 0x0F0F0F0F0F0F0F0Full << sh;
                const uint64_t ev = (st.x << sh) & m, od = (st.x >> (4 - sh)) & m;
                const uint32_t e[2] = {(uint32_t)ev, (uint32_t)(ev >> 32)};
                const uint32_t o[2] = {(uint32_t)od, (uint32_t)(od >> 32)};
                // all sixteen reads are issued before the first result is used
                M q[16];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    q[8 * h + 0] = lds_entry<M>(add_byte<0>(tb, e[h]), 8 * h + 0);
                    q[8 * h + 1] = lds_entry<M>(add_byte<0>(tb, o[h]), 8 * h + 1);
                    q[8 * h + 2] = lds_entry<M>(add_byte<1>(tb, e[h]), 8 * h + 2);
                    q[8 * h + 3] = lds_entry<M>(add_byte<1>(tb, o[h]), 8 * h + 3);
                    q[8 * h + 4] = lds_entry<M>(add_byte<2>(tb, e[h]), 8 * h + 4);
                    q[8 * h + 5] = lds_entry<M>(add_byte<2>(tb, o[h]), 8 * h + 5);
                    q[8 * h + 6] = lds_entry<M>(add_byte<3>(tb, e[h]), 8 * h + 6);
                    q[8 * h + 7] = lds_entry<M>(add_byte<3>(tb, o[h]), 8 * h + 7);
                }
                __builtin_amdgcn_sched_group_barrier(0x100, 16, 0);  // the sixteen LDS reads first
                M a = 0;
#pragma unroll
                for (int k = 0; k < 16; ++k) a |= q[k];
                const uint64_t below_hi = lane_hi >= 64 ? ~0ull : ((1ull << lane_hi) - 1ull);
                const uint64_t act = below_hi & (~0ull << lane_lo);
                if constexpr (sizeof(M) == 8)
                    a = ((uint64_t)select_by_lane(act, 0u, (uint32_t)(a >> 32)) << 32) |
                        select_by_lane(act, 0u, (uint32_t)a);
                else
                    a = select_by_lane(act, 0u, a);
                // zero results are skipped: an OR of zero still costs LDS time
                if (a) __hip_atomic_fetch_or(acc + st.r, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            __builtin_amdgcn_wave_barrier();  // later builds overwrite these tables
            // the table data counts as used here even when no table was
            // built, so that its registers are not reused while its loads are
            // in flight (which would make the next fetch wait for every load)
#pragma unroll
            for (uint32_t k = 0; k < kTbN; ++k)
                asm volatile("" ::"v"(st.tb[k].x), "v"(st.tb[k].y), "v"(st.tb[k].z), "v"(st.tb[k].w));
        };

        // the stages in rotation.  When n is not a multiple of kStages the
        // last round is processed again (fetch clamps to it), which changes
        // nothing: its tables are rebuilt with the same contents and OR is
        // idempotent.
        // the first rounds' loads are issued before the accumulators are
        // cleared, so that their latency overlaps the clearing and the
        // barrier
        Stage st[kStages];
        if (n > 0) {
#pragma unroll
            for (int k = 0; k < kStages; ++k) st[k].rec = load_rec(k);
#pragma unroll
            for (int k = 0; k + 1 < kStages; ++k) fetch(st[k], k);
        }
        for (uint32_t i = threadIdx.x; i < kRowBlock * sizeof(M) / 16; i += 64 * WAVES)
            reinterpret_cast<v4u32 *>(acc)[i] = v4u32{0u, 0u, 0u, 0u};
        __syncthreads();
        for (uint32_t i = 0; i < n; i += kStages) {
#pragma unroll
            for (int k = 0; k < kStages; ++k) {
                fetch(st[(k + kStages - 1) % kStages], i + k + kStages - 1);
                process(st[k]);
            }
        }
    }
    __syncthreads();
}

// The tile's accumulators as its partials: every row of the block at
// Pt[0 .. kRowBlock), or (compact) only the n_slot rows slot_row[..] it
// touches at Pt[0 .. n_slot).  Streaming stores: the partials are read once,
// by the combine kernel.
template <int WAVES, typename M>
__device__ __forceinline__ void write_partials(const void *lds, M *Pt)
{
    // device memory (the batch's pointer comes from its descriptors)
    typedef __attribute__((address_space(1))) v4u32 gv4;
    const v4u32 *acc = static_cast<const v4u32 *>(lds);
    gv4 *dst = (gv4 *)Pt;
    for (uint32_t i = threadIdx.x; i < kRowBlock * sizeof(M) / 16; i += 64 * WAVES)
        __builtin_nontemporal_store(acc[i], dst + i);
}

template <int WAVES, typename M>
__device__ __forceinline__ void write_partials_compact(const void *lds, M *__restrict__ Pt,
                                                       const uint16_t *__restrict__ slot_row, uint32_t n_slot)
{
    // device memory (the batch's pointers come from its descriptors)
    typedef __attribute__((address_space(1))) M gm;
    typedef __attribute__((address_space(1))) const uint16_t gu16;
    const M *acc = static_cast<const M *>(lds);
    gm *dst = (gm *)Pt;
    const gu16 *rows = (const gu16 *)slot_row;
    for (uint32_t k = threadIdx.x; k < n_slot; k += 64 * WAVES) __builtin_nontemporal_store(acc[rows[k]], dst + k);
}

// One workgroup per tile of a single frame: workgroup b runs tile
// block_tile[b], whose tasks tasks_launch holds at b * WAVES (no dependent
// load before the first task).  Partials P[tile][kRowBlock].
// With 32-bit masks a workgroup takes half the LDS, and two share a CU.
template <int WAVES, typename M>
__global__ void __launch_bounds__(64 * WAVES, sizeof(M) == 8 ? 1 : 2)
k_label_tiles(const uint32_t *__restrict__ block_tile, const SpTask *__restrict__ tasks_launch,
              const SpRound *__restrict__ rounds, const uint16_t *__restrict__ sp_row,
              const uint64_t *__restrict__ sp_val, const M *__restrict__ Tg, M *__restrict__ P,
              const uint32_t *__restrict__ tile_slot, const uint16_t *__restrict__ slot_row)
{
    extern __shared__ uint64_t lds[];
    const uint32_t tile = block_tile[blockIdx.x];
    tile_accumulate<WAVES, M>(tasks_launch + (uint64_t)blockIdx.x * WAVES, rounds, sp_row, sp_val, Tg, 256, lds);
    if (tile_slot) {
        const uint32_t s0 = tile_slot[tile], s1 = tile_slot[tile + 1];
        write_partials_compact<WAVES, M>(lds, P + s0, slot_row + s0, s1 - s0);
    } else {
        write_partials<WAVES, M>(lds, P + (uint64_t)tile * kRowBlock);
    }
}

// Frames of at most NP <= 4 propositions (the direct-mask kernel).  A label
// needs no nibble table here: bit p of an entry's label is (word value AND
// mask p of its word) != 0, with the masks Tm[word * NP + p] written by
// k_pack_masks.  Nor does a tile walk its entries by segment: the layout's
// 64-entry chunks are cut into tiles of equal chunk counts (so that tiles
// take equal time, whatever the row blocks' sizes), and a tile's chunks in
// one row block (a part) are dealt to its wavefronts in turn (chunk j to
// wavefront j % WAVES), so that the 16 wavefronts read consecutive 1 KiB
// pieces of the entry arrays together.  Per part: the masks of the part's
// segments are copied into LDS (segment i at msk[i * NP]); lane l of a chunk
// takes entry e0 + 64 j + l, whose segment is the chunk's first plus the
// start bits below l (a masked bit count), and ORs its label into the row's
// 32-bit LDS accumulator; then every row of the block with a non-zero
// accumulator gets a 1 in its label byte for each set bit.  L was zeroed by
// k_pack_masks, and the tiles sharing a row only ever store 1 into its
// bytes, so the label bytes need no combine step (concurrent stores of the
// same value to a byte are benign; stores to neighbouring bytes do not
// interfere).
//
// Only the chunk records and the entries come from memory in the chunk
// loop, all of them kDirectAhead chunks before they are processed (vector
// loads complete in issue order, and nothing waits on a later load): every
// load is unconditional and in bounds (indices clamp to the wavefront's last
// chunk of the part, the entry arrays carry kEntryPad entries of padding);
// only the processing of chunks past the last is skipped.
constexpr int kDirectAhead = 5;
// LDS of a direct-mask workgroup: the accumulators and up to
// kDirectMaskBytes of segment masks, so that two workgroups share a CU.
constexpr size_t kDirectMaskBytes = 48 * 1024;
constexpr size_t kDirectLds = kRowBlock * sizeof(uint32_t) + kDirectMaskBytes;

template <int WAVES, int NP>
__global__ void __launch_bounds__(64 * WAVES, 2)
k_label_direct(const uint32_t *__restrict__ tile_part, const DirectPart *__restrict__ parts,
               const SpChunk *__restrict__ chunks, const uint32_t *__restrict__ seg_word,
               const uint16_t *__restrict__ sp_row, const uint64_t *__restrict__ sp_val,
               const uint64_t *__restrict__ Tm, uint64_t n_traj, uint32_t n_props, uint8_t *__restrict__ L)
{
    static_assert(NP == 1 || NP == 2 || NP == 4, "direct masks: 1, 2 or 4 per word");
    constexpr int R = kDirectAhead + 1;
    extern __shared__ uint64_t lds[];
    uint32_t *acc = reinterpret_cast<uint32_t *>(lds);
    uint64_t *msk = lds + kRowBlock / 2;
    typedef __attribute__((address_space(1))) const uint32_t gu32;
    typedef __attribute__((address_space(1))) const uint16_t gu16;
    typedef __attribute__((address_space(1))) const uint64_t gu64;
    typedef __attribute__((address_space(3))) const uint64_t lu64;
    static_assert(sizeof(SpChunk) == 16, "a chunk record is four dwords");
    static_assert(sizeof(DirectPart) == 32, "a part record is eight dwords");
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t p0 = tile_part[blockIdx.x], p1 = tile_part[blockIdx.x + 1];
    for (uint32_t pi = p0; pi < p1; ++pi) {
        const DirectPart part = parts[pi];
        // chunks wave, wave + WAVES, ... of the part
        const uint32_t nc = part.c1 - part.c0;
        const uint32_t n = nc > wave ? (nc - wave + WAVES - 1) / WAVES : 0u;
        const gu32 *recs = (const gu32 *)(chunks + part.c0 + wave);
        const gu64 *vals = (const gu64 *)(sp_val + part.e0 + 64ull * wave);
        const gu16 *rows = (const gu16 *)(sp_row + part.e0 + 64ull * wave);

        struct Stage {
            uint32_t rec;  // lanes 0-3: the chunk's record
            uint64_t x;    // this lane's word value
            uint16_t r;    // its local row
        };
        Stage st[R];
        const uint32_t last = n ? n - 1 : 0u;
        auto fetch = [&](Stage &q, uint32_t k) {
            const uint32_t kk = min(k, last);
            q.rec = recs[(uint64_t)kk * (4 * WAVES) + (lane & 3u)];
            const uint64_t o = (uint64_t)kk * (64 * WAVES);
            q.x = (vals + o)[lane];
            q.r = (rows + o)[lane];
        };
        auto process = [&](const Stage &q) {
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)q.rec, 0);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)q.rec, 1);
            const uint32_t s0 = (uint32_t)__builtin_amdgcn_readlane((int)q.rec, 2);
            const uint32_t nv = (uint32_t)__builtin_amdgcn_readlane((int)q.rec, 3);
            const uint32_t seg = s0 + __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
            const lu64 *m = (const lu64 *)(msk + seg * NP);
            uint32_t a = 0;
#pragma unroll
            for (int p = 0; p < NP; ++p) a |= (uint32_t)((q.x & m[p]) != 0ull) << p;
            if (lane < nv && a) __hip_atomic_fetch_or(acc + q.r, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        };

        // the first chunks' loads are issued before the accumulators are
        // cleared and the masks copied (a wavefront without chunks loads
        // nothing: its clamped indices would point past the part)
        if (n > 0) {
#pragma unroll
            for (int k = 0; k < kDirectAhead; ++k) fetch(st[k], k);
        }
        for (uint32_t i = threadIdx.x; i < kRowBlock / 4; i += 64 * WAVES)
            reinterpret_cast<v4u32 *>(acc)[i] = v4u32{0u, 0u, 0u, 0u};
        for (uint32_t i = threadIdx.x; i < part.n_seg; i += 64 * WAVES) {
            const gu64 *src = (const gu64 *)(Tm + (uint64_t)seg_word[part.seg_first + i] * NP);
#pragma unroll
            for (int p = 0; p < NP; ++p) msk[i * NP + p] = src[p];
        }
        __syncthreads();
        for (uint32_t k0 = 0; k0 < n; k0 += R) {
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const uint32_t k = k0 + u;
                fetch(st[(u + kDirectAhead) % R], k + kDirectAhead);
                if (k < n) process(st[u]);
            }
        }
        __syncthreads();
        // the part's labels: a 1 for every set bit of a non-zero accumulator
        const uint64_t t0 = (uint64_t)part.rb * kRowBlock;
        for (uint32_t r = threadIdx.x; r < kRowBlock; r += 64 * WAVES) {
            const uint32_t v = acc[r];
            if (v && t0 + r < n_traj) {
                __attribute__((address_space(1))) uint8_t *dst =
                    (__attribute__((address_space(1))) uint8_t *)(L + (t0 + r) * n_props);
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    if ((v >> p) & 1u) dst[p] = 1;
            }
        }
        __syncthreads();  // the accumulators and masks are reused by the next part
    }
}

// OR of row t's compact partials: slots row_slots[row_slot_off[t] ..
// row_slot_off[t + 1]), four loads in flight (indices past the last slot read
// it again, which leaves the OR unchanged; a row no tile touches has none).
template <typename M>
__device__ __forceinline__ uint64_t row_slots_or(const M *__restrict__ P, const uint32_t *__restrict__ off,
                                                 const uint32_t *__restrict__ slots, uint64_t t)
{
    // device memory (the batch's pointers come from its descriptors)
    typedef __attribute__((address_space(1))) const M gm;
    typedef __attribute__((address_space(1))) const uint32_t gu32;
    const gm *Pg = (const gm *)P;
    const gu32 *og = (const gu32 *)off, *sg = (const gu32 *)slots;
    const uint32_t k0 = og[t], k1 = og[t + 1];
    uint64_t bits = 0;
    for (uint32_t kb = k0; kb < k1; kb += 4) {
        M v[4];
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) v[j] = Pg[sg[min(kb + j, k1 - 1)]];
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) bits |= v[j];
    }
    return bits;
}

// The label bytes of rows [t0, t0 + n) of one job (n <= 64), written as one
// contiguous block L[t0 * np .. (t0 + n) * np): lane r holds the job's bits
// of row t0 + r in v (bit p = proposition p).  The block is staged in LDS at
// its offset modulo 16 (each lane ORs its row's bytes into 4-byte-aligned
// words; neighbouring rows share the words at their boundary), then written
// with 16-byte stores; the units at the block's two ends, which also hold
// bytes of other rows, are written byte by byte, so no byte outside the
// block is stored.  stage: 64 * 64 + 32 bytes of this wavefront's LDS (the
// last row's words reach at most 2 bytes past the block).
__device__ __forceinline__ void emit_block(uint32_t *stage, uint32_t lane, uint32_t n, uint64_t v, uint8_t *dst,
                                           uint32_t np)
{
    const uintptr_t base = reinterpret_cast<uintptr_t>(dst);
    const uint32_t mis = (uint32_t)(base & 15u);
    const uint32_t total = mis + n * np;  // staged bytes, <= 15 + 4096
    const uint32_t n_units = (total + 15) >> 4;
    v4u32 *st4 = reinterpret_cast<v4u32 *>(stage);
    for (uint32_t u = lane; u < n_units; u += 64) st4[u] = v4u32{0u, 0u, 0u, 0u};
    __builtin_amdgcn_wave_barrier();
    if (lane < n) {
        const uint32_t o = mis + lane * np;
        const uint32_t sh = 8 * (o & 3u);
        uint32_t *w = stage + (o >> 2);
        const uint32_t nq = ((o & 3u) + np + 3) >> 2;
        uint32_t prev = 0;
        for (uint32_t q = 0; q < nq; ++q) {
            const uint32_t cur = 4 * q < np ? spread_nib((uint32_t)(v >> (4 * q)) & 0xFu) : 0u;
            const uint32_t out = sh ? (cur << sh) | (prev >> (32 - sh)) : cur;
            __hip_atomic_fetch_or(w + q, out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            prev = cur;
        }
    }
    __builtin_amdgcn_wave_barrier();
    // device memory (flat stores would also count on the LDS wait counter)
    __attribute__((address_space(1))) uint8_t *g = (__attribute__((address_space(1))) uint8_t *)(dst - mis);
    for (uint32_t u = lane; u < n_units; u += 64) {
        const v4u32 x = st4[u];
        const uint32_t lo = 16 * u, hi = lo + 16;
        if (lo >= mis && hi <= total) {
            *(__attribute__((address_space(1))) v4u32 *)(g + lo) = x;
        } else {
            const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
            for (uint32_t b = 0; b < 16; ++b)
                if (lo + b >= mis && lo + b < total) g[lo + b] = (uint8_t)(xs[b >> 2] >> (8 * (b & 3u)));
        }
    }
    __builtin_amdgcn_wave_barrier();  // the stage is reused by the next block
}

// A job's descriptor with every field in scalar registers (read through a
// pointer held in the batch's descriptors, the fields would otherwise land in
// vector registers and make the loops over them lane-divergent).
__device__ __forceinline__ SegDesc uniform_seg(const SegDesc *segs, uint32_t i)
{
    const SegDesc d = segs[i];
    auto u32 = [](uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); };
    auto ptr = [&](uintptr_t p) { return ((uintptr_t)u32((uint32_t)(p >> 32)) << 32) | u32((uint32_t)p); };
    SegDesc r;
    r.O = reinterpret_cast<const uint8_t *>(ptr(reinterpret_cast<uintptr_t>(d.O)));
    r.L = reinterpret_cast<uint8_t *>(ptr(reinterpret_cast<uintptr_t>(d.L)));
    r.n_props = u32(d.n_props);
    r.bit = u32(d.bit);
    return r;
}

// LDS of one wavefront's label-byte staging (emit_block): 64 rows of at
// most 64 bytes at an offset below 16, plus the word a row's last bytes may
// spill into.
constexpr uint32_t kStageWords = (64 * 64 + 32) / 4;
static_assert(kTileWaves * kStageWords * 4 <= kTileWaves * kRing * kTabWords * 8,
              "label staging must fit in the tile's table slots");

// Label bytes of a whole row block straight from a tile's accumulators (the
// batch tilings with one tile per row block: the accumulators hold the final
// labels of the block's rows for the lane group's 64 columns).  Wavefront w
// takes the 64-row chunks w, w + WAVES, ... of the block, and for every job
// of the lane group writes the chunk's label bytes as one contiguous block
// (emit_block), staged in the LDS the wavefronts' table slots used.
template <int WAVES>
__device__ __forceinline__ void emit_tile(uint64_t *lds, const GroupDesc &g, uint32_t gi, uint32_t rb)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t *stage = reinterpret_cast<uint32_t *>(lds + kRowBlock) + wave * kStageWords;
    const uint64_t t_base = (uint64_t)rb * kRowBlock;
    const uint32_t n_rows = (uint32_t)min<uint64_t>(kRowBlock, g.n_traj - t_base);
    const uint32_t s0 = __builtin_amdgcn_readfirstlane((int)g.lg_seg[gi]);
    const uint32_t s1 = __builtin_amdgcn_readfirstlane((int)g.lg_seg[gi + 1]);
    for (uint32_t c0 = wave * 64; c0 < n_rows; c0 += 64 * WAVES) {
        const uint32_t n = min(64u, n_rows - c0);
        const uint64_t bits = lane < n ? lds[c0 + lane] : 0ull;
        for (uint32_t sgi = s0; sgi < s1; ++sgi) {
            const SegDesc d = uniform_seg(g.segs, sgi);
            const uint64_t v = d.n_props >= 64 ? bits : (bits >> d.bit) & ((1ull << d.n_props) - 1ull);
            emit_block(stage, lane, n, v, d.L + (t_base + c0) * d.n_props, d.n_props);
        }
    }
}

// One tile item of a batch: pass it.group, tile it.tile, lane group it.gi.
// The pass's nibble tables are [w][G64][256].  Passes on a tiling with one
// tile per row block (fused) write the label bytes themselves; the others
// write partials for k_combine_batch: compact ([G64][n_slots], the rows each
// tile touches) when the tiling has slot lists, else [G64][n_tiles][kRowBlock].
template <int WAVES>
__device__ __forceinline__ void batch_tile(const GroupDesc *__restrict__ groups, const TileItem &it, uint64_t *lds)
{
    const GroupDesc &g = groups[it.group];
    tile_accumulate<WAVES, uint64_t>(g.sp_tasks + (uint64_t)it.tile * WAVES, g.sp_rounds, g.sp_row, g.sp_val,
                                     g.Ow + (uint64_t)it.gi * 256, (uint64_t)g.G64 * 256, lds);
    if (g.fused) {
        emit_tile<WAVES>(lds, g, it.gi, it.tile);
    } else if (g.tile_slot) {
        typedef __attribute__((address_space(1))) const uint32_t gu32;
        const uint32_t s0 = ((const gu32 *)g.tile_slot)[it.tile], s1 = ((const gu32 *)g.tile_slot)[it.tile + 1];
        write_partials_compact<WAVES, uint64_t>(lds, g.P + (uint64_t)it.gi * g.n_slots + s0, g.slot_row + s0,
                                                s1 - s0);
    } else {
        write_partials<WAVES, uint64_t>(lds, g.P + ((uint64_t)it.gi * g.n_tiles + it.tile) * kRowBlock);
    }
}

// One workgroup per tile item: workgroup b runs items[launch[b]].
template <int WAVES>
__global__ void __launch_bounds__(64 * WAVES)
k_label_tiles_batch(const GroupDesc *__restrict__ groups, const TileItem *__restrict__ items,
                    const uint32_t *__restrict__ launch)
{
    extern __shared__ uint64_t lds[];
    const TileItem it = items[launch[blockIdx.x]];
    batch_tile<WAVES>(groups, it, lds);
}

// Persistent: one workgroup per CU.  Items are split into kXcds queues
// (queue x = items[xcd_start[x] .. xcd_start[x + 1])) so that the items
// reading the same nibble tables run on one XCD; workgroup b starts on queue
// b % kXcds (the XCD it runs on) and, once that queue is empty, takes items
// from the others.  Every workgroup leaves when every queue is empty; no
// workgroup waits for another.
template <int WAVES>
__global__ void __launch_bounds__(64 * WAVES)
k_label_tiles_queue(const GroupDesc *__restrict__ groups, const TileItem *__restrict__ items,
                    const uint32_t *__restrict__ xcd_start, uint32_t *queues)
{
    extern __shared__ uint64_t lds[];
    __shared__ uint32_t s_item;
    const uint32_t home = blockIdx.x % kXcds;
    uint32_t k = 0;
    while (k < kXcds) {
        const uint32_t q = (home + k) % kXcds;
        // the previous item's write-back of the accumulators is complete
        // before the next item clears them
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t i = xcd_start[q] + atomicAdd(queues + q, 1u);
            s_item = i < xcd_start[q + 1] ? i : 0xFFFFFFFFu;
        }
        __syncthreads();
        const uint32_t i = s_item;
        if (i == 0xFFFFFFFFu) {
            ++k;  // uniform: this queue is empty, try the next
            continue;
        }
        const TileItem it = items[i];
        batch_tile<WAVES>(groups, it, lds);
    }
}

// Bit p set iff byte mis + p of the dwords p[0 ..] is non-zero, for p < n
// (1 <= n <= 64, mis < 4).  Reads p[0 .. (n + 6) / 4] whatever mis is (the
// caller's array extends that far); dwords past the range are dropped.
__device__ __forceinline__ uint64_t byte_mask_words(const uint32_t *p, uint32_t mis, uint32_t n)
{
    const uint32_t nd = (mis + n + 3) >> 2;  // this lane's words: 1 .. 17
    const uint32_t kmax = (n + 6) >> 2;      // an upper bound of nd for every lane
    uint64_t lo = 0;
#pragma unroll
    for (uint32_t k = 0; k < 16; ++k)
        if (k < kmax) {  // uniform
            // dwords past this lane's range are dropped by a mask, not a branch
            const uint32_t keep = 0u - (uint32_t)(k < nd);
            lo |= (uint64_t)(nz_bytes(p[k]) & keep) << (4 * k);
        }
    const uint32_t hi = kmax > 16 ? nz_bytes(p[16]) & (0u - (uint32_t)(nd > 16)) : 0u;
    const uint64_t m = mis ? (lo >> mis) | ((uint64_t)hi << (64 - mis)) : lo;
    return n >= 64 ? m : m & ((1ull << n) - 1ull);
}

// LDS words a pack wavefront stages one job's bytes of one word in: 8 runs
// of 8 cells (or one of 64) of at most 64 bytes, each from a dword boundary,
// plus the dwords byte_mask_words may read past the last run.
constexpr uint32_t kPackStaged = 8 * ((3 + 8 * 64 + 3) / 4);
static_assert(kPackStaged >= (3 + 64 * 64 + 3) / 4, "a 64-cell run must fit the stage");
constexpr uint32_t kPackStageWords = kPackStaged + 4;
// Dword loads per lane in flight while a stage is filled.
constexpr uint32_t kPackLoads = 9;

typedef __attribute__((address_space(1))) const uint32_t global_u32;
typedef __attribute__((address_space(1))) const uint64_t global_u64;

// One wavefront per pack item (pass, lane group, words [w0, w1)): for each
// word, lane b builds the proposition mask of the word's cell b over the
// lane group's columns, then the word's nibble tables for the lane group are
// written.  A job's bytes of the word's 64 cells are n_props-byte records in
// 8 runs of 8 consecutive cells (row-major ids: one run per cell row of the
// 8 x 8 tile, nx cells apart) or one run of 64 (z-order ids); they are
// staged in LDS with coalesced dword loads (every run starts at the same
// offset within a dword, since cell ids of a run start are multiples of 8),
// and each lane then reads its cell's record from LDS.
__global__ void __launch_bounds__(256)
k_pack_batch_tables(const GroupDesc *__restrict__ groups, const PackItem *__restrict__ items, uint32_t n_items)
{
    __shared__ uint32_t stage_all[4][kPackStageWords];
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t i = blockIdx.x * 4 + wv;
    if (i >= n_items) return;  // whole wavefronts
    uint32_t *stage = stage_all[wv];
    const PackItem it = items[i];
    const GroupDesc &g = groups[it.group];
    // values read through pointers held in the descriptors come back in
    // vector registers; they are wavefront-uniform, and are moved to scalar
    // registers so that the loops and offsets derived from them are scalar
    auto uni = [](uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); };
    const uint32_t s0 = uni(g.lg_seg[it.gi]), s1 = uni(g.lg_seg[it.gi + 1]);
    const bool zo = g.morton != 0;
    // lane b is the cell at (dx, dy) of the word's 8 x 8 tile, x taking the
    // odd bits of b; in z-order ids it is the word's cell b
    const uint32_t dx = ((lane >> 1) & 1u) | ((lane >> 2) & 2u) | ((lane >> 3) & 4u);
    const uint32_t dy = (lane & 1u) | ((lane >> 1) & 2u) | ((lane >> 2) & 4u);
    const uint32_t n_run = zo ? 1u : 8u, run_cells = zo ? 64u : 8u;
    const uint32_t my_run = zo ? 0u : dy, my_pos = zo ? lane : dx;
    const global_u32 *word_cell = (const global_u32 *)g.word_cell;
    for (uint32_t w = it.w0; w < it.w1; ++w) {
        // the word's first cell (dx = dy = 0), wavefront-uniform (read into
        // a scalar register, so that everything derived from it is scalar)
        const uint32_t c0 = zo ? w * 64 : word_cell[(uint64_t)w * 64];
        const uint64_t cell0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)c0);
        uint64_t m = 0;
        for (uint32_t sgi = s0; sgi < s1; ++sgi) {
            const SegDesc d = g.segs[sgi];
            const uint32_t np = uni(d.n_props), bit = uni(d.bit);
            const uintptr_t o_addr = ((uintptr_t)uni((uint32_t)((uintptr_t)d.O >> 32)) << 32) | uni((uint32_t)(uintptr_t)d.O);
            const uintptr_t a0 = o_addr + cell0 * np;
            const uint32_t mis = (uint32_t)(a0 & 3u);
            const uint32_t nd = (mis + run_cells * np + 3) >> 2;  // dwords per run, >= 2
            // byte offsets from base fit 32 bits: 7 runs of nx * np bytes
            // (nx * ny < 2^31 cells, np <= 64) plus one run's dwords
            const uint32_t run_stride = zo ? 0u : g.nx * np;
            const __attribute__((address_space(1))) uint8_t *base =
                reinterpret_cast<const __attribute__((address_space(1))) uint8_t *>(a0 - mis);
            // floor(q / nd) as umulhi(q, magic): exact for q * nd < 2^32
            const uint32_t magic = 0xFFFFFFFFu / nd + 1u;
            const uint32_t total = n_run * nd;  // <= kPackStageWords
            // the loads of a phase (up to kPackLoads per lane) are all issued
            // before the first is stored, so the wavefront waits for memory
            // once per phase: once per job and word up to 35 propositions
            // (8 runs of at most 72 dwords), twice above
            // Lanes past the end take the last dword again (loaded and
            // stored twice with the same value), so no lane branches.
            for (uint32_t q0 = 0; q0 < total; q0 += 64 * kPackLoads) {
                uint32_t v[kPackLoads], at[kPackLoads];
#pragma unroll
                for (uint32_t k = 0; k < kPackLoads; ++k)
                    if (q0 + 64 * k < total) {  // uniform
                        const uint32_t q = min(q0 + lane + 64 * k, total - 1);
                        const uint32_t r = __umulhi(q, magic), j = q - r * nd;
                        at[k] = q;
                        v[k] = *reinterpret_cast<const global_u32 *>(base + (r * run_stride + 4u * j));
                    }
#pragma unroll
                for (uint32_t k = 0; k < kPackLoads; ++k)
                    if (q0 + 64 * k < total) stage[at[k]] = v[k];
            }
            // LDS instructions of a wavefront complete in issue order; the
            // barrier keeps the compiler from moving the reads above the writes
            __builtin_amdgcn_wave_barrier();
            const uint32_t off = my_run * nd * 4 + mis + my_pos * np;
            m |= byte_mask_words(stage + (off >> 2), off & 3u, np) << bit;
            __builtin_amdgcn_wave_barrier();  // the next job overwrites the stage
        }
        write_tables(m, g.Ow + ((uint64_t)w * g.G64 + it.gi) * 256, lane);
    }
}

// OR of row t's partials over the tiles of its row block.
template <typename M>
__device__ __forceinline__ uint64_t row_partials(const M *__restrict__ P, const uint32_t *__restrict__ rb_tile,
                                                 uint64_t t)
{
    // device memory (the batch passes pointers read from its descriptors:
    // without the casts they would be flat loads)
    const __attribute__((address_space(1))) M *Pg = (const __attribute__((address_space(1))) M *)P;
    const __attribute__((address_space(1))) uint32_t *rbt = (const __attribute__((address_space(1))) uint32_t *)rb_tile;
    const uint64_t rb = t / kRowBlock, loc = t % kRowBlock;
    const uint32_t k0 = rbt[rb], k1 = rbt[rb + 1];
    uint64_t bits = 0;
    // sixteen loads in flight at a time: indices past the block's last tile
    // read that tile again, which leaves the OR unchanged
    for (uint32_t kb = k0; kb < k1; kb += 16) {
        M v[16];
#pragma unroll
        for (uint32_t j = 0; j < 16; ++j) v[j] = Pg[(uint64_t)min(kb + j, k1 - 1) * kRowBlock + loc];
#pragma unroll
        for (uint32_t j = 0; j < 16; ++j) bits |= v[j];
    }
    return bits;
}

// One wavefront per (pass, lane group, rows [row0, row1)), 64 rows at a
// time: lane j ORs the partials of row t0 + j (the 64 columns of the lane
// group), then every job of the lane group gets its block of label bytes for
// those rows (emit_block).  Each byte of L belongs to one job, one row range
// and one lane group, so exactly one wavefront writes it.
__global__ void __launch_bounds__(64)
k_combine_batch(const GroupDesc *__restrict__ groups, const CombineItem *__restrict__ items)
{
    // 64 rows of at most 64 bytes at an offset below 16, plus the word a
    // row's last bytes may spill into
    __shared__ uint32_t stage[(64 * 64 + 32) / 4];
    const uint32_t lane = threadIdx.x;
    const CombineItem it = items[blockIdx.x];
    const GroupDesc &g = groups[it.group];
    const bool compact = g.tile_slot != nullptr;
    const uint64_t *Pg = g.P + (uint64_t)it.gi * (compact ? g.n_slots : (uint64_t)g.n_tiles * kRowBlock);
    const uint32_t s0 = __builtin_amdgcn_readfirstlane((int)g.lg_seg[it.gi]);
    const uint32_t s1 = __builtin_amdgcn_readfirstlane((int)g.lg_seg[it.gi + 1]);
    for (uint64_t t0 = it.row0; t0 < it.row1; t0 += 64) {
        const uint64_t t = t0 + lane;
        uint64_t bits = 0;
        if (t < it.row1)
            bits = compact ? row_slots_or(Pg, g.row_slot_off, g.row_slots, t) : row_partials(Pg, g.sp_rb_tile, t);
        const uint32_t n = (uint32_t)min<uint64_t>(64, it.row1 - t0);
        for (uint32_t sgi = s0; sgi < s1; ++sgi) {
            const SegDesc d = uniform_seg(g.segs, sgi);
            const uint64_t v = d.n_props >= 64 ? bits : (bits >> d.bit) & ((1ull << d.n_props) - 1ull);
            emit_block(stage, lane, n, v, d.L + t0 * d.n_props, d.n_props);
        }
    }
}

// Rows' label bytes from their partials.  One wavefront takes 64 consecutive
// rows: lane j ORs the partials of row t0 + j (its compact slots when the
// tiling has them, else the row's entry in every tile of its row block).
// When n_props is a multiple of 16 (and L 16-byte aligned) the rows' bytes
// are written as consecutive 16-byte units, lane l writing units l, l + 64,
// ... of the block's n_props * 64 bytes, fetching the bits of each unit's row
// from the lane that holds them; otherwise the block is staged in LDS and
// written by emit_block.
template <typename M>
__global__ void __launch_bounds__(256)
k_combine(const M *__restrict__ P, const uint32_t *__restrict__ rb_tile,
          const uint32_t *__restrict__ row_slot_off, const uint32_t *__restrict__ row_slots, uint64_t n_traj,
          uint32_t n_props, uint8_t *__restrict__ L)
{
    __shared__ uint32_t stage[4][(64 * 64 + 32) / 4];
    const bool v16 = (n_props & 15u) == 0 && (reinterpret_cast<uintptr_t>(L) & 15u) == 0;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const uint64_t n_groups = (n_traj + 63) / 64;
    const uint32_t upr = n_props / 16;  // 16-byte units per row: 1 .. 4
    const uint32_t shift = upr == 1 ? 0 : upr == 2 ? 1 : upr == 4 ? 2 : 32;  // 32: not a power of two
    for (uint64_t grp = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; grp < n_groups; grp += n_waves) {
        const uint64_t t0 = grp * 64, t = t0 + lane;
        uint64_t bits = 0;
        if (t < n_traj)
            bits = row_slot_off ? row_slots_or(P, row_slot_off, row_slots, t) : row_partials(P, rb_tile, t);
        const uint32_t n = (uint32_t)min<uint64_t>(64, n_traj - t0);
        if (!v16) {
            emit_block(stage[wave], lane, n, bits, L + t0 * n_props, n_props);
            continue;
        }
        const uint32_t units = n * upr;
        uint4 *dst = reinterpret_cast<uint4 *>(L + t0 * n_props);
        // uniform trip count: every lane takes part in the shuffles
        for (uint32_t ub = 0; ub < units; ub += 64) {
            const uint32_t u = ub + lane;  // < 64 * upr, so row < 64
            const uint32_t row = min(shift < 32 ? u >> shift : u / upr, 63u);
            const uint32_t c = u - row * upr;
            const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)bits, (int)row);
            const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(bits >> 32), (int)row);
            const uint32_t b = (uint32_t)((((uint64_t)hi << 32) | lo) >> (16 * c)) & 0xFFFFu;
            if (u < units)
                dst[u] = make_uint4(spread_nib(b & 0xFu), spread_nib((b >> 4) & 0xFu), spread_nib((b >> 8) & 0xFu),
                                    spread_nib(b >> 12));
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

// Cost of a round, in rounds: one, plus this much when it copies a table in.
constexpr double kBuildCost = 0.25;

}  // namespace

// Relative work of wavefront w of a tile workgroup.  Wavefronts w, w + 4,
// w + 8 and w + 12 share a SIMD, and the SIMD issues for the oldest of them
// first: measured at full load, their round rates fall with age in about
// these proportions, and work sized to them lets the four finish together
// (equal shares leave the last ones running alone at a lower SIMD throughput).
double wave_share(uint32_t w)
{
    static const double share[4] = {2.6, 2.0, 1.6, 1.3};
    return share[(w % kTileWaves) / 4];
}

namespace {



// The rounds of entries [lo, hi) of one row block as one wavefront walks them
// with empty tables at the start: 64 entries per chunk from lo, at most two
// segments and one table copy per round.  sp: a segment at or before the one
// holding lo (advanced in place).  emit(c0, lane_lo, lane_hi, cut, a, build):
// the round's chunk start, lane range, first lane of the second segment (64
// if none), first segment, and -1 / 0 / 1 for no copy / copy of segment a /
// copy of segment a + 1.
template <class Emit>
void walk_rounds(const std::vector<uint64_t> &seg_start, uint64_t lo, uint64_t hi, uint64_t &sp, Emit emit)
{
    int64_t built = -1;
    for (uint64_t c0 = lo; c0 < hi; c0 += 64) {
        const uint64_t c1 = std::min(c0 + 64, hi);
        while (seg_start[sp + 1] <= c0) ++sp;
        uint64_t a = sp;
        uint32_t lane_lo = 0;
        for (;;) {
            const uint64_t end_a = seg_start[a + 1];
            const bool two = end_a < c1;  // the next segment starts inside the round
            const bool new_a = (int64_t)a > built, new_b = two && (int64_t)a + 1 > built;
            if (new_a && new_b) {
                // one table per round: the first segment's lanes alone
                emit(c0, lane_lo, (uint32_t)(end_a - c0), 64u, a, 0);
                built = (int64_t)a;
                lane_lo = (uint32_t)(end_a - c0);
                ++a;
                continue;
            }
            const uint64_t b = two ? a + 1 : a;
            const uint64_t end_r = std::min(c1, seg_start[b + 1]);
            const uint32_t lane_hi = (uint32_t)(end_r - c0);
            const uint32_t cut = two ? (uint32_t)(end_a - c0) : 64u;
            const int build = new_a ? 0 : (new_b ? 1 : -1);
            emit(c0, lane_lo, lane_hi, cut, a, build);
            if (build >= 0) built = (int64_t)a + build;
            if (end_r >= c1) break;
            a = b + 1;  // starts at end_r
            lane_lo = lane_hi;
        }
    }
}

// Cost of every 64-entry chunk of row block rb walked as one task.
std::vector<double> chunk_costs(const std::vector<uint64_t> &seg_start, const std::vector<uint64_t> &rb_seg, size_t rb)
{
    const uint64_t E0 = seg_start[rb_seg[rb]], E1 = seg_start[rb_seg[rb + 1]];
    std::vector<double> c((E1 - E0 + 63) / 64, 0.0);
    uint64_t sp = rb_seg[rb];
    walk_rounds(seg_start, E0, E1, sp, [&](uint64_t c0, uint32_t, uint32_t, uint32_t, uint64_t, int build) {
        c[(c0 - E0) / 64] += 1.0 + (build >= 0 ? kBuildCost : 0.0);
    });
    return c;
}

}  // namespace

// ---------------------------------------------------------------- host: tilings

std::vector<double> block_costs(const std::vector<uint64_t> &seg_start, const std::vector<uint64_t> &rb_seg)
{
    std::vector<double> out(rb_seg.size() - 1, 0.0);
    for (size_t rb = 0; rb + 1 < rb_seg.size(); ++rb)
        for (double x : chunk_costs(seg_start, rb_seg, rb)) out[rb] += x;
    return out;
}

std::vector<uint32_t> tiles_per_block(const std::vector<double> &cost, uint32_t target)
{
    const size_t n_rb = cost.size();
    std::vector<uint32_t> k(n_rb, 1);
    if (target <= n_rb) return k;
    double total = 0;
    for (double c : cost) total += c;
    if (total <= 0) return k;
    uint64_t sum = 0;
    for (size_t rb = 0; rb < n_rb; ++rb) {
        k[rb] = std::max<uint32_t>(1, (uint32_t)std::floor(target * cost[rb] / total));
        sum += k[rb];
    }
    // largest cost per tile gets the next tile; smallest gives one back
    while (sum < target) {
        size_t best = 0;
        for (size_t rb = 1; rb < n_rb; ++rb)
            if (cost[rb] / k[rb] > cost[best] / k[best]) best = rb;
        ++k[best];
        ++sum;
    }
    while (sum > target) {
        size_t best = n_rb;
        for (size_t rb = 0; rb < n_rb; ++rb)
            if (k[rb] > 1 && (best == n_rb || cost[rb] / (k[rb] - 1) < cost[best] / (k[best] - 1))) best = rb;
        if (best == n_rb) break;
        --k[best];
        --sum;
    }
    return k;
}

std::vector<uint32_t> choose_tiles(const std::vector<double> &cost, uint32_t n_cu)
{
    std::vector<uint32_t> best_k;
    double best_end = 0;
    for (uint32_t m = 2; m <= 8; ++m) {
        std::vector<uint32_t> k = tiles_per_block(cost, std::max<uint32_t>(1, n_cu * m / 2));
        // list schedule in row-block order: each tile to the CU that frees first
        std::priority_queue<double, std::vector<double>, std::greater<double>> cu;
        for (uint32_t i = 0; i < n_cu; ++i) cu.push(0.0);
        double end = 0;
        for (size_t rb = 0; rb < cost.size(); ++rb)
            for (uint32_t j = 0; j < k[rb]; ++j) {
                const double t = cu.top() + cost[rb] / k[rb] + kTileFixedRounds;
                cu.pop();
                cu.push(t);
                end = std::max(end, t);
            }
        for (uint32_t x : k) end += x * kTileCombineRounds;
        if (best_k.empty() || end < 0.98 * best_end) {  // more tiles only for a clear gain
            best_k = std::move(k);
            best_end = end;
        }
    }
    return best_k;
}

void make_tiling(const std::vector<uint64_t> &seg_start, const std::vector<uint32_t> &seg_word,
                 const std::vector<uint64_t> &rb_seg, const std::vector<uint32_t> &tiles_rb, TilingHost *out)
{
    const size_t n_rb = rb_seg.size() - 1;
    out->tasks.clear();
    out->rounds.clear();
    out->rb_tile.assign(n_rb + 1, 0);
    for (size_t rb = 0; rb < n_rb; ++rb) {
        out->rb_tile[rb + 1] = out->rb_tile[rb] + tiles_rb[rb];
        const uint64_t s_lo = rb_seg[rb], s_hi = rb_seg[rb + 1];
        const uint64_t E0 = seg_start[s_lo], E1 = seg_start[s_hi];
        const uint64_t m = (uint64_t)tiles_rb[rb] * kTileWaves;
        // task boundaries at chunk starts, at equal cost of the rounds walked
        // over the whole block
        const std::vector<double> cc = chunk_costs(seg_start, rb_seg, rb);
        double C = 0;
        for (double x : cc) C += x;
        // task q's share of the block's cost is proportional to
        // wave_share(q % kTileWaves)
        double Wsum = 0;
        for (uint64_t q = 0; q < m; ++q) Wsum += wave_share((uint32_t)(q % kTileWaves));
        std::vector<uint64_t> bnd(m + 1, E1);
        bnd[0] = E0;
        {
            size_t k = 0;
            double pre = 0, wq = 0;
            for (uint64_t q = 1; q < m; ++q) {
                wq += wave_share((uint32_t)((q - 1) % kTileWaves));
                const double want = C * wq / Wsum;
                while (k < cc.size() && pre + 0.5 * cc[k] < want) pre += cc[k++];
                bnd[q] = std::max(bnd[q - 1], std::min(E1, E0 + 64 * (uint64_t)k));
            }
        }
        // rounds of each task
        uint64_t sp = s_lo;  // segment containing the current entry
        for (uint64_t q = 0; q < m; ++q) {
            const uint64_t lo = bnd[q], hi = bnd[q + 1];
            SpTask t{lo, 0, (uint32_t)out->rounds.size()};
            uint32_t tword = 0;  // word of the last table copied
            walk_rounds(seg_start, lo, hi, sp,
                        [&](uint64_t c0, uint32_t lane_lo, uint32_t lane_hi, uint32_t cut, uint64_t a, int build) {
                            uint32_t meta = lane_lo | lane_hi << 8 | cut << 16;
                            if (build >= 0) {
                                meta |= build == 0 ? kMetaBuild0 : kMetaBuild1;
                                tword = seg_word[a + build];
                            }
                            if (a & 1) meta |= kMetaSlot0;  // slot of a segment = parity of its index
                            out->rounds.push_back(SpRound{(uint32_t)(c0 - lo), tword, 0, meta});
                            ++t.n_rounds;
                        });
            out->tasks.push_back(t);
        }
    }
    // launch order: tiles ranked by the word at their middle entry, the ranks
    // split into kXcds consecutive groups, group g taking blocks g, g + kXcds, ...
    const uint32_t n_tiles = (uint32_t)(out->tasks.size() / kTileWaves);
    std::vector<std::pair<uint32_t, uint32_t>> key(n_tiles);
    for (uint32_t i = 0; i < n_tiles; ++i) {
        const SpTask &f = out->tasks[(size_t)i * kTileWaves];
        const SpTask &l = out->tasks[(size_t)i * kTileWaves + kTileWaves - 1];
        uint64_t hi = l.lo;  // end of the tile's entries: its last task's end
        for (uint32_t r = 0; r < l.n_rounds; ++r) {
            const SpRound &x = out->rounds[l.round0 + r];
            hi = std::max<uint64_t>(hi, l.lo + x.e_off + ((x.meta >> 8) & 0xFFu));
        }
        const uint64_t mid = (f.lo + hi) / 2;
        uint32_t w = 0;
        if (hi > f.lo) {
            const uint64_t sidx = std::upper_bound(seg_start.begin(), seg_start.end(), mid) - seg_start.begin() - 1;
            w = seg_word[std::min<uint64_t>(sidx, seg_word.size() - 1)];
        }
        key[i] = {w, i};
    }
    std::stable_sort(key.begin(), key.end());
    out->block_tile.assign(n_tiles, 0);
    uint32_t rank = 0;
    for (uint32_t g = 0; g < kXcds; ++g)
        for (uint32_t b = g; b < n_tiles; b += kXcds) out->block_tile[b] = key[rank++].second;
}

bool make_compact(const TilingHost &h, const std::vector<uint16_t> &row, const std::vector<uint64_t> &seg_start,
                  const std::vector<uint64_t> &rb_seg, uint64_t n_traj, CompactHost *out)
{
    const size_t n_rb = rb_seg.size() - 1;
    const uint32_t n_tiles = (uint32_t)(h.tasks.size() / kTileWaves);
    out->tile_slot.assign(n_tiles + 1, 0);
    out->slot_row.clear();
    std::vector<uint32_t> row_cnt(n_traj + 1, 0);
    std::vector<uint64_t> bm(kRowBlock / 64);
    uint64_t n_slots = 0;
    for (size_t rb = 0; rb < n_rb; ++rb) {
        const uint64_t E1 = seg_start[rb_seg[rb + 1]];
        for (uint32_t i = h.rb_tile[rb]; i < h.rb_tile[rb + 1]; ++i) {
            const uint64_t lo = h.tasks[(size_t)i * kTileWaves].lo;
            const uint64_t hi = i + 1 < h.rb_tile[rb + 1] ? h.tasks[(size_t)(i + 1) * kTileWaves].lo : E1;
            std::fill(bm.begin(), bm.end(), 0ull);
            for (uint64_t e = lo; e < hi; ++e) bm[row[e] >> 6] |= 1ull << (row[e] & 63u);
            for (uint32_t q = 0; q < bm.size(); ++q)
                for (uint64_t m = bm[q]; m; m &= m - 1) {
                    const uint32_t r = q * 64 + (uint32_t)__builtin_ctzll(m);
                    out->slot_row.push_back((uint16_t)r);
                    ++row_cnt[rb * kRowBlock + r];
                }
            n_slots = out->slot_row.size();
            if (n_slots >= (1ull << 32)) return false;
            out->tile_slot[i + 1] = (uint32_t)n_slots;
        }
    }
    // a tile's slots are row-ascending, so filling row lists tile by tile
    // leaves each row's slots in tile order
    out->row_slot_off.assign(n_traj + 1, 0);
    for (uint64_t t = 0; t < n_traj; ++t) out->row_slot_off[t + 1] = out->row_slot_off[t] + row_cnt[t];
    out->row_slots.assign(n_slots, 0);
    std::vector<uint32_t> fill(out->row_slot_off.begin(), out->row_slot_off.end() - 1);
    for (size_t rb = 0; rb < n_rb; ++rb)
        for (uint32_t i = h.rb_tile[rb]; i < h.rb_tile[rb + 1]; ++i)
            for (uint32_t k = out->tile_slot[i]; k < out->tile_slot[i + 1]; ++k)
                out->row_slots[fill[rb * kRowBlock + out->slot_row[k]]++] = k;
    return true;
}

void make_direct(const std::vector<uint64_t> &seg_start, const std::vector<uint64_t> &rb_seg, uint32_t n_tiles,
                 DirectHost *out)
{
    const size_t n_rb = rb_seg.size() - 1;
    out->chunks.clear();
    out->parts.clear();
    // the chunks of every row block, and the first chunk of each block
    std::vector<uint64_t> rb_chunk(n_rb + 1, 0);
    for (size_t rb = 0; rb < n_rb; ++rb) {
        const uint64_t E0 = seg_start[rb_seg[rb]], E1 = seg_start[rb_seg[rb + 1]];
        rb_chunk[rb + 1] = rb_chunk[rb] + (E1 - E0 + 63) / 64;
    }
    const uint64_t C = rb_chunk[n_rb];
    n_tiles = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(n_tiles, C));
    out->tile_part.assign(n_tiles + 1, 0);
    // chunk records: seg0 is fixed once the parts are known (relative to the
    // part's first segment), so first record each chunk's segment
    std::vector<uint64_t> chunk_seg(C);
    for (size_t rb = 0; rb < n_rb; ++rb) {
        const uint64_t E0 = seg_start[rb_seg[rb]], E1 = seg_start[rb_seg[rb + 1]];
        uint64_t sg = rb_seg[rb];
        for (uint64_t a = E0, c = rb_chunk[rb]; a < E1; a += 64, ++c) {
            const uint64_t b = std::min(a + 64, E1);
            while (seg_start[sg + 1] <= a) ++sg;
            chunk_seg[c] = sg;
            SpChunk ch{0ull, 0u, (uint32_t)(b - a)};
            for (uint64_t q = sg + 1; q < rb_seg[rb + 1] && seg_start[q] < b; ++q)
                ch.starts |= 1ull << (seg_start[q] - a - 1);
            out->chunks.push_back(ch);
        }
    }
    // tiles of equal chunk counts, cut into one part per row block
    size_t rb = 0;
    for (uint32_t t = 0; t < n_tiles; ++t) {
        const uint64_t lo = C * t / n_tiles, hi = C * (t + 1) / n_tiles;
        uint64_t c = lo;
        while (c < hi) {
            while (rb_chunk[rb + 1] <= c) ++rb;
            const uint64_t end = std::min(hi, rb_chunk[rb + 1]);
            DirectPart p{};
            p.e0 = seg_start[rb_seg[rb]] + 64 * (c - rb_chunk[rb]);
            p.c0 = (uint32_t)c;
            p.c1 = (uint32_t)end;
            p.rb = (uint32_t)rb;
            p.seg_first = (uint32_t)chunk_seg[c];
            // the part's last segment: that of its last entry
            const uint64_t last_e = seg_start[rb_seg[rb]] + 64 * (end - 1 - rb_chunk[rb]) + out->chunks[end - 1].n_valid - 1;
            const uint64_t last_s = std::upper_bound(seg_start.begin() + (ptrdiff_t)chunk_seg[end - 1],
                                                     seg_start.begin() + (ptrdiff_t)rb_seg[rb + 1], last_e) -
                                    seg_start.begin() - 1;
            p.n_seg = (uint32_t)(last_s + 1 - chunk_seg[c]);
            for (uint64_t j = c; j < end; ++j) out->chunks[j].seg0 = (uint32_t)(chunk_seg[j] - chunk_seg[c]);
            out->parts.push_back(p);
            c = end;
        }
        out->tile_part[t + 1] = (uint32_t)out->parts.size();
    }
}

SparseLayout::~SparseLayout()
{
    (void)hipFree(row);
    (void)hipFree(val);
    (void)hipFree(used_words);
    (void)hipFree(pack_first);
    for (SpTiling &t : tilings) {
        (void)hipFree(t.tasks);
        (void)hipFree(t.rounds);
        (void)hipFree(t.rb_tile);
        (void)hipFree(t.block_tile);
        (void)hipFree(t.tasks_launch);
        (void)hipFree(t.tile_slot);
        (void)hipFree(t.slot_row);
        (void)hipFree(t.row_slot_off);
        (void)hipFree(t.row_slots);
    }
    (void)hipFree(direct.tile_part);
    (void)hipFree(direct.parts);
    (void)hipFree(direct.chunks);
    (void)hipFree(direct.seg_word);
}

void free_sparse(SparseLayout *sp) { delete sp; }

hipError_t launch_pack_batch_tables(const GroupDesc *d_groups, const PackItem *d_packs, uint32_t n_packs,
                                    hipStream_t s)
{
    if (n_packs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_batch_tables, dim3((n_packs + 3) / 4), dim3(256), 0, s, d_groups, d_packs, n_packs);
    return hipGetLastError();
}

hipError_t launch_tiles_batch(const GroupDesc *d_groups, const TileItem *d_tiles, const uint32_t *d_launch,
                              uint32_t n_tiles, hipStream_t s)
{
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_label_tiles_batch<kTileWaves>, dim3(n_tiles), dim3(64 * kTileWaves), kTileLds, s, d_groups,
                       d_tiles, d_launch);
    return hipGetLastError();
}

hipError_t launch_tiles_batch_queue(const GroupDesc *d_groups, const TileItem *d_tiles, const uint32_t *d_xcd_start,
                                    uint32_t *d_queues, uint32_t n_workgroups, hipStream_t s)
{
    if (n_workgroups == 0) return hipSuccess;
    hipLaunchKernelGGL(k_label_tiles_queue<kTileWaves>, dim3(n_workgroups), dim3(64 * kTileWaves), kTileLds, s,
                       d_groups, d_tiles, d_xcd_start, d_queues);
    return hipGetLastError();
}

hipError_t launch_combine_batch(const GroupDesc *d_groups, const CombineItem *d_items, uint32_t n_items, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(k_combine_batch, dim3(n_items), dim3(64), 0, s, d_groups, d_items);
    return hipGetLastError();
}

static lbl_status upload_compact(const CompactHost &c, SpTiling *t, size_t *bytes)
{
    t->n_slots = c.slot_row.size();
    auto up = [](void **dst, const void *src, size_t n) -> hipError_t {
        hipError_t e = hipMalloc(dst, std::max<size_t>(n, 1));
        if (e == hipSuccess && n) e = hipMemcpy(*dst, src, n, hipMemcpyHostToDevice);
        return e;
    };
    LBL_HIP_TRY(up(reinterpret_cast<void **>(&t->tile_slot), c.tile_slot.data(), c.tile_slot.size() * 4));
    LBL_HIP_TRY(up(reinterpret_cast<void **>(&t->slot_row), c.slot_row.data(), c.slot_row.size() * 2));
    LBL_HIP_TRY(up(reinterpret_cast<void **>(&t->row_slot_off), c.row_slot_off.data(), c.row_slot_off.size() * 4));
    LBL_HIP_TRY(up(reinterpret_cast<void **>(&t->row_slots), c.row_slots.data(), c.row_slots.size() * 4));
    *bytes += c.tile_slot.size() * 4 + c.slot_row.size() * 2 + c.row_slot_off.size() * 4 + c.row_slots.size() * 4;
    return LBL_OK;
}

static lbl_status upload_direct(const DirectHost &c, const std::vector<uint32_t> &seg_word, DirectLayout *d,
                                size_t *bytes)
{
    // 32-bit chunk and segment ids: larger layouts keep the nibble kernels only
    if (seg_word.size() >= (1ull << 32) || c.chunks.size() >= (1ull << 32)) return LBL_OK;
    d->n_tiles = (uint32_t)(c.tile_part.size() - 1);
    d->n_chunks = c.chunks.size();
    d->n_parts = (uint32_t)c.parts.size();
    d->max_part_segs = 0;
    for (const DirectPart &p : c.parts) d->max_part_segs = std::max(d->max_part_segs, p.n_seg);
    auto up = [](void **dst, const void *src, size_t n) -> hipError_t {
        hipError_t e = hipMalloc(dst, std::max<size_t>(n, 1));
        if (e == hipSuccess && n) e = hipMemcpy(*dst, src, n, hipMemcpyHostToDevice);
        return e;
    };
    LBL_HIP_TRY(up(reinterpret_cast<void **>(&d->tile_part), c.tile_part.data(), c.tile_part.size() * 4));
    LBL_HIP_TRY(up(reinterpret_cast<void **>(&d->parts), c.parts.data(), c.parts.size() * sizeof(DirectPart)));
    LBL_HIP_TRY(up(reinterpret_cast<void **>(&d->chunks), c.chunks.data(), c.chunks.size() * sizeof(SpChunk)));
    LBL_HIP_TRY(up(reinterpret_cast<void **>(&d->seg_word), seg_word.data(), seg_word.size() * 4));
    *bytes += c.tile_part.size() * 4 + c.parts.size() * sizeof(DirectPart) + c.chunks.size() * sizeof(SpChunk) +
              seg_word.size() * 4;
    return LBL_OK;
}

static lbl_status upload_tiling(const TilingHost &h, SpTiling *t, size_t *bytes)
{
    t->n_tiles = (uint32_t)(h.tasks.size() / kTileWaves);
    t->n_rounds = h.rounds.size();
    t->rb_tile_host = h.rb_tile;
    LBL_HIP_TRY(hipMalloc(&t->tasks, h.tasks.size() * sizeof(SpTask)));
    LBL_HIP_TRY(hipMemcpy(t->tasks, h.tasks.data(), h.tasks.size() * sizeof(SpTask), hipMemcpyHostToDevice));
    LBL_HIP_TRY(hipMalloc(&t->rounds, std::max<size_t>(h.rounds.size(), 1) * sizeof(SpRound)));
    if (!h.rounds.empty())
        LBL_HIP_TRY(hipMemcpy(t->rounds, h.rounds.data(), h.rounds.size() * sizeof(SpRound), hipMemcpyHostToDevice));
    LBL_HIP_TRY(hipMalloc(&t->rb_tile, h.rb_tile.size() * sizeof(uint32_t)));
    LBL_HIP_TRY(hipMemcpy(t->rb_tile, h.rb_tile.data(), h.rb_tile.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    LBL_HIP_TRY(hipMalloc(&t->block_tile, std::max<size_t>(h.block_tile.size(), 1) * sizeof(uint32_t)));
    LBL_HIP_TRY(hipMemcpy(t->block_tile, h.block_tile.data(), h.block_tile.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice));
    std::vector<SpTask> launch(h.tasks.size());
    for (size_t b = 0; b < h.block_tile.size(); ++b)
        for (uint32_t w = 0; w < kTileWaves; ++w)
            launch[b * kTileWaves + w] = h.tasks[(size_t)h.block_tile[b] * kTileWaves + w];
    LBL_HIP_TRY(hipMalloc(&t->tasks_launch, launch.size() * sizeof(SpTask)));
    LBL_HIP_TRY(hipMemcpy(t->tasks_launch, launch.data(), launch.size() * sizeof(SpTask), hipMemcpyHostToDevice));
    *bytes += 2 * h.tasks.size() * sizeof(SpTask) + h.rounds.size() * sizeof(SpRound) +
              (h.rb_tile.size() + h.block_tile.size()) * sizeof(uint32_t);
    return LBL_OK;
}

SparsePart::SparsePart(SparsePart &&o) noexcept
    : row(o.row), val(o.val), nnz(o.nnz), n_rb(o.n_rb), cnt(std::move(o.cnt))
{
    o.row = nullptr;
    o.val = nullptr;
}

SparsePart::~SparsePart()
{
    (void)hipFree(row);
    (void)hipFree(val);
}

lbl_status sparse_part(const uint64_t *T, uint32_t row_stride, uint64_t n_rows, uint32_t W, SparsePart *out)
{
    // 1. word-major entries (temporary)
    uint64_t *d_ptr = nullptr, *d_val = nullptr;
    uint32_t *d_row = nullptr;
    LBL_HIP_TRY(hipMalloc(&d_ptr, (size_t)(W + 1) * sizeof(uint64_t)));
    std::unique_ptr<uint64_t, decltype(&hipFree)> g_ptr(d_ptr, &hipFree);
    hipLaunchKernelGGL(k_wm_count, dim3((W + 7) / 8), dim3(512), 0, nullptr, T, row_stride, n_rows, W, d_ptr);
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
    const uint64_t nnz = run;
    LBL_HIP_TRY(hipMemcpy(d_ptr, ptr.data(), (size_t)(W + 1) * sizeof(uint64_t), hipMemcpyHostToDevice));
    LBL_HIP_TRY(hipMalloc(&d_row, std::max<uint64_t>(nnz, 1) * sizeof(uint32_t)));
    std::unique_ptr<uint32_t, decltype(&hipFree)> g_row(d_row, &hipFree);
    LBL_HIP_TRY(hipMalloc(&d_val, std::max<uint64_t>(nnz, 1) * sizeof(uint64_t)));
    std::unique_ptr<uint64_t, decltype(&hipFree)> g_val(d_val, &hipFree);
    hipLaunchKernelGGL(k_wm_fill, dim3((W + 7) / 8), dim3(512), 0, nullptr, T, row_stride, n_rows, W, d_ptr, d_row,
                       d_val);
    LBL_HIP_TRY(hipGetLastError());

    // 2. segment counts (every (rb, w), empty ones included) -> offsets (host scan) -> tiled copy
    out->n_rb = (uint32_t)((n_rows + kRowBlock - 1) / kRowBlock);
    const uint64_t n_seg = (uint64_t)out->n_rb * W;
    uint32_t *d_cnt = nullptr;
    LBL_HIP_TRY(hipMalloc(&d_cnt, std::max<uint64_t>(n_seg, 1) * sizeof(uint32_t)));
    std::unique_ptr<uint32_t, decltype(&hipFree)> g_cnt(d_cnt, &hipFree);
    hipLaunchKernelGGL(k_seg_count, dim3((unsigned)((n_seg + 255) / 256)), dim3(256), 0, nullptr, d_ptr, d_row, W,
                       out->n_rb, d_cnt);
    LBL_HIP_TRY(hipGetLastError());
    out->cnt.assign(n_seg, 0);
    LBL_HIP_TRY(hipMemcpy(out->cnt.data(), d_cnt, n_seg * sizeof(uint32_t), hipMemcpyDeviceToHost));
    std::vector<uint64_t> seg(n_seg + 1, 0);
    for (uint64_t s = 0; s < n_seg; ++s) seg[s + 1] = seg[s] + out->cnt[s];
    LBL_REQUIRE(seg[n_seg] == nnz, "sparse layout: segment counts disagree with the word counts");
    uint64_t *d_seg = nullptr;
    LBL_HIP_TRY(hipMalloc(&d_seg, (n_seg + 1) * sizeof(uint64_t)));
    std::unique_ptr<uint64_t, decltype(&hipFree)> g_seg(d_seg, &hipFree);
    LBL_HIP_TRY(hipMemcpy(d_seg, seg.data(), (n_seg + 1) * sizeof(uint64_t), hipMemcpyHostToDevice));
    LBL_HIP_TRY(hipMalloc(&out->row, std::max<uint64_t>(nnz, 1) * sizeof(uint16_t)));
    LBL_HIP_TRY(hipMalloc(&out->val, std::max<uint64_t>(nnz, 1) * sizeof(uint64_t)));
    hipLaunchKernelGGL(k_seg_fill, dim3((unsigned)((n_seg + 255) / 256)), dim3(256), 0, nullptr, d_ptr, d_row, d_val, W,
                       out->n_rb, d_seg, out->row, out->val);
    LBL_HIP_TRY(hipGetLastError());
    LBL_HIP_TRY(hipDeviceSynchronize());
    out->nnz = nnz;
    return LBL_OK;
}

lbl_status sparse_assemble(lbl_abs *a, std::vector<SparsePart> &parts)
{
    const uint32_t W = a->n_words;
    std::unique_ptr<SparseLayout> sp(new SparseLayout);
    uint64_t nnz = 0;
    for (const SparsePart &p : parts) {
        sp->n_rb += p.n_rb;
        nnz += p.nnz;
    }
    LBL_REQUIRE(sp->n_rb == (a->n_traj + kRowBlock - 1) / kRowBlock, "sparse layout: parts do not cover the rows");
    LBL_REQUIRE(nnz == a->nonzero_words, "sparse layout: entry count disagrees with the bitpacked T");
    // kEntryPad zeroed entries past the last one: a round's lanes load
    // entries up to 63 past its range without bounds checks
    LBL_HIP_TRY(hipMalloc(&sp->row, (nnz + kEntryPad) * sizeof(uint16_t)));
    LBL_HIP_TRY(hipMalloc(&sp->val, (nnz + kEntryPad) * sizeof(uint64_t)));
    LBL_HIP_TRY(hipMemset(sp->row + nnz, 0, kEntryPad * sizeof(uint16_t)));
    LBL_HIP_TRY(hipMemset(sp->val + nnz, 0, kEntryPad * sizeof(uint64_t)));
    sp->nnz = nnz;

    // 3. non-empty segments, and the tilings over them
    std::vector<uint64_t> seg_start, rb_seg(sp->n_rb + 1, 0);
    std::vector<uint32_t> seg_word;
    uint64_t at = 0;
    uint32_t rb = 0;
    for (SparsePart &p : parts) {
        if (p.nnz) {
            LBL_HIP_TRY(hipMemcpy(sp->row + at, p.row, p.nnz * sizeof(uint16_t), hipMemcpyDeviceToDevice));
            LBL_HIP_TRY(hipMemcpy(sp->val + at, p.val, p.nnz * sizeof(uint64_t), hipMemcpyDeviceToDevice));
        }
        for (uint32_t r = 0; r < p.n_rb; ++r, ++rb) {
            rb_seg[rb] = seg_word.size();
            for (uint32_t w = 0; w < W; ++w) {
                const uint32_t c = p.cnt[(uint64_t)r * W + w];
                if (c == 0) continue;
                seg_start.push_back(at);
                seg_word.push_back(w);
                at += c;
            }
        }
        SparsePart done(std::move(p));  // device arrays released here
    }
    rb_seg[sp->n_rb] = seg_word.size();
    seg_start.push_back(nnz);
    sp->n_segments = seg_word.size();
    // the words whose tables a frame needs (all of them: no list)
    std::vector<uint8_t> used(W, 0);
    for (uint32_t w : seg_word) used[w] = 1;
    std::vector<uint32_t> used_list;
    for (uint32_t w = 0; w < W; ++w)
        if (used[w]) used_list.push_back(w);
    sp->n_used = (uint32_t)used_list.size();
    // every word is packed when every word is used (or none: the tables are
    // then unread)
    if (sp->n_used == W || sp->n_used == 0) {
        used_list.resize(W);
        for (uint32_t w = 0; w < W; ++w) used_list[w] = w;
    }
    {
        std::vector<uint32_t> first(used_list.size());
        for (size_t i = 0; i < used_list.size(); ++i)
            first[i] = a->order.morton ? used_list[i] * 64u : a->order.word_cell[(uint64_t)used_list[i] * 64];
        LBL_HIP_TRY(hipMalloc(&sp->pack_first, std::max<size_t>(first.size(), 1) * sizeof(uint32_t)));
        if (!first.empty())
            LBL_HIP_TRY(hipMemcpy(sp->pack_first, first.data(), first.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    }
    if (sp->n_used < W && sp->n_used > 0) {
        LBL_HIP_TRY(hipMalloc(&sp->used_words, used_list.size() * sizeof(uint32_t)));
        LBL_HIP_TRY(hipMemcpy(sp->used_words, used_list.data(), used_list.size() * sizeof(uint32_t),
                              hipMemcpyHostToDevice));
    } else {
        sp->n_used = W;
    }
    // tile workgroups use more than 64 KB of LDS
    LBL_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_label_tiles<kTileWaves, uint64_t>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTileLds));
    LBL_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_label_tiles<kTileWaves, uint32_t>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTileLds32));
    for (const void *f : {reinterpret_cast<const void *>(&k_label_direct<kTileWaves, 1>),
                          reinterpret_cast<const void *>(&k_label_direct<kTileWaves, 2>),
                          reinterpret_cast<const void *>(&k_label_direct<kTileWaves, 4>)})
        LBL_HIP_TRY(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDirectLds));
    LBL_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_label_tiles_batch<kTileWaves>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTileLds));
    LBL_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_label_tiles_queue<kTileWaves>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTileLds));
    const uint32_t n_cu = (uint32_t)device_cu_count();
    sp->tilings.resize(kNarrowTiling + 1);
    std::vector<uint16_t> rows_host(nnz);
    if (nnz) LBL_HIP_TRY(hipMemcpy(rows_host.data(), sp->row, nnz * sizeof(uint16_t), hipMemcpyDeviceToHost));
    for (int i = 0; i <= kNarrowTiling; ++i) {
        // the 32-bit mask kernel runs two tile workgroups per CU
        const bool one_frame = i == 0 || i == kNarrowTiling;
        std::vector<uint32_t> k = one_frame ? choose_tiles(block_costs(seg_start, rb_seg), i == 0 ? n_cu : 2 * n_cu)
                                            : std::vector<uint32_t>(sp->n_rb, 1u << (i - 1));
        TilingHost h;
        make_tiling(seg_start, seg_word, rb_seg, k, &h);
        // the tile kernels address a task's entries (8 bytes each) and round
        // records with 32-bit byte offsets
        for (const SpTask &t : h.tasks)
            LBL_REQUIRE((uint64_t)t.n_rounds * sizeof(SpRound) < (1ull << 32) &&
                            (t.n_rounds == 0 || (uint64_t)h.rounds[t.round0 + t.n_rounds - 1].e_off + 64 < (1ull << 29)),
                        "a tile task spans more entries than the tile kernels address");
        lbl_status st = upload_tiling(h, &sp->tilings[i], &sp->round_bytes);
        if (st != LBL_OK) return st;
        CompactHost c;
        if (make_compact(h, rows_host, seg_start, rb_seg, a->n_traj, &c)) {
            st = upload_compact(c, &sp->tilings[i], &sp->round_bytes);
            if (st != LBL_OK) return st;
        }

    }
    {
        // the direct-mask kernel's tiles: two workgroups per CU
        DirectHost dh;
        make_direct(seg_start, rb_seg, 2 * n_cu, &dh);
        lbl_status st = upload_direct(dh, seg_word, &sp->direct, &sp->round_bytes);
        if (st != LBL_OK) return st;
    }
    LBL_HIP_TRY(hipDeviceSynchronize());
    a->sp = sp.release();
    return LBL_OK;
}

lbl_status build_sparse(lbl_abs *a)
{
    if (a->n_traj >= (1ull << 32)) return LBL_OK;  // row ids are 32-bit: keep only the bitpacked layout
    std::vector<SparsePart> parts(1);
    lbl_status st = sparse_part(a->T_bits, a->row_stride, a->n_traj, a->n_words, &parts[0]);
    if (st != LBL_OK) return st;
    return sparse_assemble(a, parts);
}

namespace {

// Whether a frame of n_props propositions takes the direct-mask kernels
// (the layout has their split and a part's segment masks fit their LDS);
// *np is then the masks per word (1, 2 or 4).
bool takes_direct(const SparseLayout &sp, uint32_t n_props, uint32_t *np)
{
    *np = n_props <= 1 ? 1 : n_props <= 2 ? 2 : 4;
    return n_props <= 4 && sp.direct.chunks != nullptr &&
           (size_t)sp.direct.max_part_segs * *np * sizeof(uint64_t) <= kDirectMaskBytes;
}

}  // namespace

size_t swm_frame_workspace_bytes(const lbl_abs *a, uint32_t n_props)
{
    const SparseLayout &sp = *a->sp;
    uint32_t np = 0;
    if (takes_direct(sp, n_props, &np)) return up256((size_t)a->n_words * np * sizeof(uint64_t));
    auto bytes = [&](int ti, size_t mask) {
        const SpTiling &tl = sp.tilings[ti];
        const size_t partials = tl.tile_slot ? (size_t)tl.n_slots : (size_t)tl.n_tiles * kRowBlock;
        return up256((size_t)a->n_words * 256 * mask) + partials * mask;
    };
    if (n_props <= 32 && (int)sp.tilings.size() > kNarrowTiling) return bytes(kNarrowTiling, sizeof(uint32_t));
    return bytes(0, sizeof(uint64_t));
}

size_t swm_workspace_bytes(const lbl_abs *a, uint32_t n_lane_groups, int t)
{
    auto bytes = [&](int ti, size_t mask) {
        const SpTiling &tl = a->sp->tilings[ti];
        const size_t partials = tl.tile_slot && n_lane_groups == 1 ? (size_t)tl.n_slots
                                                                    : (size_t)n_lane_groups * tl.n_tiles * kRowBlock;
        return up256((size_t)a->n_words * 256 * n_lane_groups * mask) + partials * mask;
    };
    size_t b = bytes(t, sizeof(uint64_t));
    if (t == 0 && n_lane_groups == 1 && (int)a->sp->tilings.size() > kNarrowTiling)
        b = std::max(b, bytes(kNarrowTiling, sizeof(uint32_t)));
    return b;
}

namespace {

// The three kernels of one frame with M-bit masks on tiling tl.
template <typename M>
lbl_status run_swm_t(const lbl_abs *a, const SpTiling &tl, size_t lds, const uint8_t *O, uint32_t n_props, void *ws,
                     uint8_t *L, hipStream_t s, bool spans)
{
    const SparseLayout &sp = *a->sp;
    M *Tg = static_cast<M *>(ws);
    M *P = Tg + up256((size_t)a->n_words * 256 * sizeof(M)) / sizeof(M);
    auto span_begin = [&](hipStream_t st) { return spans ? lbl::span_begin(st) : nullptr; };
    auto span_end = [&](void *b, hipStream_t st, int kind) {
        if (spans) lbl::span_end(b, st, kind);
    };
    void *spn = span_begin(s);
    hipLaunchKernelGGL(k_pack_tables<M>, dim3((unsigned)(((uint64_t)sp.n_used * 64 + 255) / 256)), dim3(256), 0, s, O,
                       n_props, sp.pack_first, a->nx, (uint32_t)a->order.morton, sp.used_words, sp.n_used, Tg);
    LBL_HIP_TRY(hipGetLastError());
    span_end(spn, s, 0);
    spn = span_begin(s);
    hipLaunchKernelGGL((k_label_tiles<kTileWaves, M>), dim3(tl.n_tiles), dim3(64 * kTileWaves), lds, s,
                       tl.block_tile, tl.tasks_launch, tl.rounds, sp.row, sp.val, Tg, P, tl.tile_slot, tl.slot_row);
    LBL_HIP_TRY(hipGetLastError());
    span_end(spn, s, 1);
    spn = span_begin(s);
    hipLaunchKernelGGL(k_combine<M>, dim3(grid_cap(a->n_traj, 256, 16384)), dim3(256), 0, s, P, tl.rb_tile,
                       tl.row_slot_off, tl.row_slots, a->n_traj, n_props, L);
    LBL_HIP_TRY(hipGetLastError());
    span_end(spn, s, 3);
    return LBL_OK;
}

// The two kernels of a frame of at most NP <= 4 propositions: per-word
// proposition masks (and L zeroed), then the direct-mask label kernel, which
// writes L.  The masks take the place of the nibble tables in the workspace.
template <int NP>
lbl_status run_swm_direct(const lbl_abs *a, const uint8_t *O, uint32_t n_props, void *ws, uint8_t *L,
                          hipStream_t s, bool spans)
{
    const SparseLayout &sp = *a->sp;
    const DirectLayout &d = sp.direct;
    uint64_t *Tm = static_cast<uint64_t *>(ws);
    auto span_begin = [&](hipStream_t st) { return spans ? lbl::span_begin(st) : nullptr; };
    auto span_end = [&](void *b, hipStream_t st, int kind) {
        if (spans) lbl::span_end(b, st, kind);
    };
    const uint64_t n_L = a->n_traj * n_props;
    const uint64_t pack_blocks = std::max<uint64_t>(((uint64_t)sp.n_used * 64 + 255) / 256,
                                                    std::min<uint64_t>((n_L + 4095) / 4096, 1024));
    void *spn = span_begin(s);
    hipLaunchKernelGGL(k_pack_masks<NP>, dim3((unsigned)pack_blocks), dim3(256), 0, s, O, n_props, sp.pack_first,
                       a->nx, (uint32_t)a->order.morton, sp.used_words, sp.n_used, Tm, L, n_L);
    LBL_HIP_TRY(hipGetLastError());
    span_end(spn, s, 0);
    spn = span_begin(s);
    hipLaunchKernelGGL((k_label_direct<kTileWaves, NP>), dim3(d.n_tiles), dim3(64 * kTileWaves), kDirectLds, s,
                       d.tile_part, d.parts, d.chunks, d.seg_word, sp.row, sp.val, Tm, a->n_traj, n_props, L);
    LBL_HIP_TRY(hipGetLastError());
    span_end(spn, s, 1);
    return LBL_OK;
}

}  // namespace

lbl_status run_swm(const lbl_abs *a, const uint8_t *O, uint32_t n_props, void *ws, uint8_t *L, hipStream_t s,
                   bool spans)
{
    LBL_REQUIRE(a->sp != nullptr, "the abstraction has no sparse layout");
    const SparseLayout &sp = *a->sp;
    // frames of at most 4 propositions take the direct-mask kernel (which
    // holds a part's segment masks in LDS), those of at most 32 the 32-bit
    // mask kernels
    uint32_t np = 0;
    if (takes_direct(sp, n_props, &np)) {
        if (n_props == 1) return run_swm_direct<1>(a, O, n_props, ws, L, s, spans);
        if (n_props == 2) return run_swm_direct<2>(a, O, n_props, ws, L, s, spans);
        return run_swm_direct<4>(a, O, n_props, ws, L, s, spans);
    }
    if (n_props <= 32 && (int)sp.tilings.size() > kNarrowTiling)
        return run_swm_t<uint32_t>(a, sp.tilings[kNarrowTiling], kTileLds32, O, n_props, ws, L, s, spans);
    return run_swm_t<uint64_t>(a, sp.tilings[0], kTileLds, O, n_props, ws, L, s, spans);
}

}  // namespace lbl
