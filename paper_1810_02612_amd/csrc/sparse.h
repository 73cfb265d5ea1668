// Sparse tiled layout of T (built at load time) and its frame kernels.
#pragma once

#include <memory>
#include <vector>

#include "lbl_internal.h"

namespace lbl {

// Rows per row block (local rows fit in 16 bits; a block's accumulators fill
// 64 KB of LDS).
constexpr uint32_t kRowBlock = 8192;
// Wavefronts per tile workgroup (one workgroup per CU: 16 wavefronts).
constexpr uint32_t kTileWaves = 16;
// Zeroed entries stored past the last entry of the layout, so that every lane
// of a round may load its entry without a bounds check.
constexpr uint64_t kEntryPad = 64;
// Rounds a wavefront has in flight (records, entries and table data loaded
// ahead of the round being processed).  Two: the entries and table data of
// the next round load while a round is processed, its record one round
// earlier.  Measured on the 200k x 512^2 frames (64 and 32 propositions),
// one is 35% slower and three and four 3% and 6% slower than two.
constexpr int kStages = 2;
// Nibble tables a wavefront holds at once (a round touches at most two
// segments).
constexpr uint32_t kRing = 2;
// A nibble table is 16 rows (nibble position) of 16 entries (nibble value),
// each row padded by one entry: the 64 lanes of a table build then write to
// distinct banks, and the second table of a wavefront starts half a bank
// row after the first, so lookups into the two tables in one instruction do
// not collide.
constexpr uint32_t kTabRow = 17;
constexpr uint32_t kTabWords = 16 * kTabRow;
// LDS of a tile workgroup: accumulators + every wavefront's tables.
constexpr size_t kTileLds = ((size_t)kRowBlock + (size_t)kTileWaves * kRing * kTabWords) * sizeof(uint64_t);
// The same with 32-bit masks (frames of at most 32 propositions): 66 KiB, so
// two tile workgroups share a CU.
constexpr size_t kTileLds32 = ((size_t)kRowBlock + (size_t)kTileWaves * kRing * kTabWords) * sizeof(uint32_t);

// One wavefront's share of a tile: consecutive entries lo .. of one row
// block, processed as rounds [round0, round0 + n_rounds).
struct SpTask {
    uint64_t lo;
    uint32_t n_rounds;
    uint32_t round0;
};

// One round: up to 64 consecutive entries, lane l taking entry
// task.lo + e_off + l, each lane in one of two segments (words).  A round
// builds at most one table slot: the first segment's (build0) or the
// second's (build1), from the nibble tables of word tword.
struct SpRound {
    uint32_t e_off;  // multiple of 64
    uint32_t tword;  // word whose tables the round copies (the last built word if none)
    uint32_t pad;
    uint32_t meta;   // lane_lo | lane_hi << 8 | cut << 16 | build0 << 24 | build1 << 25 | slot0 << 26
};
constexpr uint32_t kMetaBuild0 = 1u << 24, kMetaBuild1 = 1u << 25, kMetaSlot0 = 1u << 26;

// One chunk for the direct-mask kernel (frames of at most 4 propositions):
// up to 64 consecutive entries of one row block, lane l taking entry
// chunk start + l.  Bit i of `starts` is set iff entry i + 1 of the chunk
// begins a new segment, so lane l's segment is seg0 (that of entry 0,
// counted from its part's first segment) plus the popcount of the bits below
// l.  Lanes at or past n_valid hold no entry.
struct SpChunk {
    uint64_t starts;
    uint32_t seg0;
    uint32_t n_valid;
};

// A part of a direct-mask tile: the tile's chunks [c0, c1) that lie in row
// block rb, the first of them starting at entry e0; their segments are
// seg_first .. + n_seg.
struct DirectPart {
    uint64_t e0;
    uint32_t c0, c1;
    uint32_t rb;
    uint32_t seg_first, n_seg;
    uint32_t pad;
};

// The direct-mask kernel's split of the layout: the chunks of every row
// block (64 entries from the block's first, the block's last chunk
// partial), in layout order, cut into n_tiles tiles of equal chunk counts;
// a tile spanning row blocks has one part per block.  Tile t's parts are
// tile_part[t] .. tile_part[t + 1].  Empty (no device arrays) when not built.
struct DirectLayout {
    uint32_t n_tiles = 0;
    uint32_t n_parts = 0;
    uint32_t max_part_segs = 0;
    uint64_t n_chunks = 0;
    uint32_t *tile_part = nullptr;  // device [n_tiles + 1]
    DirectPart *parts = nullptr;    // device
    SpChunk *chunks = nullptr;      // device [n_chunks]
    uint32_t *seg_word = nullptr;   // device [segments]
};
struct DirectHost {
    std::vector<uint32_t> tile_part;
    std::vector<DirectPart> parts;
    std::vector<SpChunk> chunks;
};
// Host: the direct-mask split of a row-block-ordered segment list into
// n_tiles tiles (see SparseLayout::direct).
void make_direct(const std::vector<uint64_t> &seg_start, const std::vector<uint64_t> &rb_seg, uint32_t n_tiles,
                 DirectHost *out);

// A split of the layout into tiles: kTileWaves tasks per tile, every tile in
// one row block; rb_tile[rb] .. rb_tile[rb + 1] are the tiles of block rb.
struct SpTiling {
    uint32_t n_tiles = 0;
    uint64_t n_rounds = 0;
    SpTask *tasks = nullptr;     // device [n_tiles * kTileWaves]
    SpRound *rounds = nullptr;   // device [n_rounds]
    uint32_t *rb_tile = nullptr; // device [n_rb + 1]
    uint32_t *block_tile = nullptr; // device [n_tiles] launch order of a one-frame launch
    SpTask *tasks_launch = nullptr; // device [n_tiles * kTileWaves] the tasks of workgroup b at b * kTileWaves
    std::vector<uint32_t> rb_tile_host;
    // Compact partial labels (the one-frame tiling): a tile writes the
    // partials of only the rows it touches, slots tile_slot[tile] ..
    // tile_slot[tile + 1] holding local rows slot_row[..] (ascending); row t's
    // partials are the slots row_slots[row_slot_off[t] .. row_slot_off[t + 1]).
    // Null when not built (then a tile writes all kRowBlock rows).
    uint64_t n_slots = 0;
    uint32_t *tile_slot = nullptr;     // device [n_tiles + 1]
    uint16_t *slot_row = nullptr;      // device [n_slots]
    uint32_t *row_slot_off = nullptr;  // device [n_traj + 1]
    uint32_t *row_slots = nullptr;     // device [n_slots]
};

// XCDs of an MI355X.  Workgroup b of a launch runs on XCD b % kXcds, and
// each XCD has its own L2.
constexpr uint32_t kXcds = 8;

// Device-resident sparse layout of one abstraction.
struct SparseLayout {
    uint32_t n_rb = 0;
    uint64_t nnz = 0;            // entries (non-zero words of T)
    uint64_t n_segments = 0;     // non-empty (row block, word) segments
    uint16_t *row = nullptr;     // device [nnz] row within the row block
    uint64_t *val = nullptr;     // device [nnz] word value
    uint32_t n_used = 0;         // words held by some entry (their tables are packed per frame)
    uint32_t *used_words = nullptr;  // device [n_used] ascending, or null when every word is used
    uint32_t *pack_first = nullptr;  // device [n_used] the first cell id of each packed word
    // tilings[0]: one frame (about one tile per CU, tiles of equal cost);
    // tilings[1 + i]: 2^i tiles per row block (batches); tilings[kNarrowTiling]:
    // one frame of at most 32 propositions (about two tiles per CU)
    std::vector<SpTiling> tilings;
    // the direct-mask kernel's tiles (frames of at most 4 propositions)
    DirectLayout direct;
    size_t round_bytes = 0;      // device bytes of all tilings' tables
    ~SparseLayout();
};

constexpr int kBatchTilings = 4;  // 1, 2, 4, 8 tiles per row block
constexpr int kNarrowTiling = 1 + kBatchTilings;

// Build the tiled layout of a from its bitpacked T (sets a->sp).
lbl_status build_sparse(lbl_abs *a);

// Entries of a run of whole row blocks, built from that run's bitpacked rows
// (rows local to each row block, segments ordered row block by row block,
// then by word).  cnt[rb * n_words + w] is the entry count of segment
// (rb, w) of the run.  row and val are device arrays of nnz entries.
struct SparsePart {
    uint16_t *row = nullptr;
    uint64_t *val = nullptr;
    uint64_t nnz = 0;
    uint32_t n_rb = 0;
    std::vector<uint32_t> cnt;
    SparsePart() = default;
    SparsePart(const SparsePart &) = delete;
    SparsePart &operator=(const SparsePart &) = delete;
    SparsePart(SparsePart &&o) noexcept;
    ~SparsePart();
};
// Entries of rows [0, n_rows) of the bitpacked T (row_stride words apart);
// n_rows is a multiple of kRowBlock except for the abstraction's last run.
lbl_status sparse_part(const uint64_t *T, uint32_t row_stride, uint64_t n_rows, uint32_t n_words,
                       SparsePart *out);
// Concatenate the parts of a's row blocks, in row order, into a's tiled
// layout and its tilings (sets a->sp); the parts are released.
lbl_status sparse_assemble(lbl_abs *a, std::vector<SparsePart> &parts);

// Workspace bytes for one frame of n_lane_groups 64-column groups on tiling
// t (nibble tables + per-tile partial labels); for one frame (the defaults),
// the larger of the 64-bit and the 32-bit mask paths.
size_t swm_workspace_bytes(const lbl_abs *a, uint32_t n_lane_groups = 1, int t = 0);
// Workspace bytes run_swm needs for one frame of n_props propositions (the
// kernels that frame takes).
size_t swm_frame_workspace_bytes(const lbl_abs *a, uint32_t n_props);

// Pack O, label through the tiled layout, write L (device pointers).
// spans: record profiling events around the kernels (when profiling is on).
lbl_status run_swm(const lbl_abs *a, const uint8_t *O, uint32_t n_props, void *ws, uint8_t *L, hipStream_t s,
                   bool spans = true);

// Relative work of wavefront w of a tile workgroup (tasks are sized to it).
double wave_share(uint32_t w);

// Host-side: the tasks and rounds of one tiling of a row-block-ordered
// segment list (exposed for host tests).  seg_start[s] .. seg_start[s + 1]
// are the entries of segment s, seg_word[s] its word, rb_seg[rb] ..
// rb_seg[rb + 1] the segments of row block rb.  tiles_rb[rb] >= 1 tiles per
// row block; the block's tasks start at 64-entry chunk boundaries and have
// equal cost (rounds, plus a charge per table copy) as the block is walked.
// block_tile: the tile workgroup b of a one-frame launch runs; tiles are
// ranked by the word at their middle entry and the ranks split into kXcds
// consecutive groups, one per XCD, so that each XCD's L2 holds the nibble
// tables of about 1 / kXcds of the words.
struct TilingHost {
    std::vector<SpTask> tasks;
    std::vector<SpRound> rounds;
    std::vector<uint32_t> rb_tile;
    std::vector<uint32_t> block_tile;
};
void make_tiling(const std::vector<uint64_t> &seg_start, const std::vector<uint32_t> &seg_word,
                 const std::vector<uint64_t> &rb_seg, const std::vector<uint32_t> &tiles_rb, TilingHost *out);
// Compact partial slots of a tiling (host): row[e] is the local row of entry
// e; tile i of block rb covers entries [tasks[i * kTileWaves].lo, the next
// tile's first entry or the block's end).  Fails (false) if the slots
// number 2^32 or more.
struct CompactHost {
    std::vector<uint32_t> tile_slot, row_slot_off, row_slots;
    std::vector<uint16_t> slot_row;
};
bool make_compact(const TilingHost &h, const std::vector<uint16_t> &row, const std::vector<uint64_t> &seg_start,
                  const std::vector<uint64_t> &rb_seg, uint64_t n_traj, CompactHost *out);
// Cost of walking each row block's entries in rounds.
std::vector<double> block_costs(const std::vector<uint64_t> &seg_start, const std::vector<uint64_t> &rb_seg);
// Tiles per row block (at least one each) for `target` tiles in total of
// about equal cost.
std::vector<uint32_t> tiles_per_block(const std::vector<double> &cost, uint32_t target);
// Fixed cost of one tile workgroup in rounds (its start-up latency and the
// write-back of its partials, about 5 us at the ~28 rounds per microsecond a
// workgroup retires).
constexpr double kTileFixedRounds = 128.0;
// The combine's cost per tile (64 KiB of partials read by the whole chip),
// in the same units of one workgroup's rounds.
constexpr double kTileCombineRounds = 0.75;
// Tiles per row block for a one-frame launch.  Tiles cannot span row blocks,
// so with fewer row blocks than about twice the CUs one tile per CU leaves
// some tiles a whole row block; candidate totals of 1 to 4 workgroups per
// CU are scored by a list schedule (each tile to the CU that frees first,
// cost per tile plus kTileFixedRounds) plus kTileCombineRounds per tile, and
// the shortest wins, fewer tiles on near ties.
std::vector<uint32_t> choose_tiles(const std::vector<double> &cost, uint32_t n_cu);

}  // namespace lbl
