// Batched labeling: many frames over several abstractions in one persistent
// launch.  Used by lbl_label_batch (graph-cached) and by the server (direct).
#pragma once

#include "lbl_internal.h"

namespace lbl {

struct SpTask;
struct SpRound;

// Per output lane (one proposition column of one frame).
struct LaneDesc {
    const uint8_t *O;  // &O_job[p] (cell c at O[c * n_props]), null for an unused lane
    uint8_t *L;        // &L_job[p] (row t at L[t * n_props]), null for an unused lane
    uint32_t n_props;
    uint32_t pad;
};

// One job's columns inside a lane group.  Jobs are packed into lane groups
// first-fit by decreasing proposition count, so a job's columns never span
// two lane groups: lane group gi holds whole jobs, job s at columns
// [bit, bit + n_props).
struct SegDesc {
    const uint8_t *O;  // the job's O (cell c's propositions at O + c * n_props)
    uint8_t *L;        // the job's L (row t at L + t * n_props)
    uint32_t n_props;  // the job's proposition count: the row pitch of O and L
    uint32_t bit;      // first column of the job inside its lane group
};

// Per abstraction group: all jobs on one abstraction, propositions
// concatenated into G64 groups of 64 lanes.
struct GroupDesc {
    const uint64_t *T;
    const uint32_t *word_cell;
    uint64_t *Ow;             // bitpacked plans: [n_words][G64][64] masks, one per column
                              // (64 cells each); sparse plans: [n_words][G64][256] nibble
                              // tables
    const LaneDesc *lanes;    // [G64][64]
    const SegDesc *segs;      // the jobs of lane group gi: segs[lg_seg[gi] .. lg_seg[gi + 1])
    const uint32_t *lg_seg;   // [G64 + 1]
    uint64_t n_traj;
    uint32_t row_stride;
    uint32_t n_words;
    uint32_t G64;
    // sparse plans: the tiling of T's sparse layout this pass runs on, and
    // the pass's partial labels
    const SpTask *sp_tasks;
    const SpRound *sp_rounds;
    const uint32_t *sp_rb_tile;  // [n_rb + 1] first tile of each row block
    const uint16_t *sp_row;
    const uint64_t *sp_val;
    uint64_t max_entry;
    uint64_t *P;                 // [G64][n_slots] compact, else [G64][n_tiles][kRowBlock] (null when fused)
    // compact partials (the tiling's slot lists; null: full partials): tile
    // i writes slots tile_slot[i] .. tile_slot[i + 1] (local rows
    // slot_row[..]); row t's slots are row_slots[row_slot_off[t] ..
    // row_slot_off[t + 1])
    const uint32_t *tile_slot;
    const uint16_t *slot_row;
    const uint32_t *row_slot_off;
    const uint32_t *row_slots;
    uint64_t n_slots;
    uint32_t n_tiles;
    uint32_t n_rb;
    uint32_t fused;              // one tile per row block: tiles write the label bytes
    uint32_t nx;                 // grid width in cells (row-major cell ids)
    uint32_t morton;             // 1: the caller's cell ids are z-order
    uint32_t pad;
};

// Sparse plans: one wavefront per (group, lane group, words [w0, w1)) packs
// the nibble tables of those words for the lane group.
struct PackItem {
    uint32_t group, gi, w0, w1;
};

// Sparse plans: one workgroup per (group, tile, lane group).
struct TileItem {
    uint32_t group, tile, gi, pad;
};

// Sparse plans: one wavefront per (group, lane group, 64-row chunk range).
struct CombineItem {
    uint32_t group, gi;
    uint64_t row0, row1;
};

struct WorkItem {
    uint32_t group;
    uint32_t pad;
    uint64_t row0, row1;
};

// Launch choices of a batch.  Bitpacked plans use unroll, waves_per_block
// and rows_per_item; sparse plans use tiling (0: the plan's default; else
// 1 + the index of the layout's tiling: 1 = the one-frame tiling, 2..5 = 1,
// 2, 4, 8 tiles per row block) and persistent (1: one workgroup per CU
// pulling tiles from per-XCD queues; 0: one workgroup per tile).
struct BatchTile {
    int unroll = 8;
    int waves_per_block = 4;
    int rows_per_item = 128;
    int tiling = 0;
    int persistent = 1;
    bool operator==(const BatchTile &o) const
    {
        return unroll == o.unroll && waves_per_block == o.waves_per_block && rows_per_item == o.rows_per_item &&
               tiling == o.tiling && persistent == o.persistent;
    }
};

struct JobRef {
    lbl_abs *a;
    const uint8_t *O;
    uint32_t n_props;
    uint8_t *L;
};

// Host-side description of one launch: groups, lane tables, work items.
struct BatchPlan {
    std::vector<GroupDesc> groups;  // Ow and lanes fields are offsets until bound
    std::vector<LaneDesc> lanes;    // all groups' lane tables, concatenated
    std::vector<size_t> lane_off;   // first lane of each group
    std::vector<SegDesc> segs;      // all groups' job segments, by group then lane group
    std::vector<uint32_t> lg_seg;   // per group G64 + 1 entries (absolute indices into segs)
    std::vector<size_t> lgs_off;    // first lg_seg entry of each group
    std::vector<size_t> ow_off;     // byte offset of each group's Ow in the Ow region
    std::vector<WorkItem> items;
    size_t ow_bytes = 0;
    uint32_t max_g64 = 1;
    uint64_t pack_units = 0;        // sum over groups of n_words * G64
    BatchTile tile;
    uint64_t pairs = 0;             // labeled (trajectory, proposition) pairs
    std::string shape_key;
    // sparse plans (every abstraction of the batch has the sparse layout)
    bool sparse = false;
    std::vector<size_t> p_off;      // byte offset of each group's partials in the P region
    size_t p_bytes = 0;
    std::vector<TileItem> tiles;    // in queue order: XCD x's queue is tiles[xcd_start[x] .. xcd_start[x + 1])
    std::vector<uint32_t> xcd_start;  // kXcds + 1 entries (sparse plans)
    std::vector<uint32_t> launch;   // one-workgroup-per-tile launches: workgroup b runs tiles[launch[b]]
    std::vector<CombineItem> combines;  // empty for fused passes
    std::vector<PackItem> packs;
    std::vector<const lbl_abs *> group_abs;  // abstraction of each group
    int default_tiling = 1;         // sparse: tiling index used when the tile does not choose one
    int tiling = 0;                 // sparse: index of the tilings every pass uses (set by plan_finalize)

    bool finalized = false;         // tile set and items made

    // bytes of device memory the launch needs (tables + packed masks); only
    // meaningful once the plan is finalized
    size_t device_bytes() const;
};

// Build the plan (validates jobs; device >= 0 also requires every abstraction
// to live on that device).  Jobs on one abstraction are split into passes of
// at most LBL_BATCH_MAX_PROPS propositions.  Host-only.
lbl_status plan_batch(const JobRef *jobs, size_t n_jobs, int device, BatchPlan *out);

// Fix the tile and make the work items (row ranges, costliest groups first).
// Must precede device_bytes() and bind_batch().  Host-only.
void plan_finalize(BatchPlan &plan, const BatchTile &tile);

// Device buffer holding the plan's tables and masks, laid out by bind_batch.
struct BatchBuffers {
    uint8_t *base = nullptr;
    size_t bytes = 0;
    GroupDesc *d_groups = nullptr;
    WorkItem *d_items = nullptr;
    LaneDesc *d_lanes = nullptr;
    uint64_t *d_pack_prefix = nullptr;
    uint32_t *d_counter = nullptr;
    uint64_t *d_ow = nullptr;
    TileItem *d_tiles = nullptr;
    uint32_t *d_launch = nullptr;
    uint32_t *d_xcd_start = nullptr;
    uint32_t *d_queues = nullptr;   // kXcds queue counters (zeroed by a kernel before each launch)
    CombineItem *d_combines = nullptr;
    PackItem *d_packs = nullptr;
    SegDesc *d_segs = nullptr;
    uint32_t *d_lg_seg = nullptr;
    uint64_t *d_p = nullptr;
};

// Sparse batch kernels (defined with the sparse layout's kernels).
// Pack: one wavefront per pack item (group, lane group, word range) -> the
// words' nibble tables for the lane group's columns.
hipError_t launch_pack_batch_tables(const GroupDesc *d_groups, const PackItem *d_packs, uint32_t n_packs,
                                    hipStream_t s);
// Tiles: persistent (one workgroup per CU, per-XCD queues with stealing;
// d_queues zeroed first) or one workgroup per tile in launch order.
hipError_t launch_tiles_batch(const GroupDesc *d_groups, const TileItem *d_tiles, const uint32_t *d_launch,
                              uint32_t n_tiles, hipStream_t s);
hipError_t launch_tiles_batch_queue(const GroupDesc *d_groups, const TileItem *d_tiles, const uint32_t *d_xcd_start,
                                    uint32_t *d_queues, uint32_t n_workgroups, hipStream_t s);
hipError_t launch_combine_batch(const GroupDesc *d_groups, const CombineItem *d_items, uint32_t n_items,
                                hipStream_t s);

// Lay the finalized plan out in `base` (capacity bytes of device memory) and
// fill `host_image` with the bytes to copy to base (tables; masks excluded).
// LBL_EINVAL if the plan is not finalized, LBL_ENOMEM if it needs more than
// capacity.  Host-only.
lbl_status bind_batch(const BatchPlan &plan, uint8_t *base, size_t capacity, BatchBuffers *bufs,
                      std::vector<uint8_t> *host_image);
size_t batch_table_bytes(const BatchPlan &plan);

// Enqueue: counter reset, O packing for every job, persistent label kernel.
lbl_status enqueue_batch(const BatchPlan &plan, const BatchBuffers &bufs, hipStream_t s);

int device_cu_count();

// Tile recorded by lbl_tune_batch for a shape class (the default if none).
BatchTile batch_tile_for(const std::string &shape_key);
void set_batch_tile(const std::string &shape_key, const BatchTile &t);
// Every recorded (shape class, tile) pair, for the tune cache file.
std::vector<std::pair<std::string, BatchTile>> batch_tiles();
std::string batch_tile_name(const BatchPlan &p);

}  // namespace lbl
