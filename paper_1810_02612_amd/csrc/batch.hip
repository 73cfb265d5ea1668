// Batched labeling in one persistent launch.
//
// Jobs on the same abstraction form a group: their propositions are laid
// side by side in G64 lane groups of 64, so one pass over T labels all of
// them (T is read once per batch, not once per frame).  The O packing of
// every job is one kernel; the labeling is one persistent kernel whose
// workgroups pull (group, row range) items from an atomic counter, largest
// items first, so uneven abstractions share the GPU without a tail of idle
// CUs.  lbl_label_batch records the whole pipeline once as a HIP graph keyed
// by (stream, jobs, flags) and replays it.
#include <algorithm>
#include <cstring>
#include <list>
#include <map>
#include <memory>

#include "batch.h"
#include "profile.h"
#include "sparse.h"
#include "tables.h"

namespace lbl {

namespace {

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int src)
{
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// Zero the work counter (a kernel, not a memset node, so graph replays are safe).
__global__ void k_zero(uint32_t *counter) { *counter = 0u; }

// Zero n counters (n <= 64).
__global__ void k_zero_n(uint32_t *counters, uint32_t n)
{
    if (threadIdx.x < n) counters[threadIdx.x] = 0u;
}

// Bitpacked plans: one wavefront per (group, word, lane group): lane l packs
// the 64 cells of the word for the proposition column that lane (gi, l)
// stands for.
__global__ void __launch_bounds__(256)
k_pack_batch(const GroupDesc *__restrict__ groups, const uint64_t *__restrict__ prefix, uint32_t n_groups,
             uint64_t n_units)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t u = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); u < n_units; u += waves) {
        uint32_t gidx = 0;
        while (gidx + 1 < n_groups && prefix[gidx + 1] <= u) ++gidx;
        const GroupDesc g = groups[gidx];
        const uint64_t local = u - prefix[gidx];
        const uint32_t w = (uint32_t)(local / g.G64), gi = (uint32_t)(local % g.G64);
        const LaneDesc d = g.lanes[gi * 64 + lane];
        uint64_t m = 0;
        if (d.O) {
            const uint32_t *wc = g.word_cell + (uint64_t)w * 64;
#pragma unroll 16
            for (uint32_t b = 0; b < 64; ++b) m |= (uint64_t)(d.O[(uint64_t)wc[b] * d.n_props] != 0) << b;
        }
        g.Ow[((uint64_t)w * g.G64 + gi) * 64 + lane] = m;
    }
}

// Persistent labeling kernel.  Bit gi of lane l's accumulator is the label of
// the proposition column (gi, l) for the current row.
template <int UNROLL, int MAXG>
__global__ void __launch_bounds__(1024)
k_label_batch(const GroupDesc *__restrict__ groups, const WorkItem *__restrict__ items, uint32_t n_items,
              uint32_t *counter)
{
    __shared__ uint32_t s_item;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t it = s_item;
        __syncthreads();
        if (it >= n_items) return;  // uniform: every wavefront of the block leaves together
        const WorkItem item = items[it];
        const GroupDesc g = groups[item.group];
        const uint32_t G = g.G64;
        uint32_t vmask = 0;
#pragma unroll
        for (int gi = 0; gi < MAXG; ++gi)
            if ((uint32_t)gi < G && g.lanes[gi * 64 + lane].L) vmask |= 1u << gi;
        const uint32_t n_pairs = (g.n_words + 1) >> 1;
        for (uint64_t row = item.row0 + wave; row < item.row1; row += n_waves) {
            const u64x2 *Tr = reinterpret_cast<const u64x2 *>(g.T + row * (uint64_t)g.row_stride);
            uint32_t acc = 0;
            for (uint32_t base = 0; base < n_pairs; base += 64 * UNROLL) {
                u64x2 v[UNROLL];
#pragma unroll
                for (int u = 0; u < UNROLL; ++u) {
                    const uint32_t i = base + u * 64 + lane;
                    v[u] = i < n_pairs ? __builtin_nontemporal_load(Tr + i) : u64x2{0ull, 0ull};
                }
#pragma unroll
                for (int u = 0; u < UNROLL; ++u) {
                    uint64_t nz = __ballot((v[u].x | v[u].y) != 0ull);
                    while (nz) {
                        const int src = __builtin_ctzll(nz);
                        nz &= nz - 1ull;
                        const uint64_t wi = 2ull * (base + (uint32_t)(u * 64 + src));
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const uint64_t word = readlane64(h ? v[u].y : v[u].x, src);
                            if (!word) continue;
                            const uint64_t *o = g.Ow + (wi + h) * G * 64 + lane;
#pragma unroll
                            for (int gi = 0; gi < MAXG; ++gi)
                                if ((uint32_t)gi < G) acc |= (uint32_t)((word & o[gi * 64]) != 0ull) << gi;
                        }
                    }
                }
                if (__ballot((acc & vmask) != vmask) == 0ull) break;  // every column already hit
            }
#pragma unroll
            for (int gi = 0; gi < MAXG; ++gi) {
                if ((uint32_t)gi >= G) break;
                const LaneDesc d = g.lanes[gi * 64 + lane];
                if (d.L) d.L[row * d.n_props] = (uint8_t)((acc >> gi) & 1u);
            }
        }
    }
}

template <int U, int G>
hipError_t launch_label(const BatchBuffers &b, uint32_t n_items, int wpb, unsigned blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_label_batch<U, G>), dim3(blocks), dim3(64 * wpb), 0, s, b.d_groups, b.d_items, n_items,
                       b.d_counter);
    return hipGetLastError();
}

template <int U>
hipError_t launch_label_g(const BatchBuffers &b, uint32_t n_items, uint32_t maxg, int wpb, unsigned blocks,
                          hipStream_t s)
{
    if (maxg <= 1) return launch_label<U, 1>(b, n_items, wpb, blocks, s);
    if (maxg <= 2) return launch_label<U, 2>(b, n_items, wpb, blocks, s);
    if (maxg <= 4) return launch_label<U, 4>(b, n_items, wpb, blocks, s);
    if (maxg <= 8) return launch_label<U, 8>(b, n_items, wpb, blocks, s);
    return launch_label<U, 16>(b, n_items, wpb, blocks, s);
}

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

int device_cu_count()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

size_t batch_table_bytes(const BatchPlan &p)
{
    return up256(p.groups.size() * sizeof(GroupDesc)) + up256(p.items.size() * sizeof(WorkItem)) +
           up256(p.lanes.size() * sizeof(LaneDesc)) + up256((p.groups.size() + 1) * sizeof(uint64_t)) + 256 +
           up256(p.tiles.size() * sizeof(TileItem)) + up256(p.launch.size() * sizeof(uint32_t)) +
           up256(p.xcd_start.size() * sizeof(uint32_t)) + up256(p.combines.size() * sizeof(CombineItem)) +
           up256(p.segs.size() * sizeof(SegDesc)) + up256(p.lg_seg.size() * sizeof(uint32_t)) +
           up256(p.packs.size() * sizeof(PackItem));
}

size_t BatchPlan::device_bytes() const { return batch_table_bytes(*this) + ow_bytes + p_bytes; }

lbl_status plan_batch(const JobRef *jobs, size_t n_jobs, int device, BatchPlan *out)
{
    LBL_REQUIRE(jobs != nullptr && n_jobs > 0, "no jobs");
    std::vector<lbl_abs *> order;
    std::map<lbl_abs *, std::vector<size_t>> by_abs;
    bool all_sparse = true;
    for (size_t j = 0; j < n_jobs; ++j) {
        const JobRef &r = jobs[j];
        LBL_REQUIRE(r.a != nullptr, "job " + std::to_string(j) + ": abstraction is null");
        LBL_REQUIRE(r.O != nullptr && r.L != nullptr, "job " + std::to_string(j) + ": O or L is null");
        LBL_REQUIRE(r.n_props >= 1 && r.n_props <= 64, "job " + std::to_string(j) + ": n_props must be in [1, 64]");
        LBL_REQUIRE(device < 0 || r.a->device == device, "job " + std::to_string(j) + ": abstraction lives on another device");
        if (!by_abs.count(r.a)) order.push_back(r.a);
        by_abs[r.a].push_back(j);
        all_sparse = all_sparse && r.a->sp != nullptr;
    }
    if (!all_sparse)
        for (size_t j = 0; j < n_jobs; ++j)
            LBL_REQUIRE(jobs[j].a->T_bits != nullptr,
                        "job " + std::to_string(j) + ": loaded sparse only, but another job's abstraction has no "
                        "sparse layout, so the batch has no common kernel");
    BatchPlan &p = *out;
    p = BatchPlan{};
    p.sparse = all_sparse;
    const uint32_t max_g = LBL_BATCH_MAX_PROPS / 64;
    std::vector<std::string> keys;
    for (lbl_abs *a : order) {
        // first-fit by decreasing proposition count into 64-column lane
        // groups: a job's columns never span two lane groups
        std::vector<size_t> js = by_abs[a];
        std::stable_sort(js.begin(), js.end(), [&](size_t x, size_t y) { return jobs[x].n_props > jobs[y].n_props; });
        std::vector<uint32_t> used;                 // columns taken in each lane group
        std::vector<std::vector<size_t>> members;   // jobs of each lane group, in placement order
        for (size_t j : js) {
            size_t b = 0;
            while (b < used.size() && used[b] + jobs[j].n_props > 64) ++b;
            if (b == used.size()) {
                used.push_back(0);
                members.emplace_back();
            }
            members[b].push_back(j);
            used[b] += jobs[j].n_props;
        }
        // passes of at most max_g lane groups
        for (size_t b0 = 0; b0 < members.size(); b0 += max_g) {
            const size_t b1 = std::min(members.size(), b0 + max_g);
            GroupDesc g{};
            g.T = a->T_bits;
            g.word_cell = a->d_word_cell;
            g.n_traj = a->n_traj;
            g.row_stride = a->row_stride;
            g.n_words = a->n_words;
            g.G64 = (uint32_t)(b1 - b0);
            g.nx = a->nx;
            g.morton = a->order.morton ? 1u : 0u;
            if (p.sparse) {
                g.n_rb = a->sp->n_rb;
                g.sp_row = a->sp->row;
                g.sp_val = a->sp->val;
                g.max_entry = std::max<uint64_t>(a->sp->nnz, 1) - 1;
            }
            p.lane_off.push_back(p.lanes.size());
            p.lanes.resize(p.lanes.size() + (size_t)g.G64 * 64, LaneDesc{nullptr, nullptr, 0, 0});
            p.lgs_off.push_back(p.lg_seg.size());
            for (size_t b = b0; b < b1; ++b) {
                p.lg_seg.push_back((uint32_t)p.segs.size());
                uint32_t bit = 0;
                for (size_t j : members[b]) {
                    const JobRef &r = jobs[j];
                    p.segs.push_back(SegDesc{r.O, r.L, r.n_props, bit});
                    const size_t q = p.lane_off.back() + (b - b0) * 64 + bit;
                    for (uint32_t c = 0; c < r.n_props; ++c) p.lanes[q + c] = LaneDesc{r.O + c, r.L + c, r.n_props, 0};
                    bit += r.n_props;
                    p.pairs += a->n_traj * r.n_props;
                }
            }
            p.lg_seg.push_back((uint32_t)p.segs.size());
            p.ow_off.push_back(p.ow_bytes);
            // bitpacked plans: masks [w][G64][64 columns]; sparse plans:
            // nibble tables [w][G64][256]
            p.ow_bytes += up256((size_t)a->n_words * g.G64 * (p.sparse ? 256 : 64) * sizeof(uint64_t));
            p.pack_units += (uint64_t)a->n_words * g.G64;
            p.max_g64 = std::max(p.max_g64, g.G64);
            p.groups.push_back(g);
            p.group_abs.push_back(a);
            keys.push_back("W" + std::to_string(a->n_words) + "G" + std::to_string(g.G64));
        }
    }
    std::sort(keys.begin(), keys.end());
    for (auto &s : keys) p.shape_key += s + ";";
    if (p.sparse) {
        // default: the coarsest tiling (fewest partials) that still gives
        // every CU about two tile workgroups
        const uint64_t want = 2ull * (uint64_t)device_cu_count();
        p.default_tiling = kBatchTilings;
        for (int t = 1; t <= kBatchTilings; ++t) {
            uint64_t n = 0;
            for (size_t g = 0; g < p.groups.size(); ++g)
                n += (uint64_t)p.groups[g].G64 * p.group_abs[g]->sp->tilings[t].n_tiles;
            if (n >= want) {
                p.default_tiling = t;
                break;
            }
        }
        p.shape_key = "sparse;" + p.shape_key;
    }
    return LBL_OK;
}

std::string batch_tile_name(const BatchPlan &p)
{
    char buf[128];
    if (p.sparse)
        snprintf(buf, sizeof(buf), "sparse(tiling=%d,persistent=%d)", p.tiling, p.tile.persistent ? 1 : 0);
    else
        snprintf(buf, sizeof(buf), "bits(unroll=%d,waves=%d,rows=%d)", p.tile.unroll, p.tile.waves_per_block,
                 p.tile.rows_per_item);
    return buf;
}

void plan_finalize(BatchPlan &p, const BatchTile &tile)
{
    p.tile = tile;
    p.items.clear();
    p.tiles.clear();
    p.launch.clear();
    p.xcd_start.clear();
    p.combines.clear();
    p.packs.clear();
    p.p_off.clear();
    p.p_bytes = 0;
    std::vector<uint32_t> idx(p.groups.size());
    for (uint32_t i = 0; i < idx.size(); ++i) idx[i] = i;
    if (p.sparse) {
        p.tiling = tile.tiling >= 1 && tile.tiling <= kBatchTilings + 1 ? tile.tiling - 1 : p.default_tiling;
        for (size_t g = 0; g < p.groups.size(); ++g) {
            GroupDesc &d = p.groups[g];
            const SpTiling &tl = p.group_abs[g]->sp->tilings[p.tiling];
            d.sp_tasks = tl.tasks;
            d.sp_rounds = tl.rounds;
            d.sp_rb_tile = tl.rb_tile;
            d.n_tiles = tl.n_tiles;
            // one tile per row block: a tile's accumulators are its rows'
            // final labels, so it writes the label bytes and needs no partials
            d.fused = tl.n_tiles == d.n_rb ? 1u : 0u;
            // partials of only the rows each tile touches, when the tiling
            // has its slot lists
            const bool compact = !d.fused && tl.tile_slot != nullptr;
            d.tile_slot = compact ? tl.tile_slot : nullptr;
            d.slot_row = compact ? tl.slot_row : nullptr;
            d.row_slot_off = compact ? tl.row_slot_off : nullptr;
            d.row_slots = compact ? tl.row_slots : nullptr;
            d.n_slots = compact ? tl.n_slots : 0;
            p.p_off.push_back(p.p_bytes);
            if (!d.fused)
                p.p_bytes += up256((size_t)d.G64 * (compact ? tl.n_slots : (size_t)d.n_tiles * kRowBlock) *
                                   sizeof(uint64_t));
        }
        // pack items: each pass's words in runs of up to 8, at least about
        // 128 items per CU (a run's descriptors are read once for its words)
        {
            uint64_t units = 0;
            for (const GroupDesc &d : p.groups) units += (uint64_t)d.n_words * d.G64;
            const uint64_t want = 128ull * (uint64_t)device_cu_count();
            const uint32_t run = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(8, units / want));
            for (uint32_t g = 0; g < p.groups.size(); ++g)
                for (uint32_t gi = 0; gi < p.groups[g].G64; ++gi)
                    for (uint32_t w0 = 0; w0 < p.groups[g].n_words; w0 += run)
                        p.packs.push_back(PackItem{g, gi, w0, std::min(w0 + run, p.groups[g].n_words)});
        }
        // Tiles that read the same nibble tables (same pass, lane group and
        // position of the tile inside its row block, hence about the same
        // word range) share an XCD queue, so that the tables stay in that
        // XCD's L2.  Table sets go to the least loaded XCD, costliest first;
        // each queue runs its costliest tiles first.
        struct Set {
            double cost;
            std::vector<TileItem> items;
        };
        std::map<std::tuple<uint32_t, uint32_t, uint32_t>, Set> sets;
        for (uint32_t g = 0; g < p.groups.size(); ++g) {
            const GroupDesc &d = p.groups[g];
            const SpTiling &tl = p.group_abs[g]->sp->tilings[p.tiling];
            const double c = (double)(d.max_entry + 1) / (double)d.n_tiles;
            for (uint32_t rb = 0; rb + 1 < tl.rb_tile_host.size(); ++rb)
                for (uint32_t t = tl.rb_tile_host[rb]; t < tl.rb_tile_host[rb + 1]; ++t)
                    for (uint32_t gi = 0; gi < d.G64; ++gi) {
                        Set &st = sets[std::make_tuple(g, gi, t - tl.rb_tile_host[rb])];
                        st.cost += c;
                        st.items.push_back(TileItem{g, t, gi, 0});
                    }
        }
        std::vector<Set *> order;
        for (auto &kv : sets) order.push_back(&kv.second);
        std::stable_sort(order.begin(), order.end(), [](const Set *x, const Set *y) { return x->cost > y->cost; });
        std::vector<double> load(kXcds, 0.0);
        std::vector<std::vector<std::pair<double, TileItem>>> q(kXcds);
        for (Set *st : order) {
            const size_t x = std::min_element(load.begin(), load.end()) - load.begin();
            load[x] += st->cost;
            const double c = st->cost / st->items.size();
            for (const TileItem &it : st->items) q[x].push_back({c, it});
        }
        p.xcd_start.push_back(0);
        for (uint32_t x = 0; x < kXcds; ++x) {
            std::stable_sort(q[x].begin(), q[x].end(),
                             [](const std::pair<double, TileItem> &a, const std::pair<double, TileItem> &b) {
                                 return a.first > b.first;
                             });
            for (auto &e : q[x]) p.tiles.push_back(e.second);
            p.xcd_start.push_back((uint32_t)p.tiles.size());
        }
        // one workgroup per tile: workgroup b runs on XCD b % kXcds, so the
        // queues are interleaved (a queue that runs out hands its slots to
        // the others)
        std::vector<uint32_t> pos(p.xcd_start.begin(), p.xcd_start.end() - 1);
        while (p.launch.size() < p.tiles.size())
            for (uint32_t x = 0; x < kXcds; ++x) {
                uint32_t y = x;
                for (uint32_t k = 0; k < kXcds && pos[y] >= p.xcd_start[y + 1]; ++k) y = (x + k) % kXcds;
                if (pos[y] < p.xcd_start[y + 1]) p.launch.push_back(pos[y]++);
            }
        const uint64_t R = 128;  // rows per combine item (a multiple of 64)
        for (uint32_t g = 0; g < p.groups.size(); ++g)
            if (!p.groups[g].fused)
                for (uint32_t gi = 0; gi < p.groups[g].G64; ++gi)
                    for (uint64_t r0 = 0; r0 < p.groups[g].n_traj; r0 += R)
                        p.combines.push_back(CombineItem{g, gi, r0, std::min(r0 + R, p.groups[g].n_traj)});
    } else {
        auto cost = [&](uint32_t g) { return (double)p.groups[g].n_words * (4.0 + p.groups[g].G64); };
        std::stable_sort(idx.begin(), idx.end(), [&](uint32_t x, uint32_t y) { return cost(x) > cost(y); });
        const uint64_t R = (uint64_t)std::max(1, p.tile.rows_per_item);
        for (uint32_t g : idx)
            for (uint64_t r0 = 0; r0 < p.groups[g].n_traj; r0 += R)
                p.items.push_back(WorkItem{g, 0, r0, std::min(r0 + R, p.groups[g].n_traj)});
    }
    p.finalized = true;
}

lbl_status bind_batch(const BatchPlan &p, uint8_t *base, size_t capacity, BatchBuffers *b, std::vector<uint8_t> *img)
{
    LBL_REQUIRE(p.finalized, "batch plan bound before it was finalized");
    size_t off = 0;
    auto region = [&](size_t bytes) {
        const size_t o = off;
        off += up256(bytes);
        return o;
    };
    const size_t o_groups = region(p.groups.size() * sizeof(GroupDesc));
    const size_t o_items = region(p.items.size() * sizeof(WorkItem));
    const size_t o_lanes = region(p.lanes.size() * sizeof(LaneDesc));
    const size_t o_prefix = region((p.groups.size() + 1) * sizeof(uint64_t));
    const size_t o_counter = off;  // the work counter and the kXcds queue counters
    off += 256;
    const size_t o_tiles = region(p.tiles.size() * sizeof(TileItem));
    const size_t o_launch = region(p.launch.size() * sizeof(uint32_t));
    const size_t o_xcd = region(p.xcd_start.size() * sizeof(uint32_t));
    const size_t o_combines = region(p.combines.size() * sizeof(CombineItem));
    const size_t o_segs = region(p.segs.size() * sizeof(SegDesc));
    const size_t o_lgs = region(p.lg_seg.size() * sizeof(uint32_t));
    const size_t o_packs = region(p.packs.size() * sizeof(PackItem));
    const size_t o_ow = off;
    const size_t o_p = o_ow + p.ow_bytes;
    const size_t total = o_p + p.p_bytes;
    if (total > capacity || total != p.device_bytes()) {
        set_error("batch layout needs " + std::to_string(total) + " bytes, buffer holds " + std::to_string(capacity));
        return LBL_ENOMEM;
    }
    b->base = base;
    b->bytes = total;
    b->d_groups = reinterpret_cast<GroupDesc *>(base + o_groups);
    b->d_items = reinterpret_cast<WorkItem *>(base + o_items);
    b->d_lanes = reinterpret_cast<LaneDesc *>(base + o_lanes);
    b->d_pack_prefix = reinterpret_cast<uint64_t *>(base + o_prefix);
    b->d_counter = reinterpret_cast<uint32_t *>(base + o_counter);
    b->d_queues = b->d_counter + 1;
    b->d_tiles = reinterpret_cast<TileItem *>(base + o_tiles);
    b->d_launch = reinterpret_cast<uint32_t *>(base + o_launch);
    b->d_xcd_start = reinterpret_cast<uint32_t *>(base + o_xcd);
    b->d_combines = reinterpret_cast<CombineItem *>(base + o_combines);
    b->d_segs = reinterpret_cast<SegDesc *>(base + o_segs);
    b->d_lg_seg = reinterpret_cast<uint32_t *>(base + o_lgs);
    b->d_packs = reinterpret_cast<PackItem *>(base + o_packs);
    b->d_ow = reinterpret_cast<uint64_t *>(base + o_ow);
    b->d_p = reinterpret_cast<uint64_t *>(base + o_p);
    img->assign(o_ow, 0);
    std::vector<GroupDesc> gs = p.groups;
    std::vector<uint64_t> prefix(p.groups.size() + 1, 0);
    for (size_t g = 0; g < gs.size(); ++g) {
        gs[g].Ow = reinterpret_cast<uint64_t *>(base + o_ow + p.ow_off[g]);
        gs[g].lanes = b->d_lanes + p.lane_off[g];
        gs[g].segs = b->d_segs;
        gs[g].lg_seg = b->d_lg_seg + p.lgs_off[g];
        if (p.sparse && !gs[g].fused) gs[g].P = reinterpret_cast<uint64_t *>(base + o_p + p.p_off[g]);
        prefix[g + 1] = prefix[g] + (uint64_t)gs[g].n_words * gs[g].G64;
    }
    auto put = [&](size_t o, const void *src, size_t n) {
        if (n) memcpy(img->data() + o, src, n);
    };
    put(o_groups, gs.data(), gs.size() * sizeof(GroupDesc));
    put(o_items, p.items.data(), p.items.size() * sizeof(WorkItem));
    put(o_lanes, p.lanes.data(), p.lanes.size() * sizeof(LaneDesc));
    put(o_prefix, prefix.data(), prefix.size() * sizeof(uint64_t));
    put(o_tiles, p.tiles.data(), p.tiles.size() * sizeof(TileItem));
    put(o_launch, p.launch.data(), p.launch.size() * sizeof(uint32_t));
    put(o_xcd, p.xcd_start.data(), p.xcd_start.size() * sizeof(uint32_t));
    put(o_combines, p.combines.data(), p.combines.size() * sizeof(CombineItem));
    put(o_segs, p.segs.data(), p.segs.size() * sizeof(SegDesc));
    put(o_lgs, p.lg_seg.data(), p.lg_seg.size() * sizeof(uint32_t));
    put(o_packs, p.packs.data(), p.packs.size() * sizeof(PackItem));
    return LBL_OK;
}

lbl_status enqueue_batch(const BatchPlan &p, const BatchBuffers &b, hipStream_t s)
{
    LBL_REQUIRE(p.finalized && b.base != nullptr, "batch enqueued before it was bound");
    const uint64_t pack_blocks = std::max<uint64_t>(1, std::min<uint64_t>((p.pack_units + 3) / 4, 1u << 16));
    if (p.sparse) {
        if (p.tile.persistent) {
            // queue counters start at zero (a kernel, so graph replays are safe)
            hipLaunchKernelGGL(k_zero_n, dim3(1), dim3(64), 0, s, b.d_queues, kXcds);
            LBL_HIP_TRY(hipGetLastError());
        }
        LBL_HIP_TRY(launch_pack_batch_tables(b.d_groups, b.d_packs, (uint32_t)p.packs.size(), s));
        if (p.tile.persistent) {
            const uint32_t n_wg = (uint32_t)std::min<uint64_t>(p.tiles.size(), (uint64_t)device_cu_count());
            LBL_HIP_TRY(launch_tiles_batch_queue(b.d_groups, b.d_tiles, b.d_xcd_start, b.d_queues, n_wg, s));
        } else {
            LBL_HIP_TRY(launch_tiles_batch(b.d_groups, b.d_tiles, b.d_launch, (uint32_t)p.tiles.size(), s));
        }
        LBL_HIP_TRY(launch_combine_batch(b.d_groups, b.d_combines, (uint32_t)p.combines.size(), s));
        return LBL_OK;
    }
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(1), 0, s, b.d_counter);
    LBL_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_pack_batch, dim3((unsigned)pack_blocks), dim3(256), 0, s, b.d_groups,
                       b.d_pack_prefix, (uint32_t)p.groups.size(), p.pack_units);
    LBL_HIP_TRY(hipGetLastError());
    const int wpb = p.tile.waves_per_block;
    LBL_REQUIRE(wpb >= 1 && wpb <= 16, "batch tile: waves_per_block out of range");
    const uint32_t n_items = (uint32_t)p.items.size();
    const unsigned occupancy = (unsigned)std::max(1, 32 / wpb);  // resident workgroups per CU
    const unsigned blocks = (unsigned)std::min<uint64_t>(n_items, (uint64_t)device_cu_count() * occupancy);
    if (blocks == 0) return LBL_OK;
    hipError_t e;
    switch (p.tile.unroll) {
    case 4: e = launch_label_g<4>(b, n_items, p.max_g64, wpb, blocks, s); break;
    case 8: e = launch_label_g<8>(b, n_items, p.max_g64, wpb, blocks, s); break;
    default: LBL_REQUIRE(false, "batch tile: unroll must be 4 or 8");
    }
    LBL_HIP_TRY(e);
    return LBL_OK;
}

// ---------------------------------------------------------------- tuning

namespace {
std::mutex g_tile_mu;
std::map<std::string, BatchTile> g_tiles;

BatchTile tuned_tile(const std::string &key)
{
    std::lock_guard<std::mutex> lk(g_tile_mu);
    auto it = g_tiles.find(key);
    return it == g_tiles.end() ? BatchTile{} : it->second;
}

// ---------------------------------------------------------------- graph cache

struct GraphEntry {
    hipStream_t stream = nullptr;
    uint32_t flags = 0;
    std::vector<JobRef> jobs;
    BatchPlan plan;
    BatchTile asked;  // the tile the entry was built for (before defaults were resolved)
    BatchBuffers bufs;
    void *dmem = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

std::mutex g_graph_mu;
std::list<std::unique_ptr<GraphEntry>> g_graphs;  // most recent first
const size_t kMaxGraphs = 8;

bool same_jobs(const std::vector<JobRef> &a, const JobRef *b, size_t n)
{
    if (a.size() != n) return false;
    for (size_t i = 0; i < n; ++i)
        if (a[i].a != b[i].a || a[i].O != b[i].O || a[i].n_props != b[i].n_props || a[i].L != b[i].L) return false;
    return true;
}

void destroy_entry(GraphEntry *e)
{
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(e->device);
    (void)hipDeviceSynchronize();
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    if (e->dmem) (void)hipFree(e->dmem);
    (void)hipSetDevice(cur);
}

lbl_status build_entry(GraphEntry *e)
{
    const size_t bytes = e->plan.device_bytes();
    LBL_HIP_TRY(hipMalloc(&e->dmem, bytes));
    std::vector<uint8_t> img;
    lbl_status bst = bind_batch(e->plan, static_cast<uint8_t *>(e->dmem), bytes, &e->bufs, &img);
    if (bst != LBL_OK) return bst;
    LBL_HIP_TRY(hipMemcpy(e->dmem, img.data(), img.size(), hipMemcpyHostToDevice));
    hipStream_t cs = nullptr;
    LBL_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    lbl_status st = LBL_OK;
    if (err == hipSuccess) {
        st = enqueue_batch(e->plan, e->bufs, cs);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        e->graph = g;
        if (st == LBL_OK && e2 != hipSuccess) err = e2;
    }
    (void)hipStreamDestroy(cs);
    if (st != LBL_OK) return st;
    LBL_HIP_TRY(err);
    LBL_HIP_TRY(hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0));
    return LBL_OK;
}

// The cached graph for these jobs built for tile `want` (or for the tile
// recorded for their shape class when want is null), moved to the front;
// null if none.  Lock held.  Entries for the same jobs built for another
// tile are released.
GraphEntry *find_entry(const JobRef *jobs, size_t n_jobs, uint32_t flags, hipStream_t s, int device,
                       const BatchTile *want)
{
    GraphEntry *hit = nullptr;
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {
        GraphEntry *e = it->get();
        if (e->stream == s && e->flags == flags && e->device == device && same_jobs(e->jobs, jobs, n_jobs)) {
            const BatchTile w = want ? *want : tuned_tile(e->plan.shape_key);
            if (!hit && e->asked == w) {
                hit = e;
                g_graphs.splice(g_graphs.begin(), g_graphs, it++);
                continue;
            }
            if (!want) {  // built for a tile no longer recorded for the class
                destroy_entry(e);
                it = g_graphs.erase(it);
                continue;
            }
        }
        ++it;
    }
    return hit;
}

}  // namespace

BatchTile batch_tile_for(const std::string &key) { return tuned_tile(key); }

std::vector<std::pair<std::string, BatchTile>> batch_tiles()
{
    std::lock_guard<std::mutex> lk(g_tile_mu);
    return std::vector<std::pair<std::string, BatchTile>>(g_tiles.begin(), g_tiles.end());
}

void batch_forget(const lbl_abs *a)
{
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {
        bool uses = false;
        for (const JobRef &j : (*it)->jobs) uses = uses || j.a == a;
        if (uses) {
            destroy_entry(it->get());
            it = g_graphs.erase(it);
        } else {
            ++it;
        }
    }
}

void set_batch_tile(const std::string &key, const BatchTile &t)
{
    std::lock_guard<std::mutex> lk(g_tile_mu);
    g_tiles[key] = t;
}

lbl_status label_batch_graph(const JobRef *jobs, size_t n_jobs, uint32_t flags, hipStream_t s, const BatchTile *force)
{
    int cur = 0;
    LBL_HIP_TRY(hipGetDevice(&cur));
    std::lock_guard<std::mutex> lk(g_graph_mu);
    GraphEntry *hit = find_entry(jobs, n_jobs, flags, s, cur, force);
    if (!hit) {
        std::unique_ptr<GraphEntry> e(new GraphEntry());
        e->stream = s;
        e->flags = flags;
        e->device = cur;
        e->jobs.assign(jobs, jobs + n_jobs);
        lbl_status st = plan_batch(jobs, n_jobs, cur, &e->plan);
        if (st != LBL_OK) return st;
        e->asked = force ? *force : tuned_tile(e->plan.shape_key);
        plan_finalize(e->plan, e->asked);
        st = build_entry(e.get());
        if (st != LBL_OK) {
            destroy_entry(e.get());
            return st;
        }
        while (g_graphs.size() >= kMaxGraphs) {
            destroy_entry(g_graphs.back().get());
            g_graphs.pop_back();
        }
        g_graphs.push_front(std::move(e));
        hit = g_graphs.front().get();
    }
    void *span = span_begin(s);
    LBL_HIP_TRY(hipGraphLaunch(hit->exec, s));
    span_end(span, s, 2);
    return LBL_OK;
}

}  // namespace lbl

using namespace lbl;

extern "C" {

lbl_status lbl_label_batch(const lbl_job *jobs, size_t n_jobs, uint32_t flags, void *hip_stream)
{
    clear_error();
    LBL_REQUIRE(jobs != nullptr && n_jobs > 0, "no jobs");
    LBL_REQUIRE(flags == 0, "lbl_label_batch takes device pointers and no flags");
    std::vector<JobRef> refs(n_jobs);
    for (size_t j = 0; j < n_jobs; ++j) refs[j] = JobRef{jobs[j].a, jobs[j].O, jobs[j].n_props, jobs[j].L};
    return label_batch_graph(refs.data(), n_jobs, flags, reinterpret_cast<hipStream_t>(hip_stream), nullptr);
}

lbl_status lbl_tune_batch(const lbl_job *jobs, size_t n_jobs, void *hip_stream)
{
    clear_error();
    LBL_REQUIRE(jobs != nullptr && n_jobs > 0, "no jobs");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    std::vector<JobRef> refs(n_jobs);
    for (size_t j = 0; j < n_jobs; ++j) refs[j] = JobRef{jobs[j].a, jobs[j].O, jobs[j].n_props, jobs[j].L};
    BatchPlan probe;
    int cur = 0;
    LBL_HIP_TRY(hipGetDevice(&cur));
    lbl_status st = plan_batch(refs.data(), n_jobs, cur, &probe);
    if (st != LBL_OK) return st;
    // the candidates: for sparse plans every tiling of the layout, launched
    // persistent or one workgroup per tile; for bitpacked plans the
    // persistent kernel's loads in flight, workgroup size and rows per item
    std::vector<BatchTile> cands;
    if (probe.sparse) {
        for (int t = 1; t <= kBatchTilings + 1; ++t)
            for (int pers : {1, 0}) {
                BatchTile b;
                b.tiling = t;
                b.persistent = pers;
                cands.push_back(b);
            }
    } else {
        for (int u : {4, 8})
            for (int w : {4, 8, 16})
                for (int r : {32, 128, 512}) cands.push_back(BatchTile{u, w, r, 0, 1});
    }
    // each candidate: its graph built and replayed once, then `reps` replays
    // timed one by one; its score is their median.  The candidates run within
    // a few percent of each other, so the three best are timed again with
    // more replays and the lowest median wins.
    const int kEvents = 16;
    hipEvent_t ev[kEvents + 1];
    for (int i = 0; i <= kEvents; ++i) LBL_HIP_TRY(hipEventCreate(&ev[i]));
    auto score = [&](const BatchTile &t, int reps, float *out) -> lbl_status {
        lbl_status r = label_batch_graph(refs.data(), n_jobs, 0, s, &t);  // build + warm-up
        if (r != LBL_OK) return r;
        LBL_HIP_TRY(hipEventRecord(ev[0], s));
        for (int k = 0; k < reps && r == LBL_OK; ++k) {
            r = label_batch_graph(refs.data(), n_jobs, 0, s, &t);
            LBL_HIP_TRY(hipEventRecord(ev[k + 1], s));
        }
        LBL_HIP_TRY(hipEventSynchronize(ev[reps]));
        if (r != LBL_OK) return r;
        std::vector<float> ms(reps);
        for (int k = 0; k < reps; ++k) LBL_HIP_TRY(hipEventElapsedTime(&ms[k], ev[k], ev[k + 1]));
        std::nth_element(ms.begin(), ms.begin() + reps / 2, ms.end());
        *out = ms[reps / 2];
        return LBL_OK;
    };
    std::vector<std::pair<float, size_t>> scored;
    for (size_t c = 0; c < cands.size() && st == LBL_OK; ++c) {
        float ms = 0.f;
        st = score(cands[c], 5, &ms);
        scored.push_back({ms, c});
    }
    BatchTile best;
    if (st == LBL_OK) {
        std::sort(scored.begin(), scored.end());
        float best_ms = 1e30f;
        for (size_t i = 0; i < std::min<size_t>(3, scored.size()) && st == LBL_OK; ++i) {
            float ms = 0.f;
            st = score(cands[scored[i].second], kEvents, &ms);
            if (st == LBL_OK && ms < best_ms) {
                best_ms = ms;
                best = cands[scored[i].second];
            }
        }
    }
    for (int i = 0; i <= kEvents; ++i) (void)hipEventDestroy(ev[i]);
    if (st != LBL_OK) return st;
    set_batch_tile(probe.shape_key, best);
    // release the candidates' graphs except the winner's, which the next
    // lbl_label_batch of these jobs replays
    std::lock_guard<std::mutex> lk(g_graph_mu);
    (void)find_entry(refs.data(), n_jobs, 0, s, cur, nullptr);
    return LBL_OK;
}

lbl_status lbl_tune_batch_describe(const lbl_job *jobs, size_t n_jobs, void *hip_stream, char *buf, size_t buf_len)
{
    clear_error();
    LBL_REQUIRE(jobs != nullptr && n_jobs > 0, "no jobs");
    LBL_REQUIRE(buf != nullptr && buf_len > 0, "null buffer");
    std::vector<JobRef> refs(n_jobs);
    for (size_t j = 0; j < n_jobs; ++j) refs[j] = JobRef{jobs[j].a, jobs[j].O, jobs[j].n_props, jobs[j].L};
    int cur = 0;
    LBL_HIP_TRY(hipGetDevice(&cur));
    BatchPlan p;
    lbl_status st = plan_batch(refs.data(), n_jobs, cur, &p);
    if (st != LBL_OK) return st;
    std::string out;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
        GraphEntry *e = nullptr;
        for (auto &x : g_graphs)
            if (x->stream == s && x->device == cur && same_jobs(x->jobs, refs.data(), n_jobs) &&
                x->asked == tuned_tile(x->plan.shape_key)) {
                e = x.get();
                break;
            }
        if (e) {
            out = p.shape_key + " -> " + batch_tile_name(e->plan) + " cached";
        } else {
            plan_finalize(p, tuned_tile(p.shape_key));
            out = p.shape_key + " -> " + batch_tile_name(p) + " not built";
        }
    }
    snprintf(buf, buf_len, "%s", out.c_str());
    return LBL_OK;
}

}  // extern "C"
