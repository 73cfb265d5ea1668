// Host-only check of the batch planner's device layout: every table and mask
// region must lie inside the buffer the plan asks for, work items must cover
// each abstraction's rows exactly once, and lane tables must map every
// (job, proposition) column exactly once.  No device memory is touched: the
// abstractions and buffers carry fake addresses, and bind_batch only writes
// the host image.
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <map>
#include <random>
#include <set>
#include <tuple>

#include "batch.h"
#include "sparse.h"

using namespace lbl;

static int fails = 0;
#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::fprintf(stderr, "FAILED %s:%d %s\n", __FILE__, __LINE__, #c); \
            ++fails;                                                  \
        }                                                             \
    } while (0)

static void check_case(std::vector<lbl_abs> &abss, const std::vector<JobRef> &jobs, const BatchTile &tile)
{
    BatchPlan p;
    CHECK(plan_batch(jobs.data(), jobs.size(), -1, &p) == LBL_OK);
    uint8_t *base = reinterpret_cast<uint8_t *>(0x7f0000000000ull);
    BatchBuffers b;
    std::vector<uint8_t> img;
    CHECK(bind_batch(p, base, 1ull << 40, &b, &img) == LBL_EINVAL);  // not finalized
    plan_finalize(p, tile);
    const size_t bytes = p.device_bytes();
    CHECK(bind_batch(p, base, bytes - 1, &b, &img) == LBL_ENOMEM);
    CHECK(bind_batch(p, base, bytes, &b, &img) == LBL_OK);
    CHECK(b.bytes == bytes);
    auto inside = [&](const void *ptr, size_t n) {
        const uint8_t *q = static_cast<const uint8_t *>(ptr);
        return q >= base && q + n <= base + bytes;
    };
    CHECK(img.size() <= bytes);
    CHECK(inside(b.d_groups, p.groups.size() * sizeof(GroupDesc)));
    CHECK(inside(b.d_items, p.items.size() * sizeof(WorkItem)));
    CHECK(inside(b.d_lanes, p.lanes.size() * sizeof(LaneDesc)));
    CHECK(inside(b.d_pack_prefix, (p.groups.size() + 1) * sizeof(uint64_t)));
    CHECK(inside(b.d_counter, sizeof(uint32_t)));
    const GroupDesc *gs = reinterpret_cast<const GroupDesc *>(img.data() + (reinterpret_cast<uint8_t *>(b.d_groups) - base));
    std::vector<std::pair<const uint8_t *, const uint8_t *>> ow_ranges;
    for (size_t g = 0; g < p.groups.size(); ++g) {
        const size_t ow = (size_t)gs[g].n_words * gs[g].G64 * (p.sparse ? 256 : 64) * sizeof(uint64_t);
        CHECK(inside(gs[g].Ow, ow));
        CHECK(reinterpret_cast<const uint8_t *>(gs[g].Ow) >= reinterpret_cast<uint8_t *>(b.d_ow));
        CHECK(inside(gs[g].lanes, (size_t)gs[g].G64 * 64 * sizeof(LaneDesc)));
        CHECK(gs[g].G64 >= 1 && gs[g].G64 <= LBL_BATCH_MAX_PROPS / 64);
        ow_ranges.push_back({reinterpret_cast<const uint8_t *>(gs[g].Ow), reinterpret_cast<const uint8_t *>(gs[g].Ow) + ow});
    }
    for (size_t i = 0; i < ow_ranges.size(); ++i)
        for (size_t j = i + 1; j < ow_ranges.size(); ++j)
            CHECK(ow_ranges[i].second <= ow_ranges[j].first || ow_ranges[j].second <= ow_ranges[i].first);
    // items cover every group's rows exactly once
    std::vector<uint64_t> covered(p.groups.size(), 0);
    for (const WorkItem &it : p.items) {
        CHECK(it.group < p.groups.size());
        CHECK(it.row0 < it.row1 && it.row1 <= p.groups[it.group].n_traj);
        CHECK(it.row1 - it.row0 <= (uint64_t)tile.rows_per_item);
        covered[it.group] += it.row1 - it.row0;
    }
    if (!p.sparse)
        for (size_t g = 0; g < p.groups.size(); ++g) CHECK(covered[g] == p.groups[g].n_traj);
    else
        CHECK(p.items.empty());
    // lanes: every (job, proposition) exactly once, with its own stride
    std::map<const uint8_t *, int> seen;
    for (const LaneDesc &d : p.lanes)
        if (d.L) seen[d.L]++;
    size_t want = 0;
    for (const JobRef &j : jobs) {
        want += j.n_props;
        for (uint32_t c = 0; c < j.n_props; ++c) CHECK(seen[j.L + c] == 1);
    }
    CHECK(seen.size() == want);
    // segments: every job once, whole, inside one lane group, columns
    // disjoint and matching the lane tables
    CHECK(inside(b.d_segs, p.segs.size() * sizeof(SegDesc)));
    CHECK(inside(b.d_lg_seg, p.lg_seg.size() * sizeof(uint32_t)));
    std::map<const uint8_t *, int> seg_seen;
    for (size_t g = 0; g < p.groups.size(); ++g) {
        CHECK(gs[g].segs == b.d_segs);
        CHECK(inside(gs[g].lg_seg, (p.groups[g].G64 + 1) * sizeof(uint32_t)));
        const uint32_t *lgs = p.lg_seg.data() + p.lgs_off[g];
        for (uint32_t gi = 0; gi < p.groups[g].G64; ++gi) {
            CHECK(lgs[gi] <= lgs[gi + 1] && lgs[gi + 1] <= p.segs.size());
            uint64_t cols = 0;
            for (uint32_t sgi = lgs[gi]; sgi < lgs[gi + 1]; ++sgi) {
                const SegDesc &d = p.segs[sgi];
                CHECK(d.n_props >= 1 && d.bit + d.n_props <= 64);
                const uint64_t m = (d.n_props == 64 ? ~0ull : ((1ull << d.n_props) - 1)) << d.bit;
                CHECK((cols & m) == 0);
                cols |= m;
                seg_seen[d.L]++;
                for (uint32_t c = 0; c < d.n_props; ++c) {
                    const LaneDesc &ld = p.lanes[p.lane_off[g] + gi * 64 + d.bit + c];
                    CHECK(ld.L == d.L + c && ld.O == d.O + c && ld.n_props == d.n_props);
                }
            }
        }
    }
    CHECK(seg_seen.size() == jobs.size());
    for (auto &kv : seg_seen) CHECK(kv.second == 1);
    uint64_t pairs = 0;
    for (const JobRef &j : jobs) pairs += j.a->n_traj * j.n_props;
    CHECK(p.pairs == pairs);
    // sparse plans: partial regions inside and disjoint, every tile once,
    // every row of every lane group combined once
    bool sparse = true;
    for (const JobRef &j : jobs) sparse = sparse && j.a->sp != nullptr;
    CHECK(p.sparse == sparse);
    if (!p.sparse) return;
    CHECK(p.tiling >= 0 && p.tiling <= kBatchTilings);
    CHECK(tile.tiling == 0 ? p.tiling == p.default_tiling : p.tiling == tile.tiling - 1);
    std::vector<std::pair<const uint8_t *, const uint8_t *>> p_ranges;
    std::set<std::tuple<uint32_t, uint32_t, uint32_t>> tiles;
    uint64_t want_tiles = 0;
    for (size_t g = 0; g < p.groups.size(); ++g) {
        const GroupDesc &d = gs[g];
        const SpTiling &tl = p.group_abs[g]->sp->tilings[p.tiling];
        CHECK(d.n_tiles == tl.n_tiles && d.sp_tasks == tl.tasks && d.sp_rounds == tl.rounds && d.sp_rb_tile == tl.rb_tile);
        CHECK(d.n_rb == (uint32_t)((d.n_traj + kRowBlock - 1) / kRowBlock));
        // fused passes (one tile per row block) write labels from the tiles
        // and have no partials
        CHECK(d.fused == (d.n_tiles == d.n_rb ? 1u : 0u));
        want_tiles += (uint64_t)d.n_tiles * d.G64;
        if (d.fused) {
            CHECK(d.P == nullptr);
            for (uint32_t rb = 0; rb < d.n_rb; ++rb) CHECK(tl.rb_tile_host[rb] == rb);
            continue;
        }
        // compact partials ([G64][n_slots]) when the tiling has slot lists
        CHECK(d.tile_slot == tl.tile_slot && d.slot_row == tl.slot_row && d.row_slot_off == tl.row_slot_off &&
              d.row_slots == tl.row_slots && d.n_slots == (tl.tile_slot ? tl.n_slots : 0));
        const size_t pb =
            (size_t)d.G64 * (d.tile_slot ? (size_t)d.n_slots : (size_t)d.n_tiles * kRowBlock) * sizeof(uint64_t);
        CHECK(inside(d.P, pb));
        p_ranges.push_back({reinterpret_cast<const uint8_t *>(d.P), reinterpret_cast<const uint8_t *>(d.P) + pb});
    }
    // pack items: every (pass, lane group, word) exactly once
    CHECK(inside(b.d_packs, p.packs.size() * sizeof(PackItem)));
    {
        std::map<std::pair<uint32_t, uint32_t>, std::vector<uint8_t>> words;
        for (const PackItem &k : p.packs) {
            CHECK(k.group < p.groups.size() && k.gi < p.groups[k.group].G64);
            CHECK(k.w0 < k.w1 && k.w1 <= p.groups[k.group].n_words);
            auto &v = words[std::make_pair(k.group, k.gi)];
            v.resize(p.groups[k.group].n_words, 0);
            for (uint32_t w = k.w0; w < k.w1 && w < v.size(); ++w) ++v[w];
        }
        uint64_t want_pairs = 0;
        for (const GroupDesc &d : p.groups) want_pairs += d.G64;
        CHECK(words.size() == want_pairs);
        for (auto &kv : words)
            for (uint8_t c : kv.second) CHECK(c == 1);
    }
    for (size_t i = 0; i < p_ranges.size(); ++i) {
        CHECK(p_ranges[i].second <= ow_ranges.front().first || p_ranges[i].first >= ow_ranges.back().second);
        for (size_t j = i + 1; j < p_ranges.size(); ++j)
            CHECK(p_ranges[i].second <= p_ranges[j].first || p_ranges[j].second <= p_ranges[i].first);
    }
    CHECK(inside(b.d_tiles, p.tiles.size() * sizeof(TileItem)));
    CHECK(inside(b.d_combines, p.combines.size() * sizeof(CombineItem)));
    for (const TileItem &t : p.tiles) {
        CHECK(t.group < p.groups.size());
        const GroupDesc &d = p.groups[t.group];
        CHECK(t.tile < d.n_tiles && t.gi < d.G64);
        tiles.insert(std::make_tuple(t.group, t.tile, t.gi));
    }
    CHECK(tiles.size() == p.tiles.size() && p.tiles.size() == want_tiles);
    // per-XCD queues partition the tiles; the one-per-tile launch order is a
    // permutation of them
    CHECK(p.xcd_start.size() == kXcds + 1 && p.xcd_start.front() == 0 && p.xcd_start.back() == p.tiles.size());
    for (uint32_t x = 0; x < kXcds; ++x) CHECK(p.xcd_start[x] <= p.xcd_start[x + 1]);
    CHECK(inside(b.d_xcd_start, p.xcd_start.size() * sizeof(uint32_t)));
    CHECK(inside(b.d_queues, kXcds * sizeof(uint32_t)));
    CHECK(reinterpret_cast<uint8_t *>(b.d_queues) == reinterpret_cast<uint8_t *>(b.d_counter) + 4);
    CHECK(inside(b.d_launch, p.launch.size() * sizeof(uint32_t)));
    {
        std::vector<uint32_t> perm = p.launch;
        std::sort(perm.begin(), perm.end());
        CHECK(perm.size() == p.tiles.size());
        for (size_t i = 0; i < perm.size(); ++i) CHECK(perm[i] == i);
    }
    // tiles that share a table set (pass, lane group, position in the row
    // block) are on one queue
    {
        std::map<std::tuple<uint32_t, uint32_t, uint32_t>, std::set<uint32_t>> where;
        for (uint32_t x = 0; x < kXcds; ++x)
            for (uint32_t i = p.xcd_start[x]; i < p.xcd_start[x + 1]; ++i) {
                const TileItem &t = p.tiles[i];
                const auto &rbt = p.group_abs[t.group]->sp->tilings[p.tiling].rb_tile_host;
                const uint32_t rb = (uint32_t)(std::upper_bound(rbt.begin(), rbt.end(), t.tile) - rbt.begin() - 1);
                where[std::make_tuple(t.group, t.gi, t.tile - rbt[rb])].insert(x);
            }
        for (auto &kv : where) CHECK(kv.second.size() == 1);
    }
    std::map<std::pair<uint32_t, uint32_t>, uint64_t> rows;
    for (const CombineItem &c : p.combines) {
        CHECK(c.group < p.groups.size() && c.gi < p.groups[c.group].G64);
        CHECK(!p.groups[c.group].fused);
        CHECK(c.row0 < c.row1 && c.row1 <= p.groups[c.group].n_traj && c.row0 % 64 == 0);
        rows[std::make_pair(c.group, c.gi)] += c.row1 - c.row0;
    }
    // a fused pass's tile (row block rb, lane group gi) writes the rows of rb
    for (const TileItem &t : p.tiles)
        if (p.groups[t.group].fused) {
            const uint64_t r0 = (uint64_t)t.tile * kRowBlock;
            rows[std::make_pair(t.group, t.gi)] += std::min<uint64_t>(kRowBlock, p.groups[t.group].n_traj - r0);
        }
    for (size_t g = 0; g < p.groups.size(); ++g)
        for (uint32_t gi = 0; gi < p.groups[g].G64; ++gi) {
            const uint64_t covered_rows = rows[std::make_pair((uint32_t)g, gi)];
            CHECK(covered_rows == p.groups[g].n_traj);
        }
    // label bytes: every combine item writes, for each job of its lane group,
    // the contiguous block of its rows' bytes; across all items each job's
    // L is covered exactly once (no byte, hence no store unit inside a
    // block, is written by two wavefronts)
    std::map<const uint8_t *, std::vector<std::pair<uint64_t, uint64_t>>> blocks;
    std::map<const uint8_t *, uint64_t> job_bytes;
    for (const JobRef &j : jobs) job_bytes[j.L] = j.a->n_traj * j.n_props;
    auto add_rows = [&](uint32_t g, uint32_t gi, uint64_t row0, uint64_t row1) {
        const uint32_t *lgs = p.lg_seg.data() + p.lgs_off[g];
        for (uint64_t t0 = row0; t0 < row1; t0 += 64) {
            const uint64_t n = std::min<uint64_t>(64, row1 - t0);
            for (uint32_t sgi = lgs[gi]; sgi < lgs[gi + 1]; ++sgi) {
                const SegDesc &d = p.segs[sgi];
                blocks[d.L].push_back({t0 * d.n_props, (t0 + n) * d.n_props});
            }
        }
    };
    for (const CombineItem &c : p.combines) add_rows(c.group, c.gi, c.row0, c.row1);
    // fused tiles emit their block's rows in 64-row chunks (chunk starts are
    // multiples of 64 from the block start, a multiple of kRowBlock)
    for (const TileItem &t : p.tiles)
        if (p.groups[t.group].fused) {
            const uint64_t r0 = (uint64_t)t.tile * kRowBlock;
            add_rows(t.group, t.gi, r0, std::min<uint64_t>(r0 + kRowBlock, p.groups[t.group].n_traj));
        }
    CHECK(blocks.size() == job_bytes.size());
    // the store units of every block as the combine issues them: 16-byte
    // units only where they lie inside the block, single bytes where a unit
    // would reach past either end.  Blocks are disjoint (above), so no unit
    // or byte is written by two wavefronts.
    for (const auto &kv : blocks)
        for (const auto &r : kv.second) {
            const uintptr_t base = reinterpret_cast<uintptr_t>(kv.first) + r.first;
            const uint64_t len = r.second - r.first, mis = base & 15u, total = mis + len;
            uint64_t covered = 0;
            for (uint64_t lo = 0; lo < total; lo += 16) {
                if (lo >= mis && lo + 16 <= total) {
                    const uintptr_t u = base - mis + lo;
                    CHECK(u % 16 == 0 && u >= base && u + 16 <= base + len);
                    covered += 16;
                } else {
                    for (uint64_t b = lo; b < lo + 16; ++b)
                        if (b >= mis && b < total) ++covered;
                }
            }
            CHECK(covered == len);
        }
    for (auto &kv : blocks) {
        std::sort(kv.second.begin(), kv.second.end());
        uint64_t at = 0;
        for (auto &r : kv.second) {
            CHECK(r.first == at && r.second > r.first);
            at = r.second;
        }
        CHECK(at == job_bytes[kv.first]);
    }
}

// A fake sparse layout for an abstraction of `rows` rows: tilings with
// 1, 2, 4, 8 tiles per row block (and a one-frame tiling), fake addresses.
// Never freed (its destructor would release the fake addresses).
static SparseLayout *fake_layout(uint64_t rows, uint64_t base)
{
    SparseLayout *sp = new SparseLayout;
    sp->n_rb = (uint32_t)((rows + kRowBlock - 1) / kRowBlock);
    sp->nnz = rows * 50;
    sp->row = reinterpret_cast<uint16_t *>(base);
    sp->val = reinterpret_cast<uint64_t *>(base + 0x10000000ull);
    sp->tilings.resize(1 + kBatchTilings);
    for (int i = 0; i <= kBatchTilings; ++i) {
        SpTiling &t = sp->tilings[i];
        t.n_tiles = i == 0 ? std::max<uint32_t>(sp->n_rb, 256) : sp->n_rb << (i - 1);
        t.tasks = reinterpret_cast<SpTask *>(base + 0x20000000ull + 0x1000000ull * i);
        t.rounds = reinterpret_cast<SpRound *>(base + 0x30000000ull + 0x1000000ull * i);
        t.rb_tile = reinterpret_cast<uint32_t *>(base + 0x40000000ull + 0x1000000ull * i);
        // tiles of each row block: the one-frame tiling gives the first
        // blocks the extra tiles, the batch tilings 2^(i-1) each
        t.rb_tile_host.assign(sp->n_rb + 1, 0);
        for (uint32_t rb = 0; rb < sp->n_rb; ++rb) {
            const uint32_t k = i == 0 ? t.n_tiles / sp->n_rb + (rb < t.n_tiles % sp->n_rb ? 1u : 0u) : 1u << (i - 1);
            t.rb_tile_host[rb + 1] = t.rb_tile_host[rb] + k;
        }
        CHECK(t.rb_tile_host[sp->n_rb] == t.n_tiles);
        // slot lists (compact partials) on the odd tilings, fewer slots than
        // a full [n_tiles][kRowBlock] partial set
        if (i & 1) {
            t.n_slots = (uint64_t)t.n_tiles * kRowBlock / 3 + 7;
            t.tile_slot = reinterpret_cast<uint32_t *>(base + 0x50000000ull + 0x1000000ull * i);
            t.slot_row = reinterpret_cast<uint16_t *>(base + 0x60000000ull + 0x1000000ull * i);
            t.row_slot_off = reinterpret_cast<uint32_t *>(base + 0x70000000ull + 0x1000000ull * i);
            t.row_slots = reinterpret_cast<uint32_t *>(base + 0x80000000ull + 0x1000000ull * i);
        }
    }
    return sp;
}

// ---------------------------------------------------------------- tilings

// Random non-empty segments over n_rb row blocks of W words: returns the
// segment starts (with the end sentinel), words and first segment of each
// block.  mode 0: typical sizes; 1: many tiny segments; 2: few huge ones;
// 3: some empty row blocks.
static void random_segments(std::mt19937 &rng, uint32_t n_rb, uint32_t W, int mode, std::vector<uint64_t> *start,
                            std::vector<uint32_t> *word, std::vector<uint64_t> *rb_seg)
{
    start->clear();
    word->clear();
    rb_seg->assign(n_rb + 1, 0);
    uint64_t e = 0;
    for (uint32_t rb = 0; rb < n_rb; ++rb) {
        (*rb_seg)[rb] = word->size();
        if (mode == 3 && rng() % 3 == 0) continue;
        for (uint32_t w = 0; w < W; ++w) {
            uint32_t n = 0;
            if (mode == 0) n = rng() % 4 == 0 ? 0 : 1 + rng() % 120;
            if (mode == 1) n = rng() % 2 == 0 ? 0 : 1 + rng() % 5;
            if (mode == 2) n = rng() % 16 == 0 ? 200 + rng() % 3000 : 0;
            if (mode == 3) n = rng() % 3 == 0 ? 0 : 1 + rng() % 90;
            if (n == 0) continue;
            start->push_back(e);
            word->push_back(w);
            e += n;
        }
    }
    (*rb_seg)[n_rb] = word->size();
    start->push_back(e);
}

// Walk the tiling as the tile kernel does and check that every entry is
// taken by exactly one active lane, reading the table of its own segment's
// word, built before use.
static void check_tiling(const std::vector<uint64_t> &start, const std::vector<uint32_t> &word,
                         const std::vector<uint64_t> &rb_seg, const std::vector<uint32_t> &k)
{
    TilingHost h;
    make_tiling(start, word, rb_seg, k, &h);
    const size_t n_rb = rb_seg.size() - 1;
    uint64_t n_tiles = 0;
    for (uint32_t x : k) n_tiles += x;
    CHECK(h.tasks.size() == n_tiles * kTileWaves);
    CHECK(h.rb_tile.size() == n_rb + 1 && h.rb_tile[0] == 0 && h.rb_tile[n_rb] == n_tiles);
    // the launch order is a permutation of the tiles
    std::vector<uint32_t> order = h.block_tile;
    std::sort(order.begin(), order.end());
    CHECK(order.size() == n_tiles);
    for (uint32_t i = 0; i < order.size(); ++i) CHECK(order[i] == i);
    const uint64_t nnz = start.back();
    std::vector<uint8_t> seen(nnz, 0);
    for (size_t rb = 0; rb < n_rb; ++rb) {
        CHECK(h.rb_tile[rb + 1] - h.rb_tile[rb] == k[rb]);
        const uint64_t E0 = start[rb_seg[rb]], E1 = start[rb_seg[rb + 1]];
        uint64_t next = E0;  // tasks of the block cover [E0, E1) in order
        for (uint64_t t = h.rb_tile[rb]; t < h.rb_tile[rb + 1]; ++t)
            for (uint32_t wv = 0; wv < kTileWaves; ++wv) {
                const SpTask &tk = h.tasks[t * kTileWaves + wv];
                CHECK(tk.lo == next);
                int64_t slot_word[2] = {-1, -1};
                uint64_t hi = tk.lo;
                for (uint32_t i = 0; i < tk.n_rounds; ++i) {
                    CHECK((uint64_t)tk.round0 + i < h.rounds.size());
                    const SpRound &r = h.rounds[tk.round0 + i];
                    CHECK(r.e_off % 64 == 0);
                    const uint32_t lane_lo = r.meta & 0xFF, lane_hi = (r.meta >> 8) & 0xFF, cut = (r.meta >> 16) & 0xFF;
                    CHECK(lane_lo < lane_hi && lane_hi <= 64 && cut <= 64 && (r.meta >> 27) == 0);
                    const uint32_t s0 = (r.meta & kMetaSlot0) ? 1 : 0;
                    CHECK(!((r.meta & kMetaBuild0) && (r.meta & kMetaBuild1)));  // one table per round
                    if (r.meta & kMetaBuild0) slot_word[s0] = r.tword;
                    if (r.meta & kMetaBuild1) slot_word[s0 ^ 1] = r.tword;
                    for (uint32_t l = lane_lo; l < lane_hi; ++l) {
                        const uint64_t e = tk.lo + r.e_off + l;
                        CHECK(e < E1);
                        if (e >= E1) continue;
                        ++seen[e];
                        // segment of e
                        const uint64_t s = std::upper_bound(start.begin(), start.end(), e) - start.begin() - 1;
                        CHECK(s >= rb_seg[rb] && s < rb_seg[rb + 1]);
                        const uint32_t slot = s0 ^ (l >= cut ? 1 : 0);
                        CHECK(slot_word[slot] == (int64_t)word[s]);
                        CHECK(slot == (s & 1));
                        hi = std::max(hi, e + 1);
                    }
                }
                next = hi;
            }
        CHECK(next == E1);
    }
    for (uint64_t e = 0; e < nnz; ++e) CHECK(seen[e] == 1);
    // the direct-mask split: walked as the kernel does, every entry is taken
    // once, by a valid lane of a chunk of a part in the entry's own row block,
    // and every lane (valid or not) reads a segment inside its part's set,
    // the valid ones their own; tiles hold equal chunk counts (within one)
    for (uint32_t want_tiles : {1u, 7u, 512u}) {
        DirectHost dh;
        make_direct(start, rb_seg, want_tiles, &dh);
        const uint32_t nt = (uint32_t)dh.tile_part.size() - 1;
        CHECK(nt >= 1 && nt <= want_tiles && dh.tile_part[0] == 0 && dh.tile_part[nt] == dh.parts.size());
        std::vector<uint8_t> got(nnz, 0);
        uint64_t cmin = ~0ull, cmax = 0, next_chunk = 0;
        for (uint32_t t = 0; t < nt; ++t) {
            uint64_t c_t = 0;
            for (uint32_t pi = dh.tile_part[t]; pi < dh.tile_part[t + 1]; ++pi) {
                const DirectPart &p = dh.parts[pi];
                CHECK(p.c0 == next_chunk && p.c1 > p.c0 && p.c1 <= dh.chunks.size() && p.rb < n_rb);
                next_chunk = p.c1;
                c_t += p.c1 - p.c0;
                const uint64_t E1 = start[rb_seg[p.rb + 1]];
                CHECK(p.seg_first >= rb_seg[p.rb] && p.seg_first + p.n_seg <= rb_seg[p.rb + 1] && p.n_seg >= 1);
                for (uint32_t j = p.c0; j < p.c1; ++j) {
                    const SpChunk &c = dh.chunks[j];
                    const uint64_t a = p.e0 + 64ull * (j - p.c0);
                    CHECK(c.n_valid >= 1 && c.n_valid <= 64 && a + c.n_valid <= E1);
                    CHECK(c.n_valid == 64 || a + c.n_valid == E1);
                    CHECK(c.n_valid == 64 || (c.starts >> (c.n_valid - 1)) == 0);
                    for (uint32_t l = 0; l < 64; ++l) {
                        const uint32_t seg = c.seg0 + (uint32_t)__builtin_popcountll(c.starts & ((1ull << l) - 1));
                        CHECK(seg < p.n_seg);
                        if (l >= c.n_valid) continue;
                        const uint64_t e = a + l;
                        const uint64_t s = std::upper_bound(start.begin(), start.end(), e) - start.begin() - 1;
                        CHECK(p.seg_first + seg == s);
                        ++got[e];
                    }
                }
            }
            cmin = std::min(cmin, c_t);
            cmax = std::max(cmax, c_t);
        }
        CHECK(next_chunk == dh.chunks.size());
        CHECK(nnz == 0 || cmax <= cmin + 1);
        for (uint64_t e = 0; e < nnz; ++e) CHECK(got[e] == 1);
    }
    // compact partial slots: random local rows for the entries; every (row,
    // tile) pair with an entry has exactly one slot, a tile's slots ascend,
    // and each row's slot list names exactly its tiles' slots for that row
    std::mt19937 rng((uint32_t)nnz);
    const uint64_t n_traj = (uint64_t)n_rb * kRowBlock - (n_rb ? rng() % 100 : 0);
    std::vector<uint16_t> row(nnz);
    for (size_t rb = 0; rb < n_rb; ++rb)
        for (uint64_t e = start[rb_seg[rb]]; e < start[rb_seg[rb + 1]]; ++e) {
            const uint64_t lim = std::min<uint64_t>(kRowBlock, n_traj - rb * kRowBlock);
            row[e] = (uint16_t)(rng() % lim);
        }
    CompactHost c;
    CHECK(make_compact(h, row, start, rb_seg, n_traj, &c));
    CHECK(c.tile_slot.size() == n_tiles + 1 && c.tile_slot[0] == 0 && c.tile_slot[n_tiles] == c.slot_row.size());
    CHECK(c.row_slot_off.size() == n_traj + 1 && c.row_slot_off[n_traj] == c.slot_row.size());
    CHECK(c.row_slots.size() == c.slot_row.size());
    std::set<std::pair<uint64_t, uint32_t>> want_pairs, got_pairs;
    for (size_t rb = 0; rb < n_rb; ++rb)
        for (uint32_t t = h.rb_tile[rb]; t < h.rb_tile[rb + 1]; ++t) {
            const uint64_t lo = h.tasks[(size_t)t * kTileWaves].lo;
            const uint64_t hi = t + 1 < h.rb_tile[rb + 1] ? h.tasks[(size_t)(t + 1) * kTileWaves].lo
                                                           : start[rb_seg[rb + 1]];
            for (uint64_t e = lo; e < hi; ++e) want_pairs.insert({rb * kRowBlock + row[e], t});
            for (uint32_t k = c.tile_slot[t]; k < c.tile_slot[t + 1]; ++k) {
                CHECK(k == c.tile_slot[t] || c.slot_row[k] > c.slot_row[k - 1]);
                got_pairs.insert({rb * kRowBlock + c.slot_row[k], t});
            }
        }
    CHECK(got_pairs == want_pairs && got_pairs.size() == c.slot_row.size());
    std::vector<uint32_t> slot_tile(c.slot_row.size());
    for (uint32_t t = 0; t < n_tiles; ++t)
        for (uint32_t k = c.tile_slot[t]; k < c.tile_slot[t + 1]; ++k) slot_tile[k] = t;
    std::vector<uint8_t> used(c.slot_row.size(), 0);
    for (uint64_t r = 0; r < n_traj; ++r)
        for (uint32_t k = c.row_slot_off[r]; k < c.row_slot_off[r + 1]; ++k) {
            const uint32_t sl = c.row_slots[k];
            CHECK(sl < c.slot_row.size());
            if (sl >= c.slot_row.size()) continue;
            const size_t rb = r / kRowBlock;
            CHECK(c.slot_row[sl] == r % kRowBlock && slot_tile[sl] >= h.rb_tile[rb] && slot_tile[sl] < h.rb_tile[rb + 1]);
            ++used[sl];
        }
    for (uint8_t u : used) CHECK(u == 1);
}

static void check_tilings()
{
    std::mt19937 rng(11);
    std::vector<uint64_t> start, rb_seg;
    std::vector<uint32_t> word;
    for (int mode = 0; mode < 4; ++mode)
        for (int trial = 0; trial < 3; ++trial) {
            const uint32_t n_rb = 1 + rng() % 5, W = 16 + rng() % 300;
            random_segments(rng, n_rb, W, mode, &start, &word, &rb_seg);
            for (uint32_t target : {1u, 3u, 7u, 40u}) {
                const std::vector<uint32_t> k = tiles_per_block(block_costs(start, rb_seg), target);
                uint64_t sum = 0;
                for (uint32_t x : k) {
                    CHECK(x >= 1);
                    sum += x;
                }
                // a layout without entries keeps one tile per block
                CHECK(sum == (start.back() == 0 ? n_rb : std::max<uint64_t>(target, n_rb)));
                check_tiling(start, word, rb_seg, k);
            }
            check_tiling(start, word, rb_seg, std::vector<uint32_t>(n_rb, 2));
        }
    // balance: tasks of equal cost per share within a block (typical sizes, one block)
    random_segments(rng, 1, 4096, 0, &start, &word, &rb_seg);
    TilingHost h;
    make_tiling(start, word, rb_seg, std::vector<uint32_t>(1, 16), &h);
    // rounds per unit of the task's wave share (tasks are sized to the shares)
    auto per_share = [&](size_t i) { return (double)h.tasks[i].n_rounds / wave_share((uint32_t)(i % kTileWaves)); };
    double mx = 0, mn = 1e30;
    for (size_t i = 0; i < h.tasks.size(); ++i) {
        mx = std::max(mx, per_share(i));
        mn = std::min(mn, per_share(i));
    }
    CHECK(mx <= mn * 1.2 + 4);
    // balance across blocks: a full block of large segments and a short last
    // block of small ones (small segments cost more rounds per entry)
    start.clear();
    word.clear();
    rb_seg.assign(3, 0);
    uint64_t e = 0;
    for (uint32_t rb = 0; rb < 2; ++rb) {
        rb_seg[rb] = word.size();
        for (uint32_t w = 0; w < 4096; ++w) {
            start.push_back(e);
            word.push_back(w);
            e += rb == 0 ? 60 + rng() % 80 : 5 + rng() % 50;
        }
    }
    rb_seg[2] = word.size();
    start.push_back(e);
    const std::vector<uint32_t> k = tiles_per_block(block_costs(start, rb_seg), 48);
    CHECK(k[0] + k[1] == 48 && k[1] >= 1);
    make_tiling(start, word, rb_seg, k, &h);
    double sum = 0;
    mx = 0;
    for (size_t i = 0; i < h.tasks.size(); ++i) {
        mx = std::max(mx, per_share(i));
        sum += per_share(i);
    }
    const double mean = sum / h.tasks.size();
    CHECK(mx <= 1.15 * mean + 3);
    check_tiling(start, word, rb_seg, k);
}

// One-frame tile counts: one tile per CU when the row blocks split finely
// (the 200k-row headline has 25 blocks), more when a single tile per CU
// would leave some tiles a whole row block (134 blocks, as 1.1M rows have).
static void check_choose_tiles()
{
    auto total = [](const std::vector<uint32_t> &k) {
        uint64_t s = 0;
        for (uint32_t x : k) {
            CHECK(x >= 1);
            s += x;
        }
        return s;
    };
    auto max_tile = [](const std::vector<double> &c, const std::vector<uint32_t> &k) {
        double m = 0;
        for (size_t i = 0; i < c.size(); ++i) m = std::max(m, c[i] / k[i]);
        return m;
    };
    const std::vector<double> few(25, 7000.0);
    CHECK(total(choose_tiles(few, 256)) == 256);
    const std::vector<double> many(134, 4500.0);
    const std::vector<uint32_t> k = choose_tiles(many, 256);
    CHECK(total(k) > 256 && total(k) <= 1024);
    CHECK(max_tile(many, k) <= 0.5 * 4500.0);
    // more blocks than candidate tiles: one each
    const std::vector<double> huge(2000, 100.0);
    CHECK(total(choose_tiles(huge, 256)) == 2000);
    // uneven costs stay at least one tile per block, within the candidates
    std::mt19937 rng(5);
    for (int trial = 0; trial < 20; ++trial) {
        std::vector<double> c(1 + rng() % 300);
        for (double &x : c) x = 1.0 + rng() % 5000;
        const uint64_t t = total(choose_tiles(c, 256));
        CHECK(t >= c.size() && t <= std::max<uint64_t>(c.size(), 1024));
    }
}

int main()
{
    // six abstractions at the batched workload's sizes
    const uint64_t rows[6] = {25000, 100000, 50000, 200000, 150000, 10000};
    const uint32_t side[6] = {128, 128, 256, 512, 256, 512};
    std::vector<lbl_abs> abss(6);
    for (int i = 0; i < 6; ++i) {
        abss[i].n_traj = rows[i];
        abss[i].n_words = side[i] * side[i] / 64;
        abss[i].row_stride = abss[i].n_words;
        abss[i].T_bits = reinterpret_cast<uint64_t *>(0x100000000ull * (i + 1));
        abss[i].d_word_cell = reinterpret_cast<uint32_t *>(0x100000000ull * (i + 1) + 0x80000000ull);
    }
    std::mt19937 rng(7);
    uint8_t *fake = reinterpret_cast<uint8_t *>(0x200000000000ull);
    for (int trial = 0; trial < 20; ++trial) {
        std::vector<JobRef> jobs;
        const int n = 1 + (int)(rng() % 120);
        for (int k = 0; k < n; ++k) {
            lbl_abs *a = &abss[rng() % (trial % 3 == 0 ? 1 : 6)];
            const uint32_t np = 1 + rng() % 64;
            jobs.push_back(JobRef{a, fake, np, fake + 0x1000000000ull});
            fake += 0x2000000000ull;
        }
        for (int R : {1, 32, 128, 512, 4096}) check_case(abss, jobs, BatchTile{8, 4, R});
    }
    // the faulting shape: 16 frames on each of the six, 32-row items
    std::vector<JobRef> jobs;
    for (int i = 0; i < 6; ++i)
        for (int k = 0; k < 16; ++k) {
            jobs.push_back(JobRef{&abss[i], fake, (uint32_t)(4 + (k * 7 + i) % 61), fake + 0x1000000000ull});
            fake += 0x2000000000ull;
        }
    check_case(abss, jobs, BatchTile{4, 16, 32});
    // the same batches with the sparse layout present on every abstraction
    for (int i = 0; i < 6; ++i) abss[i].sp = fake_layout(rows[i], 0x300000000000ull + 0x100000000ull * i);
    check_case(abss, jobs, BatchTile{});
    for (int t = 1; t <= kBatchTilings + 1; ++t)
        for (int pers : {0, 1}) {
            BatchTile bt;
            bt.tiling = t;
            bt.persistent = pers;
            check_case(abss, jobs, bt);
        }
    for (int trial = 0; trial < 10; ++trial) {
        std::vector<JobRef> js;
        const int n = 1 + (int)(rng() % 120);
        for (int k = 0; k < n; ++k) {
            lbl_abs *a = &abss[rng() % 6];
            js.push_back(JobRef{a, fake, 1 + (uint32_t)(rng() % 64), fake + 0x1000000000ull});
            fake += 0x2000000000ull;
        }
        check_case(abss, js, BatchTile{});
    }
    // a batch mixing an abstraction without the sparse layout is planned bitpacked
    SparseLayout *keep = abss[2].sp;
    abss[2].sp = nullptr;
    check_case(abss, jobs, BatchTile{});
    abss[2].sp = keep;
    check_tilings();
    check_choose_tiles();
    // invalid jobs are rejected without touching anything
    BatchPlan p;
    JobRef bad{&abss[0], nullptr, 8, fake};
    CHECK(plan_batch(&bad, 1, -1, &p) == LBL_EINVAL);
    JobRef bad2{&abss[0], fake, 65, fake};
    CHECK(plan_batch(&bad2, 1, -1, &p) == LBL_EINVAL);
    abss[0].device = 3;
    JobRef other{&abss[0], fake, 8, fake};
    CHECK(plan_batch(&other, 1, 0, &p) == LBL_EINVAL);
    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("batch layout OK\n");
    return 0;
}
