// Host-only check of the batch planner's device layout: every table and mask
// region must lie inside the buffer the plan asks for, work items must cover
// each abstraction's rows exactly once, and lane tables must map every
// (job, proposition) column exactly once.  No device memory is touched: the
// abstractions and buffers carry fake addresses, and bind_batch only writes
// the host image.
#include <cstdio>
#include <cstdlib>
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
        const size_t ow = (size_t)gs[g].n_words * gs[g].G64 * 64 * sizeof(uint64_t);
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
    uint64_t pairs = 0;
    for (const JobRef &j : jobs) pairs += j.a->n_traj * j.n_props;
    CHECK(p.pairs == pairs);
    // sparse plans: partial regions inside and disjoint, every tile once,
    // every row of every lane group combined once
    bool sparse = true;
    for (const JobRef &j : jobs) sparse = sparse && j.a->sp_seg != nullptr;
    CHECK(p.sparse == sparse);
    if (!p.sparse) return;
    std::vector<std::pair<const uint8_t *, const uint8_t *>> p_ranges;
    std::set<std::tuple<uint32_t, uint32_t, uint32_t, uint32_t>> tiles;
    uint64_t want_tiles = 0;
    for (size_t g = 0; g < p.groups.size(); ++g) {
        const GroupDesc &d = gs[g];
        CHECK(d.n_rb == (uint32_t)((d.n_traj + kRowBlock - 1) / kRowBlock));
        CHECK(d.n_wr >= 1 && (uint64_t)d.n_wr * d.wr_words >= d.n_words && (d.n_wr - 1) * d.wr_words < d.n_words);
        const size_t pb = (size_t)d.G64 * d.n_wr * d.n_rb * kRowBlock * sizeof(uint64_t);
        CHECK(inside(d.P, pb));
        p_ranges.push_back({reinterpret_cast<const uint8_t *>(d.P), reinterpret_cast<const uint8_t *>(d.P) + pb});
        want_tiles += (uint64_t)d.n_rb * d.n_wr * d.G64;
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
        CHECK(t.rb < d.n_rb && t.wr < d.n_wr && t.gi < d.G64);
        tiles.insert(std::make_tuple(t.group, t.rb, t.wr, t.gi));
    }
    CHECK(tiles.size() == p.tiles.size() && p.tiles.size() == want_tiles);
    std::map<std::pair<uint32_t, uint32_t>, uint64_t> rows;
    for (const CombineItem &c : p.combines) {
        CHECK(c.group < p.groups.size() && c.gi < p.groups[c.group].G64);
        CHECK(c.row0 < c.row1 && c.row1 <= p.groups[c.group].n_traj && c.row0 % 64 == 0);
        rows[std::make_pair(c.group, c.gi)] += c.row1 - c.row0;
    }
    for (size_t g = 0; g < p.groups.size(); ++g)
        for (uint32_t gi = 0; gi < p.groups[g].G64; ++gi) {
            const uint64_t covered_rows = rows[std::make_pair((uint32_t)g, gi)];
            CHECK(covered_rows == p.groups[g].n_traj);
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
    for (int i = 0; i < 6; ++i) {
        abss[i].sp_seg = reinterpret_cast<uint64_t *>(0x300000000000ull + 0x10000000ull * i);
        abss[i].sp_row = reinterpret_cast<uint16_t *>(0x310000000000ull + 0x10000000ull * i);
        abss[i].sp_val = reinterpret_cast<uint64_t *>(0x320000000000ull + 0x10000000ull * i);
        abss[i].sp_nnz = rows[i] * 50;
        abss[i].sp_geom.n_rb = (uint32_t)((rows[i] + kRowBlock - 1) / kRowBlock);
    }
    check_case(abss, jobs, BatchTile{});
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
    abss[2].sp_seg = nullptr;
    check_case(abss, jobs, BatchTile{});
    abss[2].sp_seg = reinterpret_cast<uint64_t *>(0x300000000000ull + 0x20000000ull);
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
