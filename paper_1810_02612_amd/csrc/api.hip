// Host side of the C ABI: validation, abstraction loading, per-frame
// labeling, workspace management and error reporting.
#include <algorithm>
#include <cstring>
#include <memory>
#include <unordered_map>

#include "lbl_internal.h"
#include "sparse.h"
#include "tune.h"

namespace lbl {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
void clear_error() { g_err.clear(); }

uint32_t morton2(uint32_t x, uint32_t y)
{
    auto spread = [](uint32_t v) {
        uint64_t r = v & 0xFFFFu;
        r = (r | (r << 8)) & 0x00FF00FFull;
        r = (r | (r << 4)) & 0x0F0F0F0Full;
        r = (r | (r << 2)) & 0x33333333ull;
        r = (r | (r << 1)) & 0x55555555ull;
        return (uint32_t)r;
    };
    return (spread(x) << 1) | spread(y);
}

void CellOrder::build(uint32_t nx_, uint32_t ny_, bool morton_)
{
    nx = nx_;
    ny = ny_;
    morton = morton_;
    ntx = nx / 8;
    nty = ny / 8;
    n_words = ntx * nty;
    std::vector<std::pair<uint32_t, uint32_t>> key(n_words);
    for (uint32_t ty = 0; ty < nty; ++ty)
        for (uint32_t tx = 0; tx < ntx; ++tx) key[ty * ntx + tx] = {morton2(tx, ty), ty * ntx + tx};
    std::sort(key.begin(), key.end());
    tile_word.assign(n_words, 0);
    for (uint32_t r = 0; r < n_words; ++r) tile_word[key[r].second] = r;
    word_cell.assign((size_t)n_words * 64, 0);
    for (uint32_t ty = 0; ty < nty; ++ty)
        for (uint32_t tx = 0; tx < ntx; ++tx) {
            const uint32_t w = tile_word[ty * ntx + tx];
            for (uint32_t dy = 0; dy < 8; ++dy)
                for (uint32_t dx = 0; dx < 8; ++dx) {
                    const uint32_t b = morton2(dx, dy);
                    // z-order ids: the device position is the caller's id
                    word_cell[(size_t)w * 64 + b] =
                        morton ? morton2(tx * 8 + dx, ty * 8 + dy) : (ty * 8 + dy) * nx + (tx * 8 + dx);
                }
        }
}

// ---------------------------------------------------------------- workspace

namespace {
struct WsBuf {
    void *p = nullptr;
    size_t n = 0;
    int device = -1;
};
std::mutex g_ws_mu;
std::unordered_map<hipStream_t, WsBuf> g_ws;
}  // namespace

lbl_status workspace(hipStream_t s, size_t bytes, void **out)
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    int dev = 0;
    LBL_HIP_TRY(hipGetDevice(&dev));
    WsBuf &b = g_ws[s];
    if (b.p && (b.n < bytes || b.device != dev)) {
        LBL_HIP_TRY(hipStreamSynchronize(s));
        int cur = dev;
        if (b.device != dev) LBL_HIP_TRY(hipSetDevice(b.device));
        (void)hipFree(b.p);
        if (b.device != dev) LBL_HIP_TRY(hipSetDevice(cur));
        b = WsBuf{};
    }
    if (!b.p) {
        size_t n = std::max<size_t>(bytes, 1u << 20);
        n = (n + 0xFFFFF) & ~size_t(0xFFFFF);
        LBL_HIP_TRY(hipMalloc(&b.p, n));
        b.n = n;
        b.device = dev;
    }
    *out = b.p;
    return LBL_OK;
}

lbl_status check_grid(const lbl_grid *g)
{
    LBL_REQUIRE(g != nullptr, "grid is null");
    LBL_REQUIRE(g->cell_order == LBL_ROW_MAJOR || g->cell_order == LBL_MORTON,
                "grid.cell_order must be LBL_ROW_MAJOR or LBL_MORTON");
    LBL_REQUIRE(g->nx > 0 && g->ny > 0 && g->nx % 8 == 0 && g->ny % 8 == 0,
                "grid nx and ny must be positive multiples of 8");
    LBL_REQUIRE((uint64_t)g->nx * g->ny <= (1ull << 31), "grid has more than 2^31 cells");
    LBL_REQUIRE(g->cell_order != LBL_MORTON || (g->nx == g->ny && (g->nx & (g->nx - 1)) == 0),
                "LBL_MORTON cell ids need a square grid whose side is a power of two");
    return LBL_OK;
}

// Allocate the abstraction's device tables and the zeroed bitpacked T.
static lbl_status abs_alloc(const lbl_grid *g, uint64_t n_traj, std::unique_ptr<lbl_abs> &a, bool dense = true)
{
    a.reset(new lbl_abs());
    LBL_HIP_TRY(hipGetDevice(&a->device));
    a->nx = g->nx;
    a->ny = g->ny;
    a->cell_m = g->cell_m;
    a->n_traj = n_traj;
    a->n_cells = g->nx * g->ny;
    a->order.build(g->nx, g->ny, g->cell_order == LBL_MORTON);
    a->n_words = a->order.n_words;
    a->row_stride = (a->n_words + 1) & ~1u;
    LBL_HIP_TRY(hipMalloc(&a->d_tile_word, a->order.tile_word.size() * sizeof(uint32_t)));
    LBL_HIP_TRY(hipMalloc(&a->d_word_cell, a->order.word_cell.size() * sizeof(uint32_t)));
    LBL_HIP_TRY(hipMemcpy(a->d_tile_word, a->order.tile_word.data(),
                          a->order.tile_word.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    LBL_HIP_TRY(hipMemcpy(a->d_word_cell, a->order.word_cell.data(),
                          a->order.word_cell.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    if (!dense) return LBL_OK;
    const size_t bytes = (size_t)n_traj * a->row_stride * sizeof(uint64_t);
    LBL_HIP_TRY(hipMalloc(&a->T_bits, bytes));
    LBL_HIP_TRY(hipMemset(a->T_bits, 0, bytes));
    return LBL_OK;
}

static void abs_release(lbl_abs *a)
{
    if (!a) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(a->device);
    (void)hipFree(a->T_bits);
    (void)hipFree(a->T_i8);
    (void)hipFree(a->d_tile_word);
    (void)hipFree(a->d_word_cell);
    free_sparse(a->sp);
    a->sp = nullptr;
    (void)hipSetDevice(cur);
}

struct AbsDeleter {
    void operator()(lbl_abs *a) const
    {
        abs_release(a);
        delete a;
    }
};

// Statistics and the optional int8 copy, once the bitpacked T is complete.
static lbl_status abs_finish(lbl_abs *a, uint32_t flags)
{
    unsigned long long *d_cnt = nullptr;
    LBL_HIP_TRY(hipMalloc(&d_cnt, 2 * sizeof(unsigned long long)));
    LBL_HIP_TRY(hipMemset(d_cnt, 0, 2 * sizeof(unsigned long long)));
    hipError_t e = launch_count_words(a->T_bits, a->row_stride, a->n_traj, a->n_words, d_cnt, nullptr);
    unsigned long long h[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpy(h, d_cnt, sizeof(h), hipMemcpyDeviceToHost);
    (void)hipFree(d_cnt);
    LBL_HIP_TRY(e);
    a->nonzero_words = h[0];
    a->set_cells = h[1];
    if (flags & LBL_LOAD_KEEP_INT8) {
        const size_t bytes = (size_t)a->n_traj * a->n_words * 64;
        LBL_HIP_TRY(hipMalloc(&a->T_i8, bytes));
        LBL_HIP_TRY(launch_expand_i8(a->T_i8, a->T_bits, a->row_stride, a->n_traj, a->n_words, nullptr));
    }
    LBL_HIP_TRY(hipDeviceSynchronize());
    if (!(flags & LBL_LOAD_NO_SPARSE)) {
        lbl_status st = build_sparse(a);
        if (st != LBL_OK) return st;
    }
    return LBL_OK;
}

}  // namespace lbl

using namespace lbl;

extern "C" {

const char *lbl_last_error(void) { return g_err.c_str(); }

const char *lbl_version(void) { return "lbl 0.1 (gfx950)"; }

lbl_status lbl_cell_position(const lbl_grid *grid, uint32_t cell, uint32_t *word, uint32_t *bit)
{
    clear_error();
    lbl_status st = check_grid(grid);
    if (st != LBL_OK) return st;
    LBL_REQUIRE(word && bit, "null output pointer");
    LBL_REQUIRE((uint64_t)cell < (uint64_t)grid->nx * grid->ny, "cell id out of range");
    if (grid->cell_order == LBL_MORTON) {  // the z-order index is the device position
        *word = cell >> 6;
        *bit = cell & 63u;
        return LBL_OK;
    }
    // rank of the tile among the grid's tiles in z-order
    const uint32_t ix = cell % grid->nx, iy = cell / grid->nx;
    const uint32_t ntx = grid->nx / 8, nty = grid->ny / 8;
    const uint32_t key = morton2(ix >> 3, iy >> 3);
    uint32_t rank = 0;
    if ((ntx & (ntx - 1)) == 0 && ntx == nty) {
        rank = key;
    } else {
        for (uint32_t ty = 0; ty < nty; ++ty)
            for (uint32_t tx = 0; tx < ntx; ++tx) rank += morton2(tx, ty) < key;
    }
    *word = rank;
    *bit = morton2(ix & 7u, iy & 7u);
    return LBL_OK;
}

lbl_status lbl_load_abstraction(const lbl_grid *grid, uint64_t n_traj, const uint64_t *row_ptr,
                                const uint32_t *col_idx, uint32_t flags, lbl_abs_t *out)
{
    clear_error();
    lbl_status st = check_grid(grid);
    if (st != LBL_OK) return st;
    LBL_REQUIRE(out != nullptr, "out is null");
    *out = nullptr;
    LBL_REQUIRE(row_ptr != nullptr, "row_ptr is null");
    LBL_REQUIRE(n_traj > 0, "n_traj must be positive");
    LBL_REQUIRE((flags & ~(LBL_LOAD_KEEP_INT8 | LBL_LOAD_INPUT_DEVICE | LBL_LOAD_NO_SPARSE | LBL_LOAD_SPARSE_ONLY)) == 0,
                "unknown load flag");
    const bool sparse_only = flags & LBL_LOAD_SPARSE_ONLY;
    LBL_REQUIRE(!sparse_only || !(flags & (LBL_LOAD_KEEP_INT8 | LBL_LOAD_NO_SPARSE)),
                "LBL_LOAD_SPARSE_ONLY excludes LBL_LOAD_KEEP_INT8 and LBL_LOAD_NO_SPARSE");
    LBL_REQUIRE(!sparse_only || n_traj < (1ull << 32), "LBL_LOAD_SPARSE_ONLY needs fewer than 2^32 rows");
    const bool dev_in = flags & LBL_LOAD_INPUT_DEVICE;

    // row pointers on the host for validation and chunking
    std::vector<uint64_t> rp_host;
    const uint64_t *rp = row_ptr;
    if (dev_in) {
        rp_host.resize(n_traj + 1);
        LBL_HIP_TRY(hipMemcpy(rp_host.data(), row_ptr, (n_traj + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost));
        rp = rp_host.data();
    }
    LBL_REQUIRE(rp[0] == 0, "row_ptr[0] must be 0");
    for (uint64_t t = 0; t < n_traj; ++t) LBL_REQUIRE(rp[t + 1] >= rp[t], "row_ptr must be non-decreasing");
    const uint64_t nnz = rp[n_traj];
    LBL_REQUIRE(nnz == 0 || col_idx != nullptr, "col_idx is null");

    std::unique_ptr<lbl_abs> tmp;
    st = abs_alloc(grid, n_traj, tmp, !sparse_only);
    std::unique_ptr<lbl_abs, AbsDeleter> a(tmp.release());
    if (st != LBL_OK) return st;

    uint32_t *d_bad = nullptr;
    LBL_HIP_TRY(hipMalloc(&d_bad, sizeof(uint32_t)));
    std::unique_ptr<uint32_t, decltype(&hipFree)> bad_guard(d_bad, &hipFree);
    LBL_HIP_TRY(hipMemset(d_bad, 0, sizeof(uint32_t)));

    // host input is uploaded in chunks of whole rows, at most ~64M column ids
    // and 2^20 rows each (one row may exceed the column bound)
    const uint64_t chunk_cap = 64ull << 20, chunk_rows = 1ull << 20;
    uint64_t *d_rp = nullptr;
    uint32_t *d_ci = nullptr;
    std::unique_ptr<uint64_t, decltype(&hipFree)> rp_guard(nullptr, &hipFree);
    std::unique_ptr<uint32_t, decltype(&hipFree)> ci_guard(nullptr, &hipFree);
    if (!dev_in) {
        uint64_t max_row = 0;
        for (uint64_t t = 0; t < n_traj; ++t) max_row = std::max(max_row, rp[t + 1] - rp[t]);
        LBL_HIP_TRY(hipMalloc(&d_rp, (std::min(n_traj, chunk_rows) + 1) * sizeof(uint64_t)));
        rp_guard.reset(d_rp);
        LBL_HIP_TRY(hipMalloc(&d_ci, std::max<uint64_t>(std::min(nnz, std::max(chunk_cap, max_row)), 1) *
                                         sizeof(uint32_t)));
        ci_guard.reset(d_ci);
    }
    // Sets the cells of rows [t_begin, t_end) in the zeroed bitpacked rows T,
    // whose first row is row `first`.
    auto pack_rows = [&](uint64_t *T, uint64_t first, uint64_t t_begin, uint64_t t_end) -> lbl_status {
        if (dev_in) {
            LBL_HIP_TRY(launch_pack_csr(T, a->row_stride, row_ptr + t_begin, t_begin - first, t_end - t_begin,
                                        col_idx, 0, a->d_tile_word, a->nx, a->n_cells, a->order.morton, d_bad,
                                        nullptr));
            LBL_HIP_TRY(hipDeviceSynchronize());
            return LBL_OK;
        }
        for (uint64_t t0 = t_begin; t0 < t_end;) {
            uint64_t t1 = t0 + 1;
            while (t1 < t_end && rp[t1 + 1] - rp[t0] <= chunk_cap && t1 - t0 < chunk_rows) ++t1;
            const uint64_t nc = rp[t1] - rp[t0];
            LBL_HIP_TRY(hipMemcpy(d_rp, rp + t0, (t1 - t0 + 1) * sizeof(uint64_t), hipMemcpyHostToDevice));
            if (nc) LBL_HIP_TRY(hipMemcpy(d_ci, col_idx + rp[t0], nc * sizeof(uint32_t), hipMemcpyHostToDevice));
            LBL_HIP_TRY(launch_pack_csr(T, a->row_stride, d_rp, t0 - first, t1 - t0, d_ci, rp[t0], a->d_tile_word,
                                        a->nx, a->n_cells, a->order.morton, d_bad, nullptr));
            LBL_HIP_TRY(hipDeviceSynchronize());
            t0 = t1;
        }
        return LBL_OK;
    };
    auto check_bad = [&]() -> lbl_status {
        uint32_t h_bad = 0;
        LBL_HIP_TRY(hipMemcpy(&h_bad, d_bad, sizeof(uint32_t), hipMemcpyDeviceToHost));
        LBL_REQUIRE(h_bad == 0, "col_idx holds a cell id >= nx * ny");
        return LBL_OK;
    };

    if (!sparse_only) {
        st = pack_rows(a->T_bits, 0, 0, n_traj);
        if (st == LBL_OK) st = check_bad();
        if (st == LBL_OK) st = abs_finish(a.get(), flags);
        if (st != LBL_OK) return st;
        *out = a.release();
        return LBL_OK;
    }

    // Sparse only: runs of whole row blocks (about 4 GiB of bitpacked rows
    // each) are packed into one reused buffer and turned into entries.
    const uint64_t row_bytes = (uint64_t)a->row_stride * sizeof(uint64_t);
    const uint64_t run = kRowBlock * std::max<uint64_t>(1, (4ull << 30) / (row_bytes * kRowBlock));
    uint64_t *d_T = nullptr;
    LBL_HIP_TRY(hipMalloc(&d_T, std::min(run, n_traj) * row_bytes));
    std::unique_ptr<uint64_t, decltype(&hipFree)> T_guard(d_T, &hipFree);
    unsigned long long *d_cnt = nullptr;
    LBL_HIP_TRY(hipMalloc(&d_cnt, 2 * sizeof(unsigned long long)));
    std::unique_ptr<unsigned long long, decltype(&hipFree)> cnt_guard(d_cnt, &hipFree);
    LBL_HIP_TRY(hipMemset(d_cnt, 0, 2 * sizeof(unsigned long long)));
    std::vector<SparsePart> parts;
    for (uint64_t r0 = 0; r0 < n_traj; r0 += run) {
        const uint64_t r1 = std::min(n_traj, r0 + run);
        LBL_HIP_TRY(hipMemset(d_T, 0, (r1 - r0) * row_bytes));
        st = pack_rows(d_T, r0, r0, r1);
        if (st != LBL_OK) return st;
        LBL_HIP_TRY(launch_count_words(d_T, a->row_stride, r1 - r0, a->n_words, d_cnt, nullptr));
        parts.emplace_back();
        st = sparse_part(d_T, a->row_stride, r1 - r0, a->n_words, &parts.back());
        if (st != LBL_OK) return st;
    }
    st = check_bad();
    if (st != LBL_OK) return st;
    unsigned long long h[2] = {0, 0};
    LBL_HIP_TRY(hipMemcpy(h, d_cnt, sizeof(h), hipMemcpyDeviceToHost));
    a->nonzero_words = h[0];
    a->set_cells = h[1];
    T_guard.reset();
    st = sparse_assemble(a.get(), parts);
    if (st != LBL_OK) return st;
    *out = a.release();
    return LBL_OK;
}

lbl_status lbl_load_abstraction_dense(const lbl_grid *grid, uint64_t n_traj, const uint8_t *T, uint32_t flags,
                                      lbl_abs_t *out)
{
    clear_error();
    lbl_status st = check_grid(grid);
    if (st != LBL_OK) return st;
    LBL_REQUIRE(out != nullptr, "out is null");
    *out = nullptr;
    LBL_REQUIRE(T != nullptr, "T is null");
    LBL_REQUIRE(n_traj > 0, "n_traj must be positive");
    LBL_REQUIRE((flags & ~(LBL_LOAD_KEEP_INT8 | LBL_LOAD_INPUT_DEVICE | LBL_LOAD_NO_SPARSE)) == 0, "unknown load flag");
    std::unique_ptr<lbl_abs> tmp;
    st = abs_alloc(grid, n_traj, tmp);
    std::unique_ptr<lbl_abs, AbsDeleter> a(tmp.release());
    if (st != LBL_OK) return st;
    const uint64_t n_cells = a->n_cells;
    if (flags & LBL_LOAD_INPUT_DEVICE) {
        LBL_HIP_TRY(launch_pack_dense(a->T_bits, a->row_stride, T, n_traj, a->n_cells, a->d_word_cell,
                                      a->n_words, nullptr));
    } else {
        const uint64_t rows_per_chunk = std::max<uint64_t>(1, (256ull << 20) / n_cells);
        const uint64_t rows = std::min(rows_per_chunk, n_traj);
        uint8_t *d_T = nullptr;
        LBL_HIP_TRY(hipMalloc(&d_T, rows * n_cells));
        std::unique_ptr<uint8_t, decltype(&hipFree)> guard(d_T, &hipFree);
        for (uint64_t t0 = 0; t0 < n_traj; t0 += rows) {
            const uint64_t nr = std::min(rows, n_traj - t0);
            LBL_HIP_TRY(hipMemcpy(d_T, T + t0 * n_cells, nr * n_cells, hipMemcpyHostToDevice));
            LBL_HIP_TRY(launch_pack_dense(a->T_bits + t0 * a->row_stride, a->row_stride, d_T, nr, a->n_cells,
                                          a->d_word_cell, a->n_words, nullptr));
            LBL_HIP_TRY(hipDeviceSynchronize());
        }
    }
    st = abs_finish(a.get(), flags);
    if (st != LBL_OK) return st;
    *out = a.release();
    return LBL_OK;
}

lbl_status lbl_free_abstraction(lbl_abs_t a)
{
    clear_error();
    if (!a) return LBL_OK;
    batch_forget(a);
    abs_release(a);
    delete a;
    return LBL_OK;
}

lbl_status lbl_abstraction_info(lbl_abs_t a, lbl_abs_info *out)
{
    clear_error();
    LBL_REQUIRE(a && out, "null argument");
    out->n_traj = a->n_traj;
    out->nx = a->nx;
    out->ny = a->ny;
    out->n_words = a->n_words;
    out->row_stride = a->row_stride;
    out->bits_bytes = a->T_bits ? a->n_traj * a->row_stride * sizeof(uint64_t) : 0;
    out->int8_bytes = a->T_i8 ? a->n_traj * a->n_words * 64ull : 0;
    out->nonzero_words = a->nonzero_words;
    out->set_cells = a->set_cells;
    out->sparse_entries = 0;
    out->sparse_bytes = 0;
    out->sparse_frame_bytes = 0;
    out->sparse_tiles = 0;
    out->sparse_row_block = 0;
    out->sparse_frame_bytes_narrow = 0;
    out->sparse_tiles_narrow = 0;
    out->sparse_tiles_direct = 0;
    out->sparse_frame_bytes_direct = 0;
    if (a->sp) {
        const SparseLayout &sp = *a->sp;
        const SpTiling &t = sp.tilings[0];
        const uint64_t entry_bytes = sp.nnz * (sizeof(uint16_t) + sizeof(uint64_t));
        out->sparse_entries = sp.nnz;
        out->sparse_bytes = entry_bytes + sp.round_bytes;
        // the one-frame label kernel's reads of the layout: entries, its
        // tasks and rounds, and the local rows of its compact partial slots
        out->sparse_frame_bytes = entry_bytes + (uint64_t)t.n_tiles * kTileWaves * sizeof(SpTask) +
                                  t.n_rounds * sizeof(SpRound) + t.n_slots * sizeof(uint16_t);
        out->sparse_tiles = t.n_tiles;
        out->sparse_row_block = kRowBlock;
        if ((int)sp.tilings.size() > kNarrowTiling) {
            const SpTiling &u = sp.tilings[kNarrowTiling];
            out->sparse_frame_bytes_narrow = entry_bytes + (uint64_t)u.n_tiles * kTileWaves * sizeof(SpTask) +
                                             u.n_rounds * sizeof(SpRound) + u.n_slots * sizeof(uint16_t);
            out->sparse_tiles_narrow = u.n_tiles;
        }
        const DirectLayout &d = sp.direct;
        if (d.chunks) {
            out->sparse_tiles_direct = d.n_tiles;
            out->sparse_frame_bytes_direct = entry_bytes + d.n_chunks * sizeof(SpChunk) +
                                             d.n_parts * sizeof(DirectPart) + (d.n_tiles + 1ull) * sizeof(uint32_t);
        }
    }
    return LBL_OK;
}

lbl_status lbl_label_frame(lbl_abs_t a, const uint8_t *O, uint32_t n_props, uint8_t *L, uint32_t flags,
                           void *hip_stream)
{
    clear_error();
    LBL_REQUIRE(a != nullptr, "abstraction is null");
    LBL_REQUIRE(O != nullptr && L != nullptr, "O or L is null");
    LBL_REQUIRE(n_props >= 1 && n_props <= 64, "n_props must be in [1, 64]");
    LBL_REQUIRE((flags & ~(LBL_HOST_PTRS | LBL_KERNEL_MASK)) == 0, "unknown flag");
    const uint32_t kflag = flags & LBL_KERNEL_MASK;
    LBL_REQUIRE(kflag == LBL_KERNEL_AUTO || kflag == LBL_KERNEL_BITS || kflag == LBL_KERNEL_MFMA ||
                    kflag == LBL_KERNEL_MFMA_I8 || kflag == LBL_KERNEL_SPARSE,
                "unknown kernel flag");
    LBL_REQUIRE(kflag != LBL_KERNEL_MFMA_I8 || a->T_i8 != nullptr,
                "LBL_KERNEL_MFMA_I8 needs an abstraction loaded with LBL_LOAD_KEEP_INT8");
    LBL_REQUIRE(a->T_bits != nullptr || kflag == LBL_KERNEL_AUTO || kflag == LBL_KERNEL_SPARSE,
                "the abstraction was loaded with LBL_LOAD_SPARSE_ONLY: only the sparse kernel can label it");
    LBL_REQUIRE(kflag != LBL_KERNEL_SPARSE || a->sp != nullptr,
                "LBL_KERNEL_SPARSE needs the sparse layout (loaded without LBL_LOAD_NO_SPARSE, fewer than 2^32 rows)");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    int cur = 0;
    LBL_HIP_TRY(hipGetDevice(&cur));
    LBL_REQUIRE(cur == a->device, "the current device is not the abstraction's device");

    const bool host = flags & LBL_HOST_PTRS;
    Plan plan = choose(a, n_props, kflag);
    const size_t ow_bytes = plan_ow_bytes(a, n_props, plan);
    const size_t o_bytes = host ? (size_t)a->n_cells * n_props : 0;
    const size_t l_bytes = host ? (size_t)a->n_traj * n_props : 0;
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    void *ws = nullptr;
    lbl_status st = workspace(s, up(ow_bytes) + up(o_bytes) + up(l_bytes), &ws);
    if (st != LBL_OK) return st;
    uint8_t *wsb = static_cast<uint8_t *>(ws);
    void *Ow = wsb;
    const uint8_t *Od = O;
    uint8_t *Ld = L;
    if (host) {
        uint8_t *Os = wsb + up(ow_bytes);
        Ld = Os + up(o_bytes);
        LBL_HIP_TRY(hipMemcpyAsync(Os, O, o_bytes, hipMemcpyHostToDevice, s));
        Od = Os;
    }
    st = run_plan(a, plan, Od, n_props, Ow, Ld, s);
    if (st != LBL_OK) return st;
    if (host) {
        LBL_HIP_TRY(hipMemcpyAsync(L, Ld, l_bytes, hipMemcpyDeviceToHost, s));
        LBL_HIP_TRY(hipStreamSynchronize(s));
    }
    return LBL_OK;
}

}  // extern "C"
