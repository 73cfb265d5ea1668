// Kernel plans and the autotuner.
//
// A shape class is (words per row, log2 of the row count, number of 16-wide
// proposition tiles, log2 of T's non-zero word fraction).  lbl_tune times
// every candidate plan on one frame with HIP events and records the fastest
// for the class; LBL_KERNEL_AUTO looks the class up and falls back to the
// bitpacked kernel's default tile.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>

#include "batch.h"
#include "profile.h"
#include "sparse.h"
#include "tune.h"

namespace lbl {

namespace {

struct Entry {
    Plan plan;
    double us = 0.0;
};

std::mutex g_mu;
std::map<std::string, Entry> g_cache;

std::string shape_key(const lbl_abs *a, uint32_t n_props)
{
    const int tb = (int)std::ceil(std::log2((double)std::max<uint64_t>(a->n_traj, 1)));
    const double frac = a->n_traj && a->n_words
                            ? (double)std::max<uint64_t>(a->nonzero_words, 1) / ((double)a->n_traj * a->n_words)
                            : 1.0;
    const int zb = (int)std::lround(std::log2(frac));
    char buf[96];
    snprintf(buf, sizeof(buf), "W%u/T%d/P%u/Z%d", a->n_words, tb, (n_props + 15) / 16, zb);
    return buf;
}

const char *kernel_name(Kernel k)
{
    switch (k) {
    case Kernel::Bits: return "bits";
    case Kernel::Mfma: return "mfma";
    case Kernel::MfmaI8: return "mfma_i8";
    case Kernel::Sparse: return "sparse";
    }
    return "?";
}

bool kernel_from_name(const std::string &s, Kernel *k)
{
    if (s == "bits") *k = Kernel::Bits;
    else if (s == "mfma") *k = Kernel::Mfma;
    else if (s == "mfma_i8") *k = Kernel::MfmaI8;
    else if (s == "sparse") *k = Kernel::Sparse;
    else return false;
    return true;
}

// The plan used when nothing was tuned: the sparse kernel where the layout
// exists, else the bitpacked kernel.
Plan default_plan(const lbl_abs *a)
{
    Plan p;
    p.kernel = a->sp ? Kernel::Sparse : Kernel::Bits;
    return p;
}

bool plan_usable(const lbl_abs *a, const Plan &p)
{
    if (p.kernel == Kernel::Sparse) return a->sp != nullptr;
    if (!a->T_bits) return false;  // loaded sparse only
    return !(p.kernel == Kernel::MfmaI8 && !a->T_i8);
}

// Synthetic frame: every (cell, proposition) byte is 1 with probability
// density, from a counter-based hash of (seed, index).
__global__ void k_bernoulli(uint8_t *O, uint64_t n, uint32_t threshold, uint32_t seed)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t x = i * 0x9E3779B97F4A7C15ull + seed;
        x ^= x >> 30;
        x *= 0xBF58476D1CE4E5B9ull;
        x ^= x >> 27;
        x *= 0x94D049BB133111EBull;
        x ^= x >> 31;
        O[i] = (uint32_t)x < threshold ? 1 : 0;
    }
}

}  // namespace

std::string plan_name(const Plan &p)
{
    char buf[96];
    if (p.kernel == Kernel::Bits)
        snprintf(buf, sizeof(buf), "bits(unroll=%d,waves=%d)", p.bits.unroll, p.bits.waves_per_block);
    else if (p.kernel == Kernel::Sparse)
        snprintf(buf, sizeof(buf), "sparse(rows=%u,waves=%u)", kRowBlock, kTileWaves);
    else
        snprintf(buf, sizeof(buf), "%s(m_tiles=%d,waves=%d)", kernel_name(p.kernel), p.mfma.m_tiles,
                 p.mfma.waves_per_block);
    return buf;
}

Plan choose(const lbl_abs *a, uint32_t n_props, uint32_t kflag)
{
    Plan p;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(shape_key(a, n_props));
    if (kflag == LBL_KERNEL_AUTO) {
        p = it != g_cache.end() ? it->second.plan : default_plan(a);
        if (!plan_usable(a, p)) p = default_plan(a);
        return p;
    }
    p.kernel = kflag == LBL_KERNEL_BITS     ? Kernel::Bits
               : kflag == LBL_KERNEL_MFMA   ? Kernel::Mfma
               : kflag == LBL_KERNEL_SPARSE ? Kernel::Sparse
                                            : Kernel::MfmaI8;
    // keep tuned tile shapes when the cached winner is the same kernel
    if (it != g_cache.end() && it->second.plan.kernel == p.kernel) p = it->second.plan;
    return p;
}

size_t plan_ow_bytes(const lbl_abs *a, uint32_t, const Plan &p)
{
    if (p.kernel == Kernel::Sparse) return swm_workspace_bytes(a);
    return (size_t)a->n_words * 64 * sizeof(uint64_t);
}

lbl_status run_plan(const lbl_abs *a, const Plan &p, const uint8_t *O, uint32_t n_props, void *Ow, uint8_t *L,
                    hipStream_t s)
{
    if (p.kernel == Kernel::Sparse) return run_swm(a, O, n_props, Ow, L, s);
    LBL_REQUIRE(a->T_bits != nullptr, "the abstraction has no bitpacked T (loaded sparse only)");
    uint64_t *ow = static_cast<uint64_t *>(Ow);
    if (p.kernel != Kernel::Bits) {
        lbl_status st = mfma_layout_selftest();
        if (st != LBL_OK) return st;
    }
    void *span = span_begin(s);
    LBL_HIP_TRY(launch_pack_O(a, O, n_props, ow, s));
    span_end(span, s, 0);
    span = span_begin(s);
    switch (p.kernel) {
    case Kernel::Bits: LBL_HIP_TRY(launch_label_bits(a, ow, n_props, L, p.bits, s)); break;
    case Kernel::Mfma:
    case Kernel::MfmaI8:
        LBL_HIP_TRY(launch_label_mfma(a, ow, n_props, L, p.mfma, p.kernel == Kernel::MfmaI8, s));
        break;
    case Kernel::Sparse: break;  // handled above
    }
    span_end(span, s, 1);
    return LBL_OK;
}


}  // namespace lbl

using namespace lbl;

extern "C" {

lbl_status lbl_tune(lbl_abs_t a, const uint8_t *O_sample, uint32_t n_props, uint32_t density_pct, void *hip_stream)
{
    clear_error();
    LBL_REQUIRE(a != nullptr, "abstraction is null");
    LBL_REQUIRE(n_props >= 1 && n_props <= 64, "n_props must be in [1, 64]");
    LBL_REQUIRE(density_pct <= 100, "density_pct must be in [0, 100]");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const size_t o_bytes = (size_t)a->n_cells * n_props;
    const size_t l_bytes = (size_t)a->n_traj * n_props;
    // workspace large enough for every candidate plan
    size_t ws_bytes = (size_t)a->n_words * 64 * sizeof(uint64_t);
    if (a->sp) ws_bytes = std::max(ws_bytes, swm_workspace_bytes(a));
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    uint8_t *buf = nullptr;
    LBL_HIP_TRY(hipMalloc(&buf, up(ws_bytes) + up(l_bytes) + up(o_bytes)));
    std::unique_ptr<uint8_t, decltype(&hipFree)> guard(buf, &hipFree);
    uint64_t *Ow = reinterpret_cast<uint64_t *>(buf);
    uint8_t *L = buf + up(ws_bytes);
    uint8_t *O = L + up(l_bytes);
    if (O_sample) {
        O = const_cast<uint8_t *>(O_sample);
    } else {
        const uint32_t thr = (uint32_t)std::min<double>(4294967295.0, density_pct / 100.0 * 4294967296.0);
        hipLaunchKernelGGL(k_bernoulli, dim3(4096), dim3(256), 0, s, O, (uint64_t)o_bytes, thr, 0x5eedu);
        LBL_HIP_TRY(hipGetLastError());
    }
    std::vector<Plan> cands;
    if (a->sp) {
        Plan p;
        p.kernel = Kernel::Sparse;
        cands.push_back(p);
    }
    for (int u : {2, 4, 8, 16})
        for (int w : {2, 4, 8}) {
            if (!a->T_bits) break;  // loaded sparse only
            Plan p;
            p.kernel = Kernel::Bits;
            p.bits.unroll = u;
            p.bits.waves_per_block = w;
            cands.push_back(p);
        }
    if (a->T_bits && mfma_layout_selftest() == LBL_OK) {
        for (int m : {1, 2, 4})
            for (int w : {2, 4}) {
                Plan p;
                p.kernel = Kernel::Mfma;
                p.mfma.m_tiles = m;
                p.mfma.waves_per_block = w;
                cands.push_back(p);
            }
        if (a->T_i8)
            for (int m : {1, 2}) {
                Plan p;
                p.kernel = Kernel::MfmaI8;
                p.mfma.m_tiles = m;
                p.mfma.waves_per_block = 4;
                cands.push_back(p);
            }
    }
    clear_error();
    hipEvent_t e0, e1;
    LBL_HIP_TRY(hipEventCreate(&e0));
    LBL_HIP_TRY(hipEventCreate(&e1));
    Entry best;
    best.us = 1e300;
    for (const Plan &p : cands) {
        lbl_status st = run_plan(a, p, O, n_props, Ow, L, s);  // warm-up
        if (st != LBL_OK) continue;
        const int reps = 3;
        LBL_HIP_TRY(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) run_plan(a, p, O, n_props, Ow, L, s);
        LBL_HIP_TRY(hipEventRecord(e1, s));
        LBL_HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        LBL_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        const double us = 1000.0 * ms / reps;
        if (us < best.us) {
            best.us = us;
            best.plan = p;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    LBL_HIP_TRY(hipStreamSynchronize(s));
    LBL_REQUIRE(best.us < 1e299, "no candidate plan ran");
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[shape_key(a, n_props)] = best;
    return LBL_OK;
}

lbl_status lbl_tune_describe(lbl_abs_t a, uint32_t n_props, char *buf, size_t buf_len)
{
    clear_error();
    LBL_REQUIRE(a && buf && buf_len > 0, "null argument");
    LBL_REQUIRE(n_props >= 1 && n_props <= 64, "n_props must be in [1, 64]");
    const Plan p = choose(a, n_props, LBL_KERNEL_AUTO);
    std::string s = shape_key(a, n_props) + " -> " + plan_name(p);
    snprintf(buf, buf_len, "%s", s.c_str());
    return LBL_OK;
}

lbl_status lbl_tune_save(const char *path)
{
    clear_error();
    LBL_REQUIRE(path != nullptr, "path is null");
    std::ostringstream o;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        o << "[\n";
        bool first = true;
        for (const auto &kv : g_cache) {
            const Plan &p = kv.second.plan;
            o << (first ? "" : ",\n") << "  {\"key\": \"" << kv.first << "\", \"kernel\": \"" << kernel_name(p.kernel)
              << "\", \"unroll\": " << p.bits.unroll << ", \"waves\": " << p.bits.waves_per_block
              << ", \"m_tiles\": " << p.mfma.m_tiles << ", \"mfma_waves\": " << p.mfma.waves_per_block
              << ", \"us\": " << kv.second.us << "}";
            first = false;
        }
        for (const auto &kv : batch_tiles()) {
            const BatchTile &t = kv.second;
            o << (first ? "" : ",\n") << "  {\"batch\": \"" << kv.first << "\", \"unroll\": " << t.unroll
              << ", \"waves\": " << t.waves_per_block << ", \"rows\": " << t.rows_per_item
              << ", \"tiling\": " << t.tiling << ", \"persistent\": " << t.persistent << "}";
            first = false;
        }
        o << "\n]\n";
    }
    std::ofstream f(path);
    LBL_REQUIRE(f.good(), std::string("cannot write ") + path);
    f << o.str();
    return LBL_OK;
}

lbl_status lbl_tune_load(const char *path)
{
    clear_error();
    LBL_REQUIRE(path != nullptr, "path is null");
    std::ifstream f(path);
    LBL_REQUIRE(f.good(), std::string("cannot read ") + path);
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string text = ss.str();
    std::map<std::string, Entry> loaded;
    std::vector<std::pair<std::string, BatchTile>> batch_loaded;
    size_t pos = 0;
    while ((pos = text.find('{', pos)) != std::string::npos) {
        const size_t end = text.find('}', pos);
        LBL_REQUIRE(end != std::string::npos, "malformed tune cache: unterminated object");
        const std::string obj = text.substr(pos, end - pos + 1);
        auto str_field = [&](const char *name, std::string *out) {
            const std::string pat = std::string("\"") + name + "\": \"";
            size_t p = obj.find(pat);
            if (p == std::string::npos) return false;
            p += pat.size();
            size_t q = obj.find('"', p);
            if (q == std::string::npos) return false;
            *out = obj.substr(p, q - p);
            return true;
        };
        auto num_field = [&](const char *name, double *out) {
            const std::string pat = std::string("\"") + name + "\": ";
            size_t p = obj.find(pat);
            if (p == std::string::npos) return false;
            *out = std::strtod(obj.c_str() + p + pat.size(), nullptr);
            return true;
        };
        std::string key, kname;
        double unroll, waves, mt, mw, us;
        if (str_field("batch", &key)) {
            // a batch shape class and its launch choices
            double rows, tiling, pers;
            LBL_REQUIRE(num_field("unroll", &unroll) && num_field("waves", &waves) && num_field("rows", &rows) &&
                            num_field("tiling", &tiling) && num_field("persistent", &pers),
                        "malformed tune cache batch entry");
            BatchTile t{(int)unroll, (int)waves, (int)rows, (int)tiling, (int)pers};
            LBL_REQUIRE((t.unroll == 4 || t.unroll == 8) && t.waves_per_block >= 1 && t.waves_per_block <= 16 &&
                            t.rows_per_item >= 1 && t.tiling >= 0 && t.tiling <= kBatchTilings + 1 &&
                            (t.persistent == 0 || t.persistent == 1),
                        "tune cache batch entry has an unsupported tile");
            batch_loaded.push_back({key, t});
            pos = end + 1;
            continue;
        }
        LBL_REQUIRE(str_field("key", &key) && str_field("kernel", &kname) && num_field("unroll", &unroll) &&
                        num_field("waves", &waves) && num_field("m_tiles", &mt) && num_field("mfma_waves", &mw) &&
                        num_field("us", &us),
                    "malformed tune cache entry");
        Entry e;
        LBL_REQUIRE(kernel_from_name(kname, &e.plan.kernel), "unknown kernel in tune cache");
        e.plan.bits.unroll = (int)unroll;
        e.plan.bits.waves_per_block = (int)waves;
        e.plan.mfma.m_tiles = (int)mt;
        e.plan.mfma.waves_per_block = (int)mw;
        e.us = us;
        const bool ok_u = e.plan.bits.unroll == 2 || e.plan.bits.unroll == 4 || e.plan.bits.unroll == 8 ||
                          e.plan.bits.unroll == 16;
        LBL_REQUIRE(ok_u && e.plan.bits.waves_per_block >= 1 && e.plan.bits.waves_per_block <= 16 &&
                        (e.plan.mfma.m_tiles == 1 || e.plan.mfma.m_tiles == 2 || e.plan.mfma.m_tiles == 4) &&
                        e.plan.mfma.waves_per_block >= 1 && e.plan.mfma.waves_per_block <= 4,
                    "tune cache entry has an unsupported tile");
        loaded[key] = e;
        pos = end + 1;
    }
    for (auto &kv : batch_loaded) set_batch_tile(kv.first, kv.second);
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : loaded) g_cache[kv.first] = kv.second;
    return LBL_OK;
}

}  // extern "C"
