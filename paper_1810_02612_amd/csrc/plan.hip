// Minimum-cost paths on the product of a transition system and a runtime
// monitor (Sec. 3.2): product vertices are (v, q), and a transition e = (u,
// v) of cost C(e) joins (u, q) to (v, q') when the monitor moves from q to q'
// on the label of e.  A monitor with no move for a label has met a bad
// prefix, so that product edge is absent.
//
// Bellman-Ford on the device: every sweep relaxes each (edge, state) pair
// once, with a 64-bit atomic minimum of (distance << 32 | product edge id),
// until a sweep changes nothing.  Values only decrease and each is the cost
// of a real path, so the fixpoint holds the shortest distances, and in the
// low word the smallest product edge id among the edges on a shortest path
// into the vertex.  Costs are at least 1, so predecessors always have a
// smaller distance and the predecessor graph is a tree.  A graph with n
// product vertices needs at most n sweeps (each kernel ends; the host loop
// is bounded).  Sweeps run in groups of kGroup between reads of their flags
// (a sweep after the fixpoint changes nothing, so the extra ones are
// harmless), which saves a host synchronization per sweep.
#include <algorithm>

#include "lbl_internal.h"

namespace lbl {
namespace {

constexpr uint64_t kNone = ~0ull;
constexpr uint32_t kGroup = 4;  // sweeps per read of the flags

__global__ void __launch_bounds__(256) k_plan_init(uint64_t *__restrict__ best, uint64_t n, uint64_t start)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        best[i] = i == start ? 0xFFFFFFFFull : kNone;  // start: distance 0, no predecessor
}

// flags[0]: some value decreased; flags[1]: an edge names a vertex out of
// range or has cost 0.
__global__ void __launch_bounds__(256)
k_plan_relax(const uint32_t *__restrict__ src, const uint32_t *__restrict__ dst, const uint32_t *__restrict__ cost,
             const uint8_t *__restrict__ L, uint32_t l_stride, uint32_t n_props, uint32_t n_states,
             const uint8_t *__restrict__ delta,
             uint64_t n_vertices, uint64_t n_edges, uint64_t start, uint64_t *__restrict__ best,
             uint32_t *__restrict__ flags)
{
    bool changed = false, bad = false;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_edges;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t u = src[e], v = dst[e], c = cost[e];
        if (u >= n_vertices || v >= n_vertices || c == 0) {
            bad = true;
            continue;
        }
        uint32_t sigma = 0;  // the label as a proposition bit set
        for (uint32_t p = 0; p < n_props; ++p) sigma |= (L[e * l_stride + p] != 0 ? 1u : 0u) << p;
        for (uint32_t q = 0; q < n_states; ++q) {
            const uint64_t du = best[(uint64_t)u * n_states + q] >> 32;
            if (du == 0xFFFFFFFFull) continue;  // not reached yet
            const uint32_t q2 = delta[(q << n_props) | sigma];
            if (q2 >= n_states) continue;  // the monitor rejects: no product edge
            const uint64_t nd = du + c;
            if (nd >= 0xFFFFFFFFull) continue;  // beyond the representable costs
            const uint64_t to = (uint64_t)v * n_states + q2;
            if (to == start) continue;  // the start keeps distance 0 and no predecessor
            const uint64_t cand = (nd << 32) | (e * n_states + q);
            // values only decrease: a candidate no better than a value read
            // now cannot win, and most relaxations after the first sweeps are
            // such (their atomic would only cost time)
            if (cand >= best[to]) continue;
            const unsigned long long old = atomicMin(reinterpret_cast<unsigned long long *>(best + to), cand);
            changed = changed || cand < old;
        }
    }
    // one atomic per wavefront that saw a change (vector atomics only)
    const uint64_t any_changed = __ballot(changed), any_bad = __ballot(bad);
    const uint32_t lane = threadIdx.x & 63;
    if (any_changed && lane == (uint32_t)__builtin_ctzll(any_changed)) atomicOr(flags + 0, 1u);
    if (any_bad && lane == (uint32_t)__builtin_ctzll(any_bad)) atomicOr(flags + 1, 1u);
}

__global__ void __launch_bounds__(256)
k_plan_unpack(const uint64_t *__restrict__ best, uint64_t n, uint32_t *__restrict__ dist, uint32_t *__restrict__ pred)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t b = best[i];
        dist[i] = (uint32_t)(b >> 32);
        pred[i] = (uint32_t)b;
    }
}

unsigned blocks_for(uint64_t n) { return (unsigned)std::min<uint64_t>(std::max<uint64_t>((n + 255) / 256, 1), 8192); }

}  // namespace
}  // namespace lbl

using namespace lbl;

extern "C" lbl_status lbl_product_shortest_paths(uint64_t n_vertices, uint64_t n_edges, const uint32_t *src,
                                                 const uint32_t *dst, const uint32_t *cost, const uint8_t *L,
                                                 uint32_t l_stride, uint32_t n_props, uint32_t n_states,
                                                 const uint8_t *delta,
                                                 uint32_t v0, uint32_t q0, uint32_t *dist, uint32_t *pred,
                                                 uint32_t *n_sweeps, void *hip_stream)
{
    clear_error();
    LBL_REQUIRE(n_vertices > 0, "n_vertices must be positive");
    LBL_REQUIRE(n_edges == 0 || (src && dst && cost && L), "src, dst, cost or L is null");
    LBL_REQUIRE(delta && dist && pred, "delta, dist or pred is null");
    LBL_REQUIRE(n_props >= 1 && n_props <= 8, "n_props must be in [1, 8]");
    LBL_REQUIRE(l_stride >= n_props, "l_stride must be at least n_props");
    LBL_REQUIRE(n_states >= 1 && n_states <= 8, "n_states must be in [1, 8]");
    LBL_REQUIRE(v0 < n_vertices && q0 < n_states, "start vertex or state out of range");
    LBL_REQUIRE(n_vertices * n_states < 0xFFFFFFFFull, "too many product vertices (n_vertices * n_states >= 2^32 - 1)");
    LBL_REQUIRE(n_edges * n_states < 0xFFFFFFFFull, "too many product edges (n_edges * n_states >= 2^32 - 1)");
    const size_t n_delta = (size_t)n_states << n_props;
    for (size_t i = 0; i < n_delta; ++i)
        LBL_REQUIRE(delta[i] < n_states || delta[i] == LBL_MONITOR_REJECT,
                    "delta holds a state >= n_states (use LBL_MONITOR_REJECT for no move)");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    int cur = 0;
    LBL_HIP_TRY(hipGetDevice(&cur));

    const uint64_t n = n_vertices * n_states;
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    void *ws = nullptr;
    lbl_status st = workspace(s, up(n * sizeof(uint64_t)) + up(n_delta) + up(2 * kGroup * sizeof(uint32_t)), &ws);
    if (st != LBL_OK) return st;
    uint64_t *best = static_cast<uint64_t *>(ws);
    uint8_t *d_delta = reinterpret_cast<uint8_t *>(ws) + up(n * sizeof(uint64_t));
    uint32_t *d_flags = reinterpret_cast<uint32_t *>(d_delta + up(n_delta));
    LBL_HIP_TRY(hipMemcpyAsync(d_delta, delta, n_delta, hipMemcpyHostToDevice, s));
    const uint64_t start = (uint64_t)v0 * n_states + q0;
    hipLaunchKernelGGL(k_plan_init, dim3(blocks_for(n)), dim3(256), 0, s, best, n, start);
    LBL_HIP_TRY(hipGetLastError());
    // Bellman-Ford needs at most n sweeps before one that changes nothing
    uint64_t sweeps = 0;
    bool done = false;
    for (uint64_t run = 0; !done && run <= n; run += kGroup) {
        LBL_HIP_TRY(hipMemsetAsync(d_flags, 0, 2 * kGroup * sizeof(uint32_t), s));
        for (uint32_t j = 0; j < kGroup; ++j) {
            hipLaunchKernelGGL(k_plan_relax, dim3(blocks_for(n_edges)), dim3(256), 0, s, src, dst, cost, L, l_stride,
                               n_props, n_states, d_delta, n_vertices, n_edges, start, best, d_flags + 2 * j);
            LBL_HIP_TRY(hipGetLastError());
        }
        uint32_t h[2 * kGroup] = {};
        LBL_HIP_TRY(hipMemcpyAsync(h, d_flags, sizeof(h), hipMemcpyDeviceToHost, s));
        LBL_HIP_TRY(hipStreamSynchronize(s));
        for (uint32_t j = 0; j < kGroup; ++j)
            LBL_REQUIRE(h[2 * j + 1] == 0, "an edge names a vertex >= n_vertices or has cost 0");
        for (uint32_t j = 0; j < kGroup && !done; ++j) {
            ++sweeps;
            done = h[2 * j] == 0;  // this sweep changed nothing: the fixpoint
        }
    }
    LBL_REQUIRE(done, "no fixpoint within the Bellman-Ford bound (cannot happen with costs >= 1)");
    hipLaunchKernelGGL(k_plan_unpack, dim3(blocks_for(n)), dim3(256), 0, s, best, n, dist, pred);
    LBL_HIP_TRY(hipGetLastError());
    LBL_HIP_TRY(hipStreamSynchronize(s));
    if (n_sweeps) *n_sweeps = (uint32_t)std::min<uint64_t>(sweeps, 0xFFFFFFFFull);
    return LBL_OK;
}
