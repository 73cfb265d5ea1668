// Event-based kernel timing (lbl_profile_*).
#include <deque>

#include "profile.h"

namespace lbl {

namespace {

struct Span {
    hipEvent_t a, b;
    int kind;  // 0 pack, 1 label, 2 batch, 3 emit
};

std::mutex g_mu;
bool g_on = false;
std::vector<Span> g_pending;
std::vector<hipEvent_t> g_free;
uint64_t g_n[4] = {0, 0, 0, 0};
double g_ms[4] = {0.0, 0.0, 0.0, 0.0};

hipEvent_t take()
{
    if (!g_free.empty()) {
        hipEvent_t e = g_free.back();
        g_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Fold completed spans into the totals (caller holds the lock).
hipError_t drain(bool wait)
{
    std::vector<Span> keep;
    for (const Span &s : g_pending) {
        if (!wait && hipEventQuery(s.b) != hipSuccess) {
            keep.push_back(s);
            continue;
        }
        hipError_t e = hipEventSynchronize(s.b);
        if (e != hipSuccess) return e;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, s.a, s.b);
        if (e != hipSuccess) return e;
        g_n[s.kind] += 1;
        g_ms[s.kind] += ms;
        g_free.push_back(s.a);
        g_free.push_back(s.b);
    }
    g_pending.swap(keep);
    return hipSuccess;
}

}  // namespace

bool profiling() { return g_on; }

void *span_begin(hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return nullptr;
    hipEvent_t e = take();
    if (!e) return nullptr;
    if (hipEventRecord(e, s) != hipSuccess) {
        g_free.push_back(e);
        return nullptr;
    }
    return e;
}

void span_end(void *begin, hipStream_t s, int kind)
{
    if (!begin) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t a = static_cast<hipEvent_t>(begin);
    hipEvent_t b = take();
    if (!b || hipEventRecord(b, s) != hipSuccess) {
        g_free.push_back(a);
        if (b) g_free.push_back(b);
        return;
    }
    g_pending.push_back(Span{a, b, kind});
    if (g_pending.size() > 4096) (void)drain(false);
}

}  // namespace lbl

using namespace lbl;

extern "C" {

lbl_status lbl_profile_enable(int on)
{
    clear_error();
    std::lock_guard<std::mutex> lk(g_mu);
    LBL_HIP_TRY(drain(true));
    g_on = on != 0;
    for (int k = 0; k < 4; ++k) {
        g_n[k] = 0;
        g_ms[k] = 0.0;
    }
    return LBL_OK;
}

lbl_status lbl_profile_read(lbl_profile *out)
{
    clear_error();
    LBL_REQUIRE(out != nullptr, "out is null");
    std::lock_guard<std::mutex> lk(g_mu);
    LBL_HIP_TRY(drain(true));
    out->pack_launches = g_n[0];
    out->label_launches = g_n[1];
    out->batch_launches = g_n[2];
    out->emit_launches = g_n[3];
    out->pack_ms = g_ms[0];
    out->label_ms = g_ms[1];
    out->batch_ms = g_ms[2];
    out->emit_ms = g_ms[3];
    return LBL_OK;
}

}  // extern "C"
