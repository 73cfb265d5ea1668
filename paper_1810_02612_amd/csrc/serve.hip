// Serving loop with continuous batching.
//
// Clients submit frames (device pointers) from any thread.  A worker thread
// owns n_streams slots; each slot is one stream, a completion event, a
// pinned staging buffer for the batch tables and a device arena of
// hbm_budget / n_streams bytes for the batch's tables and packed masks.
// Whenever a slot is free and requests are pending, the worker forms a batch
// from the front of the queue (at most max_batch_frames requests, as many as
// fit the arena: admission by memory) and launches it with the same
// persistent kernel as lbl_label_batch (a batch of one frame: the one-frame
// kernels), while earlier batches are still running on the other slots.  Requests that arrive meanwhile join the next
// batch.  While batches are in flight the worker polls their completion
// events every few microseconds (it sleeps on a condition variable only when
// idle).  Latency is completion minus submission on the host's monotonic
// clock.  A frame's columns never share lanes with another frame's, so its
// labels do not depend on its batch-mates.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

#include "batch.h"
#include "sparse.h"

namespace {

using Clock = std::chrono::steady_clock;

double now_s()
{
    return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket;
    lbl::JobRef job;
    double t_submit;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint8_t *arena = nullptr;
    size_t arena_bytes = 0;
    uint8_t *pinned = nullptr;
    size_t pinned_bytes = 0;
    bool busy = false;
    size_t used = 0;
    std::vector<Request> reqs;
    uint64_t pairs = 0;
};

struct Outcome {
    bool finished = false;
    lbl_status st = LBL_OK;
    std::string msg;
};

}  // namespace

struct lbl_server {
    lbl_serve_cfg cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> pending;
    std::unordered_map<uint64_t, Outcome> tickets;
    uint64_t next_ticket = 1;
    std::vector<Slot> slots;
    std::thread worker;
    bool stopping = false;
    int fault_batch = -1;  // 1-based index of a batch to fail on purpose (host side), -1 = none
    // statistics
    double t_start = 0.0;
    uint64_t submitted = 0, completed = 0, rejected = 0, failed = 0, batches = 0, pairs = 0;
    uint64_t in_flight = 0, max_in_flight = 0;
    size_t budget_used = 0, budget_hw = 0;
    std::vector<double> lat_ms;
};

namespace lbl {
namespace {

void finish_slot(lbl_server *S, Slot &sl, lbl_status st, const std::string &msg)
{
    const double t = now_s();
    for (const Request &r : sl.reqs) {
        Outcome &o = S->tickets[r.ticket];
        o.finished = true;
        o.st = st;
        o.msg = msg;
        if (st == LBL_OK) {
            S->completed++;
            S->lat_ms.push_back(1000.0 * (t - r.t_submit));
        } else {
            S->failed++;
        }
    }
    if (st == LBL_OK) S->pairs += sl.pairs;
    S->in_flight -= sl.reqs.size();
    S->budget_used -= sl.used;
    sl.reqs.clear();
    sl.busy = false;
    sl.used = 0;
    sl.pairs = 0;
    S->cv_done.notify_all();
}

// Launch the requests in `take` on slot `sl` (lock held).
// Whether a batch of this one request runs the one-frame kernels on slot sl
// (the abstraction has the sparse layout and their workspace fits the arena).
bool runs_alone(const Slot &sl, const Request &r)
{
    return r.job.a->sp != nullptr && swm_frame_workspace_bytes(r.job.a, r.job.n_props) <= sl.arena_bytes;
}

// Launch the requests in take on slot sl: plan is their batch plan, or null
// for a single request that runs alone.
void launch(lbl_server *S, Slot &sl, std::vector<Request> &take, const BatchPlan *plan)
{
    S->batches++;
    sl.reqs.swap(take);
    const JobRef &j0 = sl.reqs.front().job;
    const bool alone = sl.reqs.size() == 1 && runs_alone(sl, sl.reqs.front());
    sl.pairs = plan ? plan->pairs : j0.a->n_traj * j0.n_props;
    sl.busy = true;
    sl.used = plan ? plan->device_bytes() : swm_frame_workspace_bytes(j0.a, j0.n_props);
    S->in_flight += sl.reqs.size();
    S->max_in_flight = std::max<uint64_t>(S->max_in_flight, S->in_flight);
    S->budget_used += sl.used;
    S->budget_hw = std::max(S->budget_hw, S->budget_used);
    if (S->fault_batch > 0 && (int64_t)S->batches == S->fault_batch) {
        finish_slot(S, sl, LBL_EDEVICE, "injected batch failure");
        return;
    }
    // a batch of one frame on an abstraction with the sparse layout runs the
    // one-frame kernels, with the slot's arena as their workspace: no batch
    // tables to upload and one launch fewer (the labels are the same)
    if (alone) {
        lbl_status st = run_swm(j0.a, j0.O, j0.n_props, sl.arena, j0.L, sl.stream, false);
        hipError_t e = st == LBL_OK ? hipEventRecord(sl.done, sl.stream) : hipSuccess;
        if (st != LBL_OK) finish_slot(S, sl, st, "frame launch failed");
        else if (e != hipSuccess) finish_slot(S, sl, LBL_EDEVICE, hipGetErrorString(e));
        return;
    }
    if (plan == nullptr) {
        finish_slot(S, sl, LBL_EINVAL, "batch launched without a plan");
        return;
    }
    BatchBuffers bufs;
    std::vector<uint8_t> img;
    if (bind_batch(*plan, sl.arena, sl.arena_bytes, &bufs, &img) != LBL_OK) {
        finish_slot(S, sl, LBL_ENOMEM, "batch does not fit the slot's arena");
        return;
    }
    std::string err;
    hipError_t e = hipSuccess;
    if (img.size() > sl.pinned_bytes) {
        if (sl.pinned) (void)hipHostFree(sl.pinned);
        sl.pinned = nullptr;
        sl.pinned_bytes = 0;
        e = hipHostMalloc((void **)&sl.pinned, img.size() * 2, hipHostMallocDefault);
        if (e == hipSuccess) sl.pinned_bytes = img.size() * 2;
    }
    if (e == hipSuccess) {
        memcpy(sl.pinned, img.data(), img.size());
        e = hipMemcpyAsync(sl.arena, sl.pinned, img.size(), hipMemcpyHostToDevice, sl.stream);
    }
    lbl_status st = LBL_OK;
    if (e == hipSuccess) {
        st = enqueue_batch(*plan, bufs, sl.stream);
        if (st != LBL_OK) err = "batch launch failed";
    }
    if (e == hipSuccess && st == LBL_OK) e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) {
        st = LBL_EDEVICE;
        err = hipGetErrorString(e);
    }
    if (st != LBL_OK) finish_slot(S, sl, st, err);
}

// Bytes a batch of these requests needs (0 and *ok = false if the jobs are invalid).
size_t batch_bytes(const std::vector<Request> &reqs, BatchPlan *plan, bool *ok)
{
    std::vector<JobRef> jobs;
    jobs.reserve(reqs.size());
    for (const Request &r : reqs) jobs.push_back(r.job);
    *ok = plan_batch(jobs.data(), jobs.size(), -1, plan) == LBL_OK;
    if (!*ok) return 0;
    plan_finalize(*plan, batch_tile_for(plan->shape_key));
    return plan->device_bytes();
}

void worker_main(lbl_server *S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // reap finished batches
        bool any_busy = false;
        for (Slot &sl : S->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) finish_slot(S, sl, LBL_OK, "");
            else if (q != hipErrorNotReady) finish_slot(S, sl, LBL_EDEVICE, hipGetErrorString(q));
            else any_busy = true;
        }
        // launch onto free slots
        for (Slot &sl : S->slots) {
            if (sl.busy || S->pending.empty()) continue;
            if (S->cfg.max_wait_us > 0 && any_busy && S->pending.size() < S->cfg.max_batch_frames &&
                1e6 * (now_s() - S->pending.front().t_submit) < S->cfg.max_wait_us)
                break;  // let the batch fill while the GPU is busy anyway
            std::vector<Request> take;
            // a single pending request that runs alone needs no batch plan
            if (S->pending.size() == 1 && runs_alone(sl, S->pending.front())) {
                take.push_back(S->pending.front());
                S->pending.pop_front();
                launch(S, sl, take, nullptr);
                any_busy = any_busy || sl.busy;
                continue;
            }
            BatchPlan plan;
            while (!S->pending.empty() && take.size() < S->cfg.max_batch_frames) {
                take.push_back(S->pending.front());
                bool ok = false;
                BatchPlan cand;
                const size_t need = batch_bytes(take, &cand, &ok);
                if (!ok || need > sl.arena_bytes) {
                    take.pop_back();
                    break;
                }
                plan = std::move(cand);
                S->pending.pop_front();
            }
            if (take.empty() && runs_alone(sl, S->pending.front())) {
                // the head request fits no batch but runs alone
                take.push_back(S->pending.front());
                S->pending.pop_front();
                launch(S, sl, take, nullptr);
                any_busy = any_busy || sl.busy;
                continue;
            }
            if (take.empty()) {
                // the head request cannot run (checked at submit, so only if it became invalid)
                Request r = S->pending.front();
                S->pending.pop_front();
                Outcome &o = S->tickets[r.ticket];
                o.finished = true;
                o.st = LBL_ENOMEM;
                o.msg = "request does not fit a slot's share of the HBM budget";
                S->failed++;
                S->cv_done.notify_all();
                continue;
            }
            launch(S, sl, take, &plan);
            any_busy = any_busy || sl.busy;
        }
        if (S->stopping && S->pending.empty() && !any_busy) {
            bool busy = false;
            for (Slot &sl : S->slots) busy = busy || sl.busy;
            if (!busy) break;
        }
        if (any_busy) {
            // batches are in flight: poll again after a short pause with
            // the lock released (a timed wait would sleep for the timer
            // slack, tens of microseconds, before noticing a finished batch)
            lk.unlock();
            const double t_pause = now_s() + 2e-6;
            while (now_s() < t_pause) std::this_thread::yield();
            lk.lock();
        }
        else if (S->pending.empty() && !S->stopping)
            S->cv_work.wait_for(lk, std::chrono::milliseconds(50));
    }
}

}  // namespace
}  // namespace lbl

using namespace lbl;

extern "C" {

lbl_status lbl_serve_start(const lbl_serve_cfg *cfg, lbl_server_t *out)
{
    clear_error();
    LBL_REQUIRE(cfg != nullptr && out != nullptr, "null argument");
    *out = nullptr;
    LBL_REQUIRE(cfg->max_batch_frames >= 1 && cfg->max_batch_frames <= 256, "max_batch_frames must be in [1, 256]");
    LBL_REQUIRE(cfg->n_streams >= 1 && cfg->n_streams <= 8, "n_streams must be in [1, 8]");
    LBL_REQUIRE(cfg->max_queue >= 1, "max_queue must be positive");
    LBL_REQUIRE(cfg->hbm_budget_bytes >= ((uint64_t)cfg->n_streams << 20), "hbm_budget_bytes must be >= 1 MiB per stream");
    std::unique_ptr<lbl_server> S(new lbl_server());
    S->cfg = *cfg;
    LBL_HIP_TRY(hipGetDevice(&S->device));
    if (const char *f = getenv("LBL_FAULT_BATCH")) S->fault_batch = atoi(f);
    S->slots.resize(cfg->n_streams);
    const size_t share = (size_t)(cfg->hbm_budget_bytes / cfg->n_streams) & ~size_t(255);
    auto cleanup = [&]() {
        for (Slot &sl : S->slots) {
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.arena) (void)hipFree(sl.arena);
        }
    };
    for (Slot &sl : S->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&sl.arena, share);
        if (e != hipSuccess) {
            cleanup();
            set_error(std::string("lbl_serve_start: ") + hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? LBL_ENOMEM : LBL_EDEVICE;
        }
        sl.arena_bytes = share;
    }
    S->t_start = now_s();
    lbl_server *raw = S.get();
    S->worker = std::thread(worker_main, raw);
    *out = S.release();
    return LBL_OK;
}

lbl_status lbl_serve_submit(lbl_server_t S, lbl_abs_t a, const uint8_t *O, uint32_t n_props, uint8_t *L,
                            uint64_t *ticket)
{
    clear_error();
    LBL_REQUIRE(S != nullptr && ticket != nullptr, "null argument");
    LBL_REQUIRE(a != nullptr, "abstraction is null");
    LBL_REQUIRE(O != nullptr && L != nullptr, "O or L is null");
    LBL_REQUIRE(n_props >= 1 && n_props <= 64, "n_props must be in [1, 64]");
    LBL_REQUIRE(a->device == S->device, "abstraction lives on another device than the server");
    Request r{0, JobRef{a, O, n_props, L}, now_s()};
    {
        // admission by memory: a request whose one-frame kernels fit a
        // slot's arena can always run (alone, if no batch takes it); any
        // other is admitted by the size of its batch plan
        const bool alone = runs_alone(S->slots[0], r);
        bool ok = true;
        size_t need = 0;
        if (!alone) {
            std::vector<Request> one{r};
            BatchPlan plan;
            need = batch_bytes(one, &plan, &ok);
        }
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stopping) {
            set_error("server is stopping");
            return LBL_ECLOSED;
        }
        if (!alone && (!ok || need > S->slots[0].arena_bytes)) {
            S->rejected++;
            set_error("request needs " + std::to_string(need) + " bytes, more than a slot's share of the HBM budget");
            return LBL_ENOMEM;
        }
        if (S->pending.size() >= S->cfg.max_queue) {
            S->rejected++;
            set_error("request queue is full");
            return LBL_EBUSY;
        }
        r.ticket = S->next_ticket++;
        S->tickets[r.ticket] = Outcome{};
        S->pending.push_back(r);
        S->submitted++;
    }
    S->cv_work.notify_one();
    *ticket = r.ticket;
    return LBL_OK;
}

lbl_status lbl_serve_wait(lbl_server_t S, uint64_t ticket, int64_t timeout_us)
{
    clear_error();
    LBL_REQUIRE(S != nullptr, "server is null");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    LBL_REQUIRE(it != S->tickets.end(), "unknown ticket (never issued or already waited for)");
    auto done = [&]() { return S->tickets[ticket].finished; };
    if (timeout_us < 0) {
        S->cv_done.wait(lk, done);
    } else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
        set_error("timed out");
        return LBL_ETIMEDOUT;
    }
    Outcome o = S->tickets[ticket];
    S->tickets.erase(ticket);
    if (o.st != LBL_OK) set_error(o.msg);
    return o.st;
}

lbl_status lbl_serve_stats_get(lbl_server_t S, lbl_serve_stats *out)
{
    clear_error();
    LBL_REQUIRE(S != nullptr && out != nullptr, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = lbl_serve_stats{};
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->rejected = S->rejected;
    out->failed = S->failed;
    out->batches = S->batches;
    out->pairs = S->pairs;
    out->wall_s = now_s() - S->t_start;
    out->pairs_per_s = out->wall_s > 0 ? S->pairs / out->wall_s : 0.0;
    out->max_in_flight = S->max_in_flight;
    out->budget_high_water = S->budget_hw;
    if (!S->lat_ms.empty()) {
        std::vector<double> v = S->lat_ms;
        auto pct = [&](double q) {
            const size_t k = std::min(v.size() - 1, (size_t)std::ceil(q * v.size()) - (q > 0 ? 1 : 0));
            std::nth_element(v.begin(), v.begin() + k, v.end());
            return v[k];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        double s = 0.0, mx = 0.0;
        for (double x : S->lat_ms) {
            s += x;
            mx = std::max(mx, x);
        }
        out->mean_ms = s / S->lat_ms.size();
        out->max_ms = mx;
    }
    return LBL_OK;
}

lbl_status lbl_serve_stop(lbl_server_t S)
{
    clear_error();
    if (!S) return LBL_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (Slot &sl : S->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.arena) (void)hipFree(sl.arena);
        if (sl.pinned) (void)hipHostFree(sl.pinned);
    }
    delete S;
    return LBL_OK;
}

}  // extern "C"
