// Serving: continuous batching of filter requests.
//
// A scheduler thread owns the device side.  Requests queue in arrival order;
// whenever an in-flight slot is free it admits the longest prefix of the
// queue that fits the HBM budget (the image bytes of everything in flight)
// and the slot's workspace (its share of the caller's arena, which holds the
// work list and the intermediates of two-pass images), and filters that
// group with one batched launch sequence on the slot's stream.  Planning and
// launching run outside the server lock, so submit and poll never wait
// behind a launch.  Launches on different streams overlap on the
// device, so requests that arrive while earlier ones run start as soon as a
// slot frees instead of waiting for the whole device to drain.  Completion is
// detected with one event per launch.  A request filters to the same bits
// whatever it is batched with (float tile shapes depend on each image alone;
// uint8 results are exact whatever the segment height).
#include "rsg_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace rsg {

namespace {

uint64_t now_ns()
{
    return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(
                        std::chrono::steady_clock::now().time_since_epoch())
                        .count());
}

struct Request {
    uint64_t ticket;
    rsg_image_desc desc;           // desc.boxes is NULL here; see boxes below
    bool own_boxes = false;        // the caller passed boxes: a copy is kept
    rsg_boxes boxes;
    ImgParams plan;
    size_t footprint;
    rsg_req_stats st;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void* d_ws = nullptr;             // carved from the arena: work list and two-pass intermediates
    size_t ws_bytes = 0;
    void* h_stage = nullptr;          // pinned staging for the work list header, grown on demand
    size_t stage_bytes = 0;
    bool busy = false;                // launched (or being launched) and not yet seen complete
    std::vector<uint64_t> tickets;
    size_t footprint = 0;
};

constexpr size_t kStageInit = 256 << 10;   // initial pinned staging per slot

}  // namespace
}  // namespace rsg

struct rsg_server {
    rsg_server_config cfg;
    int device = 0;
    std::vector<hipStream_t> streams;
    std::vector<rsg::Slot> slots;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<rsg::Request> pending;
    std::unordered_map<uint64_t, rsg_req_stats> state;   // queued, running or finished
    std::unordered_map<uint64_t, rsg::Request> running;
    size_t inflight_bytes = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread thread;
};

namespace rsg {
namespace {

// Plan and launch one admitted group on its slot, without the server lock
// (only the scheduler thread touches a busy slot).  Returns the status and
// the launch time.
int launch_group(Slot& slot, std::vector<Request>& group, uint64_t* t_launch)
{
    std::vector<rsg_image_desc> descs;
    for (auto& r : group) {
        descs.push_back(r.desc);
        descs.back().boxes = r.own_boxes ? &r.boxes : nullptr;
    }
    std::vector<ImgParams> imgs;
    std::vector<BatchTask> tasks;
    int rc = plan_batch(descs.data(), int(descs.size()), imgs, tasks);
    if (rc == RSG_OK) {
        // the slot's previous launch has completed, so its staging is free
        const size_t hdr = batch_header_bytes(int(imgs.size()), int64_t(tasks.size()) + pass_blocks(imgs.data(), int(imgs.size())));
        if (hdr > slot.stage_bytes) {
            if (slot.h_stage) (void)hipHostFree(slot.h_stage);
            slot.h_stage = nullptr;
            slot.stage_bytes = 0;
            if (hipHostMalloc(&slot.h_stage, hdr, hipHostMallocDefault) != hipSuccess)
                rc = set_error(RSG_ENOMEM, "cannot pin %zu bytes of staging", hdr);
            else
                slot.stage_bytes = hdr;
        }
    }
    if (rc == RSG_OK)
        rc = launch_batch(imgs.data(), int(imgs.size()), tasks.data(), int(tasks.size()), slot.d_ws, slot.ws_bytes,
                          slot.stream, slot.h_stage);
    // the event is recorded even after a partial launch, so the slot is
    // reused only once whatever was enqueued has finished
    if (hipEventRecord(slot.done, slot.stream) != hipSuccess && rc == RSG_OK) rc = RSG_EDEVICE;
    *t_launch = now_ns();
    return rc;
}

void scheduler(rsg_server* s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // completions
        for (auto& slot : s->slots) {
            if (!slot.busy) continue;
            const hipError_t q = hipEventQuery(slot.done);
            if (q == hipErrorNotReady) continue;
            const uint64_t t = now_ns();
            for (uint64_t tk : slot.tickets) {
                auto it = s->running.find(tk);
                if (it == s->running.end()) continue;
                rsg_req_stats st = it->second.st;
                st.done = 1;
                st.status = (q == hipSuccess) ? RSG_OK : RSG_EDEVICE;
                st.t_done_ns = t;
                s->state[tk] = st;
                s->running.erase(it);
            }
            s->inflight_bytes -= slot.footprint;
            slot.footprint = 0;
            slot.tickets.clear();
            slot.busy = false;
        }
        // admission: arrival order, HBM budget, the slot's workspace, one
        // group per free slot
        std::vector<std::pair<Slot*, std::vector<Request>>> work;
        for (auto& slot : s->slots) {
            if (s->pending.empty()) break;
            if (slot.busy) continue;
            std::vector<Request> group;
            size_t bytes = 0, mid = 0;
            int64_t ntasks = 0;
            while (!s->pending.empty() && int(group.size()) < s->cfg.max_batch) {
                Request& r = s->pending.front();
                const size_t fp = r.footprint;
                if (s->cfg.hbm_budget && s->inflight_bytes + bytes + fp > s->cfg.hbm_budget) break;
                const size_t mid_r = batch_mid_bytes(&r.plan, 1);
                if (batch_header_bytes(int(group.size()) + 1, ntasks + r.plan.ntasks) + mid + mid_r > slot.ws_bytes)
                    break;
                bytes += fp;
                mid += mid_r;
                ntasks += r.plan.ntasks;
                r.st.t_admit_ns = now_ns();
                group.push_back(r);
                s->pending.pop_front();
            }
            if (group.empty()) break;
            s->inflight_bytes += bytes;
            slot.busy = true;
            slot.footprint = bytes;
            for (auto& r : group) s->state[r.ticket] = r.st;
            work.emplace_back(&slot, std::move(group));
        }
        // plan and launch outside the lock: submit and poll never wait
        // behind a launch
        if (!work.empty()) {
            std::vector<std::pair<int, uint64_t>> res(work.size());
            lk.unlock();
            for (size_t i = 0; i < work.size(); ++i) res[i].first = launch_group(*work[i].first, work[i].second, &res[i].second);
            lk.lock();
            for (size_t i = 0; i < work.size(); ++i) {
                Slot& slot = *work[i].first;
                const int rc = res[i].first;
                slot.tickets.clear();
                for (auto& r : work[i].second) {
                    r.st.t_start_ns = res[i].second;
                    if (rc != RSG_OK) {               // failed: done now; the slot waits for its event
                        r.st.done = 1;
                        r.st.status = rc;
                        r.st.t_done_ns = res[i].second;
                        s->state[r.ticket] = r.st;
                        continue;
                    }
                    slot.tickets.push_back(r.ticket);
                    s->state[r.ticket] = r.st;
                    s->running.emplace(r.ticket, r);
                }
            }
        }
        bool any_busy = false;
        for (auto& slot : s->slots) any_busy |= slot.busy;
        if (s->stop && s->pending.empty() && !any_busy) break;
        if (any_busy) {
            // poll completions at a short interval while work is in flight
            s->cv.wait_for(lk, std::chrono::microseconds(20));
        } else {
            s->cv.wait(lk, [&] { return s->stop || !s->pending.empty(); });
        }
    }
}

}  // namespace
}  // namespace rsg

extern "C" {

int rsg_server_create(const rsg_server_config* cfg, rsg_server** out)
{
    using namespace rsg;
    if (!cfg || !out) return set_error(RSG_EINVAL, "rsg_server_create: NULL argument");
    if (cfg->max_inflight < 1 || cfg->max_inflight > 64) return set_error(RSG_EINVAL, "max_inflight must be in 1..64");
    if (cfg->n_streams < 1 || cfg->n_streams > 8) return set_error(RSG_EINVAL, "n_streams must be in 1..8");
    if (cfg->queue_depth < 1) return set_error(RSG_EINVAL, "queue_depth must be >= 1");
    if (cfg->max_batch < 1) return set_error(RSG_EINVAL, "max_batch must be >= 1");
    const size_t per_slot = cfg->d_arena ? (cfg->arena_bytes / size_t(cfg->max_inflight)) & ~size_t(255) : 0;
    if (!cfg->d_arena || per_slot < 4096)
        return set_error(RSG_EINVAL, "arena must hold at least 4 KiB per in-flight slot");
    rsg_server* s = new (std::nothrow) rsg_server();
    if (!s) return set_error(RSG_ENOMEM, "out of host memory");
    s->cfg = *cfg;
    if (hipGetDevice(&s->device) != hipSuccess) { delete s; return set_error(RSG_EDEVICE, "hipGetDevice failed"); }
    for (int i = 0; i < cfg->n_streams; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return set_error(RSG_EDEVICE, "stream creation failed");
        }
        s->streams.push_back(st);
    }
    s->slots.resize(cfg->max_inflight);
    for (int i = 0; i < cfg->max_inflight; ++i) {
        Slot& sl = s->slots[i];
        sl.stream = s->streams[i % cfg->n_streams];
        sl.d_ws = static_cast<char*>(cfg->d_arena) + per_slot * size_t(i);
        sl.ws_bytes = per_slot;
        sl.stage_bytes = std::min(per_slot, kStageInit);
        if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(&sl.h_stage, sl.stage_bytes, hipHostMallocDefault) != hipSuccess) {
            for (auto& x : s->slots) {
                if (x.done) (void)hipEventDestroy(x.done);
                if (x.h_stage) (void)hipHostFree(x.h_stage);
            }
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return set_error(RSG_EDEVICE, "event or staging allocation failed");
        }
    }
    // warm the sigma0 fits so the first submits do not stall on the search
    for (int K = 1; K <= RSG_MAX_K; ++K) {
        int p[RSG_MAX_K];
        double c[RSG_MAX_K], e;
        sigma0_fit(K, true, p, c, &e);
    }
    s->thread = std::thread(scheduler, s);
    *out = s;
    return RSG_OK;
}

int rsg_submit(rsg_server* s, const rsg_image_desc* req, uint64_t* ticket)
{
    using namespace rsg;
    if (!s || !req || !ticket) return set_error(RSG_EINVAL, "rsg_submit: NULL argument");
    Request r;
    std::memset(&r.st, 0, sizeof(r.st));
    r.desc = *req;
    if (req->boxes) {                     // the caller's boxes need only live during this call
        r.own_boxes = true;
        r.boxes = *req->boxes;
    }
    r.desc.boxes = nullptr;
    int rc = plan_image(*req, &r.plan);
    if (rc != RSG_OK) return rc;
    const int es = dtype_size(req->dt);
    // device bytes in flight: the caller's images (a two-pass intermediate
    // lives in the arena slot, bounded by its size)
    r.footprint = size_t(int64_t(req->H) * r.plan.src_stride * es) + size_t(int64_t(req->H) * r.plan.dst_stride * es);
    const size_t per_slot = s->slots.empty() ? 0 : s->slots[0].ws_bytes;
    if (s->cfg.hbm_budget && r.footprint > s->cfg.hbm_budget)
        return set_error(RSG_ENOMEM, "request needs %zu bytes, budget is %zu", r.footprint, s->cfg.hbm_budget);
    if (batch_workspace_bytes(&r.plan, 1, r.plan.ntasks) > per_slot)
        return set_error(RSG_ENOMEM, "request workspace (work list and intermediate) exceeds the arena slot (%zu bytes)",
                         per_slot);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return set_error(RSG_EINVAL, "server is shutting down");
    if (int(s->pending.size()) >= s->cfg.queue_depth) return set_error(RSG_EBUSY, "queue full");
    r.ticket = s->next_ticket++;
    r.st.t_submit_ns = now_ns();
    s->state[r.ticket] = r.st;
    s->pending.push_back(r);
    *ticket = r.ticket;
    s->cv.notify_all();
    return RSG_OK;
}

int rsg_poll(rsg_server* s, uint64_t ticket, rsg_req_stats* out)
{
    using namespace rsg;
    if (!s || !out) return set_error(RSG_EINVAL, "rsg_poll: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->state.find(ticket);
    if (it == s->state.end()) return set_error(RSG_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    *out = it->second;
    if (out->done) s->state.erase(it);
    return RSG_OK;
}

int rsg_server_destroy(rsg_server* s)
{
    using namespace rsg;
    if (!s) return set_error(RSG_EINVAL, "rsg_server_destroy: NULL server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->thread.joinable()) s->thread.join();
    int rc = RSG_OK;
    for (auto& sl : s->slots) {
        if (sl.done && hipEventDestroy(sl.done) != hipSuccess) rc = RSG_EDEVICE;
        if (sl.h_stage && hipHostFree(sl.h_stage) != hipSuccess) rc = RSG_EDEVICE;
    }
    for (auto st : s->streams)
        if (hipStreamDestroy(st) != hipSuccess) rc = RSG_EDEVICE;
    delete s;
    return rc == RSG_OK ? RSG_OK : set_error(rc, "teardown reported a HIP error");
}

}  // extern "C"
