// server.cpp -- request loop on top of the batched scan: submit / poll
// tickets, admission against an HBM byte budget, continuous batching of
// pending requests into one persistent launch per (dtype, operator, flags),
// and several streams so that batches overlap on the device.
//
// Co-residency: batches launch 256-thread workgroups (one wave per SIMD per
// workgroup) of the batched kernels, 4 vectors per lane (2 for the
// compensated pair, whose state is twice as wide), and the workgroups per CU
// of all streams sum to at most 3, so at most three of those waves share a
// SIMD.  Batches of one request use the plain kernel of the same shape (no
// descriptor upload).  At creation the server reads every such kernel's
// VGPR count from the code object and refuses to start unless three waves
// of the largest fit in one SIMD's 512 registers (on gfx950 they need at
// most 130 each), so the grids of all streams are always resident together.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lscan.h"
#include "runtime_internal.hpp"
#include "serve_policy.hpp"

namespace {

uint64_t now_ns()
{
    return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(
                        std::chrono::steady_clock::now().time_since_epoch())
                        .count());
}

constexpr int kServerThreads = 256;
constexpr int kMaxWorkgroupsPerCu = 3;  // summed over streams
constexpr int kSimdVgprs = 512;
constexpr int kVgprGranule = 8;

int server_vectors(uint32_t flags) { return (flags & LSCAN_F_COMPENSATED) ? 2 : 4; }

struct RequestState {
    lscan_request req;
    lscan_result res;
    uint64_t bytes = 0;
};

struct StreamSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int groups = 1;                  // workgroups per CU of this stream's launches
    uint32_t* status = nullptr;      // host word the kernel raises on a timeout
    uint32_t* status_dev = nullptr;  // its device-visible address
    bool busy = false;      // a batch was formed for this slot
    bool launched = false;  // ... and its launch and completion event are enqueued
    lscan::serve::Batch batch;
    std::thread completer;
};

uint64_t batch_key(const lscan_request& r)
{
    // every launch is deterministic, so that flag does not split batches
    const uint32_t f = r.flags & ~LSCAN_F_DETERMINISTIC;
    return uint64_t(uint32_t(r.dt)) | (uint64_t(uint32_t(r.op)) << 8) | (uint64_t(f) << 16);
}

}  // namespace

struct lscan_server {
    lscan_server_config cfg;
    std::mutex mu;
    std::condition_variable done_cv;   // waiters: a request finished
    std::condition_variable slot_cv;   // completers: a batch was launched on their slot
    std::unique_ptr<lscan::serve::Policy> policy;
    std::unordered_map<uint64_t, RequestState> reqs;
    uint64_t next_ticket = 1;
    std::vector<std::unique_ptr<StreamSlot>> slots;
    bool stopping = false;
    bool exclusive = false;  // a solo request owns the device
    lscan_server_stats stats;
};

namespace {

void fail_batch_locked(lscan_server* s, const lscan::serve::Batch& b, lscan_status st, uint64_t t)
{
    for (uint64_t t_id : b.tickets) {
        auto it = s->reqs.find(t_id);
        if (it == s->reqs.end()) continue;
        it->second.res.status = st;
        it->second.res.t_done_ns = t;
        s->stats.failed++;
    }
    s->policy->release(b.bytes);
}

// Launch batches while a stream slot is free and the policy has work.  Runs
// in whichever thread made progress possible (a submit or a completion), so
// no thread hand-off sits between an arrival and its launch.  Called with
// the lock held; drops it around each launch.
void schedule_locked(lscan_server* s, std::unique_lock<std::mutex>& lock)
{
    std::vector<lscan_array> table;
    while (s->policy->pending() > 0 && !s->exclusive) {
        StreamSlot* slot = nullptr;  // the free slot with the largest grid
        bool any_busy = false;
        for (auto& sl : s->slots) {
            any_busy |= sl->busy;
            if (!sl->busy && (!slot || sl->groups > slot->groups)) slot = sl.get();
        }
        if (!slot) return;
        if (s->policy->head_is_solo() && any_busy) return;  // a large request waits for an idle device
        lscan::serve::Batch b = s->policy->next_batch();
        if (b.tickets.empty()) return;
        const uint64_t t = now_ns();
        table.clear();
        const lscan_request& head = s->reqs[b.tickets.front()].req;
        const lscan_dtype dt = head.dt;
        const lscan_op op = head.op;
        const uint32_t flags = head.flags;
        for (uint64_t id : b.tickets) {
            RequestState& rs = s->reqs[id];
            rs.res.t_admit_ns = t;
            rs.res.batch_id = s->stats.batches;
            rs.res.batch_size = int32_t(b.tickets.size());
            table.push_back(lscan_array{rs.req.x, rs.req.y, rs.req.n});
        }
        slot->busy = true;
        slot->batch = b;
        *slot->status = 0;  // the slot's previous batch has completed
        s->stats.batches++;
        if (b.solo) s->exclusive = true;
        lscan_params prm;
        prm.block_threads = kServerThreads;
        prm.vectors_per_lane = server_vectors(flags);
        prm.groups_per_cu = slot->groups;
        prm.handoff = LSCAN_HANDOFF_WINDOW;
        lock.unlock();
        // solo: the full-device default kernel; one request: the plain kernel
        // on this stream's grid share (no descriptor upload); else batched
        lscan_status st;
        if (b.solo)
            st = lscan::launch_single(table[0].x, table[0].y, table[0].n, dt, op, flags, nullptr, slot->stream,
                                      slot->status_dev);
        else if (table.size() == 1)
            st = lscan::launch_single(table[0].x, table[0].y, table[0].n, dt, op, flags, &prm, slot->stream,
                                      slot->status_dev);
        else
            st = lscan::launch_batched(table.data(), int64_t(table.size()), dt, op, flags, &prm, slot->stream,
                                       slot->status_dev);
        if (st == LSCAN_OK && hipEventRecord(slot->done, slot->stream) != hipSuccess) st = LSCAN_ERR_DEVICE;
        const uint64_t t_launch = now_ns();
        lock.lock();
        for (uint64_t id : b.tickets) s->reqs[id].res.t_launch_ns = t_launch;
        if (st != LSCAN_OK) {
            fail_batch_locked(s, b, st, t_launch);
            slot->busy = false;
            slot->batch = lscan::serve::Batch();
            if (b.solo) s->exclusive = false;
            s->done_cv.notify_all();
        } else {
            slot->launched = true;
            s->slot_cv.notify_all();
        }
    }
}

void completer_loop(lscan_server* s, StreamSlot* sl)
{
    (void)hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lock(s->mu);
    while (true) {
        while (!sl->launched && !(s->stopping && !sl->busy)) s->slot_cv.wait(lock);
        if (!sl->launched) break;  // stopping and idle
        hipEvent_t ev = sl->done;
        lock.unlock();
        const hipError_t e = hipEventSynchronize(ev);
        const uint32_t timed_out = __atomic_load_n(sl->status, __ATOMIC_ACQUIRE);
        const lscan_status st = (e != hipSuccess) ? LSCAN_ERR_DEVICE : (timed_out ? LSCAN_ERR_TIMEOUT : LSCAN_OK);
        const uint64_t t = now_ns();
        lock.lock();
        for (uint64_t id : sl->batch.tickets) {
            auto it = s->reqs.find(id);
            if (it == s->reqs.end()) continue;
            it->second.res.status = st;
            it->second.res.t_done_ns = t;
            if (st == LSCAN_OK)
                s->stats.completed++;
            else
                s->stats.failed++;
        }
        s->policy->release(sl->batch.bytes);
        if (sl->batch.solo) s->exclusive = false;
        sl->batch = lscan::serve::Batch();
        sl->launched = false;
        sl->busy = false;
        s->done_cv.notify_all();
        schedule_locked(s, lock);  // the freed slot and bytes may admit waiting requests
    }
}

// One eager launch of every (dtype, operator, flags) on every server stream:
// runs the co-residency test and sizes the workspaces before requests
// arrive.
lscan_status warm_up(lscan_server* s)
{
    void* buf = nullptr;
    const size_t n = 4096;
    if (hipMalloc(&buf, n * 16) != hipSuccess) return LSCAN_ERR_NO_MEMORY;
    (void)hipMemset(buf, 0, n * 16);
    lscan_status st = LSCAN_OK;
    for (auto& sl : s->slots) {
        lscan_params prm;
        prm.block_threads = kServerThreads;
        prm.groups_per_cu = sl->groups;
        prm.handoff = LSCAN_HANDOFF_WINDOW;
        for (int dt = LSCAN_I32; dt <= LSCAN_BF16 && st == LSCAN_OK; ++dt)
            for (int op = LSCAN_ADD; op <= LSCAN_MIN && st == LSCAN_OK; ++op)
                for (uint32_t comp = 0; comp <= 1 && st == LSCAN_OK; ++comp) {
                    if (comp && !(op == LSCAN_ADD && (dt == LSCAN_F32 || dt == LSCAN_BF16))) continue;
                    prm.vectors_per_lane = server_vectors(comp ? LSCAN_F_COMPENSATED : 0u);
                    char* base = static_cast<char*>(buf);
                    lscan_array a[2] = {{base, base + n * 8, int64_t(n) / 2}, {base + n * 4, base + n * 12, 64}};
                    st = lscan_batched_with_params(a, 2, lscan_dtype(dt), lscan_op(op),
                                                   comp ? LSCAN_F_COMPENSATED : 0u, &prm, sl->stream);
                    if (st == LSCAN_OK)
                        st = lscan_scan_with_params(base, base + n * 8, int64_t(n), lscan_dtype(dt), lscan_op(op),
                                                    comp ? LSCAN_F_COMPENSATED : 0u, 0, &prm, sl->stream);
                }
        if (st == LSCAN_OK) st = lscan_check(sl->stream);
    }
    // the plain full-device kernels that solo requests use
    hipStream_t s0 = s->slots.front()->stream;
    for (int dt = LSCAN_I32; dt <= LSCAN_BF16 && st == LSCAN_OK; ++dt)
        for (int op = LSCAN_ADD; op <= LSCAN_MIN && st == LSCAN_OK; ++op)
            for (uint32_t comp = 0; comp <= 1 && st == LSCAN_OK; ++comp) {
                if (comp && !(op == LSCAN_ADD && (dt == LSCAN_F32 || dt == LSCAN_BF16))) continue;
                char* base = static_cast<char*>(buf);
                st = lscan_inclusive(base, base + n * 8, int64_t(n), lscan_dtype(dt), lscan_op(op),
                                     comp ? LSCAN_F_COMPENSATED : 0u, s0);
            }
    if (st == LSCAN_OK) st = lscan_check(s0);
    (void)hipDeviceSynchronize();
    (void)hipFree(buf);
    return st;
}

void destroy_slots(lscan_server* s)
{
    for (auto& o : s->slots) {
        if (o->stream) (void)hipStreamSynchronize(o->stream);
        if (o->done) (void)hipEventDestroy(o->done);
        if (o->stream) (void)hipStreamDestroy(o->stream);
        if (o->status) (void)hipHostFree(o->status);
    }
    s->slots.clear();
}

}  // namespace

extern "C" {

lscan_status lscan_server_default_config(lscan_server_config* cfg)
{
    if (!cfg) return LSCAN_ERR_INVALID_ARG;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->device = 0;
    cfg->num_streams = 2;
    cfg->groups_per_cu = 0;  // split the device: 2 + 1 workgroups per CU
    cfg->hbm_budget_bytes = uint64_t(32) << 30;
    cfg->max_queue = 1 << 16;
    cfg->max_batch = 4096;
    cfg->solo_bytes = uint64_t(64) << 20;
    return LSCAN_OK;
}

lscan_status lscan_server_create(const lscan_server_config* cfg, lscan_server** out)
{
    if (!cfg || !out) return LSCAN_ERR_INVALID_ARG;
    *out = nullptr;
    if (cfg->num_streams < 1 || cfg->num_streams > kMaxWorkgroupsPerCu || cfg->groups_per_cu < 0 ||
        cfg->num_streams * cfg->groups_per_cu > kMaxWorkgroupsPerCu || cfg->hbm_budget_bytes == 0 ||
        cfg->max_queue < 1 || cfg->max_batch < 1)
        return LSCAN_ERR_INVALID_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || cfg->device < 0 || cfg->device >= count)
        return LSCAN_ERR_INVALID_ARG;
    if (hipSetDevice(cfg->device) != hipSuccess) return LSCAN_ERR_DEVICE;
    lscan_server* s = new (std::nothrow) lscan_server();
    if (!s) return LSCAN_ERR_NO_MEMORY;
    s->cfg = *cfg;
    std::memset(&s->stats, 0, sizeof(s->stats));
    const uint64_t solo = cfg->solo_bytes ? cfg->solo_bytes : (uint64_t(64) << 20);
    s->policy.reset(
        new lscan::serve::Policy(cfg->hbm_budget_bytes, size_t(cfg->max_queue), size_t(cfg->max_batch), solo));
    for (int i = 0; i < cfg->num_streams; ++i) {
        std::unique_ptr<StreamSlot> sl(new StreamSlot());
        // groups_per_cu == 0: share kMaxWorkgroupsPerCu among the streams,
        // the larger shares first
        sl->groups = cfg->groups_per_cu > 0
                         ? cfg->groups_per_cu
                         : kMaxWorkgroupsPerCu / cfg->num_streams + (i < kMaxWorkgroupsPerCu % cfg->num_streams);
        bool ok = hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&sl->done, hipEventDisableTiming) == hipSuccess &&
                  hipHostMalloc(reinterpret_cast<void**>(&sl->status), sizeof(uint32_t),
                                hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
                  hipHostGetDevicePointer(reinterpret_cast<void**>(&sl->status_dev), sl->status, 0) == hipSuccess;
        s->slots.push_back(std::move(sl));
        if (!ok) {
            destroy_slots(s);
            delete s;
            return LSCAN_ERR_DEVICE;
        }
        *s->slots.back()->status = 0;
    }
    // every kernel the server may run must fit three waves to a SIMD
    int max_vgprs = 0;
    for (int dt = LSCAN_I32; dt <= LSCAN_BF16; ++dt)
        for (int op = LSCAN_ADD; op <= LSCAN_MIN; ++op)
            for (uint32_t comp = 0; comp <= 1; ++comp) {
                if (comp && !(op == LSCAN_ADD && (dt == LSCAN_F32 || dt == LSCAN_BF16))) continue;
                const uint32_t f = comp ? LSCAN_F_COMPENSATED : 0u;
                for (int batched = 0; batched <= 1; ++batched) {
                    const int v = lscan::kernel_vgprs(batched != 0, dt, op, f, kServerThreads, server_vectors(f));
                    max_vgprs = (v < 0) ? kSimdVgprs : std::max(max_vgprs, v);
                }
            }
    const int alloc = (max_vgprs + kVgprGranule - 1) / kVgprGranule * kVgprGranule;
    if (kMaxWorkgroupsPerCu * alloc > kSimdVgprs) {
        destroy_slots(s);
        delete s;
        return LSCAN_ERR_UNSUPPORTED;
    }
    lscan_status st = warm_up(s);
    if (st != LSCAN_OK) {
        destroy_slots(s);
        delete s;
        return st;
    }
    for (auto& sl : s->slots) sl->completer = std::thread(completer_loop, s, sl.get());
    *out = s;
    return LSCAN_OK;
}

lscan_status lscan_submit(lscan_server* s, const lscan_request* r, uint64_t* ticket)
{
    if (!s || !r || !ticket) return LSCAN_ERR_INVALID_ARG;
    lscan_status st = lscan::validate_request(r->x, r->y, r->n, r->dt, r->op, r->flags);
    if (st != LSCAN_OK) return st;
    const uint64_t t = now_ns();
    std::unique_lock<std::mutex> lock(s->mu);
    if (s->stopping) return LSCAN_ERR_INVALID_ARG;
    RequestState rs;
    rs.req = *r;
    std::memset(&rs.res, 0, sizeof(rs.res));
    rs.res.status = LSCAN_PENDING;
    rs.res.t_submit_ns = t;
    rs.bytes = lscan::request_bytes(r->n, r->dt);
    const uint64_t id = s->next_ticket;
    if (r->n == 0) {  // nothing to scan: done at once
        rs.res.status = LSCAN_OK;
        rs.res.t_admit_ns = rs.res.t_launch_ns = rs.res.t_done_ns = t;
        s->reqs.emplace(id, rs);
        s->next_ticket++;
        s->stats.submitted++;
        s->stats.completed++;
        *ticket = id;
        return LSCAN_OK;
    }
    const lscan::serve::Admit a = s->policy->submit(lscan::serve::PendingRequest{id, batch_key(*r), rs.bytes, t});
    if (a == lscan::serve::Admit::kTooLarge) return LSCAN_ERR_NO_MEMORY;
    if (a == lscan::serve::Admit::kQueueFull) return LSCAN_ERR_AGAIN;
    s->reqs.emplace(id, rs);
    s->next_ticket++;
    s->stats.submitted++;
    *ticket = id;
    schedule_locked(s, lock);
    return LSCAN_OK;
}

lscan_status lscan_poll(lscan_server* s, uint64_t ticket, lscan_result* out)
{
    if (!s || !out) return LSCAN_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return LSCAN_ERR_NOT_FOUND;
    *out = it->second.res;
    if (out->status == LSCAN_PENDING) return LSCAN_PENDING;
    const lscan_status st = out->status;
    s->reqs.erase(it);
    return st;
}

lscan_status lscan_wait(lscan_server* s, uint64_t ticket, lscan_result* out)
{
    if (!s || !out) return LSCAN_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lock(s->mu);
    while (true) {
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return LSCAN_ERR_NOT_FOUND;
        if (it->second.res.status != LSCAN_PENDING) {
            *out = it->second.res;
            const lscan_status st = out->status;
            s->reqs.erase(it);
            return st;
        }
        s->done_cv.wait(lock);
    }
}

lscan_status lscan_server_get_stats(lscan_server* s, lscan_server_stats* out)
{
    if (!s || !out) return LSCAN_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    *out = s->stats;
    out->pending = int64_t(s->policy->pending());
    out->bytes_in_flight = s->policy->in_flight_bytes();
    out->peak_bytes_in_flight = s->policy->peak_bytes();
    return LSCAN_OK;
}

lscan_status lscan_server_destroy(lscan_server* s)
{
    if (!s) return LSCAN_ERR_INVALID_ARG;
    {
        std::unique_lock<std::mutex> lock(s->mu);
        s->stopping = true;  // refuse new submits; finish what was submitted
        auto busy = [&] {
            if (s->policy->pending() > 0) return true;
            for (auto& sl : s->slots)
                if (sl->busy) return true;
            return false;
        };
        while (busy()) s->done_cv.wait(lock);
        s->slot_cv.notify_all();
    }
    for (auto& sl : s->slots)
        if (sl->completer.joinable()) sl->completer.join();
    destroy_slots(s);
    delete s;
    return LSCAN_OK;
}

}  // extern "C"
