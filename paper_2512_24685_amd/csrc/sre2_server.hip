// sre2_server.hip - continuous-batching serving loop of libsre2 (C ABI in
// include/sre2.h, sre2_server_*).
//
// Requests (one state each, mixed N) arrive from any host thread and wait in
// one of two FIFO lanes: small (N <= 14 in FP32 forms / 13 in FP64 forms,
// whole transforms in one workgroup) and large (two-pass).  A worker thread
// owned by the server:
//   * admits requests of each lane in FIFO order while a request slot is free
//     and the state fits the device arena (the HBM budget): the arena and the
//     slots are the admission control, a full arena is backpressure; the
//     large lane also keeps at most kLargeInFlight evaluations enqueued on the
//     device at a time, so a backlog of large requests waits in its host
//     lane (where the worker is never blocked by a deep device queue) and
//     small requests never wait behind it;
//   * copies every newly admitted state into its arena block and enqueues its
//     evaluation at once, without waiting for earlier work to finish: states
//     with N <= 14 (FP32 forms) / 13 (FP64 forms) that were admitted together
//     are packed by N into shared launches on the "small" stream; larger N go
//     one by one to the "large" stream, so small requests run beside a large
//     two-pass evaluation instead of queueing behind it;
//   * copies each result (M2, S, n, status) into pinned host memory behind the
//     kernels, records an event, and on its completion stamps the request done,
//     frees its slot and arena block.
// Per-request results do not depend on co-scheduling: a packed state runs the
// same kernels, grids and reduction ranges as a single sre2_m2 call, so its
// result is bitwise identical to the single call.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/sre2.h"
#include "sre2_ctx.h"
#include "sre2_internal.h"

using namespace sre2;

namespace {

double now_s() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

// First-fit allocator over one device (or pinned host) allocation,
// 256-byte granules, with coalescing of neighbouring free blocks.
class Arena {
   public:
    int init(size_t bytes, bool pinned_host = false) {
        host_ = pinned_host;
        cap_ = bytes & ~size_t(255);
        const hipError_t e = host_ ? hipHostMalloc((void**)&base_, cap_, hipHostMallocDefault)
                                   : hipMalloc((void**)&base_, cap_);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            base_ = nullptr;
            cap_ = 0;
            return SRE2_ENOMEM;
        }
        free_[0] = cap_;
        return SRE2_OK;
    }
    void release() {
        if (base_) (void)(host_ ? hipHostFree(base_) : hipFree(base_));
        base_ = nullptr;
    }
    void* alloc(size_t bytes) {
        const size_t need = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > need) free_[off + need] = len - need;
            used_[off] = need;
            in_use_ += need;
            peak_ = std::max(peak_, in_use_);
            return base_ + off;
        }
        return nullptr;
    }
    void free(void* p) {
        const size_t off = (size_t)((char*)p - base_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t len = u->second;
        in_use_ -= len;
        used_.erase(u);
        auto next = free_.lower_bound(off);
        size_t start = off;
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + (len - (off - start))) {
            len += next->second;
            free_.erase(next);
        }
        free_[start] = len;
    }
    size_t capacity() const { return cap_; }
    size_t peak() const { return peak_; }

   private:
    bool host_ = false;
    char* base_ = nullptr;
    size_t cap_ = 0, in_use_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    std::map<size_t, size_t> used_;  // offset -> length
};

struct Req {
    uint64_t ticket = 0;
    int N = 0, dtype = 0;
    size_t bytes = 0;
    std::vector<unsigned char> host;  // state copied from host memory at submit
    void* staged = nullptr;           // ... or into the pinned staging arena
    const void* src_dev = nullptr;    // caller's device state (copied at admission)
    void* d_psi = nullptr;            // arena block
    int slot = -1;
    int state = SRE2_REQ_QUEUED;
    bool cancel = false;
    double t_submit = 0.0, t_done = 0.0;
    double result[SRE2_OUT_LEN] = {0.0, 0.0, 0.0, 0.0};
};
using ReqP = std::shared_ptr<Req>;

struct Flight {
    hipEvent_t ev;
    std::vector<ReqP> reqs;
};

// Large-lane evaluations enqueued at once: two keep the large stream busy
// (the next one is queued while one runs) without a deep device queue.
constexpr int kLargeInFlight = 2;

}  // namespace

struct sre2_server {
    int device = 0, form = 0;
    int max_slots = 0;
    Arena arena;
    Arena staging;  // pinned host copies of host-submitted states
    sre2_ctx* ctx_small = nullptr;
    sre2_ctx* ctx_large = nullptr;
    hipStream_t s_small = nullptr, s_large = nullptr;
    double* d_out = nullptr;  // SRE2_OUT_LEN per slot
    double* h_out = nullptr;  // pinned mirror
    std::vector<int> free_slots;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<ReqP> queue[2];  // lanes: 0 small N, 1 large N
    int large_inflight = 0;     // admitted large-lane requests not yet retired
    std::map<uint64_t, ReqP> live;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::atomic<int> sticky{SRE2_OK};
    int64_t stat[SRE2_SERVER_STAT_COUNT] = {};
    int inflight = 0;

    std::deque<Flight> fl_small, fl_large;
    std::vector<hipEvent_t> ev_pool;
    std::thread worker;

    hipEvent_t get_event() {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }

    // Enqueue copies and evaluations of newly admitted requests (worker only,
    // without the lock); returns packs / packed states / single launches.
    void launch(std::vector<ReqP>& batch, int64_t* counts) {
        const int fmax = ctx_fused_max(form);
        for (auto& r : batch) {
            const hipStream_t st = r->N <= fmax ? s_small : s_large;
            hipError_t e;
            if (r->src_dev)
                e = hipMemcpyAsync(r->d_psi, r->src_dev, r->bytes, hipMemcpyDeviceToDevice, st);
            else if (r->staged)
                e = hipMemcpyAsync(r->d_psi, r->staged, r->bytes, hipMemcpyHostToDevice, st);
            else
                e = hipMemcpyAsync(r->d_psi, r->host.data(), r->bytes, hipMemcpyHostToDevice, st);
            if (e != hipSuccess) sticky = SRE2_EHIP;
        }
        // small N: pack requests of equal (N, dtype)
        std::map<std::pair<int, int>, std::vector<ReqP>> groups;
        for (auto& r : batch)
            if (r->N <= fmax) groups[{r->N, r->dtype}].push_back(r);
        for (auto& g : groups) {
            auto& v = g.second;
            for (size_t i0 = 0; i0 < v.size(); i0 += kMaxPack) {
                const int k = (int)std::min(v.size() - i0, (size_t)kMaxPack);
                const void* psis[kMaxPack];
                double* outs[kMaxPack];
                Flight f{get_event(), {}};
                for (int i = 0; i < k; ++i) {
                    psis[i] = v[i0 + i]->d_psi;
                    outs[i] = d_out + (size_t)SRE2_OUT_LEN * v[i0 + i]->slot;
                    f.reqs.push_back(v[i0 + i]);
                }
                if (ctx_m2_pack(ctx_small, psis, k, g.first.first, g.first.second, form, outs,
                                s_small) != SRE2_OK)
                    sticky = SRE2_EHIP;
                finish(f, s_small);
                fl_small.push_back(f);
                counts[0] += 1;
                counts[1] += k;
            }
        }
        for (auto& r : batch) {
            if (r->N <= fmax) continue;
            Flight f{get_event(), {r}};
            if (ctx_m2_one(ctx_large, r->d_psi, r->N, r->dtype, form, s_large,
                           d_out + (size_t)SRE2_OUT_LEN * r->slot) != SRE2_OK)
                sticky = SRE2_EHIP;
            finish(f, s_large);
            fl_large.push_back(f);
            counts[2] += 1;
        }
    }

    // Results to pinned host memory behind the kernels, then the event.
    void finish(Flight& f, hipStream_t st) {
        for (auto& r : f.reqs) {
            const size_t o = (size_t)SRE2_OUT_LEN * r->slot;
            if (hipMemcpyAsync(h_out + o, d_out + o, SRE2_OUT_LEN * sizeof(double),
                               hipMemcpyDeviceToHost, st) != hipSuccess)
                sticky = SRE2_EHIP;
        }
        if (!f.ev || hipEventRecord(f.ev, st) != hipSuccess) sticky = SRE2_EHIP;
    }

    bool queues_empty() const { return queue[0].empty() && queue[1].empty(); }
    int lane_of(int N) const { return N <= ctx_fused_max(form) ? 0 : 1; }

    // Retire completed flights in stream order (worker only, lock held).
    bool retire(std::deque<Flight>& q, bool large) {
        bool any = false;
        while (!q.empty()) {
            Flight& f = q.front();
            const hipError_t e = f.ev ? hipEventQuery(f.ev) : hipErrorInvalidValue;
            if (e == hipErrorNotReady) break;
            const double t = now_s();
            for (auto& r : f.reqs) {
                memcpy(r->result, h_out + (size_t)SRE2_OUT_LEN * r->slot, sizeof(r->result));
                r->t_done = t;
                r->state = (e != hipSuccess || sticky)
                               ? SRE2_REQ_FAILED
                               : (r->cancel ? SRE2_REQ_CANCELLED : SRE2_REQ_DONE);
                arena.free(r->d_psi);
                r->d_psi = nullptr;
                free_slots.push_back(r->slot);
                r->host.clear();
                r->host.shrink_to_fit();
                if (r->staged) staging.free(r->staged);
                r->staged = nullptr;
                stat[SRE2_SERVER_STAT_COMPLETED] += 1;
                --inflight;
                if (large) --large_inflight;
            }
            if (f.ev) ev_pool.push_back(f.ev);
            q.pop_front();
            any = true;
        }
        return any;
    }

    void run() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            // admission, lane by lane
            std::vector<ReqP> batch;
            for (int lane = 0; lane < 2; ++lane) {
                std::deque<ReqP>& q = queue[lane];
                while (!q.empty()) {
                    ReqP r = q.front();
                    if (r->cancel) {
                        r->state = SRE2_REQ_CANCELLED;
                        r->t_done = now_s();
                        if (r->staged) staging.free(r->staged);
                        r->staged = nullptr;
                        q.pop_front();
                        continue;
                    }
                    if (free_slots.empty()) break;
                    if (lane == 1 && large_inflight >= kLargeInFlight) break;
                    void* p = arena.alloc(r->bytes);
                    if (!p) break;  // backpressure: wait for memory
                    r->d_psi = p;
                    r->slot = free_slots.back();
                    free_slots.pop_back();
                    r->state = SRE2_REQ_RUNNING;
                    q.pop_front();
                    batch.push_back(r);
                    ++inflight;
                    if (lane == 1) ++large_inflight;
                    stat[SRE2_SERVER_STAT_ADMITTED] += 1;
                    stat[SRE2_SERVER_STAT_PEAK_INFLIGHT] =
                        std::max<int64_t>(stat[SRE2_SERVER_STAT_PEAK_INFLIGHT], inflight);
                }
            }
            if (!batch.empty()) {
                lk.unlock();
                int64_t counts[3] = {0, 0, 0};
                launch(batch, counts);
                lk.lock();
                stat[SRE2_SERVER_STAT_PACKS] += counts[0];
                stat[SRE2_SERVER_STAT_PACKED_STATES] += counts[1];
                stat[SRE2_SERVER_STAT_SINGLES] += counts[2];
            }
            const bool done_small = retire(fl_small, false);  // retire both lists
            const bool done_large = retire(fl_large, true);
            const bool done_any = done_small || done_large;
            stat[SRE2_SERVER_STAT_PEAK_BYTES] = (int64_t)arena.peak();
            if (done_any) cv.notify_all();
            const bool busy = !fl_small.empty() || !fl_large.empty();
            if (stop && queues_empty() && !busy) break;
            if (busy) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else if (batch.empty()) {
                cv.wait_for(lk, std::chrono::milliseconds(2));
            }
        }
        cv.notify_all();
    }
};

extern "C" {

int sre2_server_create(sre2_server** out, int hip_device, int form, size_t hbm_budget_bytes,
                       int max_slots) {
    if (!out || hip_device < 0 || max_slots < 1 || hbm_budget_bytes < (size_t(1) << 20))
        return SRE2_EINVAL;
    if (ctx_validate_form(1, SRE2_C64, form) == SRE2_EFORM) return SRE2_EFORM;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(hip_device) != hipSuccess)
        return SRE2_EHIP;
    sre2_server* s = new (std::nothrow) sre2_server();
    if (!s) return SRE2_ENOMEM;
    s->device = hip_device;
    s->form = form;
    s->max_slots = max_slots;
    int rc = s->arena.init(hbm_budget_bytes);
    // pinned staging for host inputs (best effort: without it, host inputs
    // are copied from pageable memory)
    if (!rc) (void)s->staging.init(std::min(hbm_budget_bytes, size_t(1) << 30), true);
    if (!rc) rc = sre2_create(&s->ctx_small, hip_device);
    if (!rc) rc = sre2_create(&s->ctx_large, hip_device);
    if (!rc) rc = sre2_set_scratch_limit(s->ctx_large, size_t(2) << 30);
    if (!rc) rc = ctx_reserve_pack(s->ctx_small, ctx_fused_max(form), form);
    if (!rc && (hipStreamCreateWithFlags(&s->s_small, hipStreamNonBlocking) != hipSuccess ||
                hipStreamCreateWithFlags(&s->s_large, hipStreamNonBlocking) != hipSuccess))
        rc = SRE2_EHIP;
    if (!rc && hipMalloc(&s->d_out, sizeof(double) * SRE2_OUT_LEN * max_slots) != hipSuccess)
        rc = SRE2_ENOMEM;
    if (!rc && hipHostMalloc(&s->h_out, sizeof(double) * SRE2_OUT_LEN * max_slots) != hipSuccess)
        rc = SRE2_ENOMEM;
    if (rc) {
        (void)hipGetLastError();
        sre2_server_destroy(s);
        (void)hipSetDevice(prev);
        return rc;
    }
    for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->worker = std::thread([s] { s->run(); });
    (void)hipSetDevice(prev);
    *out = s;
    return SRE2_OK;
}

int sre2_server_submit(sre2_server* s, const void* psi, int N, int dtype, int psi_on_device,
                       uint64_t* ticket) {
    if (!s || !psi || !ticket) return SRE2_EINVAL;
    int rc = ctx_validate_form(N, dtype, s->form);
    if (rc) return rc;
    auto r = std::make_shared<Req>();
    r->t_submit = now_s();  // latency includes the host-side copy
    r->N = N;
    r->dtype = dtype;
    r->bytes = (size_t(1) << N) * (dtype == SRE2_C64 ? 8 : 16);
    if (r->bytes + 256 > s->arena.capacity()) return SRE2_ENOMEM;  // can never be admitted
    if (psi_on_device) {
        r->src_dev = psi;
    } else {
        // host input: reject non-finite amplitudes at once, then keep a copy
        const size_t nreal = (size_t(2) << N);
        if (dtype == SRE2_C64) {
            const float* f = (const float*)psi;
            for (size_t i = 0; i < nreal; ++i)
                if (!(f[i] - f[i] == 0.0f)) return SRE2_ENORM;
        } else {
            const double* f = (const double*)psi;
            for (size_t i = 0; i < nreal; ++i)
                if (!(f[i] - f[i] == 0.0)) return SRE2_ENORM;
        }
    }
    if (!psi_on_device) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            r->staged = s->staging.capacity() ? s->staging.alloc(r->bytes) : nullptr;
        }
        if (r->staged)  // the copy itself runs outside the lock
            memcpy(r->staged, psi, r->bytes);
        else
            r->host.assign((const unsigned char*)psi, (const unsigned char*)psi + r->bytes);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        if (r->staged) s->staging.free(r->staged);
        return SRE2_EBUSY;
    }
    r->ticket = s->next_ticket++;
    s->queue[s->lane_of(N)].push_back(r);
    s->live[r->ticket] = r;
    s->stat[SRE2_SERVER_STAT_SUBMITTED] += 1;
    *ticket = r->ticket;
    s->cv.notify_all();
    return SRE2_OK;
}

int sre2_server_poll(sre2_server* s, uint64_t ticket, int* state, double* result,
                     double* latency_s) {
    if (!s || !state) return SRE2_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->live.find(ticket);
    if (it == s->live.end()) return SRE2_ENOTFOUND;
    const ReqP& r = it->second;
    *state = r->state;
    if (r->state == SRE2_REQ_DONE || r->state == SRE2_REQ_CANCELLED ||
        r->state == SRE2_REQ_FAILED) {
        if (result) memcpy(result, r->result, sizeof(r->result));
        if (latency_s) *latency_s = r->t_done - r->t_submit;
        s->live.erase(it);
    }
    return SRE2_OK;
}

int sre2_server_cancel(sre2_server* s, uint64_t ticket) {
    if (!s) return SRE2_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->live.find(ticket);
    if (it == s->live.end()) return SRE2_ENOTFOUND;
    it->second->cancel = true;
    s->stat[SRE2_SERVER_STAT_CANCELLED] += 1;
    s->cv.notify_all();
    return SRE2_OK;
}

int sre2_server_drain(sre2_server* s, double timeout_s) {
    if (!s) return SRE2_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::microseconds((int64_t)(timeout_s * 1e6));
    while (!(s->queues_empty() && s->inflight == 0)) {
        if (s->cv.wait_until(lk, deadline) == std::cv_status::timeout &&
            !(s->queues_empty() && s->inflight == 0))
            return SRE2_EBUSY;
    }
    return s->sticky;
}

int sre2_server_stats(sre2_server* s, int64_t* stats, int count) {
    if (!s || !stats || count < 0) return SRE2_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    for (int i = 0; i < count && i < SRE2_SERVER_STAT_COUNT; ++i) stats[i] = s->stat[i];
    return SRE2_OK;
}

int sre2_server_destroy(sre2_server* s) {
    if (!s) return SRE2_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    if (s->s_small) (void)hipStreamSynchronize(s->s_small);
    if (s->s_large) (void)hipStreamSynchronize(s->s_large);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    if (s->s_small) (void)hipStreamDestroy(s->s_small);
    if (s->s_large) (void)hipStreamDestroy(s->s_large);
    if (s->d_out) (void)hipFree(s->d_out);
    if (s->h_out) (void)hipHostFree(s->h_out);
    s->arena.release();
    s->staging.release();
    sre2_destroy(s->ctx_small);
    sre2_destroy(s->ctx_large);
    (void)hipSetDevice(prev);
    const int rc = s->sticky;
    delete s;
    return rc;
}

}  // extern "C"
