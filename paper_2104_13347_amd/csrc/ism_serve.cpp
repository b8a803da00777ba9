// Serving engine: continuous batching of single-room RIR requests.
//
// Requests arrive at any time (ism_server_submit, any thread).  A scheduler
// thread owns everything else:
//   * admission: strict FIFO; a request is admitted when its output fits in the
//     engine's HBM pool (a first-fit sub-allocator over one allocation) and a lane
//     is free.  The budget covers everything the engine holds on the device: the
//     output pool plus each lane's two fixed staging slots (launch buffers: room
//     table, microphones, work items, wall-power tables); a batch also stops growing
//     when its launch buffer would not fit a slot;
//   * lanes: each lane is a stream with its own library handle (own staging
//     slots); the requests admitted together become one batched launch
//     (ism_rir_batch) on a free lane, while batches on other lanes are still
//     running, so work from different arrivals overlaps on the device;
//   * completion: an event per batch, polled; completion time and latency are
//     stamped per request;
//   * release: the client frees a finished request's output, returning its
//     memory to the pool, which may admit queued requests.
// Each request's result is computed by exactly the same work items whatever the
// batch it lands in, so it is bitwise equal alone and in the mix.
//
// A mock mode runs the same scheduler without a device (batches complete after
// a host-side delay), for tests of admission and ordering.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ism.h"
#include "ism_host.h"

using Clock = std::chrono::steady_clock;

namespace {

double now_s()
{
    return std::chrono::duration<double>(Clock::now().time_since_epoch()).count();
}

struct Pool {
    // first-fit sub-allocator with coalescing, 256-byte granules
    size_t size = 0;
    size_t used = 0;
    size_t peak = 0;
    std::map<size_t, size_t> free_;  // offset -> size
    void init(size_t n)
    {
        size = n;
        free_.clear();
        if (n) free_[0] = n;
        used = peak = 0;
    }
    static size_t round(size_t n) { return (n + 255) / 256 * 256; }
    bool alloc(size_t n, size_t *off)
    {
        n = round(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                size_t rest = it->second - n, o = it->first;
                free_.erase(it);
                if (rest) free_[o + n] = rest;
                used += n;
                peak = std::max(peak, used);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = round(n);
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum ReqState { Q_QUEUED = 0, Q_RUNNING = 1, Q_DONE = 2, Q_FAILED = 3 };

struct Request {
    uint64_t ticket = 0;
    ism_room room{};
    std::vector<double> mics;
    double fs = 0, c = 0;
    int fd_taps = 0, order_mode = 0, precision = 0;
    size_t bytes = 0, off = 0;
    size_t plan_bytes = 0;  // its share of a launch buffer
    int state = Q_QUEUED;
    int status = ISM_OK;
    int64_t tag = -1;  // replay index
    double t_submit = 0, t_start = 0, t_done = 0;
};

struct Lane {
    ism_handle *h = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    unsigned long long *counts = nullptr;  // pinned: the batch's work counters, copied after its launch
    bool busy = false;
    std::vector<uint64_t> batch;
    double mock_until = 0;
};

}  // namespace

struct ism_server {
    int mock = 0;
    int max_batch = 64;
    double mock_taps_per_s = 2e12;
    size_t budget = 0;
    size_t slot_bytes = 0;   // each lane's two staging slots hold this many bytes each (0 in mock mode)
    Pool pool;
    char *base = nullptr;  // device pool
    std::vector<Lane> lanes;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    std::atomic<bool> stop{false};
    std::thread worker;
    std::string err;
    bool record_completions = false;                    // replay: queue (ticket, tag) of finished requests
    std::vector<std::pair<uint64_t, int64_t>> completed;
    // statistics
    int64_t n_submitted = 0, n_done = 0, n_batches = 0, max_inflight_batches = 0;
    int64_t rirs_done = 0;
    int64_t admission_stalls = 0;   // requests that waited at the queue head for pool memory
    uint64_t stalled_ticket = 0;
    int64_t taps_done = 0, records_done = 0;
    double busy_lane_time = 0;
    void loop();
};

static double est_taps(const Request &r)
{
    const double V = r.room.L[0] * r.room.L[1] * r.room.L[2];
    const double T = (r.room.rir_len + (r.fd_taps - 1) / 2) / r.fs;
    const double d = r.c * T;
    return 4.18879 * d * d * d / V * r.room.n_mics * r.fd_taps;
}

void ism_server::loop()
{
    std::unique_lock<std::mutex> lk(mu);
    while (!stop.load()) {
        bool progress = false;
        // 1. completions
        const double t = now_s();
        for (auto &L : lanes) {
            if (!L.busy) continue;
            bool fin = false;
            if (mock) fin = t >= L.mock_until;
            else fin = hipEventQuery(L.done) == hipSuccess;
            if (!fin) continue;
            const double td = mock ? L.mock_until : t;
            if (!mock && L.counts) {   // the counters were copied before the completion event
                taps_done += (int64_t)L.counts[0];
                records_done += (int64_t)L.counts[1];
            }
            for (uint64_t tk : L.batch) {
                auto it = reqs.find(tk);
                if (it == reqs.end()) continue;
                it->second.state = Q_DONE;
                it->second.t_done = td;
                ++n_done;
                rirs_done += it->second.room.n_mics;
                if (record_completions) completed.emplace_back(tk, it->second.tag);
            }
            L.batch.clear();
            L.busy = false;
            progress = true;
        }
        // 2. admission and launch, one batch per free lane
        int inflight = 0;
        for (auto &L : lanes) inflight += L.busy;
        for (auto &L : lanes) {
            if (L.busy || pending.empty()) continue;
            std::vector<uint64_t> batch;
            const Request &head = reqs[pending.front()];
            const double fs = head.fs, c = head.c;
            const int taps = head.fd_taps, om = head.order_mode, pr = head.precision;
            size_t plan = ism_launch_fixed_bytes(taps);
            while (!pending.empty() && (int)batch.size() < max_batch) {
                Request &r = reqs[pending.front()];
                if (r.fs != fs || r.c != c || r.fd_taps != taps || r.order_mode != om || r.precision != pr) break;
                if (slot_bytes && plan + r.plan_bytes > slot_bytes) break;  // the launch buffer is full
                size_t off;
                if (!pool.alloc(r.bytes, &off)) {  // strict FIFO: the head waits for memory
                    if (stalled_ticket != r.ticket) {
                        stalled_ticket = r.ticket;
                        ++admission_stalls;
                    }
                    break;
                }
                r.off = off;
                plan += r.plan_bytes;
                batch.push_back(r.ticket);
                pending.pop_front();
            }
            if (batch.empty()) break;
            std::vector<ism_room> rooms;
            std::vector<double> mics;
            double taps_est = 0;
            for (uint64_t tk : batch) {
                Request &r = reqs[tk];
                ism_room rm = r.room;
                rm.mic_offset = (int32_t)(mics.size() / 3);
                rm.out_offset = (int64_t)(r.off / sizeof(float));
                mics.insert(mics.end(), r.mics.begin(), r.mics.end());
                rooms.push_back(rm);
                r.state = Q_RUNNING;
                r.t_start = now_s();
                taps_est += est_taps(r);
            }
            int st = ISM_OK;
            if (mock) {
                L.mock_until = now_s() + taps_est / mock_taps_per_s;
            } else {
                lk.unlock();  // planning and launch without holding the lock
                st = ism_rir_batch(L.h, (int)rooms.size(), rooms.data(), mics.data(), fs, c, taps, om, pr,
                                   (float *)base, L.stream);
                if (st == ISM_OK && L.h->last_stats &&
                    hipMemcpyAsync(L.counts, L.h->last_stats, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                   L.stream) != hipSuccess)
                    st = ISM_EDEVICE;
                if (st == ISM_OK && hipEventRecord(L.done, L.stream) != hipSuccess) st = ISM_EDEVICE;
                lk.lock();
            }
            if (st != ISM_OK) {
                for (uint64_t tk : batch) {
                    Request &r = reqs[tk];
                    r.state = Q_FAILED;
                    r.status = st;
                    r.t_done = now_s();
                    if (r.off != (size_t)-1) pool.release(r.off, r.bytes);
                    r.off = (size_t)-1;
                    if (record_completions) completed.emplace_back(tk, r.tag);
                }
                err = ism_last_error(L.h);
                continue;
            }
            L.batch = std::move(batch);
            L.busy = true;
            ++n_batches;
            ++inflight;
            max_inflight_batches = std::max<int64_t>(max_inflight_batches, inflight);
            progress = true;
        }
        if (!progress) cv.wait_for(lk, std::chrono::microseconds(20));
    }
}

extern "C" int ism_server_create(int n_lanes, size_t hbm_budget_bytes, int max_batch_rooms, int mock,
                                 ism_server **out)
{
    if (!out) return ISM_EINVAL;
    *out = nullptr;
    if (n_lanes < 1 || n_lanes > 16 || hbm_budget_bytes < 4096 || max_batch_rooms < 1) return ISM_EINVAL;
    ism_server *s = new (std::nothrow) ism_server();
    if (!s) return ISM_ENOMEM;
    s->mock = mock ? 1 : 0;
    s->max_batch = max_batch_rooms;
    s->budget = hbm_budget_bytes;
    // staging: 64 KiB of launch buffer per room of a full batch, at most a quarter of the budget
    // over all lanes' two slots, at least 16 KiB; rounded to the pool's granule
    size_t staging = 0;
    if (!s->mock) {
        size_t sb = (size_t)max_batch_rooms << 16;
        sb = std::min(sb, hbm_budget_bytes / (8 * (size_t)n_lanes));
        sb = std::max<size_t>(Pool::round(sb), 16384);
        s->slot_bytes = sb;
        staging = 2 * (size_t)n_lanes * sb;
        if (staging + 4096 > hbm_budget_bytes) {
            delete s;
            return ISM_ENOMEM;
        }
    }
    s->pool.init((hbm_budget_bytes - staging) / 256 * 256);
    s->lanes.resize(n_lanes);
    if (!s->mock) {
        if (hipMalloc((void **)&s->base, s->pool.size) != hipSuccess) {
            delete s;
            return ISM_ENOMEM;
        }
        for (auto &L : s->lanes) {
            int st = ism_create(&L.h);
            if (st == ISM_OK && hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess) st = ISM_EDEVICE;
            if (st == ISM_OK && hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) st = ISM_EDEVICE;
            if (st == ISM_OK) st = ism_set_tuning(L.h, 0, -1, 0);  // batch shapes vary: launch directly
            if (st == ISM_OK) st = ism_reserve_staging(L.h, s->slot_bytes);
            if (st == ISM_OK && hipHostMalloc((void **)&L.counts, 8 * sizeof(unsigned long long),
                                              hipHostMallocDefault) != hipSuccess) {
                L.counts = nullptr;
                st = ISM_ENOMEM;
            }
            if (st != ISM_OK) {
                ism_server_destroy(s);
                return st == ISM_EINVAL ? ISM_EDEVICE : st;
            }
        }
    }
    s->worker = std::thread([s] { s->loop(); });
    *out = s;
    return ISM_OK;
}

extern "C" void ism_server_destroy(ism_server *s)
{
    if (!s) return;
    s->stop.store(true);
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto &L : s->lanes) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.stream) (void)hipStreamDestroy(L.stream);
        if (L.h) ism_destroy(L.h);
        if (L.counts) (void)hipHostFree(L.counts);
    }
    if (s->base) (void)hipFree(s->base);
    delete s;
}

extern "C" const char *ism_server_last_error(ism_server *s) { return s ? s->err.c_str() : ""; }

static int submit_impl(ism_server *s, const ism_room *room, const double *mics, double fs, double c, int fd_taps,
                       int order_mode, int precision, int64_t tag, uint64_t *ticket)
{
    if (!s || !room || !mics || !ticket) return ISM_EINVAL;
    ism_room r = *room;
    r.mic_offset = 0;
    r.out_offset = 0;
    // same validation as the RIR entry points (a scratch handle-free check)
    ism_handle tmp;
    int st = ism_validate_common(&tmp, fs, c, fd_taps, order_mode, precision);
    if (st == ISM_OK) st = ism_validate_room(&tmp, 0, r, mics);
    if (st != ISM_OK) {
        std::lock_guard<std::mutex> g(s->mu);
        s->err = tmp.last_error;
        return st;
    }
    const size_t bytes = sizeof(float) * (size_t)r.n_mics * (size_t)r.rir_len;
    if (Pool::round(bytes) > s->pool.size) {
        std::lock_guard<std::mutex> g(s->mu);
        s->err = "request output exceeds the engine's output pool (HBM budget less the lanes' staging)";
        return ISM_ENOMEM;
    }
    // the lanes launch with the library's default segment length (1024)
    const size_t plan_bytes = ism_room_launch_bytes(r, fs, c, fd_taps, 1024);
    if (s->slot_bytes && ism_launch_fixed_bytes(fd_taps) + plan_bytes > s->slot_bytes) {
        std::lock_guard<std::mutex> g(s->mu);
        s->err = "request's launch buffer exceeds a lane's staging slot (raise the HBM budget or max_batch_rooms)";
        return ISM_ENOMEM;
    }
    Request q;
    q.room = r;
    q.mics.assign(mics, mics + 3 * (size_t)r.n_mics);
    q.fs = fs;
    q.c = c;
    q.fd_taps = fd_taps;
    q.order_mode = order_mode;
    q.precision = precision;
    q.bytes = bytes;
    q.plan_bytes = plan_bytes;
    q.tag = tag;
    q.t_submit = now_s();
    {
        std::lock_guard<std::mutex> g(s->mu);
        q.ticket = s->next_ticket++;
        *ticket = q.ticket;
        s->pending.push_back(q.ticket);
        s->reqs.emplace(q.ticket, std::move(q));
        ++s->n_submitted;
    }
    s->cv.notify_all();
    return ISM_OK;
}

extern "C" int ism_server_submit(ism_server *s, const ism_room *room, const double *mics, double fs, double c,
                                 int fd_taps, int order_mode, int precision, uint64_t *ticket)
{
    return submit_impl(s, room, mics, fs, c, fd_taps, order_mode, precision, -1, ticket);
}

extern "C" int ism_server_poll(ism_server *s, uint64_t ticket, int *state, float **out_dev, double *latency_ms)
{
    if (!s || !state) return ISM_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return ISM_EINVAL;
    const Request &r = it->second;
    *state = r.state;
    if (out_dev) *out_dev = (r.state == Q_DONE && s->base) ? (float *)(s->base + r.off) : nullptr;
    if (latency_ms) *latency_ms = r.state >= Q_DONE ? (r.t_done - r.t_submit) * 1e3 : -1.0;
    return r.state == Q_FAILED ? r.status : ISM_OK;
}

extern "C" int ism_server_copy_result(ism_server *s, uint64_t ticket, float *dst, ism_stream stream)
{
    if (!s || !dst) return ISM_EINVAL;
    const float *src = nullptr;
    size_t bytes = 0;
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return ISM_EINVAL;
        if (it->second.state != Q_DONE) return it->second.state == Q_FAILED ? it->second.status : ISM_EBUSY;
        if (!s->base) return ISM_EDEVICE;
        src = (const float *)(s->base + it->second.off);
        bytes = it->second.bytes;
    }
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    if (e != hipSuccess) {
        std::lock_guard<std::mutex> g(s->mu);
        s->err = hipGetErrorString(e);
        return ISM_EDEVICE;
    }
    return ISM_OK;
}

extern "C" int ism_server_release(ism_server *s, uint64_t ticket)
{
    if (!s) return ISM_EINVAL;
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return ISM_EINVAL;
        if (it->second.state == Q_QUEUED || it->second.state == Q_RUNNING) return ISM_EBUSY;
        if (it->second.state == Q_DONE && it->second.off != (size_t)-1) s->pool.release(it->second.off, it->second.bytes);
        s->reqs.erase(it);
    }
    s->cv.notify_all();
    return ISM_OK;
}

extern "C" int ism_server_stats(ism_server *s, int64_t st[8])
{
    if (!s || !st) return ISM_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    st[0] = s->n_submitted;
    st[1] = s->n_done;
    st[2] = s->n_batches;
    st[3] = s->max_inflight_batches;
    st[4] = (int64_t)s->pool.size;
    st[5] = (int64_t)s->pool.peak;
    st[6] = (int64_t)s->pending.size();
    st[7] = s->rirs_done;
    return ISM_OK;
}

extern "C" int ism_server_counters(ism_server *s, int64_t v[8])
{
    if (!s || !v) return ISM_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    v[0] = (int64_t)s->budget;
    v[1] = (int64_t)s->pool.size;
    v[2] = (int64_t)(2 * s->lanes.size() * s->slot_bytes);
    v[3] = (int64_t)s->pool.peak;
    v[4] = s->admission_stalls;
    v[5] = s->taps_done;
    v[6] = s->records_done;
    v[7] = s->rirs_done;
    return ISM_OK;
}

extern "C" int ism_server_replay(ism_server *s, int n, const ism_room *rooms, const double *mics,
                                 const double *arrival_s, double fs, double c, int fd_taps, double *latency_ms,
                                 double *wall_s)
{
    if (!s || n < 0 || (n > 0 && (!rooms || !mics || !arrival_s || !latency_ms))) return ISM_EINVAL;
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->record_completions) return ISM_EBUSY;  // one replay at a time
        s->record_completions = true;
        s->completed.clear();
    }
    std::vector<int> rc(n, ISM_OK);
    std::atomic<int> n_failed_submit{0};
    const double t0 = now_s();
    std::thread client([&] {
        for (int i = 0; i < n; ++i) {
            const double due = t0 + arrival_s[i];
            while (now_s() < due) {
                const double left = due - now_s();
                if (left > 200e-6) std::this_thread::sleep_for(std::chrono::microseconds((int64_t)(left * 0.5e6)));
            }
            uint64_t tk;
            rc[i] = submit_impl(s, &rooms[i], mics + 3 * (size_t)rooms[i].mic_offset, fs, c, fd_taps, 0, 0, i, &tk);
            if (rc[i] != ISM_OK) {
                latency_ms[i] = -1.0;
                n_failed_submit.fetch_add(1);
            }
        }
    });
    int finished = 0, st = ISM_OK;
    double t_last = t0;
    std::vector<std::pair<uint64_t, int64_t>> batch;
    while (finished + n_failed_submit.load() < n) {
        {
            std::lock_guard<std::mutex> g(s->mu);
            batch.swap(s->completed);
        }
        for (auto &e : batch) {
            int state = 0;
            double lat = 0;
            int r = ism_server_poll(s, e.first, &state, nullptr, &lat);
            if (r != ISM_OK) st = r;
            if (e.second >= 0 && e.second < n) latency_ms[e.second] = lat;
            ism_server_release(s, e.first);
            ++finished;
            t_last = now_s();
        }
        if (batch.empty()) std::this_thread::sleep_for(std::chrono::microseconds(50));
        batch.clear();
    }
    client.join();
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->record_completions = false;
        s->completed.clear();
    }
    for (int i = 0; i < n; ++i)
        if (rc[i] != ISM_OK) st = rc[i];
    if (wall_s) *wall_s = t_last - t0;
    return st;
}

void ism_serve_release(ism_handle *h) { (void)h; }
