// Host side of libism.so: argument validation (the ingest step), the work plan
// of a batch (one item per room x microphone x output segment, ordered
// longest-first), staging of the plan through pinned memory, and the launch
// sequence (prologue + persistent segment kernel), optionally captured once in a
// hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ism.h"
#include "ism_host.h"
#include "ism_internal.h"

using namespace ism;

namespace ism {
struct KernelEntry { hipError_t (*fn)(const LaunchDev *, int, int, hipStream_t); const void *sym; };
KernelEntry select_segment_kernel(int K, int variant);
KernelEntry select_moment_kernel(int K, bool reduced);
hipError_t launch_prologue(const LaunchDev *P, int n_rooms, hipStream_t st);
}  // namespace ism

// ------------------------------------------------------------------ handle
void ism_set_error(ism_handle *h, const char *fmt, ...)
{
    if (!h) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    h->last_error = buf;
}

int ism_hip_fail(ism_handle *h, hipError_t e, const char *what)
{
    ism_set_error(h, "%s: %s", what, hipGetErrorString(e));
    return ISM_EDEVICE;
}

static void free_slot(Slot &s)
{
    if (s.gexec) (void)hipGraphExecDestroy(s.gexec);
    if (s.graph) (void)hipGraphDestroy(s.graph);
    if (s.event) (void)hipEventDestroy(s.event);
    if (s.host) (void)hipHostFree(s.host);
    if (s.dev) (void)hipFree(s.dev);
    s = Slot();
}

extern "C" int ism_create(ism_handle **out)
{
    if (!out) return ISM_EINVAL;
    *out = nullptr;
    ism_handle *h = new (std::nothrow) ism_handle();
    if (!h) return ISM_ENOMEM;
    // Without a HIP device the handle still validates and plans; device work
    // then fails with ISM_EDEVICE.
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1 || hipGetDevice(&h->device) != hipSuccess) {
        h->device = -1;
        h->n_cu = 0;
    } else {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, h->device) != hipSuccess) { delete h; return ISM_EDEVICE; }
        h->n_cu = prop.multiProcessorCount;
        h->lds_per_cu = (int)prop.maxSharedMemoryPerMultiProcessor;
    }
    if (const char *v = std::getenv("ISM_INTERLEAVE")) h->interleave = std::atoi(v) ? 1 : 0;
    *out = h;
    return ISM_OK;
}

extern "C" void ism_destroy(ism_handle *h)
{
    if (!h) return;
    for (auto &s : h->slots) {
        if (s.event && s.used) (void)hipEventSynchronize(s.event);
        free_slot(s);
    }
    ism_conv_release(h);
    ism_serve_release(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
}

extern "C" const char *ism_strerror(int st)
{
    switch (st) {
    case ISM_OK: return "ok";
    case ISM_EINVAL: return "invalid argument";
    case ISM_EDOMAIN: return "geometry outside the model";
    case ISM_ENOMEM: return "out of memory or size limit";
    case ISM_EDEVICE: return "HIP runtime error";
    case ISM_EBUSY: return "busy";
    default: return "unknown status";
    }
}

extern "C" const char *ism_last_error(const ism_handle *h) { return h ? h->last_error.c_str() : ""; }
extern "C" int ism_version(void) { return ISM_VERSION; }

extern "C" int ism_set_tuning(ism_handle *h, int seg_len, int wg_per_cu, int graphs)
{
    if (!h) return ISM_EINVAL;
    if (seg_len != 0 && (seg_len < 64 || seg_len > kSegMaxLimit || seg_len % 64 != 0)) {
        ism_set_error(h, "seg_len must be a multiple of 64 in [64, %d]", kSegMaxLimit);
        return ISM_EINVAL;
    }
    if (wg_per_cu < -1 || wg_per_cu > 64) { ism_set_error(h, "wg_per_cu must be in [-1, 64]"); return ISM_EINVAL; }
    if (graphs < -1 || graphs > 1) { ism_set_error(h, "graphs must be -1, 0 or 1"); return ISM_EINVAL; }
    if (seg_len) h->seg_len = seg_len;
    if (wg_per_cu >= 0) h->wg_per_cu = wg_per_cu;
    if (graphs >= 0) h->graphs = graphs;
    return ISM_OK;
}

extern "C" int ism_get_tuning(const ism_handle *h, int *seg_len, int *wg_per_cu, int *graphs)
{
    if (!h) return ISM_EINVAL;
    if (seg_len) *seg_len = h->seg_len;
    if (wg_per_cu) *wg_per_cu = h->wg_per_cu;
    if (graphs) *graphs = h->graphs;
    return ISM_OK;
}

// ------------------------------------------------------------------ validation
static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int ism_validate_common(ism_handle *h, double fs, double c, int fd_taps, int order_mode, int precision)
{
    if (!finite_pos(fs)) { ism_set_error(h, "fs must be finite and > 0"); return ISM_EINVAL; }
    if (!finite_pos(c)) { ism_set_error(h, "c must be finite and > 0"); return ISM_EINVAL; }
    if (fd_taps != kLagrangeTaps && (fd_taps < 1 || fd_taps % 2 == 0 || fd_taps > 2 * kKMax + 1)) {
        ism_set_error(h, "fd_taps must be odd and in [1, %d] (windowed sinc) or %d (Lagrange)", 2 * kKMax + 1,
                      kLagrangeTaps);
        return ISM_EINVAL;
    }
    if (fd_taps == kLagrangeTaps && precision != ISM_PREC_FP32 && precision != ISM_PREC_FP32_SPLIT) {
        ism_set_error(h, "the Lagrange filter (fd_taps = %d) runs with ISM_PREC_FP32 or ISM_PREC_FP32_SPLIT",
                      kLagrangeTaps);
        return ISM_EINVAL;
    }
    if (order_mode != ISM_ORDER_INDEX_L1 && order_mode != ISM_ORDER_REFLECTIONS) {
        ism_set_error(h, "order_mode must be ISM_ORDER_INDEX_L1 or ISM_ORDER_REFLECTIONS");
        return ISM_EINVAL;
    }
    if (precision < ISM_PREC_FP32 || precision > ISM_PREC_FP32_DIRECT) {
        ism_set_error(h, "unknown precision %d", precision);
        return ISM_EINVAL;
    }
    return ISM_OK;
}

int ism_validate_room(ism_handle *h, int idx, const ism_room &r, const double *mics)
{
    for (int a = 0; a < 3; ++a)
        if (!finite_pos(r.L[a])) { ism_set_error(h, "room %d: L must be finite and > 0", idx); return ISM_EINVAL; }
    for (int w = 0; w < 6; ++w)
        if (!std::isfinite(r.beta[w]) || r.beta[w] < 0.0 || r.beta[w] > 1.0) {
            ism_set_error(h, "room %d: beta[%d] must be in [0, 1]", idx, w);
            return ISM_EINVAL;
        }
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(r.src[a])) { ism_set_error(h, "room %d: source not finite", idx); return ISM_EINVAL; }
    if (r.n_mics < 1) { ism_set_error(h, "room %d: n_mics must be >= 1", idx); return ISM_EINVAL; }
    if (r.mic_offset < 0) { ism_set_error(h, "room %d: mic_offset < 0", idx); return ISM_EINVAL; }
    if (r.rir_len < 1 || r.rir_len > (1 << 27)) {
        ism_set_error(h, "room %d: rir_len must be in [1, 2^27]", idx);
        return ISM_EINVAL;
    }
    if (r.out_offset < 0) { ism_set_error(h, "room %d: out_offset < 0", idx); return ISM_EINVAL; }
    if (r.max_order > 100000) { ism_set_error(h, "room %d: max_order too large", idx); return ISM_EINVAL; }
    for (int a = 0; a < 3; ++a)
        if (!(r.src[a] > 0.0 && r.src[a] < r.L[a])) {
            ism_set_error(h, "room %d: source must be strictly inside the room", idx);
            return ISM_EDOMAIN;
        }
    for (int m = 0; m < r.n_mics; ++m) {
        const double *p = mics + 3 * ((int64_t)r.mic_offset + m);
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(p[a])) { ism_set_error(h, "room %d mic %d: not finite", idx, m); return ISM_EINVAL; }
            if (p[a] < 0.0 || p[a] > r.L[a]) {
                ism_set_error(h, "room %d mic %d: outside the room", idx, m);
                return ISM_EDOMAIN;
            }
            d2 += (p[a] - r.src[a]) * (p[a] - r.src[a]);
        }
        if (d2 == 0.0) { ism_set_error(h, "room %d mic %d: at the source position", idx, m); return ISM_EDOMAIN; }
    }
    return ISM_OK;
}

// ------------------------------------------------------------------ plan
// Largest wall exponent any image of the room can need, with margin.
static int pow_stride_for(const ism_room &r, double fs, double c, int K)
{
    double Lmin = std::min(r.L[0], std::min(r.L[1], r.L[2]));
    long e;
    if (r.max_order >= 0) e = (long)r.max_order + 4;
    else {
        double dmax = ((double)r.rir_len - 1.0 + K + 0.5) * c / fs;
        const double q = std::ceil(dmax / (2.0 * Lmin));
        if (!(q < (double)(1L << 22))) return 1 << 22;  // rejected by the caller
        e = (long)q + 4;
    }
    return (int)std::min<long>(e + 1, 1L << 22);
}

// Expected tap count of an output segment (ordering key only).
static double item_cost(const ism_room &r, double fs, double c, int K, int s0, int s1)
{
    const double V = r.L[0] * r.L[1] * r.L[2];
    const double lo = std::max(0.0, (s0 - K - 0.5) * c / fs), hi = (s1 - 1 + K + 0.5) * c / fs;
    double recs = 4.0 * M_PI / (3.0 * V) * (hi * hi * hi - lo * lo * lo);
    const double cols = 4.0 * hi * hi / (r.L[0] * r.L[1]) + 1.0;
    return recs * (2.0 * K + 1.0) + 30.0 * cols + 1.0;
}

// Threads for the host passes over a plan's items (large batches only).
static int host_threads(size_t n)
{
    if (n < (1u << 18)) return 1;
    const unsigned hc = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(8u, hc ? hc : 1u));
}

// Runs f(lo, hi) over [0, n) split into nt contiguous ranges, one thread each.
template <class F>
static void parallel_ranges(size_t n, int nt, F f)
{
    if (nt <= 1) { f((size_t)0, n); return; }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
        const size_t lo = n * t / nt, hi = n * (t + 1) / nt;
        th.emplace_back([=] { f(lo, hi); });
    }
    for (auto &x : th) x.join();
}

int ism_build_plan(ism_handle *h, int n_rooms, const ism_room *rooms, const double * /*mics: the plan needs none*/, double fs,
                   double c, int fd_taps, int seg_len, Plan &plan)
{
    const int K = half_length(fd_taps);
    if (fd_taps == kLagrangeTaps) seg_len = std::min(seg_len, kMomSegMax);  // moment kernel only
    plan.rooms.resize(n_rooms);
    plan.items.clear();
    plan.seg_max = 0;
    plan.n_mics_total = 0;
    plan.est_taps = 0.0;
    plan.est_records = 0.0;
    int64_t pow_total = 0;
    // a unit is one (room, output segment); its items are the room's microphones
    std::vector<int32_t> unit_first(n_rooms + 1, 0);
    int64_t n_units = 0, n_items = 0;
    for (int i = 0; i < n_rooms; ++i) {
        const ism_room &r = rooms[i];
        RoomDev &d = plan.rooms[i];
        std::memcpy(d.L, r.L, sizeof d.L);
        for (int k = 0; k < 3; ++k) d.inv_L[k] = 1.0 / r.L[k];
        std::memcpy(d.beta, r.beta, sizeof d.beta);
        std::memcpy(d.src, r.src, sizeof d.src);
        d.rir_len = r.rir_len;
        d.max_order = r.max_order < 0 ? -1 : r.max_order;
        d.n_mics = r.n_mics;
        d.mic_offset = r.mic_offset;
        d.out_offset = r.out_offset;
        d.pow_stride = pow_stride_for(r, fs, c, K);
        {   // image columns of one item (the kernels index them in 32 bits, below 2^24)
            const double dmax = r.max_order >= 0 ? 2.0 * (r.max_order + 2) * std::max(r.L[0], r.L[1])
                                                 : ((double)r.rir_len + K + 0.5) * c / fs;
            const double cols = (2.0 * dmax / r.L[0] + 5.0) * (2.0 * dmax / r.L[1] + 5.0);
            if (!(cols < 16777216.0) || d.pow_stride >= (1 << 22)) {
                ism_set_error(h, "room %d: too many images for its RIR length (room too small or RIR too long)", i);
                return ISM_EINVAL;
            }
        }
        if (pow_total + 6LL * d.pow_stride > (1LL << 30)) {
            ism_set_error(h, "wall-power tables exceed the size limit");
            return ISM_ENOMEM;
        }
        d.pow_offset = (int32_t)pow_total;
        pow_total += 6LL * d.pow_stride;
        plan.n_mics_total = std::max<int64_t>(plan.n_mics_total, (int64_t)r.mic_offset + r.n_mics);
        const int64_t nseg = ((int64_t)r.rir_len + seg_len - 1) / seg_len;
        n_units += nseg;
        n_items += nseg * r.n_mics;
        if (n_units > INT32_MAX / 2 || n_items > INT32_MAX / 2) {
            ism_set_error(h, "too many work items");
            return ISM_ENOMEM;
        }
        unit_first[i + 1] = (int32_t)n_units;
        plan.seg_max = std::max(plan.seg_max, std::min(seg_len, r.rir_len));
    }
    plan.pow_total = pow_total;
    // longest-first order: counting sort of the units on a log2 cost key (1/16 octave
    // buckets); a unit's items (its microphones) stay together.  Threads take contiguous
    // room ranges with their own histograms; their cursors are laid out bucket by bucket
    // in thread order, which gives the order of the sequential stable sort.
    const int NB = 64 * 16;
    const int nt = host_threads((size_t)n_items);
    std::vector<int32_t> bucket(n_units);
    std::vector<int64_t> th_hist((size_t)nt * NB, 0);
    std::vector<double> th_taps(nt, 0.0);
    auto room_range = [&](int t, int &lo, int &hi) {
        lo = (int)((int64_t)n_rooms * t / nt);
        hi = (int)((int64_t)n_rooms * (t + 1) / nt);
    };
    parallel_ranges((size_t)nt, nt, [&](size_t t0, size_t t1) {
        for (size_t t = t0; t < t1; ++t) {
            int lo, hi;
            room_range((int)t, lo, hi);
            int64_t *hist = th_hist.data() + t * NB;
            double taps = 0.0;
            for (int i = lo; i < hi; ++i) {
                const ism_room &r = rooms[i];
                for (int32_t u = unit_first[i]; u < unit_first[i + 1]; ++u) {
                    const int s0 = (u - unit_first[i]) * seg_len, s1 = std::min(s0 + seg_len, r.rir_len);
                    const double cst = item_cost(r, fs, c, K, s0, s1);
                    taps += (cst - 1.0) > 0 ? cst * r.n_mics : 0.0;
                    int bk = (int)std::floor(std::log2(std::max(1.0f, (float)cst)) * 16.0);
                    bk = std::min(std::max(bk, 0), NB - 1);
                    bucket[u] = NB - 1 - bk;
                    hist[bucket[u]] += r.n_mics;
                }
            }
            th_taps[t] = taps;
        }
    });
    for (int t = 0; t < nt; ++t) plan.est_taps += th_taps[t];
    plan.est_records = plan.est_taps / (2.0 * K + 1.0);
    {   // exclusive offsets: bucket-major, thread-minor
        int64_t run = 0;
        for (int bk = 0; bk < NB; ++bk)
            for (int t = 0; t < nt; ++t) {
                const int64_t v = th_hist[(size_t)t * NB + bk];
                th_hist[(size_t)t * NB + bk] = run;
                run += v;
            }
    }
    // first item of each unit in the sorted order
    std::vector<int32_t> unit_pos(n_units);
    parallel_ranges((size_t)nt, nt, [&](size_t t0, size_t t1) {
        for (size_t t = t0; t < t1; ++t) {
            int lo, hi;
            room_range((int)t, lo, hi);
            int64_t *cur = th_hist.data() + t * NB;
            for (int i = lo; i < hi; ++i)
                for (int32_t u = unit_first[i]; u < unit_first[i + 1]; ++u) {
                    unit_pos[u] = (int32_t)cur[bucket[u]];
                    cur[bucket[u]] += rooms[i].n_mics;
                }
        }
    });
    plan.items.resize(n_items);
    ItemDev *out = plan.items.data();
    parallel_ranges((size_t)n_rooms, host_threads((size_t)n_items), [&](size_t lo, size_t hi) {
        for (size_t i = lo; i < hi; ++i) {
            const ism_room &r = rooms[i];
            const RoomDev &d = plan.rooms[i];
            for (int32_t u = unit_first[i]; u < unit_first[i + 1]; ++u) {
                const int s0 = (u - unit_first[i]) * seg_len, s1 = std::min(s0 + seg_len, r.rir_len);
                ItemDev *it = out + unit_pos[u];
                for (int m = 0; m < r.n_mics; ++m)
                    it[m] = ItemDev{(int32_t)i, r.mic_offset + m, s0, s1, d.pow_offset, d.pow_stride, {0, 0}};
            }
        }
    });
    return ISM_OK;
}

extern "C" int ism_batch_plan_stats(ism_handle *h, int n_rooms, const ism_room *rooms, const double *mics,
                                    double fs, double c, int fd_taps, int64_t *n_items,
                                    double *est_records, double *est_taps)
{
    if (!h || !rooms || !mics || n_rooms < 0) return ISM_EINVAL;
    int st = ism_validate_common(h, fs, c, fd_taps, 0, 0);
    if (st) return st;
    for (int i = 0; i < n_rooms; ++i)
        if ((st = ism_validate_room(h, i, rooms[i], mics))) return st;
    Plan plan;
    if ((st = ism_build_plan(h, n_rooms, rooms, mics, fs, c, fd_taps, h->seg_len, plan))) return st;
    if (n_items) *n_items = (int64_t)plan.items.size();
    if (est_records) *est_records = plan.est_records;
    if (est_taps) *est_taps = plan.est_taps;
    return ISM_OK;
}

// ------------------------------------------------------------------ staging + launch
static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static int ensure_slot(ism_handle *h, Slot &s, size_t bytes)
{
    if (s.cap >= bytes) return ISM_OK;
    if (h->staging_fixed) {
        ism_set_error(h, "launch buffer of %zu bytes exceeds the fixed staging slot of %zu bytes", bytes,
                      h->staging_fixed);
        return ISM_ENOMEM;
    }
    if (s.event && s.used) {   // the slot's last launch must be done before its buffers go
        const hipError_t e = hipEventSynchronize(s.event);
        if (e != hipSuccess) return ism_hip_fail(h, e, "hipEventSynchronize");
    }
    free_slot(s);
    size_t cap = std::max<size_t>(bytes + bytes / 4, 1 << 20);
    hipError_t e = hipHostMalloc(&s.host, cap, hipHostMallocDefault);
    if (e != hipSuccess) { s.host = nullptr; ism_set_error(h, "pinned allocation of %zu bytes failed", cap); return ISM_ENOMEM; }
    e = hipMalloc(&s.dev, cap);
    if (e != hipSuccess) { s.dev = nullptr; ism_set_error(h, "device allocation of %zu bytes failed", cap); return ISM_ENOMEM; }
    e = hipEventCreateWithFlags(&s.event, hipEventDisableTiming);
    if (e != hipSuccess) return ism_hip_fail(h, e, "hipEventCreate");
    s.cap = cap;
    return ISM_OK;
}

int ism_reserve_staging(ism_handle *h, size_t bytes)
{
    if (!h || bytes < 4096) return ISM_EINVAL;
    if (h->device < 0) { ism_set_error(h, "no HIP device"); return ISM_EDEVICE; }
    for (Slot &s : h->slots) {
        if (s.event && s.used) {
            const hipError_t e = hipEventSynchronize(s.event);
            if (e != hipSuccess) return ism_hip_fail(h, e, "hipEventSynchronize");
        }
        free_slot(s);
        hipError_t e = hipHostMalloc(&s.host, bytes, hipHostMallocDefault);
        if (e != hipSuccess) { s.host = nullptr; ism_set_error(h, "pinned allocation failed"); return ISM_ENOMEM; }
        e = hipMalloc(&s.dev, bytes);
        if (e != hipSuccess) { s.dev = nullptr; ism_set_error(h, "device allocation failed"); return ISM_ENOMEM; }
        e = hipEventCreateWithFlags(&s.event, hipEventDisableTiming);
        if (e != hipSuccess) return ism_hip_fail(h, e, "hipEventCreate");
        s.cap = bytes;
    }
    h->staging_fixed = bytes;
    return ISM_OK;
}

// The launch buffer's layout (ism_run_plan): header | rooms | mics | items | coefficients |
// counters | wall-power tables, each part 256-byte aligned.  The per-room term counts a
// room's share of each part; the fixed part the header, the largest coefficient table, the
// counters and the alignment padding of six parts.
size_t ism_launch_fixed_bytes(int fd_taps)
{
    const int K = half_length(fd_taps);
    return align_up(sizeof(LaunchDev), 256) + sizeof(double) * kMom * (2 * K + 1) + 256 + 6 * 256;
}

size_t ism_room_launch_bytes(const ism_room &r, double fs, double c, int fd_taps, int seg_len)
{
    const int K = half_length(fd_taps);
    if (fd_taps == kLagrangeTaps) seg_len = std::min(seg_len, kMomSegMax);
    const size_t nseg = ((size_t)std::max(r.rir_len, 1) + seg_len - 1) / seg_len;
    return sizeof(RoomDev) + sizeof(double) * 3 * (size_t)r.n_mics + sizeof(ItemDev) * nseg * (size_t)r.n_mics +
           sizeof(double) * 6 * (size_t)pow_stride_for(r, fs, c, K);
}

// Chebyshev coefficients of the moment kernel's filter: for each tap k in [-K, K],
// h_k(x) = sum_{m < kMom} c[m][k] T_m(x) on x in [-1, 1], by interpolation at 32
// Chebyshev nodes in FP64 (the truncation after kMom = 9 terms is below 4.1e-8 of
// max|h| = 1, under FP32 rounding; the coefficients past 32 are below double rounding).
//  * windowed sinc: x = 2f, f in [-1/2, 1/2], h_k = h(k - f), h the Hann-windowed sinc of
//    half-length K;
//  * 7th-order Lagrange (K = 4): x = 2f - 1, f = tau - floor(tau) in [0, 1), tap k at
//    n0 + k is the basis polynomial of node j = k + 3 at D = f + 3 (zero for k = -4); a
//    polynomial of degree 7 in x, so the expansion is exact.
static void mom_coefficients(int K, bool lagrange, std::vector<double> &c)
{
    const int nk = 2 * K + 1, NN = 32;
    c.assign((size_t)kMom * nk, 0.0);
    std::vector<double> hv(NN), th(NN);
    for (int j = 0; j < NN; ++j) th[j] = M_PI * (j + 0.5) / NN;
    for (int k = -K; k <= K; ++k) {
        for (int j = 0; j < NN; ++j) {
            const double x = std::cos(th[j]);
            if (lagrange) {
                const int node = k + 3;
                double v = 0.0;
                if (node >= 0 && node < 8) {
                    const double D = 0.5 * (x + 1.0) + 3.0;
                    v = 1.0;
                    for (int i = 0; i < 8; ++i)
                        if (i != node) v *= (D - i) / (double)(node - i);
                }
                hv[j] = v;
            } else {
                const double t = k - 0.5 * x;  // never 0: no node at x = 0
                hv[j] = std::sin(M_PI * t) / (M_PI * t) * 0.5 * (1.0 + std::cos(M_PI * t / (K + 1)));
            }
        }
        for (int m = 0; m < kMom; ++m) {
            double a = 0.0;
            for (int j = 0; j < NN; ++j) a += hv[j] * std::cos(m * th[j]);
            c[(size_t)m * nk + (k + K)] = a * (m == 0 ? 1.0 : 2.0) / NN;
        }
    }
}

int ism_run_plan(ism_handle *h, const Plan &plan, const double *mics, double fs, double c, int fd_taps,
                 int order_mode, int precision, float *out, hipStream_t stream, double *t_ms)
{
    const int K = half_length(fd_taps);
    const bool lagrange = fd_taps == kLagrangeTaps;
    const int n_items = (int)plan.items.size();
    const int n_rooms = (int)plan.rooms.size();
    if (n_items == 0) return ISM_OK;
    if (h->device < 0) { ism_set_error(h, "no HIP device"); return ISM_EDEVICE; }
    const int variant = precision == ISM_PREC_FP16_LUT      ? VAR_LUT
                        : precision == ISM_PREC_FP32_ATOMIC ? VAR_F32ATOM
                                                             : VAR_FX;
    KernelEntry ke{nullptr, nullptr};
    int lds = 0, block = 64;
    int pow_max = 0;
    for (const RoomDev &r : plan.rooms) pow_max = std::max(pow_max, r.pow_stride);
    const bool reduced = precision == ISM_PREC_FP16_LUT;
    const bool moments = (precision == ISM_PREC_FP32 || precision == ISM_PREC_FP32_SPLIT || reduced) &&
                         plan.seg_max <= kMomSegMax && pow_max <= kPowCap;
    if (moments) ke = select_moment_kernel(K, reduced);
    if (ke.fn) {
        lds = mom_lds_bytes(K);
        block = 64 * kMomWaves;
        const int key = lagrange ? -1000 : K;  // distinct from every K and from the initial -1
        if (h->coef_K != key) {
            mom_coefficients(K, lagrange, h->coef);
            h->coef_K = key;
        }
    } else if (lagrange) {
        // rooms whose wall-exponent tables exceed the moment kernel's: per-tap evaluation
        ke = select_segment_kernel(K, VAR_LAG);
        lds = seg_lds_bytes(plan.seg_max, K, VAR_LAG);
    } else {
        ke = select_segment_kernel(K, variant);
        lds = seg_lds_bytes(plan.seg_max, K, variant);
    }
    const bool use_mom = block != 64;
    if (lds > 160 * 1024) { ism_set_error(h, "segment needs %d bytes of LDS", lds); return ISM_ENOMEM; }

    // layout: header | rooms | mics | items | filter coefficients | counter | pow tables
    const size_t n_coef = use_mom ? h->coef.size() : 0;
    size_t off_rooms = align_up(sizeof(LaunchDev), 256);
    size_t off_mics = align_up(off_rooms + sizeof(RoomDev) * n_rooms, 256);
    size_t off_items = align_up(off_mics + sizeof(double) * 3 * plan.n_mics_total, 256);
    size_t off_coef = align_up(off_items + sizeof(ItemDev) * n_items, 256);
    size_t off_cnt = align_up(off_coef + sizeof(double) * n_coef, 256);
    size_t off_pow = align_up(off_cnt + 256, 256);  // counter at +0, stats at +64
    size_t total = off_pow + sizeof(double) * (size_t)plan.pow_total;
    size_t upload = off_cnt;

    Slot &s = h->slots[h->next_slot];
    h->next_slot ^= 1;
    int st = ensure_slot(h, s, total);
    if (st) return st;
    if (s.used) {
        hipError_t e = hipEventSynchronize(s.event);
        if (e != hipSuccess) return ism_hip_fail(h, e, "hipEventSynchronize");
    }
    char *hb = (char *)s.host, *db = (char *)s.dev;
    LaunchDev L{};
    L.fs = fs;
    L.c = c;
    L.rooms = (const RoomDev *)(db + off_rooms);
    L.mics = (const double *)(db + off_mics);
    L.items = (const ItemDev *)(db + off_items);
    L.counter = (uint32_t *)(db + off_cnt);
    L.stats = (unsigned long long *)(db + off_cnt + 64);
    L.pow_tab = (double *)(db + off_pow);
    L.out = out;
    L.n_rooms = n_rooms;
    L.n_items = n_items;
    L.K = K;
    L.order_mode = order_mode;
    L.split32 = precision == ISM_PREC_FP32_SPLIT ? 1 : 0;
    L.lagrange = lagrange ? 1 : 0;
    L.seg_max = plan.seg_max;
    L.interleave = h->interleave;
    L.coef = use_mom ? (const double *)(db + off_coef) : nullptr;
    L.coef_exp = 0;
    L.reserved1 = 0;
    if (use_mom) {  // power-of-two scale that brings the largest coefficient to (2^13, 2^14]
        double cmax = 0.0;
        for (double v : h->coef) cmax = std::max(cmax, std::fabs(v));
        int E = 0;
        (void)std::frexp(cmax, &E);  // cmax = m 2^E, m in [1/2, 1)
        L.coef_exp = cmax > 0.0 ? 14 - E : 0;
    }
    std::memcpy(hb, &L, sizeof L);
    if (n_coef) std::memcpy(hb + off_coef, h->coef.data(), sizeof(double) * n_coef);
    std::memcpy(hb + off_rooms, plan.rooms.data(), sizeof(RoomDev) * n_rooms);
    std::memcpy(hb + off_mics, mics, sizeof(double) * 3 * plan.n_mics_total);
    {   // the item table is the bulk of the upload: copy it on several threads when large
        char *dst = hb + off_items;
        const char *src = (const char *)plan.items.data();
        const size_t bytes = sizeof(ItemDev) * (size_t)n_items;
        parallel_ranges(bytes / 4096 + 1, host_threads((size_t)n_items), [&](size_t lo, size_t hi) {
            const size_t b0 = std::min(bytes, lo * 4096), b1 = std::min(bytes, hi * 4096);
            if (b1 > b0) std::memcpy(dst + b0, src + b0, b1 - b0);
        });
    }

    int per_cu = 0;
    hipError_t e = hipSuccess;
    if (h->occ_sym == ke.sym && h->occ_lds == lds) {
        per_cu = h->occ_per_cu;
    } else {
        if (lds > 64 * 1024) {
            e = hipFuncSetAttribute(ke.sym, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            if (e != hipSuccess) return ism_hip_fail(h, e, "hipFuncSetAttribute");
        }
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ke.sym, block, lds);
        if (e != hipSuccess || per_cu < 1) per_cu = 1;
        h->occ_sym = ke.sym;
        h->occ_lds = lds;
        h->occ_per_cu = per_cu;
    }
    if (h->wg_per_cu > 0) per_cu = std::min(per_cu, h->wg_per_cu);
    const int grid = (int)std::min<int64_t>(n_items, (int64_t)per_cu * h->n_cu);
    const LaunchDev *Pd = (const LaunchDev *)db;

    auto enqueue = [&](hipStream_t q) -> hipError_t {
        hipError_t r = hipMemcpyAsync(db, hb, upload, hipMemcpyHostToDevice, q);
        if (r != hipSuccess) return r;
        r = launch_prologue(Pd, n_rooms, q);
        if (r != hipSuccess) return r;
        return ke.fn(Pd, grid, lds, q);
    };

    if (h->graphs) {
        GraphKey key{(const void *)ke.fn, upload, grid, lds, n_rooms};
        if (!s.gexec || !(s.key == key)) {
            if (s.gexec) { (void)hipGraphExecDestroy(s.gexec); s.gexec = nullptr; }
            if (s.graph) { (void)hipGraphDestroy(s.graph); s.graph = nullptr; }
            // capture on the handle's own stream (the caller's may be the legacy
            // default stream, which cannot be captured); replay on the caller's
            if (!h->cap_stream) {
                e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
                if (e != hipSuccess) { h->cap_stream = nullptr; return ism_hip_fail(h, e, "hipStreamCreate"); }
            }
            e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return ism_hip_fail(h, e, "hipStreamBeginCapture");
            hipError_t e2 = enqueue(h->cap_stream);
            e = hipStreamEndCapture(h->cap_stream, &s.graph);
            if (e2 != hipSuccess) return ism_hip_fail(h, e2, "capture of the batch launch");
            if (e != hipSuccess) return ism_hip_fail(h, e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&s.gexec, s.graph, nullptr, nullptr, 0);
            if (e != hipSuccess) { s.gexec = nullptr; return ism_hip_fail(h, e, "hipGraphInstantiate"); }
            s.key = key;
        }
        e = hipGraphLaunch(s.gexec, stream);
        if (e != hipSuccess) return ism_hip_fail(h, e, "hipGraphLaunch");
    } else {
        e = enqueue(stream);
        if (e != hipSuccess) return ism_hip_fail(h, e, "segment launch");
    }
    e = hipEventRecord(s.event, stream);
    if (e != hipSuccess) return ism_hip_fail(h, e, "hipEventRecord");
    s.used = true;
    h->last_slot = &s;
    h->last_stats = db + off_cnt + 64;
    (void)t_ms;
    return ISM_OK;
}

extern "C" int ism_last_counts(ism_handle *h, int64_t counts[8])
{
    if (!h || !counts) return ISM_EINVAL;
    for (int i = 0; i < 8; ++i) counts[i] = 0;
    if (!h->last_slot || !h->last_stats) return ISM_OK;
    hipError_t e = hipEventSynchronize(h->last_slot->event);
    if (e != hipSuccess) return ism_hip_fail(h, e, "hipEventSynchronize");
    unsigned long long v[8];
    e = hipMemcpy(v, h->last_stats, sizeof v, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return ism_hip_fail(h, e, "hipMemcpy of the work counters");
    for (int i = 0; i < 8; ++i) counts[i] = (int64_t)v[i];
    return ISM_OK;
}

static int tune_batch(ism_handle *h, int n_rooms, const ism_room *rooms, const double *mics, double fs, double c,
                      int fd_taps, int order_mode, int precision, float *out, hipStream_t stream,
                      const std::vector<int> &seg_cands, TuneVal &best);

static TuneKey tune_key(int n_rooms, const ism_room *rooms, double fs, int fd_taps, int order_mode, int precision)
{
    int len = 1, nm = 1;
    int64_t nr = 0;
    for (int i = 0; i < n_rooms; ++i) {
        len = std::max(len, rooms[i].rir_len);
        nm = std::max(nm, rooms[i].n_mics);
        nr += rooms[i].n_mics;
    }
    auto clog2 = [](int64_t v) { int b = 0; while ((1LL << b) < v) ++b; return b; };
    return TuneKey{precision, fd_taps, order_mode, (long long)std::llround(fs * 1e3), clog2(len), clog2(nm), clog2(nr)};
}

static int rir_batch_impl(ism_handle *h, int n_rooms, const ism_room *rooms, const double *mics, double fs,
                          double c, int fd_taps, int order_mode, int precision, float *out, hipStream_t stream)
{
    Plan &plan = h->plan;
    int st = ism_build_plan(h, n_rooms, rooms, mics, fs, c, fd_taps, h->seg_len, plan);
    if (st) return st;
    return ism_run_plan(h, plan, mics, fs, c, fd_taps, order_mode, precision, out, stream, nullptr);
}

extern "C" int ism_rir_batch(ism_handle *h, int n_rooms, const ism_room *rooms, const double *mics,
                             double fs, double c, int fd_taps, int order_mode, int precision, float *out,
                             ism_stream stream)
{
    if (!h) return ISM_EINVAL;
    h->last_error.clear();
    if (n_rooms < 0 || (n_rooms > 0 && (!rooms || !mics || !out))) {
        ism_set_error(h, "NULL argument or negative room count");
        return ISM_EINVAL;
    }
    int st = ism_validate_common(h, fs, c, fd_taps, order_mode, precision);
    if (st) return st;
    for (int i = 0; i < n_rooms; ++i)
        if ((st = ism_validate_room(h, i, rooms[i], mics))) return st;
    if (n_rooms == 0) return ISM_OK;
    if (h->autotune && h->device >= 0) {
        const TuneKey key = tune_key(n_rooms, rooms, fs, fd_taps, order_mode, precision);
        auto hit = h->tune_cache.find(key);
        if (hit == h->tune_cache.end()) {
            TuneVal best{};
            // the tuner leaves the batch's result (with the chosen configuration) in out
            if ((st = tune_batch(h, n_rooms, rooms, mics, fs, c, fd_taps, order_mode, precision, out,
                                 (hipStream_t)stream, {}, best)))
                return st;
            h->tune_cache[key] = best;
            return ISM_OK;
        }
        h->seg_len = hit->second.seg_len;
        h->wg_per_cu = hit->second.wg_per_cu;
        h->interleave = hit->second.interleave;
    }
    return rir_batch_impl(h, n_rooms, rooms, mics, fs, c, fd_taps, order_mode, precision, out, (hipStream_t)stream);
}

extern "C" int ism_rir(ism_handle *h, const double L[3], const double beta[6], const double src[3], int M,
                       const double *mics, double fs, double c, int max_order, int order_mode, int rir_len,
                       int fd_taps, int precision, float *out, ism_stream stream)
{
    if (!h) return ISM_EINVAL;
    if (!L || !beta || !src || !mics || !out) {
        ism_set_error(h, "NULL argument");
        return ISM_EINVAL;
    }
    ism_room r;
    std::memcpy(r.L, L, sizeof r.L);
    std::memcpy(r.beta, beta, sizeof r.beta);
    std::memcpy(r.src, src, sizeof r.src);
    r.mic_offset = 0;
    r.n_mics = M;
    r.max_order = max_order;
    r.rir_len = rir_len;
    r.out_offset = 0;
    return ism_rir_batch(h, 1, &r, mics, fs, c, fd_taps, order_mode, precision, out, stream);
}

// ------------------------------------------------------------------ autotuner
// Launch configuration of a batch: segment length (output samples per work item; the
// moment kernel takes at most kMomSegMax, so longer candidates are not tried where it
// would otherwise run), and for the per-tap kernel (single-wave workgroups) the cap on
// resident workgroups per CU and the enumeration order of a column chunk.  Coordinate
// search: segment lengths first, then (per-tap kernel only) the occupancy cap, then the
// order; each candidate runs once untimed (graph capture, caches) and twice timed, and the
// fastest time counts.  The last launch uses the winner, so `out` holds its result.
static bool moment_path(int fd_taps, int precision)
{
    const int K = half_length(fd_taps);
    const bool compiled = fd_taps == kLagrangeTaps || K == 4 || K == 40 || K == 63;
    return compiled && (precision == ISM_PREC_FP32 || precision == ISM_PREC_FP32_SPLIT);
}

static int tune_batch(ism_handle *h, int n_rooms, const ism_room *rooms, const double *mics, double fs, double c,
                      int fd_taps, int order_mode, int precision, float *out, hipStream_t q,
                      const std::vector<int> &seg_cands, TuneVal &best)
{
    const bool mom = moment_path(fd_taps, precision);
    std::vector<int> segs = seg_cands;
    if (segs.empty()) segs = mom ? std::vector<int>{256, 512, 1024} : std::vector<int>{256, 512, 1024, 2048};
    std::vector<int> ok;
    for (int sl : segs)
        if (sl >= 64 && sl % 64 == 0 && sl <= (mom ? kMomSegMax : kSegMaxLimit)) ok.push_back(sl);
    if (ok.empty()) {
        ism_set_error(h, "no valid segment-length candidate (multiples of 64 up to %d)", mom ? kMomSegMax : kSegMaxLimit);
        return ISM_EINVAL;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) { ism_set_error(h, "hipEventCreate failed"); return ISM_EDEVICE; }
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        ism_set_error(h, "hipEventCreate failed");
        return ISM_EDEVICE;
    }
    const int s_seg = h->seg_len, s_wg = h->wg_per_cu, s_il = h->interleave;
    best = TuneVal{s_seg, s_wg, s_il, 1e30f};
    int st = ISM_OK;
    auto trial = [&](int sl, int wg, int il) -> int {
        h->seg_len = sl;
        h->wg_per_cu = wg;
        h->interleave = il;
        int rc = rir_batch_impl(h, n_rooms, rooms, mics, fs, c, fd_taps, order_mode, precision, out, q);
        if (rc) return rc;
        float t = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
            if (hipEventRecord(e0, q) != hipSuccess) return ISM_EDEVICE;
            if ((rc = rir_batch_impl(h, n_rooms, rooms, mics, fs, c, fd_taps, order_mode, precision, out, q)))
                return rc;
            if (hipEventRecord(e1, q) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return ISM_EDEVICE;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return ISM_EDEVICE;
            t = std::min(t, ms);
        }
        if (t < best.ms) best = TuneVal{sl, wg, il, t};
        return ISM_OK;
    };
    for (int sl : ok)
        if ((st = trial(sl, s_wg, s_il))) break;
    if (!st && !mom) {
        const int caps[] = {0, 4, 8, 16};
        const int sl = best.seg_len, il = best.interleave;
        for (int wg : caps)
            if (wg != s_wg && (st = trial(sl, wg, il))) break;
        if (!st) st = trial(best.seg_len, best.wg_per_cu, 1 - best.interleave);
    }
    if (!st) {   // the winner's launch last: out holds its result
        h->seg_len = best.seg_len;
        h->wg_per_cu = best.wg_per_cu;
        h->interleave = best.interleave;
        st = rir_batch_impl(h, n_rooms, rooms, mics, fs, c, fd_taps, order_mode, precision, out, q);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) {
        h->seg_len = s_seg;
        h->wg_per_cu = s_wg;
        h->interleave = s_il;
        if (st == ISM_EDEVICE && h->last_error.empty()) ism_set_error(h, "HIP event call failed while tuning");
    }
    return st;
}

extern "C" int ism_autotune(ism_handle *h, int n_rooms, const ism_room *rooms, const double *mics, double fs,
                            double c, int fd_taps, int order_mode, int precision, float *out, ism_stream stream,
                            const int *cand, int n_cand, int *best_seg_len)
{
    if (!h) return ISM_EINVAL;
    h->last_error.clear();
    if (n_rooms < 1 || !rooms || !mics || !out || (n_cand > 0 && !cand)) {
        ism_set_error(h, "NULL argument or empty batch");
        return ISM_EINVAL;
    }
    int st = ism_validate_common(h, fs, c, fd_taps, order_mode, precision);
    if (st) return st;
    for (int i = 0; i < n_rooms; ++i)
        if ((st = ism_validate_room(h, i, rooms[i], mics))) return st;
    if (h->device < 0) { ism_set_error(h, "no HIP device"); return ISM_EDEVICE; }
    std::vector<int> cands;
    if (cand && n_cand > 0) cands.assign(cand, cand + n_cand);
    TuneVal best{};
    if ((st = tune_batch(h, n_rooms, rooms, mics, fs, c, fd_taps, order_mode, precision, out, (hipStream_t)stream,
                         cands, best)))
        return st;
    h->tune_cache[tune_key(n_rooms, rooms, fs, fd_taps, order_mode, precision)] = best;
    if (best_seg_len) *best_seg_len = best.seg_len;
    return ISM_OK;
}

extern "C" int ism_set_autotune(ism_handle *h, int enable)
{
    if (!h) return ISM_EINVAL;
    if (enable < 0 || enable > 1) { ism_set_error(h, "enable must be 0 or 1"); return ISM_EINVAL; }
    h->autotune = enable;
    return ISM_OK;
}

extern "C" int ism_get_launch_tuning(const ism_handle *h, int *seg_len, int *wg_per_cu, int *interleave,
                                     int *autotune, int *n_tuned_buckets, float *last_tuned_ms)
{
    if (!h) return ISM_EINVAL;
    if (seg_len) *seg_len = h->seg_len;
    if (wg_per_cu) *wg_per_cu = h->wg_per_cu;
    if (interleave) *interleave = h->interleave;
    if (autotune) *autotune = h->autotune;
    if (n_tuned_buckets) *n_tuned_buckets = (int)h->tune_cache.size();
    if (last_tuned_ms) {
        *last_tuned_ms = 0.f;
        for (const auto &kv : h->tune_cache)
            if (kv.second.seg_len == h->seg_len && kv.second.wg_per_cu == h->wg_per_cu &&
                kv.second.interleave == h->interleave)
                *last_tuned_ms = kv.second.ms;
    }
    return ISM_OK;
}
