// Host-side state of a libism handle.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ism.h"
#include "ism_internal.h"

namespace ism {

// Allocator whose value-less construct leaves trivially constructible elements
// uninitialised: resizing the item table writes nothing, its threaded fill is the only pass.
template <class T>
struct DefaultInitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = DefaultInitAlloc<U>;
    };
    DefaultInitAlloc() = default;
    template <class U>
    DefaultInitAlloc(const DefaultInitAlloc<U> &) noexcept {}
    template <class U>
    void construct(U *p) noexcept { ::new ((void *)p) U; }
    template <class U, class... Args>
    void construct(U *p, Args &&...args) { ::new ((void *)p) U(std::forward<Args>(args)...); }
};

struct Plan {
    std::vector<RoomDev> rooms;
    std::vector<ItemDev, DefaultInitAlloc<ItemDev>> items;
    int64_t n_mics_total = 0;
    int64_t pow_total = 0;
    int seg_max = 0;
    double est_taps = 0.0;
    double est_records = 0.0;
};

struct GraphKey {
    const void *fn = nullptr;
    size_t upload = 0;
    int grid = 0;
    int lds = 0;
    int n_rooms = 0;
    bool operator==(const GraphKey &o) const
    {
        return fn == o.fn && upload == o.upload && grid == o.grid && lds == o.lds && n_rooms == o.n_rooms;
    }
};

// A staging slot: pinned host image of the launch buffer, its device copy, the
// event that marks the end of the last launch that read it, and the captured
// launch graph.  Two slots alternate so that the host can plan the next batch
// while the device still works on the previous one.
struct Slot {
    void *host = nullptr;
    void *dev = nullptr;
    size_t cap = 0;
    hipEvent_t event = nullptr;
    bool used = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    GraphKey key;
};

// Autotuner cache: one launch configuration per shape bucket of a batch.
struct TuneKey {
    int precision, fd_taps, order_mode;
    long long fs_mhz;   // sample rate in mHz
    int len_bucket;     // ceil(log2(longest RIR))
    int mic_bucket;     // ceil(log2(most microphones of a room))
    int rir_bucket;     // ceil(log2(RIRs in the batch)): one RIR and thousands of RIRs of the
                        // same shape fill the chip differently and tune differently
    bool operator<(const TuneKey &o) const
    {
        if (precision != o.precision) return precision < o.precision;
        if (fd_taps != o.fd_taps) return fd_taps < o.fd_taps;
        if (order_mode != o.order_mode) return order_mode < o.order_mode;
        if (fs_mhz != o.fs_mhz) return fs_mhz < o.fs_mhz;
        if (len_bucket != o.len_bucket) return len_bucket < o.len_bucket;
        if (mic_bucket != o.mic_bucket) return mic_bucket < o.mic_bucket;
        return rir_bucket < o.rir_bucket;
    }
};
struct TuneVal {
    int seg_len, wg_per_cu, interleave;
    float ms;           // time of the winning configuration on the batch it was tuned on
};

struct ConvState;
struct ServeState;

}  // namespace ism

struct ism_handle {
    int device = 0;
    int n_cu = 256;
    int lds_per_cu = 160 * 1024;
    int seg_len = 1024;
    int wg_per_cu = 0;  // 0: as many as fit
    int graphs = 1;
    int interleave = 1;
    const void *occ_sym = nullptr;  // cached occupancy of the last segment kernel / LDS size
    int occ_lds = -1;
    int occ_per_cu = 1;
    std::string last_error;
    ism::Slot slots[2];
    int next_slot = 0;
    ism::Plan plan;
    hipStream_t cap_stream = nullptr; // stream used only to capture launch graphs
    ism::Slot *last_slot = nullptr;   // slot of the last batch launch
    void *last_stats = nullptr;       // its device work counters
    ism::ConvState *conv = nullptr;
    int coef_K = -1;                  // Chebyshev filter coefficients of the moment kernel, for coef_K
    std::vector<double> coef;
    size_t staging_fixed = 0;         // nonzero: both staging slots fixed at this capacity (no growth)
    int autotune = 0;                 // 1: tune each new shape bucket on its first batch
    std::map<ism::TuneKey, ism::TuneVal> tune_cache;
};

void ism_set_error(ism_handle *h, const char *fmt, ...);
int ism_hip_fail(ism_handle *h, hipError_t e, const char *what);
int ism_validate_common(ism_handle *h, double fs, double c, int fd_taps, int order_mode, int precision);
int ism_validate_room(ism_handle *h, int idx, const ism_room &r, const double *mics);
int ism_build_plan(ism_handle *h, int n_rooms, const ism_room *rooms, const double *mics, double fs, double c,
                   int fd_taps, int seg_len, ism::Plan &plan);
int ism_run_plan(ism_handle *h, const ism::Plan &plan, const double *mics, double fs, double c, int fd_taps,
                 int order_mode, int precision, float *out, hipStream_t stream, double *t_ms);
// Device bytes of the launch buffer of a batch: a fixed part plus one term per room
// (room record, microphones, work items, wall-power tables), for segments of seg_len.
size_t ism_launch_fixed_bytes(int fd_taps);
size_t ism_room_launch_bytes(const ism_room &r, double fs, double c, int fd_taps, int seg_len);
// Allocates both staging slots of the handle at `bytes` each and fixes them there: a batch
// whose launch buffer is larger then fails with ISM_ENOMEM instead of growing the slots.
int ism_reserve_staging(ism_handle *h, size_t bytes);
void ism_conv_release(ism_handle *h);
void ism_serve_release(ism_handle *h);
