/*
 * ism.h -- C-ABI of libism.so: image-source-method room impulse responses on
 * AMD Instinct MI355X (gfx950).
 *
 * The operation (paper, section II.A, synthetic dataset generation): for a
 * shoebox room with walls at x = 0, Lx, y = 0, Ly, z = 0, Lz, every image of
 * the source (image method of Allen and Berkley) is found, its distance d to
 * each microphone, its damping = product over the walls it was reflected by of
 * that wall's pressure reflection coefficient, times 1/(4 pi d), and its delay
 * d*fs/c, split into an integer part n0 = floor(tau + 1/2) and a fraction
 * f = tau - n0.  A fractional-delay filter centred on tau is added into the
 * RIR at samples n0-K .. n0+K.  The filter is the Hann-windowed sinc
 * h(t) = sinc(t) * (1 + cos(pi t / (K+1))) / 2, K = (fd_taps - 1) / 2 (odd
 * fd_taps, the filter of the workloads this library serves), or, for
 * fd_taps = 8, the paper's own 7th-order Lagrange interpolator: n0 = floor(tau),
 * taps at n0-3 .. n0+4, tap j = prod_{i != j} (D - i) / (j - i) with
 * D = tau - (n0 - 3) in [3, 4).  Taps outside [0, rir_len) are dropped.  Image n,l,q in Z, u,v,w in {0,1} sits at
 * ((1-2u) sx + 2n Lx, (1-2v) sy + 2l Ly, (1-2w) sz + 2q Lz) and is damped by
 * beta[0]^|n-u| beta[1]^|n| beta[2]^|l-v| beta[3]^|l| beta[4]^|q-w| beta[5]^|q|
 * (beta order: x0, xL, y0, yL, z0, zL).
 *
 * Image sets:
 *   max_order >= 0, ISM_ORDER_INDEX_L1:    |n| + |l| + |q| <= max_order
 *   max_order >= 0, ISM_ORDER_REFLECTIONS: |2n-u| + |2l-v| + |2q-w| <= max_order
 *   max_order <  0: every image whose taps reach [0, rir_len) (the paper keeps
 *                   every reflection arriving within the reverberation time).
 *
 * Conventions for every entry point:
 *   - Host pointers (room geometry, microphone positions, room tables) are read
 *     before the call returns; the caller may free them afterwards.
 *   - Device pointers (out, rirs, src, z) must stay valid until the work queued
 *     on `stream` has finished.  The caller owns them.  `out` is overwritten in
 *     full, zeros included.
 *   - Work is queued asynchronously on `stream` (a hipStream_t; NULL means the
 *     default stream).  Calls return once the work is queued.
 *   - Errors are return codes; nothing throws or aborts.  Arguments are
 *     validated before any device work is queued, so a failed call leaves
 *     `out` untouched.  ism_last_error() gives a one-line description.
 *   - Summation order is fixed by the data: the same inputs give bitwise the
 *     same outputs, alone or batched with other rooms.
 *   - A handle is not thread-safe; use one handle per host thread.
 */
#ifndef ISM_H
#define ISM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ISM_VERSION 100

typedef struct ism_handle ism_handle;
typedef void *ism_stream; /* hipStream_t */

enum ism_status {
    ISM_OK = 0,
    ISM_EINVAL = -1,  /* malformed argument: taps even or < 1 or > 255, rir_len < 1, n_mics < 1,
                         fs/c/L not finite and > 0, beta outside [0,1], NULL pointer, bad enum */
    ISM_EDOMAIN = -2, /* geometry outside the model: source not strictly inside the room,
                         microphone outside [0, L], or microphone at the source position */
    ISM_ENOMEM = -3,  /* device or pinned host allocation failed, or a size limit was exceeded */
    ISM_EDEVICE = -4, /* a HIP runtime call failed (text in ism_last_error) */
    ISM_EBUSY = -5    /* serving engine: no capacity for the request right now */
};

enum ism_order_mode { ISM_ORDER_INDEX_L1 = 0, ISM_ORDER_REFLECTIONS = 1 };

/*
 * Arithmetic.  In every mode the image positions, distances, delays and the
 * integer/fractional delay split are computed in FP64 (except the FP32-split
 * ablation).
 *   ISM_PREC_FP32        for fd_taps 9, 81 and 127 with segments of at most
 *                        1024 samples (the default): moment evaluation.  For
 *                        each tap k, h(k - f) is expanded in Chebyshev
 *                        polynomials of 2f (9 terms; truncation below 4.1e-8 of
 *                        max|h| = 1).  Each record adds g T_m(2f), m < 9, in
 *                        FP64 and quantised to 32-bit fixed point, into the bin of
 *                        its integer delay n0; the bin sums are exact 64-bit
 *                        integers (deterministic), rounded once to FP32 and
 *                        split into FP16 pairs (hi + lo, 22 significant bits);
 *                        each output sample is then a 2K+1-tap filter over the 9
 *                        bin sequences on the matrix cores (FP16 pair products,
 *                        FP32 sums).
 *                        Other fd_taps or longer segments: as ISM_PREC_FP32_DIRECT.
 *   ISM_PREC_FP16_LUT    the windowed sinc read from an FP16 table (64 steps per
 *                        sample, linear interpolation); exact accumulation as in
 *                        ISM_PREC_FP32_DIRECT.
 *   ISM_PREC_FP32_SPLIT  ablation: distance and delay split in FP32, otherwise as
 *                        ISM_PREC_FP32.
 *   ISM_PREC_FP32_ATOMIC ablation: FP32 taps summed with FP32 LDS atomics (plain
 *                        FP32 accumulation; the order of the adds at each output
 *                        sample is still fixed).
 *   ISM_PREC_FP32_DIRECT every tap evaluated in FP32 (the sinc by one reciprocal,
 *                        the window by angle addition), quantised to a 32-bit
 *                        fixed-point value (step below 1e-9 of a bound on the
 *                        largest image gain of its output segment) and summed
 *                        exactly in 64-bit integers: deterministic, and the only
 *                        accumulation error is one quantisation per tap.
 */
enum ism_precision {
    ISM_PREC_FP32 = 0,
    ISM_PREC_FP16_LUT = 1,
    ISM_PREC_FP32_SPLIT = 2,
    ISM_PREC_FP32_ATOMIC = 3,
    ISM_PREC_FP32_DIRECT = 4
};

/* One room of a batch.  Microphones of room i are mics[mic_offset .. mic_offset+n_mics);
 * the RIR of its m-th microphone is out[out_offset + m*rir_len .. + rir_len). */
typedef struct ism_room {
    double L[3];
    double beta[6];
    double src[3];
    int32_t mic_offset;
    int32_t n_mics;
    int32_t max_order;
    int32_t rir_len;
    int64_t out_offset;
} ism_room;

/* Create a handle bound to the current HIP device; the handle owns its device
 * work buffers, pinned staging buffers and tuning state.  *h is NULL on error. */
int ism_create(ism_handle **h);
/* Waits for the handle's queued work, then releases everything it owns. */
void ism_destroy(ism_handle *h);
/* Static text for a status code. */
const char *ism_strerror(int status);
/* Text of the last error on this handle ("" if none); valid until the next call. */
const char *ism_last_error(const ism_handle *h);
int ism_version(void);

/*
 * One room, M microphones (section II.A).
 *   L[3], beta[6], src[3]: host, room geometry (m) and reflection coefficients.
 *   mics: host, M x 3 positions (m), row-major.
 *   fs (Hz), c (m/s): sample rate and speed of sound.
 *   max_order, order_mode: image set (see above).
 *   rir_len: samples per RIR; fd_taps: odd windowed-sinc length 2K+1 (<= 255), or
 *            8 for the 7th-order Lagrange filter (ISM_PREC_FP32 / _SPLIT only; segments of
 *            at most 1024 samples are planned for it; it runs on the moment kernel, or on
 *            the per-tap kernel with FP32 coefficients for rooms whose RIR length needs
 *            wall exponents of 128 or more).
 *   precision: ism_precision.
 *   out: device, M x rir_len floats, row-major, fully overwritten.
 */
int ism_rir(ism_handle *h, const double L[3], const double beta[6], const double src[3],
            int M, const double *mics, double fs, double c, int max_order, int order_mode,
            int rir_len, int fd_taps, int precision, float *out, ism_stream stream);

/*
 * Many rooms in one launch (the batched form of ism_rir): every (room, mic,
 * output segment) of the batch is one work item of a single persistent launch.
 *   rooms: host, n_rooms entries; mics: host, positions referenced by the rooms.
 *   out: device; room i writes out[out_offset + m*rir_len + n].
 * Results are bitwise equal to calling ism_rir room by room.
 */
int ism_rir_batch(ism_handle *h, int n_rooms, const ism_room *rooms, const double *mics,
                  double fs, double c, int fd_taps, int order_mode, int precision, float *out,
                  ism_stream stream);

/*
 * Counts of the work a batch implies, computed on the host without device work:
 * work items (room, mic, segment), and upper-bound estimates of images and taps.
 * Any output pointer may be NULL.
 */
int ism_batch_plan_stats(ism_handle *h, int n_rooms, const ism_room *rooms, const double *mics,
                         double fs, double c, int fd_taps, int64_t *n_items,
                         double *est_records, double *est_taps);

/*
 * Work counters of the last ism_rir / ism_rir_batch call on this handle, written
 * to counts[0..7]: [0] taps that landed in the outputs (one per image, microphone
 * and output sample of its filter inside [0, rir_len)), [1] image records
 * processed (an image near a segment boundary is processed once per segment it
 * reaches), [2] candidate images evaluated, [3] tap rounds (64 lanes each),
 * [4] column chunks, [5] enumeration steps, [6] records deferred by an equal
 * delay in the same round, [7] reserved.  Waits for that call to finish.
 */
int ism_last_counts(ism_handle *h, int64_t counts[8]);

/*
 * Tuning of the segment kernel: seg_len = output samples per work item
 * (multiple of 64, 64..2048; 0 keeps the current value), wg_per_cu = cap on
 * resident single-wave workgroups per compute unit of the persistent launch
 * (0 = as many as fit, -1 keeps the current value), graphs = capture each batch
 * launch sequence in a hipGraph and replay it (1) or launch directly (0; -1
 * keeps the current value).  Settings apply to later calls on this handle.
 */
int ism_set_tuning(ism_handle *h, int seg_len, int wg_per_cu, int graphs);
int ism_get_tuning(const ism_handle *h, int *seg_len, int *wg_per_cu, int *graphs);

/*
 * Autotuner of the batched launch (section II.A: the paper batches its RIR
 * computation on the GPU; the launch shape is tuned per workload).  Knobs: the
 * segment length (output samples per work item: 256, 512, 1024, and 2048 where the
 * per-tap kernel runs; the moment kernel takes at most 1024, so longer candidates
 * are never tried where it runs), and for the per-tap kernel the cap on resident
 * single-wave workgroups per compute unit (0, 4, 8, 16) and the image order within a
 * column chunk.  Coordinate search on the caller's batch: each candidate is launched
 * once untimed and twice timed with HIP events on `stream` (the faster run counts).
 * The winner is kept in the handle and in its cache under the batch's shape bucket
 * (precision, fd_taps, order_mode, fs, ceil(log2 longest RIR), ceil(log2 most
 * microphones), ceil(log2 RIRs in the batch)).  out receives the batch's result with the winning configuration.
 * cand / n_cand: segment lengths to try instead of the built-in list (n_cand = 0).
 * *best_seg_len (may be NULL): the chosen segment length.  Synchronises `stream`.
 */
int ism_autotune(ism_handle *h, int n_rooms, const ism_room *rooms, const double *mics,
                 double fs, double c, int fd_taps, int order_mode, int precision, float *out,
                 ism_stream stream, const int *cand, int n_cand, int *best_seg_len);

/*
 * enable = 1: ism_rir_batch (and ism_rir) look up each batch's shape bucket in the
 * handle's tuning cache; the first batch of a bucket not yet cached is tuned as by
 * ism_autotune (that call then synchronises `stream` and takes several launches), later
 * batches of the bucket launch with the cached configuration.  enable = 0 (default):
 * every launch uses the handle's current tuning.
 * ism_get_launch_tuning: the configuration the next launch uses, the autotune mode,
 * the number of cached buckets, and the tuned time (ms) of the cache entry that matches
 * the current configuration (0 if none).  Any pointer may be NULL.
 */
int ism_set_autotune(ism_handle *h, int enable);
int ism_get_launch_tuning(const ism_handle *h, int *seg_len, int *wg_per_cu, int *interleave, int *autotune,
                          int *n_tuned_buckets, float *last_tuned_ms);

/*
 * Source convolution and sensor noise for a batch of rooms (paper section III.A:
 * the RIRs are convolved with source signals; Gaussian noise at a drawn SNR is
 * added to the multichannel result).
 *   rirs: device FP32; room r, mic m: rirs[rir_offset[r] + m*rir_len[r] + j].
 *   rir_offset, rir_len: host arrays of n_rooms entries.
 *   src: device FP32, n_rooms x src_len; out: device FP32, n_rooms x M x out_len.
 *   y[r][m][n] = sum_{j <= min(n, rir_len-1)} h[r][m][j] * x[r][n-j], n < out_len.
 *   snr_db: host, n_rooms entries, or NULL for no noise.  With noise,
 *   y += sigma_r * z, sigma_r^2 = mean over m,n of y^2 * 10^(-snr_db[r]/10), where
 *   z[r][m][n] are the standard normal deviates that ism_normal_deviates writes for
 *   (n_rooms, M, out_len, noise_seed): they are drawn inside the noise pass and never
 *   stored.  r is the room's index within this call, so a caller that splits one
 *   dataset over several calls gives each call its own seed.
 *   use_mfma: 1 = block-Toeplitz GEMM on MFMA, BF16 inputs, FP32 accumulation
 *             (M must be 8); 0 = FP32 direct convolution on the vector units.
 *   Limits: 0 <= n_rooms <= 65535, 1 <= M <= 65535, rir_len in [1, 2^24],
 *   src_len and out_len in [1, 2^28]; otherwise ISM_EINVAL before any device work.
 *   Asynchronous on `stream`.  The handle keeps two workspaces (BF16 RIRs, tile power
 *   sums, room table) used by alternate calls: a call waits on the host only for the
 *   work of the call before the previous one, so back-to-back calls overlap their host
 *   work with the device work of the last.  Calls may go to different streams (a
 *   workspace is reused only after the host has waited for the call that last used it,
 *   on whatever stream): calls in turn on two streams, with separate outputs, overlap
 *   one call's noise pass with the next call's convolution.
 */
int ism_convolve_batch(ism_handle *h, int n_rooms, int M, const float *rirs,
                       const int64_t *rir_offset, const int32_t *rir_len, const float *src,
                       int src_len, int out_len, const float *snr_db, uint64_t noise_seed,
                       int use_mfma, float *out, ism_stream stream);

/*
 * As ism_convolve_batch, with the noise deviates supplied by the caller: z is device
 * FP32, n_rooms x M x out_len standard normal deviates, required if snr_db != NULL.
 * The form that lets a test give the GPU and the reference the same numbers.
 */
int ism_convolve_batch_z(ism_handle *h, int n_rooms, int M, const float *rirs,
                         const int64_t *rir_offset, const int32_t *rir_len, const float *src,
                         int src_len, int out_len, const float *snr_db, const float *z,
                         int use_mfma, float *out, ism_stream stream);

/*
 * Kernel timing of the convolution calls, for measurement.  With timing on, each
 * ism_convolve_batch / ism_convolve_batch_z call records HIP events on its stream around
 * its kernels; ism_conv_last_timing waits for the last call on this handle and writes
 * the durations in ms of its RIR packing ([0], 0-length on the FP32 direct path), its
 * convolution kernel ([1]) and its noise pass ([2], 0 without noise).  ISM_EINVAL when
 * the last call was not timed.  Timing is off by default.
 */
int ism_conv_set_timing(ism_handle *h, int on);
int ism_conv_last_timing(ism_handle *h, float ms[3]);

/*
 * Seeded standard normal deviates (the sensor noise of paper section III.A), written
 * to the device FP32 array z[r][m][n], r < n_rooms, m < M, n < n_samples.  Generator:
 * Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011) with key
 * (seed mod 2^32, seed >> 32); samples 4j .. 4j+3 of (r, m) come from counter
 * (j, m, r, 0), whose output words x0..x3 become uniforms ((x >> 9) + 1/2) 2^-23;
 * Box-Muller (1958) turns (x0, x1) into samples 4j (cosine) and 4j+1 (sine), and
 * (x2, x3) into 4j+2 and 4j+3.  FP32 arithmetic on the hardware's log2, square root,
 * sine and cosine: each deviate is within 1.3e-6 of its exact value (checked over all
 * 2^23 possible uniforms), |z| <= sqrt(48 ln 2).
 * Limits as for ism_convolve_batch (n_samples in place of out_len).  Asynchronous.
 */
int ism_normal_deviates(ism_handle *h, int n_rooms, int M, int n_samples, uint64_t seed, float *z,
                        ism_stream stream);

/*
 * Reverberation time of an RIR and the uniform-absorption fit (paper section III.A:
 * the simulated rooms get homogeneous wall absorption chosen so that their RIRs have
 * the target reverberation time; the paper cites Lehmann and Johansson's prediction
 * for it, which is not reproduced here: the fit measures the simulated RIR itself).
 *
 * ism_rir_t30: T30 of the device FP32 RIR rir[0 .. rir_len) (ISO 3382: Schroeder
 *   backward-integrated energy in dB, least-squares line over the samples from the
 *   first one 5 dB down to the first one 35 dB down, time for that line to fall
 *   60 dB), written as one double to the device pointer t30; +inf when the decay
 *   does not reach -35 dB within the RIR.  Queued on `stream`.
 * ism_fit_beta: the uniform beta (all six walls) whose time-bounded RIR of rir_len
 *   samples from src to mic (fd_taps filter, FP32 precision) has T30 = rt_target:
 *   `iters` bisection steps on beta in [0, 1), T30 being increasing in beta.
 *   work: device buffer of ism_rt_work_bytes(rir_len) bytes, owned by the caller.
 *   *beta_out, *rt_out (host): the fitted beta and the T30 of its RIR.  Blocking: it
 *   waits for `stream` after every step.  rir_len should cover the decay to -35 dB
 *   (about 1.5 x rt_target x fs or more).  Validation as for ism_rir, plus
 *   ISM_EINVAL for rt_target <= 0, iters outside [1, 60] or a short work buffer;
 *   ISM_EDOMAIN (beta_out and rt_out still written) when the final T30 misses the
 *   target by more than 1 % (an RIR too short for the decay, or too few steps).
 */
size_t ism_rt_work_bytes(int rir_len);
/*
 * ism_fit_beta_mean: room-level form of ism_fit_beta (section III.A asks for the room's
 *   reverberation time, not one pair's): the uniform beta whose RIRs from every source
 *   srcs[i] (host, n_src x 3) to every microphone mics[m] (host, M x 3) have a mean T30
 *   of rt_target.  Each bisection step is one batched launch of the n_src x M RIRs
 *   (time-bounded, fd_taps filter, ISM_PREC_FP32) and one T30 per RIR; the mean is
 *   summed on the host in RIR order (source-major) and is +inf when any decay does not
 *   reach -35 dB.  work: device buffer of ism_rt_mean_work_bytes(n_src, M, rir_len)
 *   bytes, owned by the caller.  Requires n_src x M <= 65535.  Blocking, errors and the
 *   1 % check as for ism_fit_beta (ISM_EDOMAIN when the mean misses the target).
 */
size_t ism_rt_mean_work_bytes(int n_src, int M, int rir_len);
int ism_fit_beta_mean(ism_handle *h, const double L[3], int n_src, const double *srcs, int M, const double *mics,
                      double fs, double c, int fd_taps, double rt_target, int rir_len, int iters, void *work,
                      size_t work_bytes, double *beta_out, double *rt_out, ism_stream stream);
int ism_rir_t30(ism_handle *h, const float *rir, int rir_len, double fs, double *t30, ism_stream stream);
int ism_fit_beta(ism_handle *h, const double L[3], const double src[3], const double mic[3], double fs, double c,
                 int fd_taps, double rt_target, int rir_len, int iters, void *work, size_t work_bytes,
                 double *beta_out, double *rt_out, ism_stream stream);

/*
 * Serving engine: continuous batching of single-room requests (the dataset
 * generator of section II.A run as a service, for requests of uneven room size,
 * RIR length and microphone count arriving at any time).
 *
 * ism_server_create: n_lanes streams (1..16), each with its own launch state;
 *   hbm_budget_bytes bounds all the device memory the engine holds: each lane's two
 *   fixed staging slots (launch buffers; 64 KiB per room of a full batch, at most a
 *   quarter of the budget over all lanes) and the output pool (the rest, allocated
 *   once).  A request is admitted, in strict FIFO order, when its output
 *   (M x rir_len floats) fits in the pool and a lane is free; up to max_batch_rooms
 *   admitted requests with equal fs, c, fd_taps, order_mode and precision whose
 *   launch buffer fits a slot form one batched launch.  Batches on different lanes
 *   run concurrently.  mock = 1 runs the scheduler without a device (batches
 *   complete after a host-side delay; outputs are NULL; no staging is reserved).
 *   ISM_ENOMEM if the budget cannot hold the staging slots.
 * ism_server_submit: copies the room and its microphones (host), returns a ticket;
 *   room->mic_offset and room->out_offset are ignored.  Thread-safe.
 *   ISM_ENOMEM if the output can never fit the pool or its launch buffer a staging
 *   slot; validation errors as for ism_rir.
 * ism_server_poll: *state = 0 queued, 1 running, 2 done, 3 failed; when done,
 *   *out_dev = device pointer to the M x rir_len result (owned by the engine until
 *   release) and *latency_ms = completion - submission (host clock at the
 *   engine's observation of the batch's completion event).  Returns the failure
 *   status for a failed request.
 * ism_server_copy_result: queues a device-to-device copy of a finished request's
 *   result (M x rir_len floats) into dst on `stream` (ISM_EBUSY if not done yet).
 * ism_server_release: frees a finished request (ISM_EBUSY while queued/running);
 *   copies queued before release must have completed.
 * ism_server_stats: [submitted, done, batches, max concurrent batches, pool
 *   bytes, peak pool bytes in use, queued now, RIRs done].
 * ism_server_replay: benchmark driver; submits rooms[i] (microphones at
 *   mics + 3*rooms[i].mic_offset) at arrival_s[i] seconds after the call from a
 *   client thread, releases each result when done, writes per-request latency
 *   (ms) and the wall time from the call to the last completion.
 * ism_server_destroy: stops the scheduler, waits for running batches, frees all.
 */
typedef struct ism_server ism_server;
int ism_server_create(int n_lanes, size_t hbm_budget_bytes, int max_batch_rooms, int mock, ism_server **s);
void ism_server_destroy(ism_server *s);
int ism_server_submit(ism_server *s, const ism_room *room, const double *mics, double fs, double c, int fd_taps,
                      int order_mode, int precision, uint64_t *ticket);
int ism_server_poll(ism_server *s, uint64_t ticket, int *state, float **out_dev, double *latency_ms);
int ism_server_copy_result(ism_server *s, uint64_t ticket, float *dst, ism_stream stream);
int ism_server_release(ism_server *s, uint64_t ticket);
int ism_server_stats(ism_server *s, int64_t stats[8]);
/*
 * ism_server_counters: v[0] HBM budget, v[1] output pool bytes, v[2] staging bytes
 * (two fixed launch-buffer slots per lane; the pool is the budget less these), v[3] peak
 * pool bytes in use, v[4] admission stalls (requests that waited at the head of the queue
 * for pool memory), v[5] taps and v[6] image records of finished batches (exact device
 * counts, as ism_last_counts), v[7] RIRs done.
 */
int ism_server_counters(ism_server *s, int64_t v[8]);
const char *ism_server_last_error(ism_server *s);
int ism_server_replay(ism_server *s, int n, const ism_room *rooms, const double *mics, const double *arrival_s,
                      double fs, double c, int fd_taps, double *latency_ms, double *wall_s);

#ifdef __cplusplus
}
#endif
#endif /* ISM_H */
