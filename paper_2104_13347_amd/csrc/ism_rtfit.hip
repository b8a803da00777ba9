// Reverberation time of an RIR and the uniform-absorption fit (paper section III.A:
// the simulated rooms get homogeneous wall absorption chosen so that their RIRs have
// the target reverberation time).
//
// T30 (ISO 3382): E(n) = sum_{m >= n} h[m]^2 (Schroeder backward integration),
// L(n) = 10 log10(E(n) / E(0)); a least-squares line through L over the samples from
// the first with L <= -5 dB to the first with L <= -35 dB; T30 = -60 / slope.  One
// workgroup of 1024 threads: each thread takes a contiguous chunk, the chunk energies
// are suffix-summed in LDS (FP64), and each thread walks its chunk backwards twice
// (threshold crossings, then the regression sums).
//
// Fit: bisection on a uniform beta in [0, 1) (T30 increases with beta), one RIR from
// the moment kernel and one T30 per step.  Room-level fit: each step is one batched
// launch of every (source, microphone) RIR of the room, one T30 workgroup per RIR, and
// the mean of the T30s (summed on the host in RIR order).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include <climits>
#include <cmath>
#include <vector>

#include "../../include/ism.h"
#include "ism_host.h"

namespace ism {

namespace {

constexpr int RT_THREADS = 1024;

__device__ __forceinline__ double rt_block_sum(double v, double *red)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < RT_THREADS / 64; ++i) s += red[i];
    return s;
}

__device__ __forceinline__ int rt_block_min(int v, int *red)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int s = red[0];
    for (int i = 1; i < RT_THREADS / 64; ++i) s = min(s, red[i]);
    return s;
}

// grid: one workgroup per RIR; RIR i is h[i * n .. (i + 1) n), its T30 goes to out[i]
__global__ __launch_bounds__(RT_THREADS) void rt_t30_kernel(const float *__restrict__ h, int n, double fs,
                                                            double *__restrict__ out)
{
    h += (int64_t)blockIdx.x * n;
    out += blockIdx.x;
    __shared__ double suf[RT_THREADS + 1];
    __shared__ double red[RT_THREADS / 64];
    __shared__ int redi[RT_THREADS / 64];
    const int tid = threadIdx.x;
    const int C = (n + RT_THREADS - 1) / RT_THREADS;
    const int a = min(n, tid * C), b = min(n, a + C);
    double s = 0.0;
    for (int i = a; i < b; ++i) s += (double)h[i] * (double)h[i];
    suf[tid] = s;
    if (tid == 0) suf[RT_THREADS] = 0.0;
    __syncthreads();
    // suffix sums: suf[t] = sum of the chunk energies of threads t .. 1023
    for (int d = 1; d < RT_THREADS; d <<= 1) {
        const double v = suf[tid] + (tid + d < RT_THREADS ? suf[tid + d] : 0.0);
        __syncthreads();
        suf[tid] = v;
        __syncthreads();
    }
    const double E0 = suf[0];
    const double th5 = E0 * 0.31622776601683794, th35 = E0 * 3.1622776601683794e-4;
    // first samples 5 dB and 35 dB down: E is non-increasing, so the samples at or
    // below a threshold form a suffix; a backward walk keeps the smallest index
    int i5 = INT_MAX, i35 = INT_MAX;
    {
        double e = suf[tid + 1];
        for (int i = b - 1; i >= a; --i) {
            e += (double)h[i] * (double)h[i];
            if (e <= th5) i5 = i;
            if (e <= th35) i35 = i;
        }
    }
    const int n5 = rt_block_min(i5, redi);
    const int n35 = rt_block_min(i35, redi);
    if (!(E0 > 0.0) || n5 == INT_MAX || n35 == INT_MAX || n35 - n5 < 2) {
        if (tid == 0) *out = INFINITY;
        return;
    }
    double sx = 0.0, sy = 0.0, sxy = 0.0, sxx = 0.0, cnt = 0.0;
    {
        double e = suf[tid + 1];
        for (int i = b - 1; i >= a; --i) {
            e += (double)h[i] * (double)h[i];
            if (i >= n5 && i <= n35) {
                const double x = (double)i / fs, y = 10.0 * log10(e / E0);
                sx += x;
                sy += y;
                sxy += x * y;
                sxx += x * x;
                cnt += 1.0;
            }
        }
    }
    sx = rt_block_sum(sx, red);
    sy = rt_block_sum(sy, red);
    sxy = rt_block_sum(sxy, red);
    sxx = rt_block_sum(sxx, red);
    cnt = rt_block_sum(cnt, red);
    if (tid == 0) {
        const double slope = (cnt * sxy - sx * sy) / (cnt * sxx - sx * sx);
        *out = slope < 0.0 ? -60.0 / slope : INFINITY;
    }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

}  // namespace ism

using namespace ism;

extern "C" size_t ism_rt_work_bytes(int rir_len)
{
    if (rir_len < 1) return 0;
    return align256((size_t)rir_len * sizeof(float)) + 256;
}

extern "C" int ism_rir_t30(ism_handle *h, const float *rir, int rir_len, double fs, double *t30, ism_stream stream)
{
    if (!h) return ISM_EINVAL;
    if (!rir || !t30 || rir_len < 1) { ism_set_error(h, "NULL argument or rir_len < 1"); return ISM_EINVAL; }
    if (!(fs > 0.0) || !std::isfinite(fs)) { ism_set_error(h, "fs must be finite and > 0"); return ISM_EINVAL; }
    hipLaunchKernelGGL(rt_t30_kernel, dim3(1), dim3(RT_THREADS), 0, (hipStream_t)stream, rir, rir_len, fs, t30);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ism_hip_fail(h, e, "rt_t30_kernel launch");
    return ISM_OK;
}

extern "C" int ism_fit_beta(ism_handle *h, const double L[3], const double src[3], const double mic[3], double fs,
                            double c, int fd_taps, double rt_target, int rir_len, int iters, void *work,
                            size_t work_bytes, double *beta_out, double *rt_out, ism_stream stream)
{
    if (!h) return ISM_EINVAL;
    if (!L || !src || !mic || !work || !beta_out || !rt_out) { ism_set_error(h, "NULL argument"); return ISM_EINVAL; }
    if (!(rt_target > 0.0) || !std::isfinite(rt_target)) {
        ism_set_error(h, "rt_target must be finite and > 0");
        return ISM_EINVAL;
    }
    if (iters < 1 || iters > 60) { ism_set_error(h, "iters must be in [1, 60]"); return ISM_EINVAL; }
    if (rir_len < 1 || work_bytes < ism_rt_work_bytes(rir_len)) {
        ism_set_error(h, "rir_len < 1 or work of %zu bytes, %zu needed", work_bytes, ism_rt_work_bytes(rir_len));
        return ISM_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    float *rir = (float *)work;
    double *dev_rt = (double *)((char *)work + align256((size_t)rir_len * sizeof(float)));
    auto trial = [&](double beta, double &rt) -> int {
        const double b6[6] = {beta, beta, beta, beta, beta, beta};
        int rc = ism_rir(h, L, b6, src, 1, mic, fs, c, -1, ISM_ORDER_INDEX_L1, rir_len, fd_taps, ISM_PREC_FP32,
                         rir, stream);
        if (rc) return rc;
        if ((rc = ism_rir_t30(h, rir, rir_len, fs, dev_rt, stream))) return rc;
        hipError_t e = hipMemcpyAsync(&rt, dev_rt, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return ism_hip_fail(h, e, "T30 read-back");
        return ISM_OK;
    };
    double lo = 0.0, hi = 1.0, rt = 0.0;
    for (int it = 0; it < iters; ++it) {
        const double mid = 0.5 * (lo + hi);
        const int rc = trial(mid, rt);
        if (rc) return rc;
        if (rt < rt_target) lo = mid;
        else hi = mid;
    }
    const double beta = 0.5 * (lo + hi);
    const int rc = trial(beta, rt);
    if (rc) return rc;
    *beta_out = beta;
    *rt_out = rt;
    if (!(std::fabs(rt - rt_target) <= 0.01 * rt_target)) {
        ism_set_error(h, "target T30 %.4g s not reached: T30 %.4g s at beta %.6g after %d steps (rir_len too short "
                      "for the decay, or fewer steps than the target needs)", rt_target, rt, beta, iters);
        return ISM_EDOMAIN;
    }
    return ISM_OK;
}

extern "C" size_t ism_rt_mean_work_bytes(int n_src, int M, int rir_len)
{
    if (n_src < 1 || M < 1 || rir_len < 1) return 0;
    const size_t n = (size_t)n_src * (size_t)M;
    return align256(n * (size_t)rir_len * sizeof(float)) + align256(n * sizeof(double));
}

extern "C" int ism_fit_beta_mean(ism_handle *h, const double L[3], int n_src, const double *srcs, int M,
                                 const double *mics, double fs, double c, int fd_taps, double rt_target,
                                 int rir_len, int iters, void *work, size_t work_bytes, double *beta_out,
                                 double *rt_out, ism_stream stream)
{
    if (!h) return ISM_EINVAL;
    h->last_error.clear();
    if (!L || !srcs || !mics || !work || !beta_out || !rt_out) { ism_set_error(h, "NULL argument"); return ISM_EINVAL; }
    if (n_src < 1 || M < 1 || (int64_t)n_src * M > 65535) {
        ism_set_error(h, "n_src >= 1, M >= 1 and n_src * M <= 65535 required");
        return ISM_EINVAL;
    }
    if (!(rt_target > 0.0) || !std::isfinite(rt_target)) {
        ism_set_error(h, "rt_target must be finite and > 0");
        return ISM_EINVAL;
    }
    if (iters < 1 || iters > 60) { ism_set_error(h, "iters must be in [1, 60]"); return ISM_EINVAL; }
    if (rir_len < 1 || work_bytes < ism_rt_mean_work_bytes(n_src, M, rir_len)) {
        ism_set_error(h, "rir_len < 1 or work of %zu bytes, %zu needed", work_bytes,
                      ism_rt_mean_work_bytes(n_src, M, rir_len));
        return ISM_EINVAL;
    }
    const int n = n_src * M;
    hipStream_t st = (hipStream_t)stream;
    float *rirs = (float *)work;
    double *dev_rt = (double *)((char *)work + align256((size_t)n * rir_len * sizeof(float)));
    std::vector<ism_room> rooms(n_src);
    for (int i = 0; i < n_src; ++i) {
        ism_room &r = rooms[i];
        for (int k = 0; k < 3; ++k) {
            r.L[k] = L[k];
            r.src[k] = srcs[3 * i + k];
        }
        r.mic_offset = 0;
        r.n_mics = M;
        r.max_order = -1;
        r.rir_len = rir_len;
        r.out_offset = (int64_t)i * M * rir_len;
    }
    std::vector<double> rt(n);
    auto trial = [&](double beta, double &mean) -> int {
        for (ism_room &r : rooms)
            for (int k = 0; k < 6; ++k) r.beta[k] = beta;
        int rc = ism_rir_batch(h, n_src, rooms.data(), mics, fs, c, fd_taps, ISM_ORDER_INDEX_L1, ISM_PREC_FP32, rirs,
                               stream);
        if (rc) return rc;
        hipLaunchKernelGGL(rt_t30_kernel, dim3(n), dim3(RT_THREADS), 0, st, rirs, rir_len, fs, dev_rt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return ism_hip_fail(h, e, "rt_t30_kernel launch");
        e = hipMemcpyAsync(rt.data(), dev_rt, sizeof(double) * n, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return ism_hip_fail(h, e, "T30 read-back");
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += rt[i];
        mean = s / n;
        return ISM_OK;
    };
    double lo = 0.0, hi = 1.0, mean = 0.0;
    for (int it = 0; it < iters; ++it) {
        const double mid = 0.5 * (lo + hi);
        const int rc = trial(mid, mean);
        if (rc) return rc;
        if (mean < rt_target) lo = mid;
        else hi = mid;
    }
    const double beta = 0.5 * (lo + hi);
    const int rc = trial(beta, mean);
    if (rc) return rc;
    *beta_out = beta;
    *rt_out = mean;
    if (!(std::fabs(mean - rt_target) <= 0.01 * rt_target)) {
        ism_set_error(h, "target mean T30 %.4g s not reached: %.4g s at beta %.6g after %d steps", rt_target, mean,
                      beta, iters);
        return ISM_EDOMAIN;
    }
    return ISM_OK;
}
