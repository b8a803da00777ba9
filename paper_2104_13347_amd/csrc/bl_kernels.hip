// BeamLearning forward pass on gfx950 (paper section II.B): three cascaded
// filterbank modules of depthwise-separable atrous convolutions with layer norm,
// tanh and residual connections, the pseudo-energy of the valid samples, and a
// layer norm, SELU and fully connected head.
//
// Design:
//  * Folding.  The depthwise taps of a layer are folded into its pointwise
//    weights once per model: W[k][c][o] = sum_j dw[c][j][k] pw[4c+j][o].  A layer
//    is then one dilated convolution, a GEMM over K = 3 x 128 (3 time taps of the
//    128 input channels) instead of a depthwise pass plus a GEMM over K = 512.
//  * Matrix cores.  Layers 1..17 run on v_mfma_f32_16x16x32_f16 with FP16 pairs
//    (x = hi + lo, W = hi + lo; hi*hi + hi*lo + lo*hi summed in FP32).  The
//    activations are scaled by 2^11 and each layer's weights by a power of two
//    chosen from its largest weight, so both halves of a pair stay normal FP16
//    numbers; the output is scaled back exactly.  The folded weights are laid out
//    in MFMA fragment order: one 1 KB contiguous load per wave and operand.
//  * Layer norm across kernels.  The statistics of a layer span the whole
//    n_t x 128 map of a frame, so a layer ends at a kernel boundary: kernel l
//    writes a_l (before its norm) and (sum, M2) partials per 16 rows; kernel l+1
//    combines the partials in FP64 (Chan's formula), forms
//    x_{l+1} = x_l + tanh(LN(a_l)) on the fly while it stages its input tile, and
//    writes x_{l+1} for the next residual.  Per layer and frame that is two reads
//    and two writes of the 128-channel map, the HBM floor of this structure.
//  * Tiles.  A workgroup (4 waves) takes 64 time samples of one frame plus a halo of D
//    on each side; each wave computes the 64 rows for 32 of the 128 output channels, its
//    weight fragments streamed from L2 and its activation fragments read from LDS (row
//    pitch 272 B: the 16 rows of a fragment fall on distinct banks).  Workgroups are
//    renumbered so that each XCD runs a contiguous range of tiles (halo rows in its L2).
//    Batches too small to fill the chip take 16- or 32-row tiles instead (more, shorter
//    workgroups); the layer-norm partials are per 16 rows in every form, so the tile
//    height changes the schedule, not a single bit of the result.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <new>

#include "../../include/beamlearning.h"
#include "ism_host.h"

#define DEV __device__ __forceinline__

namespace {

constexpr int NF = 128;
constexpr int MULT = 4;
constexpr int NL = 18;
// Build constants (measured choices; alternatives in the design notes)
#ifndef BL_PREFETCH
#define BL_PREFETCH 1
#endif
#ifndef BL_STAGE_U
#define BL_STAGE_U 4
#endif
#ifndef BL_LOWLAT_U
#define BL_LOWLAT_U 4
#endif
constexpr int SB = 16;           // rows per layer-norm partial (the finest tile height)
constexpr int BPF = BL_PREFETCH; // weight-fragment steps loaded ahead of the one in use
#ifndef BL_CHUNK
#define BL_CHUNK 0
#endif
constexpr int CHUNK = BL_CHUNK;  // frames per pass through the 18 layers (0: the whole batch)
constexpr int MT0 = 64;         // time samples per layer-0 tile
constexpr int KSTEPS = 12;       // K = 3 taps x 128 channels in steps of 32
constexpr int XROW = 136;        // LDS pitch of a staged input row, in halves
constexpr int MAX_D = 32;
constexpr int MARGIN = BL_MARGIN;
constexpr int XEXP = 11;         // activations are split after scaling by 2^11
constexpr int FRAG_HALVES = 8 * KSTEPS * 2 * 512;  // per layer: [nb][ks][hi/lo][lane][8]
constexpr int MAX_NT = 1 << 20;

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4_t __attribute__((ext_vector_type(4)));

// Offsets (in floats) of each layer's tensors in the flat parameter array.
struct ParamOffsets {
    int64_t dw[NL], pw[NL], b[NL], g[NL], be[NL];
    int64_t g_e, be_e, fc_w, fc_b;
};

struct ModelLayout {
    size_t hdr, w0, vec, frag, head, total;
};

ModelLayout model_layout(int c_in, int n_out)
{
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    ModelLayout m;
    m.hdr = 0;
    m.w0 = al(m.hdr + 64 * sizeof(int));
    m.vec = al(m.w0 + (size_t)3 * c_in * NF * sizeof(float));
    m.frag = al(m.vec + (size_t)NL * 3 * NF * sizeof(float));
    m.head = al(m.frag + (size_t)(NL - 1) * FRAG_HALVES * sizeof(_Float16));
    m.total = al(m.head + (size_t)(2 * NF + NF * n_out + n_out) * sizeof(float));
    return m;
}

struct WsLayout {
    size_t a[2], x[2], st[2], part, total;
    int nst, ne;
};

int cdiv(int a, int b) { return (a + b - 1) / b; }

WsLayout ws_layout(int batch, int n_t)
{
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    WsLayout w;
    w.nst = cdiv(n_t, SB);
    w.ne = cdiv(n_t - 2 * MARGIN, MT0);
    const size_t map = (size_t)batch * n_t * NF * sizeof(float);
    const size_t st = (size_t)batch * w.nst * 2 * sizeof(double);
    size_t o = 0;
    for (int i = 0; i < 2; ++i) { w.a[i] = o; o = al(o + map); }
    for (int i = 0; i < 2; ++i) { w.x[i] = o; o = al(o + map); }
    for (int i = 0; i < 2; ++i) { w.st[i] = o; o = al(o + st); }
    w.part = o;
    o = al(o + (size_t)batch * w.ne * NF * sizeof(float));
    w.total = o;
    return w;
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Renumber them so that each XCD
// takes one contiguous range of (frame, tile) blocks: the neighbouring tiles of a frame,
// which read each other's halo rows, then share that XCD's L2.
DEV int xcd_block()
{
    const int n = gridDim.x, i = blockIdx.x;
    const int per = n >> 3, rem = n & 7, x = i & 7, k = i >> 3;
    return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// ------------------------------------------------------------------ reductions
DEV double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Wave totals of RB per-lane values at the cost of about one: at the xor-32 step the two
// halves of the wave each keep half of the values (and at xor 16 half again), sending the
// partner only what it keeps.  Every kept value sees the same additions, in the same
// order, as in wave_sum, so lane l returns exactly wave_sum(v[rb]) for rb = l / (64 / RB).
template <int RB>
DEV double wave_sum_split(const float (&s)[RB])
{
    static_assert(RB == 1 || RB == 2 || RB == 4, "RB is 1, 2 or 4");
    const int lane = threadIdx.x & 63;
    double k;
    int m0 = 32;
    if constexpr (RB == 1) {
        k = (double)s[0];
    } else if constexpr (RB == 2) {
        const bool hi = lane & 32;
        k = (double)(hi ? s[1] : s[0]);
        k += __shfl_xor((double)(hi ? s[0] : s[1]), 32, 64);
        m0 = 16;
    } else {
        const bool hi = lane & 32;
        double k0 = (double)(hi ? s[2] : s[0]), k1 = (double)(hi ? s[3] : s[1]);
        k0 += __shfl_xor((double)(hi ? s[0] : s[2]), 32, 64);
        k1 += __shfl_xor((double)(hi ? s[1] : s[3]), 32, 64);
        const bool h16 = lane & 16;
        k = h16 ? k1 : k0;
        k += __shfl_xor(h16 ? k0 : k1, 16, 64);
        m0 = 8;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        if (m <= m0) k += __shfl_xor(k, m, 64);
    return k;
}

DEV double wave_max(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
    return v;
}

// Sum over the workgroup (nw waves); every thread gets the total.  `red` holds nw doubles.
DEV double block_sum(double v, double *red, int nw)
{
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

// Layer-norm statistics of one frame from its per-block (sum, M2 about the block mean)
// partials, one per SB rows (Chan et al.'s pairwise update, written as two sums), each sum
// spread over the lanes of a wave; every wave computes them for itself.  The partials are
// per SB rows whatever the tile height of the kernels that wrote them, so a frame's
// statistics, and with them its result, do not depend on the batch it runs in.
//
// One load round (nst <= 64): lane i holds partial i (si, mi; zero beyond nst).
DEV void ln_stats_lanes(double si, double mi, int nst, int T, float eps, double &mean, double &rstd)
{
    const int lane = threadIdx.x & 63;
    const double N = (double)T * NF;
    mean = wave_sum(si) / N;
    double m2 = 0.0;
    if (lane < nst) {
        const double ni = (double)min(SB, T - lane * SB) * NF;
        const double d = si / ni - mean;
        m2 = mi + ni * d * d;
    }
    rstd = 1.0 / sqrt(wave_sum(m2) / N + (double)eps);
}

DEV void ln_stats(const double *st, int nst, int T, float eps, double &mean, double &rstd)
{
    const int lane = threadIdx.x & 63;
    if (nst <= 64) {
        const bool ok = lane < nst;
        ln_stats_lanes(ok ? st[2 * lane] : 0.0, ok ? st[2 * lane + 1] : 0.0, nst, T, eps, mean, rstd);
        return;
    }
    const double N = (double)T * NF;
    double s = 0.0;
    for (int i = lane; i < nst; i += 64) s += st[2 * i];
    mean = wave_sum(s) / N;
    double m2 = 0.0;
    for (int i = lane; i < nst; i += 64) {
        const double ni = (double)min(SB, T - i * SB) * NF;
        const double d = st[2 * i] / ni - mean;
        m2 += st[2 * i + 1] + ni * d * d;
    }
    rstd = 1.0 / sqrt(wave_sum(m2) / N + (double)eps);
}

// tanh(y) = sign(y) (1 - 2 r), r = 1 / (2^(2 log2(e) |y|) + 1), with the hardware exp2
// and reciprocal (about one ulp each).  Absolute error below about 2e-7: near y = 0 it
// is the rounding of 1 - 2r, for large |y| it shrinks with r.
DEV float tanh_fast(float y)
{
    const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * fabsf(y));
    const float t = fmaf(-2.f, __builtin_amdgcn_rcpf(e + 1.f), 1.f);
    return copysignf(t, y);
}

// ------------------------------------------------------------------ model preparation
struct FoldArgs {
    const float *params;
    ParamOffsets po;
    int c_in, n_out;
    int *hdr;
    float *w0, *vec, *head;
    _Float16 *frag;
};

DEV double folded(const float *dw, const float *pw, int k, int o)
{
    // k = tap * 128 + c
    const int tap = k / NF, c = k % NF;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < MULT; ++j) s += (double)dw[(c * MULT + j) * 3 + tap] * (double)pw[(c * MULT + j) * NF + o];
    return s;
}

__global__ __launch_bounds__(256) void bl_fold(FoldArgs A)
{
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const int l = blockIdx.x;
    const float *P = A.params;
    if (l == 0) {
        // layer 0 stays FP32: w0[tap][c][o]
        const int n = 3 * A.c_in * NF;
        for (int i = tid; i < n; i += 256) {
            const int o = i % NF, c = (i / NF) % A.c_in, tap = i / (NF * A.c_in);
            double s = 0.0;
            for (int j = 0; j < MULT; ++j)
                s += (double)P[A.po.dw[0] + (c * MULT + j) * 3 + tap] * (double)P[A.po.pw[0] + (c * MULT + j) * NF + o];
            A.w0[i] = (float)s;
        }
        if (tid == 0) A.hdr[0] = 0;
        return;
    }
    if (l == NL) {
        for (int ll = 0; ll < NL; ++ll)
            for (int i = tid; i < NF; i += 256) {
                A.vec[(ll * 3 + 0) * NF + i] = P[A.po.b[ll] + i];
                A.vec[(ll * 3 + 1) * NF + i] = P[A.po.g[ll] + i];
                A.vec[(ll * 3 + 2) * NF + i] = P[A.po.be[ll] + i];
            }
        const int nh = 2 * NF + NF * A.n_out + A.n_out;
        for (int i = tid; i < nh; i += 256) {
            float v;
            if (i < NF) v = P[A.po.g_e + i];
            else if (i < 2 * NF) v = P[A.po.be_e + i - NF];
            else if (i < 2 * NF + NF * A.n_out) v = P[A.po.fc_w + i - 2 * NF];
            else v = P[A.po.fc_b + i - 2 * NF - NF * A.n_out];
            A.head[i] = v;
        }
        return;
    }
    const float *dw = P + A.po.dw[l];
    const float *pw = P + A.po.pw[l];
    double mx = 0.0;
    for (int i = tid; i < 3 * NF * NF; i += 256) mx = fmax(mx, fabs(folded(dw, pw, i / NF, i % NF)));
    mx = wave_max(mx);
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    int e = 0;
    if (mx > 0.0) frexp(mx, &e);
    const int wexp = 14 - e;  // max |W| 2^wexp < 2^14
    if (tid == 0) A.hdr[l] = wexp;
    _Float16 *fr = A.frag + (size_t)(l - 1) * FRAG_HALVES;
    // fragment order [nb][ks][hi/lo][lane][e]: lane holds B[k = 32 ks + 8 (lane / 16) + e][n = 16 nb + lane % 16]
    for (int i = tid; i < FRAG_HALVES / 2; i += 256) {
        const int e8 = i & 7, lane = (i >> 3) & 63, ks = (i >> 9) % KSTEPS, nb = (i >> 9) / KSTEPS;
        const int k = 32 * ks + 8 * (lane >> 4) + e8, n = 16 * nb + (lane & 15);
        const double v = ldexp(folded(dw, pw, k, n), wexp);
        const _Float16 hi = (_Float16)(float)v;
        const _Float16 lo = (_Float16)(float)(v - (double)(float)hi);
        const size_t base = ((size_t)(nb * KSTEPS + ks) * 2) * 512 + lane * 8 + e8;
        fr[base] = hi;
        fr[base + 512] = lo;
    }
}

// ------------------------------------------------------------------ layer 0 (FP32, vector units)
struct Layer0Args {
    const float *x;
    const int64_t *offs;
    int64_t base, ex_stride, ch_stride;
    const float *w0;    // [3][c_in][128]
    const float *bias;  // [128]
    float *a_out;       // [B][T][128]
    double *st_out;     // [B][nst][2]
    int T, ntiles, nst, c_in;
};

// One thread per output channel and 16-row block of the tile (its 16 outputs in
// registers): block p is computed by waves 2p and 2p + 1, which also give its layer-norm
// partial.  The folded weights and each channel's input window sit in LDS; the window
// is read as 16-byte broadcasts, one channel at a time.
constexpr int L0THREADS = 512;
constexpr int L0XP = MT0 + 4;  // LDS pitch of an input channel: 16-byte aligned rows

__global__ __launch_bounds__(L0THREADS) void bl_layer0(Layer0Args A)
{
    constexpr int R = MT0 / (L0THREADS / NF);  // rows per thread
    static_assert(R == SB, "one 16-row block per group of 128 threads");
    extern __shared__ __align__(16) unsigned char smem[];
    const int c_in = A.c_in;
    float *xin = (float *)smem;          // [c_in][L0XP]: xin[c][p] holds sample t0 - 1 + p
    float *wl = xin + c_in * L0XP;       // [3][c_in][128]
    double *red = (double *)(wl + 3 * c_in * NF);  // [2][8]
    const int tid = threadIdx.x, wave = tid >> 6;
    const int blk = xcd_block();
    const int b = blk / A.ntiles, tile = blk % A.ntiles;
    const int t0 = tile * MT0, T = A.T;
    const int64_t off = A.offs ? A.offs[b] : A.base + (int64_t)b * A.ex_stride;
    for (int i = tid; i < c_in * L0XP; i += L0THREADS) {
        const int c = i / L0XP, p = i % L0XP;
        const int t = t0 - 1 + p;
        xin[i] = (p < MT0 + 2 && t >= 0 && t < T) ? A.x[off + (int64_t)c * A.ch_stride + t] : 0.f;
    }
    {
        // 16-byte copies (the weights and wl are 16-byte aligned; 3 c_in NF is a multiple of 4)
        const float4 *__restrict__ w4 = (const float4 *)A.w0;
        float4 *wl4 = (float4 *)wl;
        for (int i = tid; i < 3 * c_in * NF / 4; i += L0THREADS) wl4[i] = w4[i];
    }
    __syncthreads();
    const int o = tid & (NF - 1), part = tid / NF;
    const int r0 = part * R;
    const int nr = min(R, T - t0 - r0);  // valid rows of this block (<= 0 past the frame)
    const float bo = A.bias[o];
    float v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = bo;
#pragma unroll 1
    for (int c = 0; c < c_in; ++c) {
        const float w0 = wl[c * NF + o], w1 = wl[(c_in + c) * NF + o], w2 = wl[(2 * c_in + c) * NF + o];
        float xs[R + 4];
        const float4 *src = (const float4 *)(xin + c * L0XP + r0);
#pragma unroll
        for (int q = 0; q < R / 4 + 1; ++q) {
            const float4 f = src[q];
            xs[4 * q] = f.x; xs[4 * q + 1] = f.y; xs[4 * q + 2] = f.z; xs[4 * q + 3] = f.w;
        }
#pragma unroll
        for (int i = 0; i < R; ++i) v[i] = fmaf(w2, xs[i + 2], fmaf(w1, xs[i + 1], fmaf(w0, xs[i], v[i])));
    }
    float *dst = A.a_out + ((size_t)b * T + t0 + r0) * NF + o;
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < R; ++i)
        if (i < nr) {
            dst[(size_t)i * NF] = v[i];
            s += v[i];
        }
    const double ws = wave_sum((double)s);
    if ((tid & 63) == 0) red[wave] = ws;
    __syncthreads();
    const double S = red[2 * part] + red[2 * part + 1];
    const float mt = nr > 0 ? (float)(S / ((double)nr * NF)) : 0.f;
    float m2 = 0.f;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const float d = v[i] - mt;
        if (i < nr) m2 = fmaf(d, d, m2);
    }
    const double wm = wave_sum((double)m2);
    if ((tid & 63) == 0) red[8 + wave] = wm;
    __syncthreads();
    if (o == 0 && nr > 0) {
        double *so = A.st_out + ((size_t)b * A.nst + tile * (MT0 / SB) + part) * 2;
        so[0] = S;
        so[1] = red[8 + 2 * part] + red[8 + 2 * part + 1];
    }
}

// ------------------------------------------------------------------ layers 1..17 (matrix cores)
struct LayerArgs {
    const float *a_in;     // a_{l-1}
    const float *x_in;     // x_{l-1} (l >= 2)
    float *x_out;          // x_l
    float *a_out;          // a_l
    const double *st_in;   // partials of a_{l-1}
    double *st_out;        // partials of a_l
    const float *vec_prev; // b, g, be of layer l-1
    const float *bias;     // b of layer l
    const _Float16 *frag;  // layer l's weight fragments
    const int *hdr;
    int T, ntiles, nst, layer, D;
    float eps;
};

constexpr int LWAVES = 4;              // waves per layer workgroup: one per 32 output channels
constexpr int LTHREADS = 64 * LWAVES;

DEV void load_b(f16x8_t (&bq)[4], const _Float16 *fr, int nb0, int ks)
{
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int p = 0; p < 2; ++p)
            bq[2 * cb + p] = *(const f16x8_t *)(fr + ((size_t)((nb0 + cb) * KSTEPS + ks) * 2 + p) * 512);
}

// Stage x_l = (l >= 2 ? x_{l-1} : 0) + tanh(LN(a_{l-1})) for rows t0 - D .. t0 + MT + D of
// frame b into LDS as the scaled FP16 split (hi in xh, lo in xl), and write the tile's own
// rows of x_l to HBM.  256 threads (ptid), 8 rows per pass; U passes' loads are issued
// before any is used.
template <int MT, int U>
DEV void stage_tile(const LayerArgs &A, int b, int tile, _Float16 *xh, _Float16 *xl, int ptid)
{
    const int D = A.D, T = A.T;
    const int rows = MT + 2 * D;
    const int t0 = tile * MT;
    const size_t fb = (size_t)b * T;
    const float *__restrict__ a_in = A.a_in;
    const float *__restrict__ x_in = A.x_in;
    float *__restrict__ x_out = A.x_out;
    const bool resid = A.layer >= 2;
    double mean, rstd;
    ln_stats(A.st_in + (size_t)b * A.nst * 2, A.nst, T, A.eps, mean, rstd);
    const int c4 = (ptid & 31) * 4;
    const float4 g = *(const float4 *)(A.vec_prev + NF + c4);
    const float4 be = *(const float4 *)(A.vec_prev + 2 * NF + c4);
    const float mu = (float)mean, rs = (float)rstd;
    const float4 sc = make_float4(g.x * rs, g.y * rs, g.z * rs, g.w * rs);
    constexpr int RS = 256 / 32;  // rows per pass
    for (int rb = ptid >> 5; rb < rows; rb += RS * U) {
        float4 av[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = rb + RS * u, t = t0 - D + r;
            const bool ok = r < rows && t >= 0 && t < T;
            av[u] = ok ? *(const float4 *)(a_in + (fb + t) * NF + c4) : make_float4(0.f, 0.f, 0.f, 0.f);
            xv[u] = ok && resid ? *(const float4 *)(x_in + (fb + t) * NF + c4) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = rb + RS * u, t = t0 - D + r;
            if (r < rows) {
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (t >= 0 && t < T) {
                    v.x = xv[u].x + tanh_fast(fmaf(av[u].x - mu, sc.x, be.x));
                    v.y = xv[u].y + tanh_fast(fmaf(av[u].y - mu, sc.y, be.y));
                    v.z = xv[u].z + tanh_fast(fmaf(av[u].z - mu, sc.z, be.z));
                    v.w = xv[u].w + tanh_fast(fmaf(av[u].w - mu, sc.w, be.w));
                    if (r >= D && r < D + MT) *(float4 *)(x_out + (fb + t) * NF + c4) = v;
                }
                const float s = (float)(1 << XEXP);
                const float vs[4] = {v.x * s, v.y * s, v.z * s, v.w * s};
                f16x4_t h, lo;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    h[i] = (_Float16)vs[i];
                    lo[i] = (_Float16)(vs[i] - (float)h[i]);
                }
                *(f16x4_t *)(xh + r * XROW + c4) = h;
                *(f16x4_t *)(xl + r * XROW + c4) = lo;
            }
        }
    }
}

// a_l[t][n] = sum over taps and channels of x_l[t + (tap-1) D][c] W[tap][c][n] for the
// 16 RB rows of a staged tile and the 32 output channels of column group cg (one wave).
// The weight fragments sit in a ring of P + 1 steps: step ks in slot ks % (P + 1), step
// ks + P loaded while step ks runs.  preload_b fills the first P slots.
template <int P>
DEV void preload_b(f16x8_t (&bq)[P + 1][4], const LayerArgs &A, int cg, int lane)
{
#pragma unroll
    for (int i = 0; i < P; ++i) load_b(bq[i], A.frag + lane * 8, 2 * cg, i);
}

template <int P, int RB>
DEV void gemm_tile(const LayerArgs &A, const _Float16 *xh, const _Float16 *xl, int cg, int lane,
                   f16x8_t (&bq)[P + 1][4], f32x4_t (&acc)[RB][2])
{
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    const _Float16 *fr = A.frag + lane * 8;
    const int nb0 = 2 * cg, D = A.D;
    const int rowl = lane & 15;
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
        if (ks + P < KSTEPS) load_b(bq[(ks + P) % (P + 1)], fr, nb0, ks + P);
        const f16x8_t *bc = bq[ks % (P + 1)];
        const int tap = ks >> 2;
        const int off = (tap * D + rowl) * XROW + (ks & 3) * 32 + 8 * (lane >> 4);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const f16x8_t ah = *(const f16x8_t *)(xh + off + rb * 16 * XROW);
            const f16x8_t al = *(const f16x8_t *)(xl + off + rb * 16 * XROW);
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bc[2 * cb], acc[rb][cb], 0, 0, 0);
                acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bc[2 * cb + 1], acc[rb][cb], 0, 0, 0);
                acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bc[2 * cb], acc[rb][cb], 0, 0, 0);
            }
        }
    }
}

// Scale back, add the bias and store the wave's 16 RB x 32 block of a_l; s[rb] gets the
// lane's sum over the valid rows of 16-row block rb.
template <int RB>
DEV void store_tile(const LayerArgs &A, int b, int tile, int cg, int lane, f32x4_t (&acc)[RB][2], float (&s)[RB])
{
    constexpr int MT = 16 * RB;
    const int T = A.T, t0 = tile * MT;
    const int nrows = min(MT, T - t0);
    const float osc = ldexpf(1.f, -(XEXP + A.hdr[A.layer]));
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const float bn_ = A.bias[32 * cg + 16 * cb + (lane & 15)];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[rb][cb][v] = fmaf(acc[rb][cb][v], osc, bn_);
    }
    float *__restrict__ dst = A.a_out + ((size_t)b * T + t0 + 4 * (lane >> 4)) * NF + 32 * cg + (lane & 15);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) s[rb] = 0.f;
    if (nrows == MT) {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    dst[(16 * rb + v) * NF + 16 * cb] = acc[rb][cb][v];
                    s[rb] += acc[rb][cb][v];
                }
    } else {
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (16 * rb + 4 * (lane >> 4) + v < nrows) {
                        dst[(16 * rb + v) * NF + 16 * cb] = acc[rb][cb][v];
                        s[rb] += acc[rb][cb][v];
                    }
    }
}

// Sums of squared deviations from each 16-row block's mean over its valid rows.
template <int RB>
DEV void m2_tile(int nrows, int lane, const float (&mean)[RB], const f32x4_t (&acc)[RB][2], float (&m2)[RB])
{
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) m2[rb] = 0.f;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float d = acc[rb][cb][v] - mean[rb];
                if (16 * rb + 4 * (lane >> 4) + v < nrows) m2[rb] = fmaf(d, d, m2[rb]);
            }
}

// One tile of 16 RB rows per workgroup (4 waves): stage, barrier, GEMM, store, and the
// layer-norm partial of each 16-row block (a fixed-order sum over the four waves, so the
// same for every RB).  The low-latency form (at most one workgroup per CU, small batches)
// issues the first 7 steps' weight-fragment loads before staging, so their latency hides
// behind it, and stages in fewer, wider passes.
template <bool LOWLAT, int RB>
__global__ __launch_bounds__(LTHREADS) void bl_layer(LayerArgs A)
{
    constexpr int MT = 16 * RB;
    constexpr int P = LOWLAT ? 7 : BPF;
    constexpr int U = LOWLAT ? BL_LOWLAT_U : BL_STAGE_U;
    extern __shared__ __align__(16) unsigned char smem[];
    const int rows = MT + 2 * A.D;
    _Float16 *xh = (_Float16 *)smem;
    _Float16 *xl = xh + rows * XROW;
    double *red = (double *)(xl + rows * XROW);  // [2][LWAVES][RB]
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int blk = xcd_block();
    const int b = blk / A.ntiles, tile = blk % A.ntiles;
    f16x8_t bq[P + 1][4];
    if (LOWLAT) preload_b<P>(bq, A, wave, lane);
    stage_tile<MT, U>(A, b, tile, xh, xl, tid);
    __syncthreads();
    if (!LOWLAT) preload_b<P>(bq, A, wave, lane);
    f32x4_t acc[RB][2];
    gemm_tile<P, RB>(A, xh, xl, wave, lane, bq, acc);
    const int nrows = min(MT, A.T - tile * MT);
    float s[RB];
    store_tile<RB>(A, b, tile, wave, lane, acc, s);
    constexpr int LPB = 64 / RB;  // lanes per 16-row block in wave_sum_split's result
    {
        const double w = wave_sum_split<RB>(s);
        if (lane % LPB == 0) red[wave * RB + lane / LPB] = w;
    }
    __syncthreads();
    float mean[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        double S = 0.0;
        for (int w = 0; w < LWAVES; ++w) S += red[w * RB + rb];
        const int nr = min(16, nrows - 16 * rb);
        mean[rb] = nr > 0 ? (float)(S / ((double)nr * NF)) : 0.f;
    }
    float m2[RB];
    m2_tile<RB>(nrows, lane, mean, acc, m2);
    double *red2 = red + LWAVES * RB;
    {
        const double w = wave_sum_split<RB>(m2);
        if (lane % LPB == 0) red2[wave * RB + lane / LPB] = w;
    }
    __syncthreads();
    if (tid < RB && 16 * tid < nrows) {
        double S = 0.0, M2 = 0.0;
        for (int w = 0; w < LWAVES; ++w) {
            S += red[w * RB + tid];
            M2 += red2[w * RB + tid];
        }
        double *so = A.st_out + ((size_t)b * A.nst + tile * RB + tid) * 2;
        so[0] = S;
        so[1] = M2;
    }
}

// ------------------------------------------------------------------ pseudo-energy partials
struct EnergyArgs {
    const float *a_in;    // a_17
    const float *x_in;    // x_17
    const double *st_in;  // partials of a_17
    const float *vec;     // b, g, be of layer 17
    float *part;          // [B][ne][128] sums of S^2
    int T, nst, ne;
    float eps;
};

__global__ __launch_bounds__(256) void bl_energy(EnergyArgs A)
{
    __shared__ float4 sm[8][32];
    const int tid = threadIdx.x;
    const int blk = xcd_block();
    const int b = blk / A.ne, et = blk % A.ne;
    const int T = A.T;
    const int r0 = MARGIN + et * MT0, r1 = min(r0 + MT0, T - MARGIN);
    double mean, rstd;
    ln_stats(A.st_in + (size_t)b * A.nst * 2, A.nst, T, A.eps, mean, rstd);
    const int c4 = (tid & 31) * 4;
    const float4 g = *(const float4 *)(A.vec + NF + c4);
    const float4 be = *(const float4 *)(A.vec + 2 * NF + c4);
    const float mu = (float)mean, rs = (float)rstd;
    const float4 sc = make_float4(g.x * rs, g.y * rs, g.z * rs, g.w * rs);
    const size_t fb = (size_t)b * T;
    const float *__restrict__ a_in = A.a_in;
    const float *__restrict__ x_in = A.x_in;
    float4 e = make_float4(0.f, 0.f, 0.f, 0.f);
    constexpr int U = 4;
    for (int tb = r0 + (tid >> 5); tb < r1; tb += 8 * U) {
        float4 av[U], xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = tb + 8 * u;
            const bool ok = t < r1;
            av[u] = ok ? *(const float4 *)(a_in + (fb + t) * NF + c4) : make_float4(0.f, 0.f, 0.f, 0.f);
            xv[u] = ok ? *(const float4 *)(x_in + (fb + t) * NF + c4) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (tb + 8 * u < r1) {
                const float sx = xv[u].x + tanh_fast(fmaf(av[u].x - mu, sc.x, be.x));
                const float sy = xv[u].y + tanh_fast(fmaf(av[u].y - mu, sc.y, be.y));
                const float sz = xv[u].z + tanh_fast(fmaf(av[u].z - mu, sc.z, be.z));
                const float sw = xv[u].w + tanh_fast(fmaf(av[u].w - mu, sc.w, be.w));
                e.x = fmaf(sx, sx, e.x); e.y = fmaf(sy, sy, e.y); e.z = fmaf(sz, sz, e.z); e.w = fmaf(sw, sw, e.w);
            }
    }
    sm[tid >> 5][tid & 31] = e;
    __syncthreads();
    if (tid < 32) {
        float4 t = sm[0][tid];
        for (int i = 1; i < 8; ++i) {
            const float4 u = sm[i][tid];
            t.x += u.x; t.y += u.y; t.z += u.z; t.w += u.w;
        }
        *(float4 *)(A.part + ((size_t)b * A.ne + et) * NF + 4 * tid) = t;
    }
}

// ------------------------------------------------------------------ head
struct HeadArgs {
    const float *part;
    const float *head;  // g_e[128], be_e[128], fc_w[128][n_out], fc_b[n_out]
    float *feat;
    float *out;
    int ne, n_out, n_valid, mode;
    float eps;
};

constexpr int HEAD_SMALL = 16;  // outputs up to which the dot products run on all 128 threads

__global__ __launch_bounds__(128) void bl_head(HeadArgs A)
{
    __shared__ double f[NF];
    __shared__ double o[BL_MAX_NOUT];
    __shared__ double red[2];
    __shared__ double part[2 * HEAD_SMALL];
    const int c = threadIdx.x, b = blockIdx.x;
    const float *W = A.head + 2 * NF;
    const float *bias = W + NF * A.n_out;
    const bool small = A.n_out <= HEAD_SMALL;
    // small heads: thread c holds input channel c's weights, loaded before the reductions
    double wv[HEAD_SMALL];
#pragma unroll
    for (int j = 0; j < HEAD_SMALL; ++j) wv[j] = small && j < A.n_out ? (double)W[c * A.n_out + j] : 0.0;
    double e = 0.0;
#pragma unroll 8
    for (int i = 0; i < A.ne; ++i) e += (double)A.part[((size_t)b * A.ne + i) * NF + c];
    e /= (double)A.n_valid;
    const double mean = block_sum(e, red, 2) / NF;
    const double d = e - mean;
    const double var = block_sum(d * d, red, 2) / NF;
    const double y = d / sqrt(var + (double)A.eps) * (double)A.head[c] + (double)A.head[NF + c];
    const double sel = 1.0507009873554804934 * (y > 0.0 ? y : 1.6732632423543772848 * expm1(y));
    f[c] = sel;
    if (A.feat) A.feat[(size_t)b * NF + c] = (float)sel;
    if (small) {
        // o[j] = bias[j] + sum over c of f[c] W[c][j]: a wave sum per output, then the two waves
#pragma unroll
        for (int j = 0; j < HEAD_SMALL; ++j)
            if (j < A.n_out) {
                const double w = wave_sum(sel * wv[j]);
                if ((c & 63) == 0) part[2 * j + (c >> 6)] = w;
            }
        __syncthreads();
        if (c < A.n_out) o[c] = (double)bias[c] + (part[2 * c] + part[2 * c + 1]);
    } else {
        __syncthreads();
        for (int j = c; j < A.n_out; j += NF) {
            double s = (double)bias[j];
#pragma unroll 16
            for (int k = 0; k < NF; ++k) s += f[k] * (double)W[k * A.n_out + j];
            o[j] = s;
        }
    }
    __syncthreads();
    double mx = -INFINITY;
    for (int j = c; j < A.n_out; j += NF) mx = fmax(mx, o[j]);
    if (A.mode == BL_CLASSIFICATION) {
        mx = wave_max(mx);
        __syncthreads();
        if ((c & 63) == 0) red[c >> 6] = mx;
        __syncthreads();
        mx = fmax(red[0], red[1]);
        double se = 0.0;
        for (int j = c; j < A.n_out; j += NF) {
            o[j] = exp(o[j] - mx);
            se += o[j];
        }
        se = block_sum(se, red, 2);
        for (int j = c; j < A.n_out; j += NF) o[j] /= se;
    }
    for (int j = c; j < A.n_out; j += NF) A.out[(size_t)b * A.n_out + j] = (float)o[j];
}

int layer_lds_bytes(int rb, int D) { return 2 * (16 * rb + 2 * D) * XROW * 2 + 2 * 8 * LWAVES * rb; }

// The layer kernel's LDS can exceed the 64 KB default: raise each form's limit once per
// device (the attribute is per device).  A device reset in the process clears the
// attribute but not this cache; the next launch above 64 KB then fails, and bl_forward
// reports it as ISM_EDEVICE.
int set_layer_lds_limits()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    static std::atomic<unsigned long long> done{0};
    if (dev < 64 && (done.load() >> dev & 1ull)) return 0;
    const void *fn[4] = {(const void *)bl_layer<false, 4>, (const void *)bl_layer<true, 4>,
                         (const void *)bl_layer<true, 2>, (const void *)bl_layer<true, 1>};
    const int rb[4] = {4, 4, 2, 1};
    for (int i = 0; i < 4 && e == hipSuccess; ++i)
        e = hipFuncSetAttribute(fn[i], hipFuncAttributeMaxDynamicSharedMemorySize, layer_lds_bytes(rb[i], MAX_D));
    if (e == hipSuccess && dev < 64) done.fetch_or(1ull << dev);
    return (int)e;
}

}  // namespace

struct bl_model {
    int c_in, n_out, mode;
    float eps;
    void *dev;
    ModelLayout lay;
};

extern "C" size_t bl_param_count(int c_in, int n_out)
{
    if (c_in < 1 || c_in > BL_MAX_CIN || n_out < 1 || n_out > BL_MAX_NOUT) return 0;
    size_t n = 0;
    for (int l = 0; l < NL; ++l) {
        const size_t ci = l == 0 ? c_in : NF;
        n += ci * MULT * 3 + ci * MULT * NF + 3 * NF;
    }
    return n + 2 * NF + (size_t)NF * n_out + n_out;
}

extern "C" int bl_model_create(ism_handle *h, int c_in, int n_out, int mode, float ln_eps, const float *params,
                               ism_stream stream, bl_model **model)
{
    if (!h || !model) return ISM_EINVAL;
    *model = nullptr;
    if (c_in < 1 || c_in > BL_MAX_CIN || n_out < 1 || n_out > BL_MAX_NOUT) {
        ism_set_error(h, "c_in must be in [1, %d] and n_out in [1, %d]", BL_MAX_CIN, BL_MAX_NOUT);
        return ISM_EINVAL;
    }
    if (mode != BL_REGRESSION && mode != BL_CLASSIFICATION) {
        ism_set_error(h, "mode must be BL_REGRESSION or BL_CLASSIFICATION");
        return ISM_EINVAL;
    }
    if (!(ln_eps > 0.f) || !std::isfinite(ln_eps)) {
        ism_set_error(h, "ln_eps must be finite and > 0");
        return ISM_EINVAL;
    }
    if (!params) { ism_set_error(h, "NULL params"); return ISM_EINVAL; }
    bl_model *m = new (std::nothrow) bl_model;
    if (!m) return ISM_ENOMEM;
    m->c_in = c_in;
    m->n_out = n_out;
    m->mode = mode;
    m->eps = ln_eps;
    m->lay = model_layout(c_in, n_out);
    if (hipMalloc(&m->dev, m->lay.total) != hipSuccess) {
        ism_set_error(h, "hipMalloc of %zu bytes for the model failed", m->lay.total);
        delete m;
        return ISM_ENOMEM;
    }
    FoldArgs F;
    int64_t o = 0;
    for (int l = 0; l < NL; ++l) {
        const int64_t ci = l == 0 ? c_in : NF;
        F.po.dw[l] = o; o += ci * MULT * 3;
        F.po.pw[l] = o; o += ci * MULT * NF;
        F.po.b[l] = o; o += NF;
        F.po.g[l] = o; o += NF;
        F.po.be[l] = o; o += NF;
    }
    F.po.g_e = o; o += NF;
    F.po.be_e = o; o += NF;
    F.po.fc_w = o; o += (int64_t)NF * n_out;
    F.po.fc_b = o;
    F.params = params;
    F.c_in = c_in;
    F.n_out = n_out;
    char *base = (char *)m->dev;
    F.hdr = (int *)(base + m->lay.hdr);
    F.w0 = (float *)(base + m->lay.w0);
    F.vec = (float *)(base + m->lay.vec);
    F.frag = (_Float16 *)(base + m->lay.frag);
    F.head = (float *)(base + m->lay.head);
    hipLaunchKernelGGL(bl_fold, dim3(NL + 1), dim3(256), 0, (hipStream_t)stream, F);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        (void)hipFree(m->dev);
        delete m;
        return ism_hip_fail(h, e, "bl_fold launch");
    }
    *model = m;
    return ISM_OK;
}

extern "C" void bl_model_destroy(bl_model *m)
{
    if (!m) return;
    (void)hipDeviceSynchronize();  // forward passes may still read the model
    if (m->dev) (void)hipFree(m->dev);
    delete m;
}

extern "C" size_t bl_workspace_bytes(int batch, int n_t)
{
    if (batch < 0 || n_t < 2 * MARGIN + 1 || n_t > MAX_NT) return 0;
    return ws_layout(CHUNK > 0 && batch > CHUNK ? CHUNK : batch, n_t).total;
}

// The forward pass over `batch` frames, `chunk` frames per pass through the layers, with the
// workspace laid out for `chunk` frames (arguments already checked).
static int forward_impl(ism_handle *h, const bl_model *m, int batch, int chunk, int n_t, const float *x,
                        const int64_t *x_offsets, int64_t ex_stride, int64_t ch_stride, void *workspace,
                        float *features, float *out, ism_stream stream)
{
    const WsLayout w = ws_layout(chunk, n_t);
    if ((int64_t)chunk * w.nst > 0x7fffffff) { ism_set_error(h, "batch too large"); return ISM_EINVAL; }
    const int ea = set_layer_lds_limits();
    if (ea != 0) return ism_hip_fail(h, (hipError_t)ea, "hipFuncSetAttribute");
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    const char *mb = (const char *)m->dev;
    float *Abuf[2] = {(float *)(ws + w.a[0]), (float *)(ws + w.a[1])};
    float *Xbuf[2] = {(float *)(ws + w.x[0]), (float *)(ws + w.x[1])};
    double *Sbuf[2] = {(double *)(ws + w.st[0]), (double *)(ws + w.st[1])};
    const float *vec = (const float *)(mb + m->lay.vec);
    for (int c0 = 0; c0 < batch; c0 += chunk) {
        const int nb = batch - c0 < chunk ? batch - c0 : chunk;
        const int nt0 = cdiv(n_t, MT0);
        // Tile height of layers 1..17: the tallest whose grid still fits one workgroup per
        // CU takes the low-latency form; larger batches take 64-row tiles at full occupancy.
        int rb = 4;
        bool lowlat = false;
        for (int r = 1; r <= 4; r *= 2)
            if ((int64_t)nb * cdiv(n_t, 16 * r) <= h->n_cu) {
                rb = r;
                lowlat = true;
                break;
            }

        Layer0Args L0;
        L0.x = x;
        L0.offs = x_offsets ? x_offsets + c0 : nullptr;
        L0.base = (int64_t)c0 * ex_stride;
        L0.ex_stride = ex_stride;
        L0.ch_stride = ch_stride;
        L0.w0 = (const float *)(mb + m->lay.w0);
        L0.bias = vec;
        L0.a_out = Abuf[0];
        L0.st_out = Sbuf[0];
        L0.T = n_t;
        L0.ntiles = nt0;
        L0.nst = w.nst;
        L0.c_in = m->c_in;
        const int l0_lds = (m->c_in * L0XP + 3 * m->c_in * NF) * 4 + 2 * 8 * (L0THREADS / 64);
        hipLaunchKernelGGL(bl_layer0, dim3(nb * nt0), dim3(L0THREADS), l0_lds, st, L0);

        for (int l = 1; l < NL; ++l) {
            LayerArgs L;
            L.a_in = Abuf[(l - 1) & 1];
            L.x_in = Xbuf[(l - 1) & 1];
            L.x_out = Xbuf[l & 1];
            L.a_out = Abuf[l & 1];
            L.st_in = Sbuf[(l - 1) & 1];
            L.st_out = Sbuf[l & 1];
            L.vec_prev = vec + (size_t)(l - 1) * 3 * NF;
            L.bias = vec + (size_t)l * 3 * NF;
            L.frag = (const _Float16 *)(mb + m->lay.frag) + (size_t)(l - 1) * FRAG_HALVES;
            L.hdr = (const int *)(mb + m->lay.hdr);
            L.T = n_t;
            L.ntiles = cdiv(n_t, 16 * rb);
            L.nst = w.nst;
            L.layer = l;
            L.D = 1 << (l % 6);
            L.eps = m->eps;
            const dim3 grid(nb * L.ntiles), blk(LTHREADS);
            const int lds = layer_lds_bytes(rb, L.D);
            if (!lowlat) hipLaunchKernelGGL((bl_layer<false, 4>), grid, blk, lds, st, L);
            else if (rb == 4) hipLaunchKernelGGL((bl_layer<true, 4>), grid, blk, lds, st, L);
            else if (rb == 2) hipLaunchKernelGGL((bl_layer<true, 2>), grid, blk, lds, st, L);
            else hipLaunchKernelGGL((bl_layer<true, 1>), grid, blk, lds, st, L);
        }

        EnergyArgs E;
        E.a_in = Abuf[(NL - 1) & 1];
        E.x_in = Xbuf[(NL - 1) & 1];
        E.st_in = Sbuf[(NL - 1) & 1];
        E.vec = vec + (size_t)(NL - 1) * 3 * NF;
        E.part = (float *)(ws + w.part);
        E.T = n_t;
        E.nst = w.nst;
        E.ne = w.ne;
        E.eps = m->eps;
        hipLaunchKernelGGL(bl_energy, dim3(nb * w.ne), dim3(256), 0, st, E);

        HeadArgs Hd;
        Hd.part = E.part;
        Hd.head = (const float *)(mb + m->lay.head);
        Hd.feat = features ? features + (size_t)c0 * NF : nullptr;
        Hd.out = out + (size_t)c0 * m->n_out;
        Hd.ne = w.ne;
        Hd.n_out = m->n_out;
        Hd.n_valid = n_t - 2 * MARGIN;
        Hd.mode = m->mode;
        Hd.eps = m->eps;
        hipLaunchKernelGGL(bl_head, dim3(nb), dim3(128), 0, st, Hd);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ism_hip_fail(h, e, "bl_forward launch");
    return ISM_OK;
}

static int check_forward_args(ism_handle *h, const bl_model *m, int batch, int n_t, int64_t ex_stride,
                              int64_t ch_stride)
{
    if (!m) { ism_set_error(h, "NULL model"); return ISM_EINVAL; }
    if (batch < 0) { ism_set_error(h, "batch must be >= 0"); return ISM_EINVAL; }
    if (n_t < 2 * MARGIN + 1 || n_t > MAX_NT) {
        ism_set_error(h, "n_t must be in [%d, %d]", 2 * MARGIN + 1, MAX_NT);
        return ISM_EINVAL;
    }
    if (ex_stride < 0 || ch_stride < 0) { ism_set_error(h, "strides must be >= 0"); return ISM_EINVAL; }
    return ISM_OK;
}

extern "C" int bl_forward(ism_handle *h, const bl_model *m, int batch, int n_t, const float *x,
                          const int64_t *x_offsets, int64_t ex_stride, int64_t ch_stride, void *workspace,
                          size_t workspace_bytes, float *features, float *out, ism_stream stream)
{
    if (!h) return ISM_EINVAL;
    int rc = check_forward_args(h, m, batch, n_t, ex_stride, ch_stride);
    if (rc) return rc;
    if (batch == 0) return ISM_OK;
    if (!x || !workspace || !out) { ism_set_error(h, "NULL argument"); return ISM_EINVAL; }
    const int chunk = CHUNK > 0 && batch > CHUNK ? CHUNK : batch;
    const size_t need = ws_layout(chunk, n_t).total;
    if (workspace_bytes < need) {
        ism_set_error(h, "workspace of %zu bytes, %zu needed", workspace_bytes, need);
        return ISM_EINVAL;
    }
    return forward_impl(h, m, batch, chunk, n_t, x, x_offsets, ex_stride, ch_stride, workspace, features, out,
                        stream);
}

// ------------------------------------------------------------------ form without allocation
// The workspace of bl_forward_noalloc: one file-scope device array per GPU, held until the
// process ends.  Host code never passes the array's name to a kernel (in host code it is a
// stand-in, not a device address): the entry point takes the device address of its copy
// from hipGetSymbolAddress once per device, with that device current, and uses only that.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::atomic<void *> g_scratch_addr[kMaxDevices];

static int scratch_address(ism_handle *h, void **p)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return ism_hip_fail(h, e, "hipGetDevice");
    if (dev != h->device) {
        ism_set_error(h, "call with the handle's device (%d) current, not %d", h->device, dev);
        return ISM_EINVAL;
    }
    if (dev < 0 || dev >= kMaxDevices) { ism_set_error(h, "device index %d out of range", dev); return ISM_EINVAL; }
    void *a = g_scratch_addr[dev].load(std::memory_order_acquire);
    if (!a) {   // a race between threads only repeats the same query
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !a) return ism_hip_fail(h, e == hipSuccess ? hipErrorInvalidSymbol : e,
                                                       "hipGetSymbolAddress of the workspace array");
        g_scratch_addr[dev].store(a, std::memory_order_release);
    }
    *p = a;
    return ISM_OK;
}

extern "C" size_t bl_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int bl_forward_noalloc(ism_handle *h, const bl_model *m, int batch, int n_t, const float *x,
                                  const int64_t *x_offsets, int64_t ex_stride, int64_t ch_stride,
                                  float *features, float *out, ism_stream stream)
{
    if (!h) return ISM_EINVAL;
    h->last_error.clear();
    int rc = check_forward_args(h, m, batch, n_t, ex_stride, ch_stride);
    if (rc) return rc;
    if (batch == 0) return ISM_OK;
    if (!x || !out) { ism_set_error(h, "NULL argument"); return ISM_EINVAL; }
    if (h->device < 0) { ism_set_error(h, "no HIP device"); return ISM_EDEVICE; }
    // frames per pass: as many as the array holds (the results do not depend on it)
    if (ws_layout(1, n_t).total > kScratchBytes) {
        ism_set_error(h, "one frame of %d samples needs %zu bytes of workspace, more than the %zu of the "
                      "no-allocation form (at most about %d samples)", n_t, ws_layout(1, n_t).total, kScratchBytes,
                      (int)(kScratchBytes / ws_layout(1, 1024).total * 1024));
        return ISM_EINVAL;
    }
    int chunk = (int)std::min<size_t>((size_t)batch, kScratchBytes / ws_layout(1, n_t).total);
    while (chunk > 1 && ws_layout(chunk, n_t).total > kScratchBytes) --chunk;
    void *ws = nullptr;
    if ((rc = scratch_address(h, &ws))) return rc;
    return forward_impl(h, m, batch, chunk, n_t, x, x_offsets, ex_stride, ch_stride, ws, features, out, stream);
}
