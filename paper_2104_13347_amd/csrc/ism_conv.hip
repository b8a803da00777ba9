// Source convolution + sensor noise for a batch of rooms (paper section III.A:
// the multichannel RIRs are convolved with source signals, then Gaussian noise
// at a drawn SNR is added).
//
//   y[r][m][n] = sum_{j <= min(n, L_r - 1)} h[r][m][j] x[r][n - j],  n < out_len
//   y += sigma_r z,  sigma_r^2 = mean_{m,n} y^2 * 10^(-snr_r / 10)
//
// MFMA path (block-Toeplitz GEMM, BF16 inputs, FP32 accumulation).  With
// 32-sample output blocks t and 32-tap RIR blocks b,
//   Y_t (32 x M) = sum_s T_s (32 x 32) H_{t-s} (32 x M),  T_s[i][j] = x[32 s + i - j].
// T_s depends on s only, so one workgroup (one wave) keeps 16 output blocks x 8
// microphones = 128 columns (four 32-column MFMA tiles sharing every A operand) and
// walks s.  Per s: A = T_s from a 128-sample source ring in LDS (BF16, reversed and
// stored twice, so each lane's eight K values are consecutive there, plus a copy one
// entry later, so they start on a 4-byte boundary of one of the two: four dword reads),
// the ring gaining one 32-sample block per step;
// B = the RIR blocks b = t - s from a 16-slot LDS ring that gains one block per
// step, of which three tiles' operands carry over from the previous step in
// registers; eight v_mfma_f32_32x32x16_bf16, issued while the next step's operands
// are read (software pipeline).  MACs on zeros: the Toeplitz triangles of a tile's
// first and last 15 steps (where t - s leaves [0, nb)) and up to three padding
// steps, about 12 % of the products on a workload of 1 s sources.
//
// FP32 path: direct convolution on the vector units (register-blocked, four
// outputs per lane, RIR chunks and the matching source window staged in LDS).
//
// Noise: every output tile writes the sum of y^2 of its samples (FP64,
// fixed-order wave reduction); the noise kernel adds those partial sums in a fixed
// order for its room, derives sigma, and adds sigma * z.  z is either supplied by
// the caller or drawn inside the noise pass from a counter-based generator
// (Philox4x32-10 and the Box-Muller transform), so the seeded form reads y once,
// writes it once and reads no deviates from memory.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/ism.h"
#include "ism_host.h"

namespace ism {

#define DEV __device__ __forceinline__

struct alignas(16) ConvRoom {
    int64_t rir_off;   // FP32 RIRs: rirs[rir_off + m * rir_len + j]
    int64_t h_off;     // BF16 padded RIRs: hb[h_off + m * nb * 32 + j]
    int32_t rir_len;
    int32_t nb;        // ceil(rir_len / 32)
    float snr_db;
    int32_t order;     // grid row j of the convolution kernels takes room rooms[j].order
                       // (rooms by decreasing RIR length, so the longest start first)
    double nscale;     // 10^(-snr_db / 10), FP64, from the host
};

// Two slots used in turn: a call waits only for the call before the previous one, so the
// host work of a call (room table, upload, launches) overlaps the kernels of the last.
struct ConvSlot {
    void *ws = nullptr;       // device: BF16 RIRs | tile power sums | room table
    size_t cap = 0;
    void *stage = nullptr;    // pinned staging for the room table
    size_t stage_cap = 0;
    hipEvent_t ev = nullptr;  // end of the last call's kernels that used this slot
    bool used = false;
    hipEvent_t tev[4] = {};   // with kernel timing on: before pack, convolution, noise, and after
    bool timed = false;       // the last call on this slot recorded tev
    bool noise = false;       // ... and had a noise pass
};
struct ConvState {
    ConvSlot slot[2];
    int next = 0;
    bool timing = false;
    int last = -1;            // slot of the last call
};

constexpr int CB = 32;            // block length (samples / taps)
#ifndef CONV_CG
#define CONV_CG 16
#endif
constexpr int CG = CONV_CG;       // output blocks per MFMA workgroup
constexpr int CTILE = CB * CG;    // output samples per workgroup
constexpr int NT = CG / 4;        // 32-column MFMA tiles per workgroup (4 blocks x 8 microphones)
constexpr int LNT = NT == 2 ? 1 : NT == 4 ? 2 : 3;
constexpr int UN = NT > 4 ? NT : 4;   // steps per loop group: a multiple of NT and of 4
static_assert(NT == 2 || NT == 4 || NT == 8, "CG must be 8, 16 or 32");
constexpr int CM = 8;             // microphones per room on the MFMA path

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

DEV uint16_t f2bf(float f)
{   // round to nearest even: gfx950's v_cvt_pk_bf16_f32 (one instruction)
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

// ------------------------------------------------------------------ RIRs -> padded BF16
// grid (chunks, rooms, M), 256 threads of 4 consecutive taps each (one 8-byte store; a
// microphone's padded row starts 64-byte aligned)
__global__ __launch_bounds__(256) void conv_pack_h(const float *__restrict__ rirs,
                                                   const ConvRoom *__restrict__ rooms,
                                                   uint16_t *__restrict__ hb)
{
    const int r = blockIdx.y, m = blockIdx.z;
    const ConvRoom R = rooms[r];
    const int n = R.nb * CB;
    const float *src = rirs + R.rir_off + (int64_t)m * R.rir_len;
    uint16_t *dst = hb + R.h_off + (int64_t)m * n;
    for (int j = 4 * (blockIdx.x * blockDim.x + threadIdx.x); j < n; j += 4 * gridDim.x * blockDim.x) {
        uint32_t w[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const uint32_t lo = j + 2 * q < R.rir_len ? f2bf(src[j + 2 * q]) : 0u;
            const uint32_t hi = j + 2 * q + 1 < R.rir_len ? f2bf(src[j + 2 * q + 1]) : 0u;
            w[q] = lo | (hi << 16);
        }
        *(uint2 *)(dst + j) = make_uint2(w[0], w[1]);
    }
}

// ------------------------------------------------------------------ MFMA block-Toeplitz
// grid (tiles, rooms), one wave.  LDS: a 128-sample source ring (BF16, reversed,
// stored twice so that any 8-sample window is contiguous, and a copy shifted by one
// entry) and a CG-slot RIR ring.
constexpr int XR = 128;   // source ring length (samples)
constexpr int kBufWord3 = 0x00020000;   // buffer descriptor word 3 (gfx9 family: raw 32-bit data)
// RIR ring: two halves (taps 0-15 and 16-31 of a block), each CG x 8 rows (a slot per block,
// 8 microphones) of two 16-byte chunks.  Chunk c of the row of block b sits at position
// c ^ ((b / NT) & 1): the 16 rows that 16 lanes of a read instruction touch (blocks b and
// b + NT, 8 microphones each) fill all 16 chunk positions of 256 bytes, so the reads have no
// bank conflicts and the ring needs no padding.
constexpr int CRH = CG * CM * 16;   // one half (u16): CG slots
DEV int ring_pos(int b, int m, int c) { return ((b & (CG - 1)) * CM + m) * 16 + 8 * (c ^ ((b >> LNT) & 1)); }

// Registers: the software pipeline keeps two steps' operands live (accumulators 16 NT, B
// operands 8 NT + 8, A operands 2 x 8, prefetch queue 12): 3 waves per SIMD for 16 blocks.
#ifndef CONV_MW
#define CONV_MW 3
#endif
__global__ __launch_bounds__(64, CONV_MW) void conv_mfma(const float *__restrict__ x, int src_len, int out_len,
                                                const uint16_t *__restrict__ hb,
                                                const ConvRoom *__restrict__ rooms,
                                                float *__restrict__ y, double *__restrict__ psum,
                                                int tiles_per_room)
{
    // source ring (below) and its copy one entry later, so that a fragment starting at an
    // odd entry starts on a 4-byte boundary of the copy; the copy starts 160 dwords after
    // the ring, so dword d of either sits in banks d and d + 32 (mod 64): the two dword
    // ranges a read instruction touches (about 20 dwords each) never share a bank
    __shared__ __attribute__((aligned(16))) uint16_t xrings[2 * XR + 64 + 2 * XR + 8];
    uint16_t *const xring = xrings, *const xring1 = xrings + 2 * XR + 64;
    __shared__ __attribute__((aligned(16))) uint16_t ring[2 * CRH];
    const int lane = threadIdx.x;
    // Workgroups are dealt to the 8 XCDs round-robin in launch order, and each XCD has
    // its own L2.  With the room count a multiple of 8, the k-th workgroup on XCD x takes
    // tile k mod T of room row x + 8 (k / T): all tiles of a room share one L2, and the
    // XCDs still take the rooms longest-first.
    int row = blockIdx.y, tile = blockIdx.x;
    if ((gridDim.y & 7) == 0) {
        const int L = blockIdx.x + gridDim.x * blockIdx.y;
        const int x = L & 7, k = L >> 3;
        row = x + 8 * (k / (int)gridDim.x);
        tile = k % (int)gridDim.x;
    }
    const int r = rooms[row].order;
    const int t0 = tile * CG;
    const ConvRoom R = rooms[r];
    const int nb = R.nb;
    const int s_end = t0 + CG - 1;
    // Steps s_start .. s_end, with s_start moved down so that s_end - s_start is a multiple
    // of UN (whole groups below; up to UN - 1 extra steps, whose source samples before 0 or
    // RIR blocks past nb read as zeros).
    const int s_start = s_end - UN * ((s_end - max(0, t0 - nb + 1) + UN - 1) / UN);
    // The source and the RIR blocks of the room are read through buffer descriptors: a read
    // outside the buffer returns zero, which is the zero padding of both signals (samples
    // before 0 or past the end, blocks outside [0, nb)), with no clamp or select.
    const __amdgpu_buffer_rsrc_t xrs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(x + (int64_t)r * src_len), (short)0, src_len * 4, kBufWord3);
    const __amdgpu_buffer_rsrc_t hrs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(hb + R.h_off), (short)0, CM * nb * CB * 2, kBufWord3);
    auto load_x = [&](int sb) -> float {           // lane covers sample 32 sb + lane % 32
        const int X = CB * sb + (lane & 31);    // X < 0: a byte offset of 2^32 - 4|X|, outside
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(xrs, X * 4, 0, 0));
    };
    // source ring: sample X sits at (-X) mod 128 and again 128 entries later, so that any
    // 8 consecutive samples read downwards in time are contiguous
    auto store_x = [&](int sb, float v) {
        if (lane < 32) {
            const int X = CB * sb + lane;
            const uint16_t bv = f2bf(v);
            const int p = (-X) & (XR - 1);
            xring[p] = bv;
            xring[p + XR] = bv;
            xring1[p + 1] = bv;
            xring1[p + 1 + XR] = bv;
        }
    };
    // RIR ring: slot (b mod CG) holds block b of all microphones (zeros outside [0, nb));
    // lane covers 4 taps: mic = lane / 8, taps (lane % 8) * 4 .. + 3
    const int hlane = ((lane >> 3) * nb * CB + (lane & 7) * 4) * 2;   // byte offset in block 0
    auto load_block = [&](int b) -> uint2 {
        const int off = (b >= 0 && b < nb) ? b * CB * 2 : (1 << 30);   // (1 << 30): outside
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(hrs, hlane + off, 0, 0);
        return make_uint2(v[0], v[1]);
    };
    auto store_block = [&](int b, uint2 v) {
        const int k = (lane & 7) * 4;   // first tap
        *(uint2 *)(ring + (k >> 4) * CRH + ring_pos(b, lane >> 3, (k >> 3) & 1) + (k & 7)) = v;
    };
    {
        float x0[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) x0[j] = load_x(s_start - 2 + j);
#pragma unroll
        for (int j = 0; j < 3; ++j) store_x(s_start - 2 + j, x0[j]);
#pragma unroll
        for (int g = 0; g < CG; g += 8) {   // the first CG blocks, eight at a time
            uint2 h0[8];
#pragma unroll
            for (int tl = 0; tl < 8; ++tl) h0[tl] = load_block(t0 - s_start + g + tl);
#pragma unroll
            for (int tl = 0; tl < 8; ++tl) store_block(t0 - s_start + g + tl, h0[tl]);
        }
    }
    // prefetch queue: the blocks entering the rings at step u sit in slot (u - s_start - 1) % PD
#ifndef CONV_PD
#define CONV_PD 4
#endif
    constexpr int PD = CONV_PD;   // steps of global prefetch (2 or 4)
    float xq[PD];
    uint2 hq[PD];
#pragma unroll
    for (int j = 0; j < PD; ++j) {
        xq[j] = load_x(s_start + 1 + j);
        hq[j] = load_block(t0 - s_start - 1 - j);
    }
    __syncthreads();

    f32x16_t acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
        for (int q = 0; q < 16; ++q) acc[nt][q] = 0.0f;

    const int i = lane & 31;           // A row / B column within a tile
    const int kk0 = (lane >> 5) * 8;   // first K index of this lane's eight
    const uint32_t *xr32 = (const uint32_t *)xring, *xr32s = (const uint32_t *)xring1;
    // one step: Y_t += T_s H_{t - s} for the CG output blocks t0 .. t0 + CG - 1.  The A
    // fragments of T_s are x[X - e], X = 32 s + i - 16 ks - kk0, e = 0..7: ring entry
    // p = (-X) mod 128 for ks = 0 and p + 16 for ks = 1 (the ring is stored twice, so no
    // wrap); read as four dwords from the ring (p even) or its shifted copy (p odd).
    // B operand: column i of MFMA tile nt is output block tl = NT (i / 8) + nt of microphone
    // i % 8, so from one step to the next the operand of tile nt is the previous step's
    // operand of tile nt - 1 (the same registers): each step reads only tile 0's operand,
    // blocks t0 - s + NT k (k = 0..3), from the ring.  bq slot (nt - ph) mod NT holds tile
    // nt's operand at phase ph = (s - s_start) mod NT (a constant in the unrolled loop).
    u32x4_t bq[2][NT];
    auto read_b = [&](int s, int nt, u32x4_t &b0, u32x4_t &b1) {
        const int b = t0 + (i >> 3) * NT + nt - s;
        const uint16_t *bp = ring + ring_pos(b, i & 7, kk0 >> 3);
        b0 = *(const u32x4_t *)bp;
        b1 = *(const u32x4_t *)(bp + CRH);
    };
    // A operand of step s: the Toeplitz fragments starting at ring entry p, read as four
    // dwords from the ring (p even) or from its copy one entry later (p odd)
    auto read_a = [&](int p, bf16x8_t (&a)[2]) {
        const uint32_t *src = (p & 1) ? xr32s + ((p + 1) >> 1) : xr32 + (p >> 1);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            u32x4_t v;
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = src[8 * ks + k];
            a[ks] = __builtin_bit_cast(bf16x8_t, v);
        }
    };
    // the products of one step; K step outermost: the four tiles' MFMAs are independent
    auto mma = [&](const bf16x8_t (&a)[2], int ph) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    a[ks], __builtin_bit_cast(bf16x8_t, bq[ks][(nt - ph) & (NT - 1)]), acc[nt], 0, 0, 0);
    };
    auto ring_entry = [&](int s) { return (-(CB * s + i - kk0)) & (XR - 1); };
    // Step u = s_start + 1 + 4 k + j enters source block u at ring entry (-32 u - lane) mod 128
    // and reads T_u from entry (-(32 u + i - kk0)) mod 128: both depend on j mod 4 only (four
    // steps make one lap of the ring), so they are computed once.  Lanes below 32 store, and for
    // them the two entries coincide.
    const int p1 = ring_entry(s_start + 1);
    // Software pipeline: step u's ring entries are written and its operands read before the
    // products of step u - 1 are issued, so the LDS reads run under those products.
    bf16x8_t a_cur[2];
    auto advance = [&](int u, int j) {   // u = s_start + 1 + UN k + j
        const int q = j & (PD - 1);   // prefetch slot
        const int pe = (p1 - CB * (j & 3)) & (XR - 1);   // ring entry of step u
        __syncthreads();   // the ring reads of step u - 1 precede these writes
        store_block(t0 - u, hq[q]);
        if (lane < 32) {
            const uint16_t bv = f2bf(xq[q]);
            xring[pe] = bv;
            xring[pe + XR] = bv;
            xring1[pe + 1] = bv;
            xring1[pe + 1 + XR] = bv;
        }
        hq[q] = load_block(t0 - u - PD);
        xq[q] = load_x(u + PD);
        __syncthreads();
        bf16x8_t a_nx[2];
        u32x4_t bn0, bn1;
        read_a(pe, a_nx);
        read_b(u, 0, bn0, bn1);
        mma(a_cur, j & (NT - 1));   // step u - 1: (u - 1 - s_start) mod NT = j mod NT
        const int sl = (-(1 + j)) & (NT - 1);   // tile 0's slot at step u
        bq[0][sl] = bn0;
        bq[1][sl] = bn1;
        a_cur[0] = a_nx[0];
        a_cur[1] = a_nx[1];
    };
    {
        const int p0 = ring_entry(s_start);
        read_a(p0, a_cur);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) read_b(s_start, nt, bq[0][nt], bq[1][nt]);
    }
    for (int u0 = s_start + 1; u0 <= s_end; u0 += UN) {
#pragma unroll
        for (int j = 0; j < UN; ++j) advance(u0 + j, j);
    }
    mma(a_cur, 0);   // step s_end: (s_end - s_start) mod NT = 0

    // store: register q of tile nt holds row 8 (q / 4) + 4 (lane / 32) + (q % 4), column lane % 32
    double pw = 0.0;
    float *yr = y + (int64_t)r * CM * out_len;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int tl = (i >> 3) * NT + nt, m = i & 7;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int row = 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
            const int n = CB * (t0 + tl) + row;
            if (n < out_len) {
                const float v = acc[nt][q];
                yr[(int64_t)m * out_len + n] = v;
                pw += (double)v * (double)v;
            }
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) pw += __shfl_xor(pw, d, 64);
    if (lane == 0) psum[(int64_t)r * tiles_per_room + tile] = pw;
}

// ------------------------------------------------------------------ FP32 direct
// grid (tiles of 1024 outputs, M, rooms), 256 threads x 4 outputs; RIR chunks of 256 taps.
constexpr int DT = 1024, DJ = 256;

__global__ __launch_bounds__(256) void conv_direct(const float *__restrict__ rirs, const ConvRoom *__restrict__ rooms,
                                                   const float *__restrict__ x, int src_len, int out_len, int M,
                                                   float *__restrict__ y, double *__restrict__ psum,
                                                   int tiles_per_room)
{
    __shared__ float hs[DJ];
    __shared__ float xw[DT + DJ + 4];
    const int tid = threadIdx.x;
    const int tile = blockIdx.x, m = blockIdx.y, r = rooms[blockIdx.z].order;
    const ConvRoom R = rooms[r];
    const float *h = rirs + R.rir_off + (int64_t)m * R.rir_len;
    const float *xs = x + (int64_t)r * src_len;
    const int n0 = tile * DT;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    const int jmax = min(R.rir_len, n0 + DT);   // taps beyond the last output are never used
    for (int j0 = 0; j0 < jmax; j0 += DJ) {
        __syncthreads();
        hs[tid] = (j0 + tid < R.rir_len) ? h[j0 + tid] : 0.0f;
        // window: xw[q] = x[n0 - j0 - DJ + q], q in [0, DT + DJ)
        for (int q = tid; q < DT + DJ + 4; q += 256) {
            const int xi = n0 - j0 - DJ + q;
            xw[q] = (q < DT + DJ && xi >= 0 && xi < src_len) ? xs[xi] : 0.0f;
        }
        __syncthreads();
        // output n = n0 + 4 tid + u needs x[n - j] = xw[4 tid + u + DJ - jj] for j = j0 + jj
        const int base = 4 * tid + DJ;
        float x0 = xw[base + 0], x1 = xw[base + 1], x2 = xw[base + 2], x3 = xw[base + 3];
#pragma unroll 8
        for (int jj = 0; jj < DJ; ++jj) {
            const float hv = hs[jj];
            acc[0] = fmaf(hv, x0, acc[0]);
            acc[1] = fmaf(hv, x1, acc[1]);
            acc[2] = fmaf(hv, x2, acc[2]);
            acc[3] = fmaf(hv, x3, acc[3]);
            x3 = x2; x2 = x1; x1 = x0;
            x0 = xw[base - jj - 1];
        }
    }
    double pw = 0.0;
    float *yo = y + ((int64_t)r * M + m) * out_len;
    for (int u = 0; u < 4; ++u) {
        const int n = n0 + 4 * tid + u;
        if (n < out_len) {
            yo[n] = acc[u];
            pw += (double)acc[u] * (double)acc[u];
        }
    }
    // fixed-order block reduction
    __shared__ double red[256];
    red[tid] = pw;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) psum[((int64_t)r * M + m) * tiles_per_room + tile] = red[0];
}

// ------------------------------------------------------------------ seeded deviates
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds on a 128-bit
// counter under a 64-bit key.  Each round takes the two 64-bit products
// w0 * 0xD2511F53 and w2 * 0xCD9E8D57 and forms (hi2 ^ w1 ^ k0, lo2, hi0 ^ w3 ^ k1,
// lo0); the key is advanced by the Weyl increments 0x9E3779B9, 0xBB67AE85 after each
// round (the bump after the tenth round is never used).
DEV uint4 philox4x32_10(uint4 w, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // each 64-bit product (high and low words) is one v_mad_u64_u32
        const uint64_t p0 = (uint64_t)w.x * 0xD2511F53u, p2 = (uint64_t)w.z * 0xCD9E8D57u;
        w = make_uint4((uint32_t)(p2 >> 32) ^ w.y ^ k0, (uint32_t)p2, (uint32_t)(p0 >> 32) ^ w.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return w;
}

// Box and Muller (1958): uniforms u1, u2 in (0, 1) give the independent standard
// normals sqrt(-2 ln u1) cos(2 pi u2) and sqrt(-2 ln u1) sin(2 pi u2).  A 32-bit word
// x becomes the uniform ((x >> 9) + 1/2) 2^-23 (exact in FP32), so |z| <= sqrt(48 ln 2).
// The hardware's log2, square root, sine and cosine (the last two take turns, not
// radians) on these 2^23 possible uniforms: over all of them, the radius
// sqrt(-2 ln 2 log2 u1) is within 4.9e-7 of its exact value and the sine and cosine
// within 1.3e-7, so a deviate is within 1.3e-6.
DEV float2 box_muller(uint32_t a, uint32_t b)
{
    const float u1 = ((float)(a >> 9) + 0.5f) * 0x1p-23f;
    const float u2 = ((float)(b >> 9) + 0.5f) * 0x1p-23f;
    const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
    return make_float2(rad * __builtin_amdgcn_cosf(u2), rad * __builtin_amdgcn_sinf(u2));
}

// The four deviates of samples 4j .. 4j+3 of room r, microphone m (the counter layout
// of ism_normal_deviates): counter (j, m, r, 0); words (x0, x1) give samples 4j, 4j+1,
// (x2, x3) samples 4j+2, 4j+3.
DEV float4 deviates4(uint32_t j, uint32_t m, uint32_t r, uint32_t k0, uint32_t k1)
{
    const uint4 w = philox4x32_10(make_uint4(j, m, r, 0u), k0, k1);
    const float2 a = box_muller(w.x, w.y), b = box_muller(w.z, w.w);
    return make_float4(a.x, a.y, b.x, b.y);
}

// grid (chunks, rooms): z[r][m][n] for n < n_samples
__global__ __launch_bounds__(256) void normal_deviates_kernel(float *__restrict__ z, int M, int n_samples,
                                                              uint32_t k0, uint32_t k1)
{
    const int r = blockIdx.y;
    const int nq = (n_samples + 3) >> 2;
    float *zr = z + (int64_t)r * M * n_samples;
    const bool vec = (n_samples & 3) == 0 && ((uintptr_t)z & 15) == 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (int64_t)M * nq;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(t / nq), j = (int)(t - (int64_t)m * nq);
        const float4 d = deviates4((uint32_t)j, (uint32_t)m, (uint32_t)r, k0, k1);
        float *p = zr + (int64_t)m * n_samples + 4 * j;
        if (vec) {
            *(float4 *)p = d;
        } else {
            const float e[4] = {d.x, d.y, d.z, d.w};
            for (int q = 0; q < 4 && 4 * j + q < n_samples; ++q) p[q] = e[q];
        }
    }
}

// per-room noise scale from the convolution's partial power sums (fixed order)
// sigma_r = sqrt(mean of y^2 over the room x 10^(-snr/10)), by the first wave of a block (all
// 64 lanes): lane k adds parts k, k + 64, ... in order, then a fixed shuffle reduction; lane
// 0 writes the result.
DEV void room_sigma(const double *__restrict__ psum, int r, int n_parts, int64_t per_room, double nscale,
                    float *sigma)
{
    const int lane = threadIdx.x;
    double P = 0.0;
    for (int k = lane; k < n_parts; k += 64) P += psum[(int64_t)r * n_parts + k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) P += __shfl_xor(P, d, 64);
    if (lane == 0) *sigma = (float)sqrt(P / (double)per_room * nscale);
}

// grid (chunks, rooms): y += sigma_r z with z drawn here (one Philox call per 4 samples).
// Each thread takes kNoiseQ groups of 4 samples per pass: their loads are issued first, the
// deviates computed while they are in flight, and the room's sigma (thread 0) is awaited
// only before the stores.
constexpr int kNoiseQ = 2;
__global__ __launch_bounds__(256) void conv_noise_seeded(float *__restrict__ y, const double *__restrict__ psum,
                                                         const ConvRoom *__restrict__ rooms, int n_parts, int M,
                                                         int out_len, uint32_t k0, uint32_t k1)
{
    const int r = blockIdx.y;
    __shared__ float sigma_s;
    const int nq = (out_len + 3) >> 2;
    const int64_t nall = (int64_t)M * nq;
    float *yr = y + (int64_t)r * M * out_len;
    const bool vec = (out_len & 3) == 0 && ((uintptr_t)y & 15) == 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool have_sigma = false;
    float sg = 0.0f;
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t0 - (int64_t)threadIdx.x < nall;
         t0 += stride * kNoiseQ) {
        float4 v[kNoiseQ], d[kNoiseQ];
        float *pq[kNoiseQ];
        int jq[kNoiseQ];
#pragma unroll
        for (int u = 0; u < kNoiseQ; ++u) {
            const int64_t t = t0 + u * stride;
            const int64_t tc = t < nall ? t : nall - 1;   // clamped: always a valid group
            const int m = (int)(tc / nq), j = (int)(tc - (int64_t)m * nq);
            jq[u] = t < nall ? j : -1;
            pq[u] = yr + (int64_t)m * out_len + 4 * j;
            if (vec) v[u] = *(const float4 *)pq[u];
            d[u] = deviates4((uint32_t)j, (uint32_t)m, (uint32_t)r, k0, k1);
        }
        if (!have_sigma) {   // once per block, after its first loads are in flight
            if (threadIdx.x < 64) room_sigma(psum, r, n_parts, (int64_t)M * out_len, rooms[r].nscale, &sigma_s);
            __syncthreads();
            sg = sigma_s;
            have_sigma = true;
        }
#pragma unroll
        for (int u = 0; u < kNoiseQ; ++u) {
            if (jq[u] < 0) continue;
            float *p = pq[u];
            if (vec) {
                float4 w = v[u];
                w.x = fmaf(sg, d[u].x, w.x);
                w.y = fmaf(sg, d[u].y, w.y);
                w.z = fmaf(sg, d[u].z, w.z);
                w.w = fmaf(sg, d[u].w, w.w);
                *(float4 *)p = w;
            } else {
                const float e[4] = {d[u].x, d[u].y, d[u].z, d[u].w};
                for (int q = 0; q < 4 && 4 * jq[u] + q < out_len; ++q) p[q] = fmaf(sg, e[q], p[q]);
            }
        }
    }
}

// ------------------------------------------------------------------ noise (caller's deviates)
// grid (chunks, rooms); psum holds n_parts partial sums of y^2 per room, in order.
__global__ void conv_noise(float *__restrict__ y, const float *__restrict__ z, const double *__restrict__ psum,
                           const ConvRoom *__restrict__ rooms, int n_parts, int64_t per_room)
{
    const int r = blockIdx.y;
    __shared__ float sigma_s;
    if (threadIdx.x < 64) room_sigma(psum, r, n_parts, per_room, rooms[r].nscale, &sigma_s);
    __syncthreads();
    const float sg = sigma_s;
    float *yr = y + (int64_t)r * per_room;
    const float *zr = z + (int64_t)r * per_room;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_room; i += (int64_t)gridDim.x * blockDim.x)
        yr[i] = fmaf(sg, zr[i], yr[i]);
}

}  // namespace ism

using namespace ism;

void ism_conv_release(ism_handle *h)
{
    if (!h || !h->conv) return;
    ConvState *c = h->conv;
    for (ConvSlot &S : c->slot) {
        if (S.ev) {
            if (S.used) (void)hipEventSynchronize(S.ev);
            (void)hipEventDestroy(S.ev);
        }
        for (hipEvent_t &t : S.tev)
            if (t) (void)hipEventDestroy(t);
        if (S.ws) (void)hipFree(S.ws);
        if (S.stage) (void)hipHostFree(S.stage);
    }
    delete c;
    h->conv = nullptr;
}

static size_t al256(size_t v) { return (v + 255) / 256 * 256; }

// noise: none (snr_db NULL), caller's deviates z, or deviates drawn from noise_seed
static int convolve_impl(ism_handle *h, int n_rooms, int M, const float *rirs, const int64_t *rir_offset,
                         const int32_t *rir_len, const float *src, int src_len, int out_len, const float *snr_db,
                         const float *z, bool seeded, uint64_t noise_seed, int use_mfma, float *out,
                         ism_stream stream)
{
    if (!h) return ISM_EINVAL;
    h->last_error.clear();
    if (n_rooms < 0 || n_rooms > 65535 || M < 1 || M > 65535 || src_len < 1 || out_len < 1) {
        ism_set_error(h, "0 <= n_rooms <= 65535, 1 <= M <= 65535, src_len >= 1 and out_len >= 1 required");
        return ISM_EINVAL;
    }
    if (n_rooms == 0) return ISM_OK;
    if (!rirs || !rir_offset || !rir_len || !src || !out) {
        ism_set_error(h, "NULL argument");
        return ISM_EINVAL;
    }
    if (snr_db && !z && !seeded) {
        ism_set_error(h, "noise deviates z are required when snr_db is given");
        return ISM_EINVAL;
    }
    if (use_mfma && M != CM) {
        ism_set_error(h, "the MFMA path takes %d microphones per room", CM);
        return ISM_EINVAL;
    }
    if ((int64_t)out_len > (1LL << 28) || (int64_t)src_len > (1LL << 28)) {
        ism_set_error(h, "signal length limit exceeded");
        return ISM_EINVAL;
    }
    std::vector<ConvRoom> rooms(n_rooms);
    int64_t hb_total = 0;
    int nb_max = 0;
    for (int r = 0; r < n_rooms; ++r) {
        if (rir_len[r] < 1 || rir_len[r] > (1 << 24) || rir_offset[r] < 0) {
            ism_set_error(h, "room %d: rir_len must be in [1, 2^24] and rir_offset >= 0", r);
            return ISM_EINVAL;
        }
        if (snr_db && !std::isfinite(snr_db[r])) {
            ism_set_error(h, "room %d: snr_db not finite", r);
            return ISM_EINVAL;
        }
        ConvRoom &c = rooms[r];
        c.rir_off = rir_offset[r];
        c.rir_len = rir_len[r];
        c.nb = (rir_len[r] + CB - 1) / CB;
        c.h_off = hb_total;
        c.snr_db = snr_db ? snr_db[r] : 0.0f;
        c.nscale = std::pow(10.0, -(double)c.snr_db / 10.0);
        c.order = r;
        hb_total += (int64_t)M * c.nb * CB;
        nb_max = std::max(nb_max, c.nb);
    }
    {
        std::vector<int32_t> ord(n_rooms);
        for (int r = 0; r < n_rooms; ++r) ord[r] = r;
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return rooms[a].nb > rooms[b].nb; });
        for (int r = 0; r < n_rooms; ++r) rooms[r].order = ord[r];
    }
    if (h->device < 0) { ism_set_error(h, "no HIP device"); return ISM_EDEVICE; }
    if (!h->conv) h->conv = new (std::nothrow) ConvState();
    if (!h->conv) return ISM_ENOMEM;
    ConvSlot &C = h->conv->slot[h->conv->next];
    hipStream_t q = (hipStream_t)stream;

    const int mt_tiles = (out_len + CTILE - 1) / CTILE;
    const int dt_tiles = (out_len + DT - 1) / DT;
    const int64_t n_parts = use_mfma ? mt_tiles : (int64_t)M * dt_tiles;
    const size_t off_hb = 0;
    const size_t off_ps = al256(off_hb + (use_mfma ? (size_t)hb_total * 2 : 0));
    const size_t off_rm = al256(off_ps + sizeof(double) * (size_t)n_rooms * n_parts);
    const size_t need = al256(off_rm + sizeof(ConvRoom) * n_rooms);
    if (C.ev && C.used) {
        hipError_t e = hipEventSynchronize(C.ev);
        if (e != hipSuccess) return ism_hip_fail(h, e, "hipEventSynchronize");
        C.used = false;
    }
    if (C.cap < need) {
        if (C.ws) (void)hipFree(C.ws);
        C.ws = nullptr;
        C.cap = 0;
        if (hipMalloc(&C.ws, need) != hipSuccess) { ism_set_error(h, "conv workspace allocation failed"); return ISM_ENOMEM; }
        C.cap = need;
    }
    const size_t rbytes = sizeof(ConvRoom) * n_rooms;
    if (C.stage_cap < rbytes) {
        if (C.stage) (void)hipHostFree(C.stage);
        C.stage = nullptr;
        C.stage_cap = 0;
        if (hipHostMalloc(&C.stage, rbytes, hipHostMallocDefault) != hipSuccess) {
            ism_set_error(h, "pinned allocation failed");
            return ISM_ENOMEM;
        }
        C.stage_cap = rbytes;
    }
    if (!C.ev && hipEventCreateWithFlags(&C.ev, hipEventDisableTiming) != hipSuccess) {
        ism_set_error(h, "hipEventCreate failed");
        return ISM_EDEVICE;
    }
    std::memcpy(C.stage, rooms.data(), rbytes);
    char *ws = (char *)C.ws;
    uint16_t *hb = (uint16_t *)(ws + off_hb);
    double *ps = (double *)(ws + off_ps);
    ConvRoom *rm = (ConvRoom *)(ws + off_rm);
    hipError_t e = hipMemcpyAsync(rm, C.stage, rbytes, hipMemcpyHostToDevice, q);
    if (e != hipSuccess) return ism_hip_fail(h, e, "hipMemcpyAsync");
    const bool timed = h->conv->timing;
    C.timed = false;
    if (timed) {
        for (hipEvent_t &t : C.tev)
            if (!t && (e = hipEventCreate(&t)) != hipSuccess) return ism_hip_fail(h, e, "hipEventCreate");
        if ((e = hipEventRecord(C.tev[0], q)) != hipSuccess) return ism_hip_fail(h, e, "hipEventRecord");
    }
    if (use_mfma) {
        hipLaunchKernelGGL(conv_pack_h, dim3(std::max(1, (nb_max * CB + 1023) / 1024), n_rooms, M), dim3(256), 0, q,
                           rirs, rm, hb);
        if ((e = hipGetLastError()) != hipSuccess) return ism_hip_fail(h, e, "conv_pack_h launch");
        if (timed && (e = hipEventRecord(C.tev[1], q)) != hipSuccess) return ism_hip_fail(h, e, "hipEventRecord");
        hipLaunchKernelGGL(conv_mfma, dim3(mt_tiles, n_rooms), dim3(64), 0, q, src, src_len, out_len, hb, rm, out, ps,
                           mt_tiles);
        if ((e = hipGetLastError()) != hipSuccess) return ism_hip_fail(h, e, "conv_mfma launch");
    } else {
        if (timed && (e = hipEventRecord(C.tev[1], q)) != hipSuccess) return ism_hip_fail(h, e, "hipEventRecord");
        hipLaunchKernelGGL(conv_direct, dim3(dt_tiles, M, n_rooms), dim3(256), 0, q, rirs, rm, src, src_len, out_len, M,
                           out, ps, dt_tiles);
        if ((e = hipGetLastError()) != hipSuccess) return ism_hip_fail(h, e, "conv_direct launch");
    }
    if (timed && (e = hipEventRecord(C.tev[2], q)) != hipSuccess) return ism_hip_fail(h, e, "hipEventRecord");
    if (snr_db && seeded) {
        const int64_t quads = (int64_t)M * ((out_len + 3) / 4);
        const int chunks = (int)std::min<int64_t>(256, (quads + 256 * kNoiseQ - 1) / (256 * kNoiseQ));
        hipLaunchKernelGGL(conv_noise_seeded, dim3(chunks, n_rooms), dim3(256), 0, q, out, ps, rm, (int)n_parts, M,
                           out_len, (uint32_t)noise_seed, (uint32_t)(noise_seed >> 32));
        if ((e = hipGetLastError()) != hipSuccess) return ism_hip_fail(h, e, "conv_noise_seeded launch");
    } else if (snr_db) {
        const int64_t per_room = (int64_t)M * out_len;
        const int chunks = (int)std::min<int64_t>(64, (per_room + 255) / 256);
        hipLaunchKernelGGL(conv_noise, dim3(chunks, n_rooms), dim3(256), 0, q, out, z, ps, rm, (int)n_parts, per_room);
        if ((e = hipGetLastError()) != hipSuccess) return ism_hip_fail(h, e, "conv_noise launch");
    }
    if (timed && (e = hipEventRecord(C.tev[3], q)) != hipSuccess) return ism_hip_fail(h, e, "hipEventRecord");
    if ((e = hipEventRecord(C.ev, q)) != hipSuccess) return ism_hip_fail(h, e, "hipEventRecord");
    C.used = true;
    C.timed = timed;
    C.noise = snr_db != nullptr;
    h->conv->last = h->conv->next;
    h->conv->next ^= 1;
    return ISM_OK;
}

extern "C" int ism_convolve_batch(ism_handle *h, int n_rooms, int M, const float *rirs, const int64_t *rir_offset,
                                  const int32_t *rir_len, const float *src, int src_len, int out_len,
                                  const float *snr_db, uint64_t noise_seed, int use_mfma, float *out,
                                  ism_stream stream)
{
    return convolve_impl(h, n_rooms, M, rirs, rir_offset, rir_len, src, src_len, out_len, snr_db, nullptr, true,
                         noise_seed, use_mfma, out, stream);
}

extern "C" int ism_convolve_batch_z(ism_handle *h, int n_rooms, int M, const float *rirs, const int64_t *rir_offset,
                                    const int32_t *rir_len, const float *src, int src_len, int out_len,
                                    const float *snr_db, const float *z, int use_mfma, float *out, ism_stream stream)
{
    return convolve_impl(h, n_rooms, M, rirs, rir_offset, rir_len, src, src_len, out_len, snr_db, z, false, 0,
                         use_mfma, out, stream);
}

extern "C" int ism_conv_set_timing(ism_handle *h, int on)
{
    if (!h) return ISM_EINVAL;
    h->last_error.clear();
    if (!h->conv) h->conv = new (std::nothrow) ConvState();
    if (!h->conv) return ISM_ENOMEM;
    h->conv->timing = on != 0;
    return ISM_OK;
}

extern "C" int ism_conv_last_timing(ism_handle *h, float ms[3])
{
    if (!h) return ISM_EINVAL;
    h->last_error.clear();
    if (!ms) { ism_set_error(h, "NULL argument"); return ISM_EINVAL; }
    if (!h->conv || h->conv->last < 0 || !h->conv->slot[h->conv->last].timed) {
        ism_set_error(h, "no timed convolution call on this handle (ism_conv_set_timing first)");
        return ISM_EINVAL;
    }
    ConvSlot &C = h->conv->slot[h->conv->last];
    hipError_t e = hipEventSynchronize(C.tev[3]);
    if (e != hipSuccess) return ism_hip_fail(h, e, "hipEventSynchronize");
    for (int k = 0; k < 3; ++k) {
        if ((e = hipEventElapsedTime(&ms[k], C.tev[k], C.tev[k + 1])) != hipSuccess)
            return ism_hip_fail(h, e, "hipEventElapsedTime");
    }
    if (!C.noise) ms[2] = 0.0f;
    return ISM_OK;
}

extern "C" int ism_normal_deviates(ism_handle *h, int n_rooms, int M, int n_samples, uint64_t seed, float *z,
                                   ism_stream stream)
{
    if (!h) return ISM_EINVAL;
    h->last_error.clear();
    if (n_rooms < 0 || M < 1 || n_samples < 1 || n_rooms > 65535 || (int64_t)n_samples > (1LL << 28)) {
        ism_set_error(h, "0 <= n_rooms <= 65535, M >= 1 and 1 <= n_samples <= 2^28 required");
        return ISM_EINVAL;
    }
    if (n_rooms == 0) return ISM_OK;
    if (!z) { ism_set_error(h, "NULL argument"); return ISM_EINVAL; }
    if (h->device < 0) { ism_set_error(h, "no HIP device"); return ISM_EDEVICE; }
    const int64_t quads = (int64_t)M * ((n_samples + 3) / 4);
    const int chunks = (int)std::min<int64_t>(256, (quads + 255) / 256);
    hipLaunchKernelGGL(normal_deviates_kernel, dim3(chunks, n_rooms), dim3(256), 0, (hipStream_t)stream, z, M,
                       n_samples, (uint32_t)seed, (uint32_t)(seed >> 32));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ism_hip_fail(h, e, "normal_deviates launch");
    return ISM_OK;
}
