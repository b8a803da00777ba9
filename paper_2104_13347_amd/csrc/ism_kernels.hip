// Image-source RIR kernels for gfx950 (paper section II.A: every image of the
// source in a shoebox room adds a fractional-delay filter, centred on its delay,
// into the RIR of each microphone).
//
// Two kernels compute the same sum over work items (an item is the output segment
// [s0, s1) of one microphone's RIR; both are persistent over a queue of items):
//  * ism_moments, the default for the compiled filter lengths and segments of at most
//    1024 samples: 16 waves own an item; they enumerate its images in column chunks,
//    add each image's 9 Chebyshev moments of its fractional delay (FP64, exact 64-bit
//    fixed point) into LDS bins by integer delay, and then evaluate the filter once
//    per output sample as a GEMM on the matrix cores (see the kernel's comments).
//  * ism_segments, the per-tap kernel described next (the other filters, longer
//    segments, rooms beyond the moment kernel's wall-power tables, and the ablations).
//
// Per-tap design (one wave64 per workgroup):
//
//  * Enumeration in registers.  Only images whose rounded delay n0 can put a tap
//    into the segment are visited: they lie in a spherical shell around the
//    microphone.  The wave walks the (x, y) image columns 64 at a time; each
//    lane derives the z-index intervals of its column that fall into the shell
//    (at most four: two parities, each an interval with the inner hole cut
//    out); a wave prefix sum flattens the images of 64 columns so that every
//    lane evaluates one image per step.  Distance, delay and the integer /
//    fractional split are FP64 and follow the same operation order as the
//    definition ((dx^2 + dy^2) + dz^2, sqrt, (d fs) / c, floor(tau + 1/2)).
//  * Records (f, g, n0) of valid images go to a 256-entry ring in LDS (stable,
//    in enumeration order, via ballot + mbcnt).
//  * Rounds: 64 records at a time, one per lane, the 2K+1 taps with k uniform
//    across the wave (unrolled, constants folded).  Each tap is converted to a
//    32-bit fixed-point value and added with a 64-bit integer LDS atomic into
//    the segment accumulator.  Integer addition is associative, so the result
//    does not depend on the order of the adds: it is deterministic by
//    construction and exact apart from one quantisation per tap.  The scale is
//    a power of two per work item, 2^30 / (a bound on the item's largest image
//    gain), so no tap exceeds 2^30 and no 64-bit sum can overflow; the
//    quantisation step is below 1e-9 of that gain bound.  (On gfx950 an LDS
//    FP32 atomic add costs about 190 CU cycles per wave instruction, a 64-bit
//    integer one about 6.)
//  * The FP32-atomic ablation keeps FP32 LDS atomics; there the lanes of one
//    round must hold distinct n0, so that no ds_add sees two lanes on one
//    address: a claim array with an LDS atomic min keeps the lowest lane of
//    each n0 and defers the others to the ring's tail, which fixes the order
//    of the adds at every address.
//  * The segment is written once, coalesced (lane-contiguous samples).
//
// Tap formula.  With t = k - f, sinc(t) = -(-1)^k sin(pi f) / (pi t), and the
// Hann window w(t) = (1 + cos(P t)) / 2, P = pi / (K+1), expands by angle
// addition into constants of k times per-record values of f:
//     g h(k - f) = (-1)^k / (k - f) * (a0 + a1 cos(P k) + a2 sin(P k)),
//     a0 = -g sin(pi f) / (2 pi), a1 = a0 cos(P f), a2 = a0 sin(P f).
// Per tap: one subtraction (the sign (-1)^k folds into its operand order), one
// v_rcp_f32, two FMAs, one multiply, a float-to-int conversion, a sign
// extension and one ds_add_u64.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ism_internal.h"

namespace ism {

#define DEV __device__ __forceinline__

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- compile-time trig
constexpr double cx_sin_red(double x)
{  // |x| <= pi: Taylor series to well below double rounding
    double x2 = x * x, term = x, sum = x;
    for (int i = 1; i < 30; ++i) {
        term *= -x2 / ((2.0 * i) * (2.0 * i + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double cx_cos_red(double x)
{
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int i = 1; i < 30; ++i) {
        term *= -x2 / ((2.0 * i - 1.0) * (2.0 * i));
        sum += term;
    }
    return sum;
}

template <int K>
struct TapConst {
    float c[2 * K + 1];
    float s[2 * K + 1];
    constexpr TapConst() : c(), s()
    {
        for (int i = 0; i <= 2 * K; ++i) {
            double x = kPi * (double)(i - K) / (double)(K + 1);  // |x| < pi
            c[i] = (float)cx_cos_red(x);
            s[i] = (float)cx_sin_red(x);
        }
    }
};

// ---------------------------------------------------------------- wave helpers
DEV int lane_id() { return __lane_id(); }
DEV uint64_t ballot(bool p) { return __ballot(p); }
DEV int mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}
DEV int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

DEV int wave_excl_scan(int v, int &total)
{
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane_id() >= d) x += y;
    }
    total = __shfl(x, 63, 64);
    return x - v;
}

// Inclusive prefix sum over the 64 lanes of a wave by DPP moves (no LDS round trips):
// row_shr 1, 2, 4, 8 within rows of 16 lanes, then row_bcast:15 and row_bcast:31 carry
// the row totals into the later rows.
DEV int wave_incl_scan_dpp(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    return x;
}

// The same pattern with max: lane 63 ends with the largest of the 64 values (x >= 0;
// lanes with no source take 0).
DEV uint32_t wave_incl_max_dpp(uint32_t x)
{
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false));
    return x;
}

DEV void lds_add(float *p, float v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Per-record coefficients a0, a1, a2 of the tap formula (FP32; |f| <= 1/2).
DEV void tap_coeffs(float f, float g, float P, bool wide, float &a0, float &a1, float &a2)
{
    const float x = 3.14159265358979f * f;  // |x| <= pi/2
    const float x2 = x * x;
    // sin(x)/x, Taylor series through x^12 (truncation < 5e-10 on |x| <= pi/2)
    float p = fmaf(x2, 1.0f / 6227020800.0f, -1.0f / 39916800.0f);
    p = fmaf(x2, p, 1.0f / 362880.0f);
    p = fmaf(x2, p, -1.0f / 5040.0f);
    p = fmaf(x2, p, 1.0f / 120.0f);
    p = fmaf(x2, p, -1.0f / 6.0f);
    p = fmaf(x2, p, 1.0f);
    a0 = -0.5f * g * (f * p);  // -g sin(pi f) / (2 pi)
    const float y = P * f;     // |y| <= pi / (2(K+1))
    const float y2 = y * y;
    float cy, sy;
    if (!wide) {
        // K >= 4: |y| <= pi/10, truncation below 3e-9
        cy = fmaf(y2, fmaf(y2, fmaf(y2, -1.0f / 720.0f, 1.0f / 24.0f), -0.5f), 1.0f);
        sy = y * fmaf(y2, fmaf(y2, fmaf(y2, -1.0f / 5040.0f, 1.0f / 120.0f), -1.0f / 6.0f), 1.0f);
    } else {
        // K < 4: |y| up to pi/2, Taylor series through y^12 / y^13 (truncation < 7e-8)
        cy = fmaf(y2, 1.0f / 479001600.0f, -1.0f / 3628800.0f);
        cy = fmaf(y2, cy, 1.0f / 40320.0f);
        cy = fmaf(y2, cy, -1.0f / 720.0f);
        cy = fmaf(y2, cy, 1.0f / 24.0f);
        cy = fmaf(y2, cy, -0.5f);
        cy = fmaf(y2, cy, 1.0f);
        float q = fmaf(y2, 1.0f / 6227020800.0f, -1.0f / 39916800.0f);
        q = fmaf(y2, q, 1.0f / 362880.0f);
        q = fmaf(y2, q, -1.0f / 5040.0f);
        q = fmaf(y2, q, 1.0f / 120.0f);
        q = fmaf(y2, q, -1.0f / 6.0f);
        q = fmaf(y2, q, 1.0f);
        sy = y * q;
    }
    a1 = a0 * cy;
    a2 = a0 * sy;
}

DEV void lds_add_fx(long long *p, float x)
{
    // x is already scaled; |x| < 2^31, truncation toward zero
    const long long v = (long long)(int)x;
    __hip_atomic_fetch_add((unsigned long long *)p, (unsigned long long)v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// 2K+1 taps of one record, K known at compile time: constants fold to literals.
// FX: fixed-point accumulation into acc64; otherwise FP32 LDS atomics into acc32.
// Taps +k and -k share one reciprocal: with p = f^2 - k^2 = (k - f)(-k - f),
// 1/(k - f) = (-k - f)/p and 1/(-k - f) = (k - f)/p; the sign (-1)^k (the same
// for +k and -k) is folded into the two numerators' factors.
template <int K, bool FX>
DEV void taps_fp32_ct(long long *acc64, float *acc32, float f, float a0, float a1, float a2)
{
    constexpr TapConst<K> T{};
    {   // k = 0: (-1)^0 / (0 - f)
        const float r = __builtin_amdgcn_rcpf(-f);
        const float num = fmaf(a2, T.s[K], fmaf(a1, T.c[K], a0));
        if (FX) lds_add_fx(acc64, num * r);
        else lds_add(acc32, num * r);
    }
    const float f2 = f * f;
#pragma unroll
    for (int k = 1; k <= K; ++k) {
        const float rp = __builtin_amdgcn_rcpf(f2 - (float)(k * k));
        // (-1)^k / (k - f) = tp * rp and (-1)^k / (-k - f) = tm * rp
        const float tp = (k & 1) ? ((float)k + f) : (-(float)k - f);
        const float tm = (k & 1) ? (f - (float)k) : ((float)k - f);
        const float np = fmaf(a2, T.s[K + k], fmaf(a1, T.c[K + k], a0));
        const float nm = fmaf(a2, T.s[K - k], fmaf(a1, T.c[K - k], a0));
        const float vp = (np * tp) * rp;
        const float vm = (nm * tm) * rp;
        if (FX) {
            lds_add_fx(acc64 + k, vp);
            lds_add_fx(acc64 - k, vm);
        } else {
            lds_add(acc32 + k, vp);
            lds_add(acc32 - k, vm);
        }
    }
}

// 7th-order Lagrange interpolation on the per-tap kernel: taps k = -3..4 at n0 + k,
// n0 = floor(tau), f = tau - n0 in [0, 1); the coefficient of node j = k + 3 at D = f + 3 is
// prod_{i != j} (D - i) / (j - i), from prefix and suffix products of w_i = D - i (each
// w_i = f + (3 - i) rounded once) and the node denominators prod_{i != j} (j - i).
DEV void taps_lagrange(long long *acc64, float f, float gs)
{
    constexpr float inv_den[8] = {-1.0f / 5040.0f, 1.0f / 720.0f, -1.0f / 240.0f, 1.0f / 144.0f,
                                  -1.0f / 144.0f, 1.0f / 240.0f, -1.0f / 720.0f, 1.0f / 5040.0f};
    float w[8], pre[8], suf[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = f + (float)(3 - i);
    pre[0] = 1.0f;
#pragma unroll
    for (int i = 1; i < 8; ++i) pre[i] = pre[i - 1] * w[i - 1];
    suf[7] = 1.0f;
#pragma unroll
    for (int i = 6; i >= 0; --i) suf[i] = suf[i + 1] * w[i + 1];
#pragma unroll
    for (int j = 0; j < 8; ++j) lds_add_fx(acc64 + (j - 3), (pre[j] * suf[j]) * (inv_den[j] * gs));
}

// Runtime K: constants from an LDS table (uniform address, broadcast read).
template <bool FX>
DEV void taps_fp32_rt(long long *acc64, float *acc32, int K, const float2 *trig, float f, float a0, float a1,
                      float a2)
{
    for (int k = -K; k <= K; ++k) {
        const float2 cs = trig[k + K];
        const float kf = (float)k;
        const float t = (k & 1) ? (f - kf) : (kf - f);
        const float r = __builtin_amdgcn_rcpf(t);
        const float num = fmaf(a2, cs.y, fmaf(a1, cs.x, a0));
        if (FX) lds_add_fx(acc64 + k, num * r);
        else lds_add(acc32 + k, num * r);
    }
}

// FP16 table variant: h(k - f) from pairs (h(k - f_j), h(k - f_{j+1})), f_j = -1/2 + j/Q,
// linear interpolation, times the (scaled) gain; fixed-point accumulation.
template <int KT>
DEV void taps_lut(long long *acc64, int Krt, const uint32_t *lut, float f, float gs)
{
    const int K = KT > 0 ? KT : Krt;
    const float p = (f + 0.5f) * (float)kLutQ;
    int j = (int)p;
    j = j > kLutQ - 1 ? kLutQ - 1 : (j < 0 ? 0 : j);
    const float al = p - (float)j;
    const uint32_t *row = lut + j;
#pragma unroll 9
    for (int k = -K; k <= K; ++k) {
        const uint32_t pr = row[(k + K) * kLutQ];
        const float h0 = (float)__builtin_bit_cast(_Float16, (unsigned short)(pr & 0xFFFFu));
        const float h1 = (float)__builtin_bit_cast(_Float16, (unsigned short)(pr >> 16));
        lds_add_fx(acc64 + k, gs * fmaf(al, h1 - h0, h0));
    }
}

DEV double hann_sinc(double t, int K)
{
    double s = (t == 0.0) ? 1.0 : sin(kPi * t) / (kPi * t);
    return s * 0.5 * (1.0 + cos(kPi * t / (double)(K + 1)));
}

// ---------------------------------------------------------------- prologue
// Zero the work counter and build the wall-power tables beta^e (repeated
// multiplication, so beta^0 = 1 for beta = 0), one thread per (room, wall).
__global__ void ism_prologue(const LaunchDev *P)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid == 0) *P->counter = 0u;
    if (gid < 8) P->stats[gid] = 0ull;
    if (gid >= P->n_rooms * 6) return;
    const int room = gid / 6, wall = gid % 6;
    const RoomDev &R = P->rooms[room];
    double *t = P->pow_tab + R.pow_offset + wall * R.pow_stride;
    const double b = R.beta[wall];
    double v = 1.0;
    for (int e = 0; e < R.pow_stride; ++e) {
        t[e] = v;
        v *= b;
    }
}

// ---------------------------------------------------------------- segment kernel
struct Lds {
    long long *acc64;   // fixed-point accumulator (FX, LUT)
    float *acc32;       // FP32 accumulator (FP32-atomic ablation), aliases acc64
    uint32_t *claim;    // FP32-atomic ablation only
    float *bf, *bg;
    int32_t *bn;
    int32_t *coff;      // kCols + 1 prefix offsets
    double *crho2, *cbxy;
    int32_t *cord;      // order index of the column (x and y part)
    int32_t *iq0, *icum, *iw;  // 4 intervals per column
    float2 *trig;
    uint32_t *lut;
};

DEV Lds carve(char *base, int seg_max, int K, int variant)
{
    Lds s;
    const int acc = (seg_max + 4 * K + 63) / 64 * 64;
    const int clm = variant == VAR_F32ATOM ? (seg_max + 2 * K + 63) / 64 * 64 : 0;
    char *p = base;
    s.crho2 = (double *)p; p += kCols * 8;
    s.cbxy = (double *)p; p += kCols * 8;
    s.acc64 = (long long *)p;
    s.acc32 = (float *)p; p += acc * 8;
    s.claim = (uint32_t *)p; p += clm * 4;
    s.bf = (float *)p; p += kBufCap * 4;
    s.bg = (float *)p; p += kBufCap * 4;
    s.bn = (int32_t *)p; p += kBufCap * 4;
    s.coff = (int32_t *)p; p += (kCols + 4) * 4;
    s.cord = (int32_t *)p; p += kCols * 4;
    s.iq0 = (int32_t *)p; p += kCols * 4 * 4;
    s.icum = (int32_t *)p; p += kCols * 4 * 4;
    s.iw = (int32_t *)p; p += kCols * 4 * 4;
    s.trig = (float2 *)p; p += (2 * K + 1) * 8;
    s.lut = (uint32_t *)p;
    return s;
}

extern __shared__ __attribute__((aligned(16))) char ism_lds[];


// ---------------------------------------------------------------- read-only launch tables
// Rooms, items and microphones do not change while a kernel runs.  Read through the
// constant address space, a wave-uniform index becomes a scalar load (scalar cache, no
// vector registers, no wait on the vector-memory counter).
typedef const __attribute__((address_space(4))) ItemDev CItemDev;
typedef const __attribute__((address_space(4))) RoomDev CRoomDev;
typedef const __attribute__((address_space(4))) double CDouble;

DEV ItemDev load_item(const LaunchDev *P, int i)
{
    CItemDev *p = (CItemDev *)P->items + i;
    ItemDev it;
    it.room = p->room;
    it.mic = p->mic;
    it.s0 = p->s0;
    it.s1 = p->s1;
    return it;
}

DEV CRoomDev *room_ptr(const LaunchDev *P, int room) { return (CRoomDev *)P->rooms + room; }

// Writes through generic pointers compile to flat instructions, which a wave counts among
// its LDS operations as well: every later wait for LDS (each barrier) would also wait for
// an output store or the item counter's atomic to complete.  The kernels write through
// the global address space instead.
typedef __attribute__((address_space(1))) float GFloat;
DEV GFloat *global_out(float *p) { return (GFloat *)p; }

// Next work item, fetched by one lane.  The counter's address goes through an empty asm
// (a value the compiler cannot see to be uniform), so the atomic is not rewritten into a
// wave-wide one, whose result the compiler would wait for at once: the wait comes where
// the index is used.
DEV int fetch_item(uint32_t *counter)
{
    uint64_t a = (uint64_t)counter;
    asm volatile("" : "+v"(a));
    return (int)__hip_atomic_fetch_add((__attribute__((address_space(1))) uint32_t *)a, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- item geometry
// Everything about one work item (room, microphone, output segment [s0, s1)) that the
// enumeration needs, derived once per item.  Table pointers carry the global address space
// (generic pointers would make their loads flat instructions, which waves count among
// their LDS operations).
typedef const __attribute__((address_space(1))) double GConstDouble;
struct ItemGeom {
    double Lx, Ly, Lz, sx, sy, sz, rx, ry, rz;
    double dlo2, dhi2;            // squared distance shell of the item's records
    double zeps;                  // margin of the column intervals' z bounds (in z-index units)
    double inv2Lz;                // 1 / (2 Lz) (its rounding is inside the margin)
    GConstDouble *px0, *pz0, *pzL; // the room's wall-power tables (global memory)
    int alo, blo;                 // first (x, y) image column indices
    float inv_nb;                 // 1 / nb
    int pow_stride, pmax;
    int rir_len, N, s0, s1, Sn;
    int nlo, nhi;                 // record delays n0 in [nlo, nhi] can reach the segment
    int rel;                      // n0 - rel indexes the item's delay bins / accumulator
    int nb, ncols;                // columns: (a, b) = (alo + c / nb, blo + c % nb)
    int escale;                   // fixed-point scale 2^escale
};

DEV ItemGeom item_geom(const LaunchDev *P, const ItemDev &it, int K)
{
    ItemGeom G;
    CRoomDev &R = *room_ptr(P, it.room);
    CDouble *mic = (CDouble *)P->mics + 3 * it.mic;
    const double fs = P->fs, cs = P->c;
    G.Lx = R.L[0]; G.Ly = R.L[1]; G.Lz = R.L[2];
    G.sx = R.src[0]; G.sy = R.src[1]; G.sz = R.src[2];
    G.rx = mic[0]; G.ry = mic[1]; G.rz = mic[2];
    G.rir_len = R.rir_len;
    G.N = R.max_order;
    G.s0 = it.s0; G.s1 = it.s1; G.Sn = it.s1 - it.s0;
    // taps k = kmin..kmax about n0 reach [s0, s1) for n0 in [s0 - kmax, s1 - 1 - kmin]
    const int kmin = P->lagrange ? -3 : -K, kmax = P->lagrange ? 4 : K;
    G.nlo = max(G.s0 - kmax, 0);
    G.nhi = min(G.s1 - 1 - kmin, G.rir_len - 1 - kmin);
    G.rel = G.s0 - K;
    G.px0 = (GConstDouble *)(P->pow_tab + R.pow_offset);
    G.pz0 = G.px0 + 4 * R.pow_stride;
    G.pzL = G.pz0 + R.pow_stride;
    G.pow_stride = R.pow_stride;
    G.pmax = R.pow_stride - 1;
    // distance shell of the records this segment needs (widened: every test below is exact);
    // n0 = floor(tau + half) puts tau in [n0 - half, n0 + 1 - half)
    const double half = P->lagrange ? 0.0 : 0.5;
    const double csf = cs / fs;  // the margins cover its rounding
    const double dlo = fmax(0.0, ((double)G.nlo - half) * csf * (1.0 - 1e-12) - 1e-12);
    const double dhi = ((double)G.nhi + 1.0 - half) * csf * (1.0 + 1e-12) + 1e-12;
    G.dlo2 = dlo * dlo;
    G.dhi2 = dhi * dhi;
    // the column intervals' z bounds come from FP32 square roots (relative error below
    // 2^-22 with the FP32 rounding of the argument): widened by this margin in z-index
    // units they still hold every image of the shell
    G.inv2Lz = 0.5 * R.inv_L[2];
    G.zeps = 1e-9 + 4e-7 * dhi * G.inv2Lz;
    // Fixed-point scale 2^e: no image is closer than the direct path and every
    // beta <= 1, so g <= 1/(4 pi max(dlo, |s - r|)) =: gb for every record of the
    // item, and |tap| <= g (|h| <= 1); e is the largest exponent with 2^e gb < 2^30.
    {
        const double ddx = G.sx - G.rx, ddy = G.sy - G.ry, ddz = G.sz - G.rz;
        const double ddir = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
        const double gb = 1.0 / (4.0 * kPi * fmax(dlo, ddir));
        int E;
        (void)frexp(gb, &E);  // gb = m 2^E, m in [1/2, 1)
        G.escale = 30 - E;
    }
    // image index bounds (with a margin of one, which also covers the reciprocal's rounding)
    const double ilx = R.inv_L[0], ily = R.inv_L[1];
    long alo = (long)floor((G.rx - dhi) * ilx) - 1, ahi = (long)ceil((G.rx + dhi) * ilx) + 1;
    long blo = (long)floor((G.ry - dhi) * ily) - 1, bhi = (long)ceil((G.ry + dhi) * ily) + 1;
    if (G.N >= 0) {
        const long lim = P->order_mode == 0 ? 2L * G.N + 2 : (long)G.N + 1;
        alo = max(alo, -lim); ahi = min(ahi, lim);
        blo = max(blo, -lim); bhi = min(bhi, lim);
    }
    G.alo = (int)alo;
    G.blo = (int)blo;
    G.nb = (int)(bhi - blo + 1);
    G.ncols = (int)(ahi - alo + 1) * G.nb;
    G.inv_nb = 1.0f / (float)G.nb;
    return G;
}

// An item's geometry as one wave wrote it to LDS, read back word by word into scalar
// registers (every lane reads the same words).
static_assert(sizeof(ItemGeom) <= kMomGeomBytes && sizeof(ItemGeom) % 4 == 0, "geometry fits its LDS area");
DEV ItemGeom geom_from_lds(const ItemGeom *g)
{
    constexpr int NW = sizeof(ItemGeom) / 4;
    const uint32_t *src = (const uint32_t *)g;
    uint32_t w[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) w[i] = __builtin_amdgcn_readfirstlane(src[i]);
    ItemGeom G;
    __builtin_memcpy(&G, w, sizeof G);
    return G;
}

// One (x, y) image column: the z-index intervals whose images lie in the item's
// distance shell (two parities w, each an interval with the inner hole cut out, so
// at most four), the squared horizontal distance, the x/y wall-power product and the
// x/y part of the reflection order.
struct Column {
    int q0[4], len[4], wv[4];
    double rho2, bxy;
    int ord;
};

// px: x0, xL, y0, yL wall-power tables, `ps` apart (exponents 0 .. pmax)
DEV Column column_setup(const ItemGeom &G, int ci, int order_mode, GConstDouble *px, int ps)
{
    Column C;
#pragma unroll
    for (int i = 0; i < 4; ++i) { C.q0[i] = 0; C.len[i] = 0; C.wv[i] = 0; }
    C.rho2 = 0.0;
    C.bxy = 0.0;
    C.ord = 0;
    if (ci >= G.ncols) return C;
    const int N = G.N;
    // ci / nb from a float reciprocal, corrected to the exact quotient (ci < 2^24)
    int ca = (int)((float)ci * G.inv_nb);
    ca -= ca * G.nb > ci;
    ca += (ca + 1) * G.nb <= ci;
    const int a = G.alo + ca, b = G.blo + (ci - ca * G.nb);
    const int u = a & 1, v = b & 1;
    const int n = (a + u) >> 1, l = (b + v) >> 1;
    const double X = (u ? -G.sx : G.sx) + (2.0 * (double)n) * G.Lx;
    const double Y = (v ? -G.sy : G.sy) + (2.0 * (double)l) * G.Ly;
    const double dx = X - G.rx, dy = Y - G.ry;
    const double rho2 = dx * dx + dy * dy;
    C.rho2 = rho2;
    int qlim_lo = -(1 << 30), qlim_hi = 1 << 30;
    bool ok = rho2 < G.dhi2;
    int ordxy = 0;
    if (N >= 0) {
        ordxy = order_mode == 0 ? abs(n) + abs(l) : abs(2 * n - u) + abs(2 * l - v);
        if (ordxy > N) ok = false;
    }
    C.ord = ordxy;
    if (!ok) return C;
    const int pmax = G.pmax;
    const int ex0 = min(abs(n - u), pmax), exL = min(abs(n), pmax);
    const int ey0 = min(abs(l - v), pmax), eyL = min(abs(l), pmax);
    C.bxy = ((px[ex0] * px[ps + exL]) * px[2 * ps + ey0]) * px[3 * ps + eyL];
    // z extent of the shell on this column; FP32 square roots, the bounds below widen the
    // intervals (and narrow the hole) by G.zeps, so any extra image lies outside the
    // shell and fails the delay test
    const double zb = (double)__builtin_amdgcn_sqrtf((float)(G.dhi2 - rho2));
    const double za = G.dlo2 > rho2 ? (double)__builtin_amdgcn_sqrtf((float)(G.dlo2 - rho2)) : 0.0;
    const double inv2L = G.inv2Lz;
    int ni = 0;
    // interval slot ni (unrolled selects keep the slots in registers)
    auto put = [&](int qq, int ll, int ww) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (i == ni) { C.q0[i] = qq; C.len[i] = ll; C.wv[i] = ww; }
        ++ni;
    };
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        // dz = (+-sz + 2 q Lz) - rz; |q| stays far below 2^31 (wall exponents < 2^22, host)
        const double off = G.rz - (w ? -G.sz : G.sz);
        int qlo = (int)ceil((off - zb) * inv2L - G.zeps);
        int qhi = (int)floor((off + zb) * inv2L + G.zeps);
        if (N >= 0) {
            const int rem = N - ordxy;
            if (order_mode == 0) { qlim_lo = -rem; qlim_hi = rem; }
            else { qlim_lo = (w - rem + 1) >> 1; qlim_hi = (w + rem) >> 1; }
            // (w - rem + 1) >> 1 = ceil((w - rem) / 2)
            qlo = max(qlo, qlim_lo); qhi = min(qhi, qlim_hi);
        }
        if (qlo > qhi) continue;
        int hlo = 1, hhi = 0;  // empty hole
        if (za > 0.0) {
            hlo = (int)ceil((off - za) * inv2L + G.zeps);
            hhi = (int)floor((off + za) * inv2L - G.zeps);
        }
        if (hlo <= hhi && hhi >= qlo && hlo <= qhi) {
            if (hlo > qlo) put(qlo, hlo - qlo, w);
            if (hhi < qhi) put(hhi + 1, qhi - hhi, w);
        } else {
            put(qlo, qhi - qlo + 1, w);
        }
    }
    return C;
}

// Square root of a normal positive double (a >= 2^-767), correctly rounded:
// Goldschmidt iteration from the hardware reciprocal-square-root estimate with two
// Newton corrections of the root (the general sqrt adds only range scaling and
// special-value handling, which the squared distances here never need).
DEV double sqrt_normal(double a)
{
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, hh = y * 0.5;
    const double r = fma(-hh, g, 0.5);
    g = fma(g, r, g);
    hh = fma(hh, r, hh);
    double e = fma(-g, g, a);
    g = fma(e, hh, g);
    e = fma(-g, g, a);
    return fma(e, hh, g);
}

// Square root of a normal positive double to within about one ulp: the first iteration
// and one correction of sqrt_normal (which adds a second correction for correct rounding).
// The iteration also refines the reciprocal square root: *rinv = 2 hh = 1 / sqrt(a) to
// about the square of the hardware estimate's relative error.
DEV double sqrt_close(double a, double *rinv)
{
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, hh = y * 0.5;
    const double r = fma(-hh, g, 0.5);
    g = fma(g, r, g);
    hh = fma(hh, r, hh);
    *rinv = hh + hh;
    const double e = fma(-g, g, a);
    return fma(e, hh, g);
}

// One image of a column: distance (FP64, (dx^2 + dy^2) + dz^2), delay and its
// integer / fractional split.  Returns whether the record belongs to the item
// (delay in [nlo, nhi], order within the limit).
DEV bool image_eval(const ItemGeom &G, double rho2, int cord, int q, int w, int order_mode, double fs, double cs,
                    double fsc, int split32, double half, int &n0, double &fr, double &d)
{
    bool ordok = true;
    if (G.N >= 0) {
        const int oz = order_mode == 0 ? abs(q) : abs(2 * q - w);
        ordok = cord + oz <= G.N;
    }
    const double Z = (w ? -G.sz : G.sz) + (2.0 * (double)q) * G.Lz;
    const double dz = Z - G.rz;
    const double d2 = rho2 + dz * dz;
    d = sqrt_normal(d2);  // d2 >= (closest image distance)^2, far above 2^-767
    // tau = (d fs) / c as in the definition; d * (fs/c) differs by at most an
    // ulp or two, which can change floor(tau + half) only right at a rounding
    // boundary: there the exact quotient is taken
    double tau = d * fsc;
    {
        const double h = tau + half, fl = floor(h);
        if (h - fl < 1e-12 * h || (fl + 1.0) - h < 1e-12 * h) tau = d * fs / cs;
    }
    const double n0d = floor(tau + half);
    n0 = (int)n0d;
    fr = tau - n0d;
    if (split32) {
        // ablation: the same split in FP32 arithmetic
        const float d2f = (float)rho2 + (float)dz * (float)dz;
        const float tauf = sqrtf(d2f) * (float)fs / (float)cs;
        const float n0f = floorf(tauf + (float)half);
        n0 = (int)n0f;
        fr = (double)(tauf - n0f);
    }
    return ordok && n0 >= G.nlo && n0 <= G.nhi;
}

// image_eval for the moment kernel's walk: the z image offset zw = +-sz is held per interval,
// and the rounding-boundary test works on the fractional part: |fr + ec| > ethr, with
// ec = half - 1/2 and ethr = 1/2 - 1e-12 H for an H at least tau + half of every image
// that can become a record (a superset of image_eval's test).  The distance first comes
// from sqrt_close (about one ulp, so tau is off by far less than the test's margin); near
// a boundary it is recomputed correctly rounded and tau taken as the definition's exact
// quotient, so n0 is the definition's everywhere.
DEV bool image_eval_z(const ItemGeom &G, double rho2, int cord, int q, int w, double zw, int order_mode,
                      double fs, double cs, double fsc, int split32, double half, double ec, double ethr,
                      int &n0, double &fr, double &d, double &rd)
{
    bool ordok = true;
    if (G.N >= 0) {
        const int oz = order_mode == 0 ? abs(q) : abs(2 * q - w);
        ordok = cord + oz <= G.N;
    }
    const double Z = zw + (2.0 * (double)q) * G.Lz;
    const double dz = Z - G.rz;
    const double d2 = rho2 + dz * dz;
    d = sqrt_close(d2, &rd);
    double tau = d * fsc;
    double fl = floor(tau + half);
    fr = tau - fl;
    if (fabs(fr + ec) > ethr) {
        d = sqrt_normal(d2);
        tau = d * fs / cs;
        fl = floor(tau + half);
        fr = tau - fl;
    }
    n0 = (int)fl;
    if (split32) {
        const float d2f = (float)rho2 + (float)dz * (float)dz;
        const float tauf = sqrtf(d2f) * (float)fs / (float)cs;
        const float n0f = floorf(tauf + (float)half);
        n0 = (int)n0f;
        fr = (double)(tauf - n0f);
    }
    return ordok && n0 >= G.nlo && n0 <= G.nhi;
}

template <int KT, int VAR>
__global__ __launch_bounds__(64) void ism_segments(const LaunchDev *__restrict__ P)
{
    constexpr bool LAG = VAR == VAR_LAG;  // the Lagrange filter (K = 4, taps -3..4 about floor(tau))
    const int lane = lane_id();
    const int K = KT > 0 ? KT : P->K;
    const int seg_max = P->seg_max;
    Lds S = carve(ism_lds, seg_max, K, VAR);
    const double fs = P->fs, cs = P->c;
    const double fsc = fs / cs;
    const int order_mode = P->order_mode;
    const int split32 = P->split32;
    const float Pw = (float)(kPi / (double)(K + 1));

    // per-launch tables
    for (int i = lane; i <= 2 * K; i += 64) {
        const double x = kPi * (double)(i - K) / (double)(K + 1);
        S.trig[i] = make_float2((float)cos(x), (float)sin(x));
    }
    if (VAR == VAR_LUT) {
        const int n = (2 * K + 1) * kLutQ;
        for (int idx = lane; idx < n; idx += 64) {
            const int k = idx / kLutQ - K, j = idx % kLutQ;
            const double f0 = -0.5 + (double)j / kLutQ, f1 = -0.5 + (double)(j + 1) / kLutQ;
            const unsigned short h0 = __builtin_bit_cast(unsigned short, (_Float16)(float)hann_sinc(k - f0, K));
            const unsigned short h1 = __builtin_bit_cast(unsigned short, (_Float16)(float)hann_sinc(k - f1, K));
            S.lut[idx] = (uint32_t)h0 | ((uint32_t)h1 << 16);
        }
    }
    {
        const int acc_n = (seg_max + 4 * K + 63) / 64 * 64;
        for (int i = lane; i < acc_n; i += 64) S.acc64[i] = 0;
    }
    __syncthreads();

    for (;;) {
        int item = 0;
        if (lane == 0) item = fetch_item(P->counter);
        item = uniform(__shfl(item, 0, 64));
        if (item >= P->n_items) break;

        const ItemDev it = load_item(P, item);
        const ItemGeom G = item_geom(P, it, K);
        const int s0 = G.s0, s1 = G.s1, Sn = G.Sn;
        const int rel = G.rel;  // n0rel = n0 - rel in [0, Sn + 2K)
        const int escale = G.escale;
        const float fscale = VAR == VAR_F32ATOM ? 1.0f : ldexpf(1.0f, escale);
        const int ncols = G.ncols;

        int head = 0, cnt = 0;
        uint32_t n_taps = 0, n_rec = 0, n_img = 0;  // per lane
        uint32_t n_rounds = 0, n_chunks = 0, n_steps = 0, n_defer = 0;  // per wave (uniform)

        auto round = [&]() {
            const int nact = cnt < 64 ? cnt : 64;
            const bool act = lane < nact;
            const int slot = (head + lane) & (kBufCap - 1);
            float f = 0.0f, g = 0.0f;
            int nr = 0;
            if (act) { f = S.bf[slot]; g = S.bg[slot]; nr = S.bn[slot]; }
            bool lead = act;
            int nd = 0;
            if (VAR == VAR_F32ATOM) {
                if (act) S.claim[nr] = 0xFFFFFFFFu;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                if (act) atomicMin(&S.claim[nr], (uint32_t)lane);
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                lead = act && (S.claim[nr] == (uint32_t)lane);
                const bool dfr = act && !lead;
                const uint64_t dm = ballot(dfr);
                nd = __popcll(dm);
                if (dfr) {
                    const int ts = (head + cnt + mbcnt(dm)) & (kBufCap - 1);
                    S.bf[ts] = f; S.bg[ts] = g; S.bn[ts] = nr;
                }
            }
            head = (head + nact) & (kBufCap - 1);
            cnt = cnt - nact + nd;
            ++n_rounds;
            n_defer += nd;
            if (lead) {
                // taps of this record that land in [s0, s1): n0 + k with n0 = nr + rel
                const int lo = max(nr + rel - (LAG ? 3 : K), s0), hi = min(nr + rel + K, s1 - 1);
                n_taps += hi >= lo ? (uint32_t)(hi - lo + 1) : 0u;
                ++n_rec;
                long long *a64 = S.acc64 + (nr + K);  // acc index of tap k is nr + K + k
                float *a32 = S.acc32 + (nr + K);
                if (LAG) {
                    taps_lagrange(a64, f, g * fscale);
                } else if (VAR == VAR_LUT) {
                    taps_lut<KT>(a64, K, S.lut, f, g * fscale);
                } else {
                    float a0, a1, a2;
                    tap_coeffs(f, g * fscale, Pw, K < 4, a0, a1, a2);
                    constexpr bool FX = VAR == VAR_FX;
                    if (KT > 0) taps_fp32_ct<(KT > 0 ? KT : 1), FX>(a64, a32, f, a0, a1, a2);
                    else taps_fp32_rt<FX>(a64, a32, K, S.trig, f, a0, a1, a2);
                }
            }
        };

        for (int c0 = 0; c0 < ncols; c0 += kCols) {
            // ---- column chunk: one (a, b) column per lane
            const Column C = column_setup(G, c0 + lane, order_mode, G.px0, G.pow_stride);
            ++n_chunks;
            const int ctot = C.len[0] + C.len[1] + C.len[2] + C.len[3];
            int T;
            const int off = wave_excl_scan(ctot, T);
            __syncthreads();
            S.coff[lane] = off;
            if (lane == 63) S.coff[64] = T;
            S.crho2[lane] = C.rho2;
            S.cbxy[lane] = C.bxy;
            S.cord[lane] = C.ord;
            int cum = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                cum += C.len[i];
                S.iq0[lane * 4 + i] = C.q0[i];
                S.icum[lane * 4 + i] = cum;
                S.iw[lane * 4 + i] = C.wv[i];
            }
            __syncthreads();

            // ---- flattened images of the chunk, one per lane per step
            const int nsteps = (T + 63) / 64;
            // each lane walks increasing flattened indices: find its first column once,
            // then advance column and interval incrementally
            int c = 0;
            {
                const int xs = P->interleave ? lane * nsteps : lane;
#pragma unroll
                for (int st = 32; st >= 1; st >>= 1)
                    if (S.coff[c + st] <= xs) c += st;
            }
            for (int js = 0; js < nsteps; ++js) {
                // interleaved: the 64 lanes of a step take images spread over the whole
                // chunk (different columns), so that their delays rarely coincide
                const int x = P->interleave ? lane * nsteps + js : js * 64 + lane;
                ++n_steps;
                bool valid = false;
                float rf = 0.0f, rg = 0.0f;
                int rn = 0;
                if (x < T) {
                    ++n_img;
                    while (S.coff[c + 1] <= x) ++c;
                    const int loc = x - S.coff[c];
                    const int e0 = S.icum[c * 4 + 0], e1 = S.icum[c * 4 + 1], e2 = S.icum[c * 4 + 2];
                    const int iv = (loc >= e0) + (loc >= e1) + (loc >= e2);
                    const int before = iv == 0 ? 0 : S.icum[c * 4 + iv - 1];
                    const int q = S.iq0[c * 4 + iv] + (loc - before);
                    const int w = S.iw[c * 4 + iv];
                    int n0;
                    double fr, d;
                    valid = image_eval(G, S.crho2[c], S.cord[c], q, w, order_mode, fs, cs, fsc, split32,
                                       LAG ? 0.0 : 0.5, n0, fr, d);
                    if (valid) {
                        const int ez0 = min(abs(q - w), G.pmax), ezL = min(abs(q), G.pmax);
                        const double B = (S.cbxy[c] * G.pz0[ez0]) * G.pzL[ezL];
                        // g = B / (4 pi d) to FP32 accuracy
                        rg = (float)B * (0.0795774715459477f * __builtin_amdgcn_rcpf((float)d));
                        rf = (float)fr;
                        if (!LAG && rf == 0.0f) rf = 0x1p-40f;  // integer delay: exact Kronecker limit
                        rn = n0 - rel;
                    }
                }
                const uint64_t vm = ballot(valid);
                if (valid) {
                    const int ts = (head + cnt + mbcnt(vm)) & (kBufCap - 1);
                    S.bf[ts] = rf; S.bg[ts] = rg; S.bn[ts] = rn;
                }
                cnt += __popcll(vm);
                while (cnt >= 64) round();
            }
        }
        while (cnt > 0) round();
        __syncthreads();

        // ---- store the segment (coalesced), then clear the accumulator
        CRoomDev &R = *room_ptr(P, it.room);
        GFloat *o = global_out(P->out) + R.out_offset + (long)(it.mic - R.mic_offset) * G.rir_len + s0;
        if (VAR == VAR_F32ATOM) {
            for (int i = lane; i < Sn; i += 64) o[i] = S.acc32[2 * K + i];
        } else {
            for (int i = lane; i < Sn; i += 64) o[i] = (float)ldexp((double)S.acc64[2 * K + i], -escale);
        }
        const int acc_n = Sn + 4 * K;
        __syncthreads();
        for (int i = lane; i < acc_n; i += 64) S.acc64[i] = 0;
        // work counters of the item (one atomic per wave)
        unsigned long long t = n_taps, r = n_rec, im = n_img;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            t += __shfl_xor(t, d, 64);
            r += __shfl_xor(r, d, 64);
            im += __shfl_xor(im, d, 64);
        }
        if (lane == 0) {
            atomicAdd(P->stats + 0, t);
            atomicAdd(P->stats + 1, r);
            atomicAdd(P->stats + 2, im);
            atomicAdd(P->stats + 3, (unsigned long long)n_rounds);
            atomicAdd(P->stats + 4, (unsigned long long)n_chunks);
            atomicAdd(P->stats + 5, (unsigned long long)n_steps);
            atomicAdd(P->stats + 6, (unsigned long long)n_defer);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- moment kernel
// One column of the moment kernel's enumeration batch, set up without branches (the same
// images as column_setup): horizontal distance, x/y wall powers, and per parity w the
// z-index range [qlo, qhi] of the shell minus the hole [hlo, hhi] under it, as the
// intervals "below" [qlo, hlo - 1] and "above" [hhi + 1, qhi] (or the whole range when
// the hole misses it).  The four candidate intervals are packed with the non-empty ones
// first, as 16-bit lengths and 2 q0 + w values.  Columns past the item's last and
// columns outside the shell get length 0.  Issue priority steps down through the stages
// (3, 2, 1) so that the waves set up their columns side by side.
struct MomColSetup {
    double rho2, bxy;
    uint64_t lens, qws;  // 4 x 16 bits each, non-empty intervals first
    int ctot, ord;
};

DEV MomColSetup mom_column(const ItemGeom &G, int ci, int order_mode, const double *px, int ps)
{
    __builtin_amdgcn_s_setprio(3);
    MomColSetup R;
    const int N = G.N;
    const bool inrange = ci < G.ncols;
    ci = inrange ? ci : 0;
    // ci / nb from a float reciprocal, corrected to the exact quotient (ci < 2^24)
    int ca = (int)((float)ci * G.inv_nb);
    ca -= ca * G.nb > ci;
    ca += (ca + 1) * G.nb <= ci;
    const int a = G.alo + ca, b = G.blo + (ci - ca * G.nb);
    const int u = a & 1, v = b & 1;
    const int n = (a + u) >> 1, l = (b + v) >> 1;
    const double X = (u ? -G.sx : G.sx) + (2.0 * (double)n) * G.Lx;
    const double Y = (v ? -G.sy : G.sy) + (2.0 * (double)l) * G.Ly;
    const double dx = X - G.rx, dy = Y - G.ry;
    const double rho2 = dx * dx + dy * dy;
    R.rho2 = rho2;
    __builtin_amdgcn_s_setprio(2);
    const int ordxy = order_mode == 0 ? abs(n) + abs(l) : abs(2 * n - u) + abs(2 * l - v);
    R.ord = ordxy;
    const bool ok = inrange && rho2 < G.dhi2 && (N < 0 || ordxy <= N);
    const int pmax = G.pmax;
    const int ex0 = min(abs(n - u), pmax), exL = min(abs(n), pmax);
    const int ey0 = min(abs(l - v), pmax), eyL = min(abs(l), pmax);
    R.bxy = ((px[ex0] * px[ps + exL]) * px[2 * ps + ey0]) * px[3 * ps + eyL];
    // z extent of the shell on this column; FP32 square roots, the bounds below widen the
    // intervals (and narrow the hole) by G.zeps, so any extra image lies outside the
    // shell and fails the delay test
    const double zb = (double)__builtin_amdgcn_sqrtf((float)fmax(G.dhi2 - rho2, 0.0));
    const double za = (double)__builtin_amdgcn_sqrtf((float)fmax(G.dlo2 - rho2, 0.0));
    const bool hole = G.dlo2 > rho2;
    const double inv2L = G.inv2Lz;
    uint32_t len[4];
    int qw[4];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        // dz = (+-sz + 2 q Lz) - rz; |q| stays far below 2^31 (wall exponents < 2^22, host)
        const double off = G.rz - (w ? -G.sz : G.sz);
        int qlo = (int)ceil((off - zb) * inv2L - G.zeps);
        int qhi = (int)floor((off + zb) * inv2L + G.zeps);
        if (N >= 0) {
            const int rem = N - ordxy;
            // (w - rem + 1) >> 1 = ceil((w - rem) / 2)
            const int lo = order_mode == 0 ? -rem : (w - rem + 1) >> 1;
            const int hi = order_mode == 0 ? rem : (w + rem) >> 1;
            qlo = max(qlo, lo);
            qhi = min(qhi, hi);
        }
        const int hlo = hole ? (int)ceil((off - za) * inv2L + G.zeps) : 1;
        const int hhi = hole ? (int)floor((off + za) * inv2L - G.zeps) : 0;
        const bool cut = hlo <= hhi && hhi >= qlo && hlo <= qhi;
        const int lb = cut ? hlo - qlo : qhi - qlo + 1;  // "below" (or the whole range)
        const int la = cut ? qhi - hhi : 0;              // "above"
        len[2 * w] = ok ? (uint32_t)max(lb, 0) : 0u;
        len[2 * w + 1] = ok ? (uint32_t)max(la, 0) : 0u;
        qw[2 * w] = 2 * qlo + w;
        qw[2 * w + 1] = 2 * (hhi + 1) + w;
    }
    __builtin_amdgcn_s_setprio(1);
    // pack: slot i goes to field pos_i = number of non-empty slots before it (an empty
    // slot contributes zero wherever it lands)
    uint64_t lens = 0, qws = 0;
    int pos = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t sh = 16u * (uint32_t)pos;
        lens |= (uint64_t)len[i] << sh;
        qws |= (uint64_t)(len[i] ? ((uint32_t)qw[i] & 0xFFFFu) : 0u) << sh;
        pos += len[i] ? 1 : 0;
    }
    R.lens = lens;
    R.qws = qws;
    R.ctot = (int)(len[0] + len[1] + len[2] + len[3]);
    return R;
}

// Same sum, reorganised around delay bins.  For fixed k, h(k - f) is an entire
// function of the fractional delay f in [-1/2, 1/2], so its Chebyshev series in
// x = 2f converges fast: with kMom = 9 terms, h(k - f) = sum_m c[m][k] T_m(2f) up to
// 3.3e-8 of max|h| = 1 (K = 40 and 63; 4.1e-8 for K = 4), below FP32 rounding; the
// 7th-order Lagrange filter is a polynomial of degree 7 in f, so its series is exact.
// A record (n0, f, g) then contributes sum_m c[m][k] (g T_m(2f)) to sample n0 + k, and
//     out[n] = sum_m sum_k c[m][k] U_m[n - k],   U_m[b] = sum over records with
//                                                n0 = b of g T_m(2 f),
// so each record only adds kMom moments into the bins of its n0 (a counting sort
// of the records by delay, with the sum per bin taken at once), and the 2K+1 taps
// per sample become a dense 2K+1-tap filter over kMom moment sequences.
//  * Moments are FP64 (recurrence T_{m+1} = 2x T_m - T_{m-1}), scaled by the item's
//    2^e, made non-negative (channel m >= 1 adds g (T_m + 1)), truncated to 32 bits and
//    added with ds_add_u64: the bin sums are exact integers, independent of the order
//    of the adds.  Channel 0's sum is taken off the others when the bins are read.
//  * One workgroup of kMomWaves waves owns one item.  Columns are set up 64 per
//    wave (kMomWaves chunks at a time); every thread then takes a contiguous slice
//    of the flattened images of those chunks, so all waves share the work of small
//    and large items alike.
//  * The filter is a GEMM on the matrix cores over the FP32 bins (see the kernel);
//    the partial tiles of the waves are summed in a fixed order and stored once per
//    sample.
constexpr int kMomThreads = 64 * kMomWaves;
static_assert(kMomSetupWaves == kMomWaves, "every wave sets up 64 columns of a batch");
constexpr int kMomCols = 64 * kMomSetupWaves;  // columns per enumeration batch

DEV int mpad(int i) { return i + (i >> 4); }

// One column of an enumeration batch: squared horizontal distance, x/y wall-power
// product, the column's images [start, end) in the batch's flattened order, and its
// intervals (non-empty ones first) as 16-bit fields: lengths, and first z index times 2
// plus parity.  16 bits hold them: with wall exponents below kPowCap, |q| < kPowCap and
// an interval has fewer than 2 kPowCap + 1 images.
struct alignas(16) MomCol {
    double rho2, bxy;
    int32_t start, end;
    uint32_t len01, len23;  // lengths of intervals 0, 1 (low, high half) and 2, 3
    int32_t qw01, qw23;     // 2 q0 + w of intervals 0, 1 and 2, 3 (signed halves)
    int32_t cord;           // x/y part of the reflection order
    int32_t pad;
};

DEV int col_len(const MomCol &m, int iv)
{
    const uint32_t v = iv < 2 ? m.len01 : m.len23;
    return (int)((v >> (16 * (iv & 1))) & 0xFFFFu);
}

DEV int col_qw(const MomCol &m, int iv)
{
    const int32_t v = iv < 2 ? m.qw01 : m.qw23;
    return (iv & 1) ? (v >> 16) : (int32_t)(int16_t)(v & 0xFFFF);
}

struct MomLds {
    long long *U;          // kMom x ustride int64 bins; then the filter's partial tiles
    MomCol *col;           // [kMomCols] column records; then the FP16 bins (hi, lo)
    int32_t *chunk;        // [1] next 64-column chunk of the item
    double *pzz;           // [4 kPowCap] z wall powers by (2 q + w), q in (-kPowCap, kPowCap)
    double *pxy;           // [4 kPowCap] x0, xL, y0, yL wall powers, kPowCap apart
    _Float16 *c16;         // [2 shifts][hi, lo][kMom][CL] FP16 coefficient rows (see the kernel)
    int32_t *item;         // [2] current and next item
    uint32_t *bmax;        // [4] largest channel-0 bin of the item (FP32 bits), its records,
                           // waves out of columns
    ItemGeom *gnext;       // the next item's geometry
};

DEV MomLds mom_carve(char *base, int K)
{
    MomLds s;
    char *p = base;
    s.U = (long long *)p; p += mom_u_bytes(K);
    s.col = (MomCol *)p; p += kMomCols * sizeof(MomCol);
    s.pzz = (double *)p; p += 4 * kPowCap * 8;
    s.pxy = (double *)p; p += 4 * kPowCap * 8;
    s.c16 = (_Float16 *)p; p += (size_t)4 * kMom * mom_cl(K) * 2;
    s.chunk = (int32_t *)p; p += kMomSetupWaves * 4;
    s.item = (int32_t *)p; p += 16;
    s.bmax = (uint32_t *)p; p += 16;
    s.gnext = (ItemGeom *)p;   // 16-byte aligned: every area above is a multiple of 16 bytes
    return s;
}

DEV void lds_add_u31(long long *p, double v)
{
    // 0 <= v < 2^31 (a slightly negative rounding result saturates to 0): truncated,
    // zero high word
    const unsigned long long q = (unsigned long long)(uint32_t)v;
    __hip_atomic_fetch_add((unsigned long long *)p, q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

typedef float f32x4_t __attribute__((ext_vector_type(4)));

typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));

// 8 consecutive FP16 values from a 4-byte aligned LDS address (four dword reads).
DEV f16x8_t lds_f16x8_a4(const _Float16 *p)
{
    const uint32_t *q = (const uint32_t *)p;
    typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
    u32x4_t v;
    v[0] = q[0];
    v[1] = q[1];
    v[2] = q[2];
    v[3] = q[3];
    return __builtin_bit_cast(f16x8_t, v);
}

// Partial tiles of the filter, one per (channel, tile of 256 output samples): 16 rows of 16
// floats, kPartPitch floats apart, at the start of the bins' area; kPartU4 16-byte units.
constexpr int kPartPitch = 17;
constexpr int kPartTiles = kMom * 4;
constexpr int kPartU4 = kPartTiles * 16 * kPartPitch * 4 / 16;
static_assert(kPartTiles * 16 * kPartPitch * 4 % 16 == 0, "whole 16-byte units");

// RED = true: the reduced-precision form (ISM_PREC_FP16_LUT on this kernel): kMomRed = 6
// Chebyshev terms (truncation below 1.3e-4 of max|h|), FP16 bins and FP16 coefficients
// without their low halves, one matrix-core product per step; delays, distances and the
// exact integer binning as in the full form.
template <int KT, bool RED>
__global__ __launch_bounds__(kMomThreads) void ism_moments(const LaunchDev *__restrict__ P)
{
    constexpr int K = KT;
    constexpr int NM = RED ? kMomRed : kMom;   // moment channels
    static_assert(kMom * mom_ustride(KT) * 4 <= kMomCols * (int)sizeof(MomCol),
                  "the FP32 bins fit the column-record area");
    static_assert(NM % 3 == 0 && NM <= kMom, "channels in groups of 3");
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = uniform(tid >> 6);
    const int ustride = mom_ustride(K);
    MomLds S = mom_carve(ism_lds, K);
    const double fs = P->fs, cs = P->c;
    const double fsc = fs / cs;
    const int order_mode = P->order_mode;
    const int split32 = P->split32;
    const bool lagrange = P->lagrange != 0;
    const double half = lagrange ? 0.0 : 0.5, xoff = lagrange ? 1.0 : 0.0;
    const int kmin = lagrange ? -3 : -K, kmax = lagrange ? 4 : K;
    uint64_t n_taps = 0;
    uint32_t n_rec = 0, n_img = 0;
    const int nU = NM * ustride;

    // wall-power tables of an item's room into LDS, one entry i < kTab per thread:
    // pzz[i = 2 (q + kPowCap) + w] = beta_z0^|q - w| beta_zL^|q|; pxy[i] = x0, xL, y0, yL
    // powers, kPowCap apart (|q|, exponents <= pmax < kPowCap: pow_stride <= kPowCap on the
    // host).  The entry's loads (table_load, into registers) are issued well before its
    // stores (table_store), with other work between.
    constexpr int kTab = 4 * kPowCap;
    typedef const __attribute__((address_space(1))) double GDouble;
    auto table_load = [&](int pow_offset, int stride, int i, double (&v)[3]) {
        // opaque copy of i: keeps the index arithmetic here instead of being hoisted out
        // of the item loop, where it would hold registers through the walk
        asm volatile("" : "+v"(i));
        const int pmax = stride - 1;
        GDouble *px = (GDouble *)P->pow_tab + pow_offset;
        GDouble *pz0 = px + 4 * stride, *pzL = pz0 + stride;
        const int q = (i >> 1) - kPowCap, w = i & 1;
        v[0] = pz0[min(abs(q - w), pmax)];
        v[1] = pzL[min(abs(q), pmax)];
        v[2] = px[(i / kPowCap) * stride + min(i % kPowCap, pmax)];
    };
    auto table_store = [&](int i, const double (&v)[3]) {
        S.pzz[i] = v[0] * v[1];
        S.pxy[i] = v[2];
    };
    // The index of the current item alternates between S.item[0] and S.item[1]: the first
    // wave to run out of columns fetches the next item and writes its geometry to LDS; its
    // tables are filled during the filter.
    // FP16 coefficient rows of the filter (see there): row (sh, hl, m) holds at index i the
    // reversed tap t = i + sh - 16 of channel m, c[m][2K - t] (zero outside [0, 2K]),
    // scaled by 2^coef_exp, as hi = fp16(c) (hl = 0) and lo = fp16(c - hi) (hl = 1); the
    // copy shifted by one (sh = 1) lets every lane read its 8 taps from a 4-byte boundary
    constexpr int CL = mom_cl(K);
    {
        const float cscale = ldexpf(1.0f, P->coef_exp);
        for (int i = tid; i < 2 * kMom * CL; i += kMomThreads) {
            const int row = i / CL, idx = i - row * CL;
            const int sh = row / kMom, m = row - sh * kMom;
            const int t = idx + sh - 16;
            const float c = (t >= 0 && t <= 2 * K) ? (float)(P->coef[m * (2 * K + 1) + 2 * K - t] * cscale) : 0.0f;
            const _Float16 hi = (_Float16)c;
            const _Float16 lo = (_Float16)(c - (float)hi);
            S.c16[((sh * 2 + 0) * kMom + m) * CL + idx] = hi;
            S.c16[((sh * 2 + 1) * kMom + m) * CL + idx] = lo;
        }
    }
    // The bins are cleared here for the first item; for later items their area beyond the
    // partial tiles is cleared during the previous item's filter and the partial tiles'
    // area at the item's start, once the store has read it.
    typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
    u32x4_t *const zb = (u32x4_t *)S.U;
    const u32x4_t zero4 = {0u, 0u, 0u, 0u};
    static_assert(NM * mom_ustride(KT) / 2 >= kPartU4, "the bins cover the partial tiles");
    for (int i = tid; i < nU / 2; i += kMomThreads) zb[i] = zero4;
    if (tid == 0) S.item[0] = fetch_item(P->counter);
    __syncthreads();
    {
        const int first = uniform(S.item[0]);
        if (first < P->n_items && wave == 0) {
            const ItemGeom G0 = item_geom(P, load_item(P, first), K);
            if (lane == 0) *S.gnext = G0;
        }
        if (first < P->n_items && tid < kTab) {
            CItemDev &f = ((CItemDev *)P->items)[first];
            double tv[3];
            table_load(f.pow_offset, f.pow_stride, tid, tv);
            table_store(tid, tv);
        }
    }
    __syncthreads();  // the first item's geometry
    for (int iter = 0;; ++iter) {
        const int item = uniform(S.item[iter & 1]);
        if (item >= P->n_items) break;
        // the partial tiles' area of the bins (the rest was cleared during the last filter)
        for (int i = tid; i < kPartU4; i += kMomThreads) zb[i] = zero4;
        if (tid == 0) {
            S.bmax[0] = 0u;
            S.bmax[1] = 0u;
            S.bmax[2] = 0u;
            S.chunk[0] = 0;
        }
        const ItemDev it = load_item(P, item);
        // the geometry the first wave out of columns derived during the last item (the first
        // item's, by wave 0 before the loop)
        const ItemGeom G = geom_from_lds(S.gnext);
        const double gk = 0.07957747154594767 * ldexp(1.0, G.escale);  // 2^e / (4 pi), exact scaling
        // taps landing in [s0, s1) per record: W minus those cut at either end,
        // max(0, tL - n0) + max(0, n0 - tR) = |med3(n0, lo, hi) - n0| + max(0, tL - tR)
        const int tL = G.s0 - kmin, tR = G.s1 - 1 - kmax;
        const int tlo = min(tL, tR), thi = max(tL, tR);
        uint32_t rec_item = 0, loss_item = 0;
        // rounding-boundary test of the delay split (image_eval_z)
        const double ec = half - 0.5, ethr = 0.5 - 1e-12 * ((double)G.nhi + 2.0);
        __syncthreads();  // bins zeroed, tables of this item complete

        // ---- records: moments into the delay bins.  Each wave takes chunks of 64 columns
        //      from a workgroup counter, sets them up (one per lane), writes their records
        //      to its own 64 slots and walks their images; no workgroup barrier until the
        //      item's columns are done, so waves never wait for each other's batches.
        MomCol *wcol = S.col + 64 * wave;
        for (;;) {
            int ch = 0;
            if (lane == 0) ch = atomicAdd(S.chunk, 1);
            const int c0 = 64 * __builtin_amdgcn_readfirstlane(__shfl(ch, 0, 64));
            if (c0 >= G.ncols) {
                // The first wave out of columns fetches the next item and derives its
                // geometry into LDS (while the other waves finish their chunks); the index
                // is published for the table loads after the enumeration barrier.
                uint32_t out = 0;
                if (lane == 0) out = atomicAdd(S.bmax + 2, 1u);
                if (__builtin_amdgcn_readfirstlane(out) == 0) {
                    int nx = 0;
                    if (lane == 0) nx = fetch_item(P->counter);
                    nx = __builtin_amdgcn_readfirstlane(nx);
                    if (nx < P->n_items) {
                        const ItemGeom GN = item_geom(P, load_item(P, nx), K);
                        if (lane == 0) *S.gnext = GN;
                    }
                    if (lane == 0) S.item[(iter + 1) & 1] = nx;
                }
                break;
            }
            const MomColSetup C = mom_column(G, c0 + lane, order_mode, S.pxy, kPowCap);
            __builtin_amdgcn_s_setprio(0);
            const int ctot = C.ctot;
            const int incl = wave_incl_scan_dpp(ctot);
            const int Tall = __builtin_amdgcn_readlane(incl, 63);
            const int off = incl - ctot;
            {
                MomCol mc;
                mc.rho2 = C.rho2;
                mc.bxy = C.bxy * gk;  // x/y wall powers times 2^e / (4 pi)
                mc.start = off;
                mc.end = off + ctot;
                mc.len01 = (uint32_t)C.lens;
                mc.len23 = (uint32_t)(C.lens >> 32);
                mc.qw01 = (int32_t)(uint32_t)C.qws;
                mc.qw23 = (int32_t)(uint32_t)(C.qws >> 32);
                mc.cord = C.ord;
                mc.pad = 0;
                wcol[lane] = mc;  // read back by this wave only (LDS keeps a wave's order)
            }

            // lane t takes the images [t n, (t + 1) n) of the chunk: consecutive lanes sit in
            // different columns, so their delays rarely coincide.  The walk state (column
            // record, interval, z index, images left in the interval, z-power table index)
            // stays in registers; the next record is read only when the column ends.  The
            // loop runs n times in every wave (scalar control); lanes past their last image
            // idle.
            const int n = (Tall + 63) >> 6;
            const int x0 = lane * n;
            const int cnt = max(0, min(n, Tall - x0));
            n_img += (uint32_t)cnt;
            if (cnt > 0) {
                int c = 0;
#pragma unroll
                for (int st = 32; st >= 1; st >>= 1)
                    if (wcol[c + st].start <= x0) c += st;
                MomCol mc = wcol[c];
                int loc = x0 - mc.start, iv = 0;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const int l = col_len(mc, iv);
                    if (loc >= l) { loc -= l; ++iv; }
                }
                int qwv = col_qw(mc, iv);
                int q = (qwv >> 1) + loc, w = qwv & 1, rem = col_len(mc, iv) - loc;
                double zw = w ? -G.sz : G.sz;
                int pz = 2 * (q + kPowCap) + w;  // S.pzz index of (q, w); |q| <= pmax < kPowCap
                for (int k = 0; k < n; ++k) {
                    if (k >= cnt) continue;
                    int n0;
                    double fr, d, rd;
                    if (image_eval_z(G, mc.rho2, mc.cord, q, w, zw, order_mode, fs, cs, fsc, split32, half, ec,
                                     ethr, n0, fr, d, rd)) {
                        const double Bg = mc.bxy * S.pzz[pz];
                        ++rec_item;
                        {   // loss += |med3(n0, tlo, thi) - n0| (both non-negative)
                            const uint32_t a = (uint32_t)min(max(n0, tlo), thi);
                            asm("v_sad_u32 %0, %1, %2, %0" : "+v"(loss_item) : "v"(a), "v"(n0));
                        }
                        // g 2^e = B 2^e / (4 pi d) in FP64, 1/d from the square root's iteration
                        // (relative error far below the 2^-30 fixed-point step)
                        const double gs = Bg * rd;
                        // Chebyshev variable: x = 2f for f in [-1/2, 1/2) (sinc), 2f - 1 for f in [0, 1)
                        const double xx = fma(2.0, fr, -xoff), x2 = xx + xx;
                        // bins: channel 0 adds g, channel m >= 1 adds g (T_m + 1) in [0, 2g]:
                        // non-negative, so no sign extension; the bias (channel 0's sum) is
                        // taken off when the bins are read
                        long long *u = S.U + (n0 - G.rel);
                        // channels 7.. from a second base (LDS instruction offsets have 16 bits);
                        // the opaque index keeps the compiler from folding it back per channel
                        int i7 = n0 - G.rel + 7 * ustride;
                        asm("" : "+v"(i7));
                        long long *u7 = S.U + i7;
                        double tp = 1.0, tc = xx;
                        lds_add_u31(u, gs);
                        lds_add_u31(u + ustride, fma(gs, xx, gs));
#pragma unroll
                        for (int m = 2; m < NM; ++m) {
                            const double tn = fma(x2, tc, -tp);
                            lds_add_u31(m < 7 ? u + m * ustride : u7 + (m - 7) * ustride, fma(gs, tn, gs));
                            tp = tc;
                            tc = tn;
                        }
                    }
                    ++q;
                    pz += 2;
                    if (--rem == 0 && k + 1 < cnt) {  // next non-empty interval, in this column or a later one
                        ++iv;
                        int l = iv < 4 ? col_len(mc, iv) : 0;
                        while (l == 0) {
                            mc = wcol[++c];
                            iv = 0;
                            l = col_len(mc, 0);
                        }
                        qwv = col_qw(mc, iv);
                        q = qwv >> 1;
                        w = qwv & 1;
                        zw = w ? -G.sz : G.sz;
                        pz = 2 * (q + kPowCap) + w;
                        rem = l;
                    }
                }
            }
        }
        __syncthreads();  // every chunk of the item is binned; the next item's index and geometry

        n_rec += rec_item;
        n_taps += (unsigned long long)rec_item * (unsigned)(kmax - kmin + 1 - max(0, tL - tR)) - loss_item;

        // the next item's wall-power table location, loaded now (vector memory: its wait
        // does not hold up the LDS work below) for the table entries loaded during the filter
        const int nxt = uniform(S.item[(iter + 1) & 1]);
        const bool fill = nxt < P->n_items && tid < kTab;
        int nxt_pow_offset = 0, nxt_pow_stride = 1;
        if (fill) {
            const __attribute__((address_space(1))) ItemDev *ni =
                (const __attribute__((address_space(1))) ItemDev *)P->items + nxt;
            nxt_pow_offset = ni->pow_offset;
            nxt_pow_stride = ni->pow_stride;
        }

        // ---- bins to FP16 pairs in the column-record area: V_m = U_m - U_0 for m >= 1 (the
        //      bias), exact in int64 and in the double; scaled by 2^bexp so that |V| <= 2^13;
        //      hi = fp16(V), lo = fp16(V - hi) (22 significant bits); zeros past the last delay.
        //      Each record adds to bin i of channel m >= 1 a value within 1 of g (T_m + 1) and
        //      to channel 0 one within 1 of g, so |V_m[i]| < U_0[i] + 2 (records in bin i): the
        //      scale comes from max U_0 + 2 (records of the item).
        constexpr int NB = kMomSegMax + 2 * K;
        constexpr int NBP = mom_nbp(K);
        {
            long long mx = 0;
            for (int i = tid; i < NB; i += kMomThreads) mx = max(mx, S.U[i]);
            // the wave's largest bin and record total by DPP moves, in lane 63 (mx >= 0, so
            // FP32 bit patterns order as the values)
            const uint32_t fb = wave_incl_max_dpp(__float_as_uint((float)mx));
            const int rc = wave_incl_scan_dpp((int)rec_item);
            if (lane == 63) {
                if (fb) atomicMax(S.bmax, fb);
                atomicAdd(S.bmax + 1, (uint32_t)rc);
            }
        }
        __syncthreads();
        int bexp;
        {
            int E = 0;
            // bound <= 2^E; the FP32 roundings may raise it by a few ulps, below 2^13 of margin
            (void)frexpf(__uint_as_float(S.bmax[0]) + 2.0f * (float)S.bmax[1], &E);
            bexp = 13 - E;
        }
        _Float16 *Uh = (_Float16 *)S.col, *Ul = Uh + kMom * NBP;
        {
            // work units (bins i, i + 1, group of 3 channels); the bin sums are below 2^53, so the
            // doubles are exact, and so is fma(U_m, 2^bexp, -U_0 2^bexp); one rounding to FP32
            const double bs = ldexp(1.0, bexp);
            auto u64d = [](long long v) {  // exact for 0 <= v < 2^53
                const unsigned long long u = (unsigned long long)v;
                return fma((double)(uint32_t)(u >> 32), 4294967296.0, (double)(uint32_t)u);
            };
            // two consecutive bins per work unit: 16-byte reads of the int64 pairs and 4-byte
            // writes of the FP16 pairs (NB, NBP and the channel stride are even)
            static_assert(NB % 2 == 0 && NBP % 2 == 0 && mom_ustride(KT) % 2 == 0, "bin pairs");
            typedef long long i64x2_t __attribute__((ext_vector_type(2)));
            typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
            auto put2 = [&](int e, float xa, float xb) {
                const f16x2_t hi = {(_Float16)xa, (_Float16)xb};
                *(f16x2_t *)(Uh + e) = hi;
                if (!RED) *(f16x2_t *)(Ul + e) = f16x2_t{(_Float16)(xa - (float)hi[0]), (_Float16)(xb - (float)hi[1])};
            };
            constexpr int NB2 = NB / 2;
            for (int w = tid; w < (NM / 3) * NB2; w += kMomThreads) {
                const int g = w / NB2, i = 2 * (w - g * NB2);
                // all four reads first (the stores below may alias them as far as the compiler
                // knows, and would otherwise wait for each read in turn)
                const i64x2_t v0 = *(const i64x2_t *)(S.U + i);
                i64x2_t v[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) v[k] = *(const i64x2_t *)(S.U + (3 * g + k) * ustride + i);
                const double u0a = u64d(v0[0]) * bs, u0b = u64d(v0[1]) * bs;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int m = 3 * g + k;
                    const double da = fma(u64d(v[k][0]), bs, -u0a), db = fma(u64d(v[k][1]), bs, -u0b);
                    put2(m * NBP + i, (float)(m ? da : u0a), (float)(m ? db : u0b));
                }
            }
            if constexpr (NBP > NB) {  // zeros past the last delay
                for (int e = tid; e < NM * (NBP - NB); e += kMomThreads) {
                    const int m = e / (NBP - NB), i = NB + e - m * (NBP - NB);
                    Uh[m * NBP + i] = (_Float16)0.0f;
                    if (!RED) Ul[m * NBP + i] = (_Float16)0.0f;
                }
            }
        }
        __syncthreads();

        // ---- the filter as a GEMM on the matrix cores, split FP16 products with FP32 sums
        //      (v_mfma_f32_16x16x32_f16: hi*hi + hi*lo + lo*hi per step):
        //      OUT[r][b] = sum_m sum_j A_m[r][j] B_m[j][b], output sample 16 b + r of a tile,
        //      A_m[r][j] = c_m[2K - (j - r)] (zero outside the band), B_m[j][b] = bin 16 b + j,
        //      j in [0, JP), 32 per step.  Lane l holds A[l % 16][8 (l / 16) + e] and
        //      B[8 (l / 16) + e][l % 16], e < 8, and D[4 (l / 16) + v][l % 16] in acc[v].
        // Wave w < 8 takes channel w over the 4 tiles of 256 output samples (one accumulator
        // per tile), so a step's coefficient fragments are read once for the four tiles; a
        // ninth channel goes one tile each to waves 12..15 (one per SIMD).  The partial tile
        // of each (channel, tile) is summed over the channels in the store.
        {
            constexpr int JP = mom_jp(K), NS = JP / 32;
            const int r16 = lane & 15, kq = lane >> 4;
            // the next item's wall-power table entries: loads issued before the tasks, stored
            // after them (this item no longer reads the tables)
            double tv[3];
            if (fill) table_load(nxt_pow_offset, nxt_pow_stride, tid, tv);
            // A fragments of channel m, step s: taps j - r = 32 s + 8 kq + e - r, stored at
            // index + 16; odd starts read the copy shifted by one
            auto coef_row = [&](int m, int s) {
                const int t0 = 32 * s + 8 * kq - r16 + 16, sh = t0 & 1;
                return S.c16 + ((sh * 2) * kMom + m) * CL + (t0 - sh);
            };
            // the int64 bins are no longer read: their area takes the partial tiles, rows
            // kPartPitch floats apart (the store below reads down a column without bank
            // conflicts); D[i][b]: b = lane % 16, i = 4 (lane / 16) + v
            auto put_part = [&](int m, int tile, const f32x4_t &acc) {
                float *part = (float *)S.U + (m * 4 + tile) * 16 * kPartPitch;
#pragma unroll
                for (int v = 0; v < 4; ++v) part[(4 * kq + v) * kPartPitch + r16] = acc[v];
            };
            if (wave < 8 && wave < NM) {
                const int m = wave;
                f32x4_t acc[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[t] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
                for (int s = 0; s < NS; ++s) {
                    const _Float16 *crow = coef_row(m, s);
                    const f16x8_t ah = lds_f16x8_a4(crow);
                    f16x8_t al;
                    if (!RED) al = lds_f16x8_a4(crow + kMom * CL);
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int bb = m * NBP + 256 * t + 16 * r16 + 8 * kq + 32 * s;
                        const f16x8_t bh = *(const f16x8_t *)(Uh + bb);
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, acc[t], 0, 0, 0);
                        if (!RED) {
                            const f16x8_t bl = *(const f16x8_t *)(Ul + bb);
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, acc[t], 0, 0, 0);
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, acc[t], 0, 0, 0);
                        }
                    }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) put_part(m, t, acc[t]);
            } else if (NM > 8 && wave >= 12) {
                const int m = 8, t = wave - 12;
                f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const _Float16 *crow = coef_row(m, s);
                    const int bb = m * NBP + 256 * t + 16 * r16 + 8 * kq + 32 * s;
                    const f16x8_t ah = lds_f16x8_a4(crow);
                    const f16x8_t bh = *(const f16x8_t *)(Uh + bb);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, acc, 0, 0, 0);
                    if (!RED) {
                        const f16x8_t al = lds_f16x8_a4(crow + kMom * CL);
                        const f16x8_t bl = *(const f16x8_t *)(Ul + bb);
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, acc, 0, 0, 0);
                        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, acc, 0, 0, 0);
                    }
                }
                put_part(m, t, acc);
            }
            if (fill) table_store(tid, tv);
            // the rest of the bins' area is cleared for the next item
            for (int i = kPartU4 + tid; i < nU / 2; i += kMomThreads) zb[i] = zero4;
        }
        __syncthreads();
        {
            CRoomDev &R = *room_ptr(P, it.room);
            GFloat *o = global_out(P->out) + R.out_offset + (long)(it.mic - R.mic_offset) * G.rir_len + G.s0;
            const double inv = ldexp(1.0, -G.escale - bexp - P->coef_exp);
            const float *part = (const float *)S.U;
            for (int i = tid; i < G.Sn; i += kMomThreads) {
                const int blk = i >> 4, row = i & 15, tl = blk >> 4, col = blk & 15;
                double v = 0.0;
#pragma unroll
                for (int m = 0; m < NM; ++m) v += (double)part[(m * 4 + tl) * 16 * kPartPitch + row * kPartPitch + col];
                o[i] = (float)(v * inv);
            }
        }
        __syncthreads();
    }

    // work counters (one atomic per wave and counter)
    unsigned long long t = n_taps, r = n_rec, im = n_img;
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1) {
        t += __shfl_xor(t, dd, 64);
        r += __shfl_xor(r, dd, 64);
        im += __shfl_xor(im, dd, 64);
    }
    if (lane == 0) {
        atomicAdd(P->stats + 0, t);
        atomicAdd(P->stats + 1, r);
        atomicAdd(P->stats + 2, im);
    }
}

// ---------------------------------------------------------------- launch glue
template <int KT, int VAR>
static hipError_t launch_t(const LaunchDev *P, int grid, int lds, hipStream_t st)
{
    hipLaunchKernelGGL((ism_segments<KT, VAR>), dim3(grid), dim3(64), lds, st, P);
    return hipGetLastError();
}

typedef hipError_t (*LaunchFn)(const LaunchDev *, int, int, hipStream_t);
typedef const void *KernelSym;

template <int KT, int VAR>
static const void *sym_t() { return reinterpret_cast<const void *>(&ism_segments<KT, VAR>); }

struct KernelEntry { LaunchFn fn; const void *sym; };

KernelEntry select_segment_kernel(int K, int variant)
{
    if (variant == VAR_LAG) return {launch_t<4, VAR_LAG>, sym_t<4, VAR_LAG>()};
#define ISM_CASE(KK)                                                                      \
    if (K == KK) {                                                                        \
        if (variant == VAR_LUT) return {launch_t<KK, VAR_LUT>, sym_t<KK, VAR_LUT>()};      \
        if (variant == VAR_F32ATOM) return {launch_t<KK, VAR_F32ATOM>, sym_t<KK, VAR_F32ATOM>()}; \
        return {launch_t<KK, VAR_FX>, sym_t<KK, VAR_FX>()};                                \
    }
    ISM_CASE(4)
    ISM_CASE(40)
    ISM_CASE(63)
#undef ISM_CASE
    if (variant == VAR_LUT) return {launch_t<0, VAR_LUT>, sym_t<0, VAR_LUT>()};
    if (variant == VAR_F32ATOM) return {launch_t<0, VAR_F32ATOM>, sym_t<0, VAR_F32ATOM>()};
    return {launch_t<0, VAR_FX>, sym_t<0, VAR_FX>()};
}

template <int KT, bool RED>
static hipError_t launch_m(const LaunchDev *P, int grid, int lds, hipStream_t st)
{
    hipLaunchKernelGGL((ism_moments<KT, RED>), dim3(grid), dim3(kMomThreads), lds, st, P);
    return hipGetLastError();
}

template <int KT, bool RED>
static const void *sym_m() { return reinterpret_cast<const void *>(&ism_moments<KT, RED>); }

// Moment kernel for the compiled half-lengths (full or reduced precision); {nullptr,
// nullptr} otherwise.
KernelEntry select_moment_kernel(int K, bool reduced)
{
    if (K == 4) return reduced ? KernelEntry{launch_m<4, true>, sym_m<4, true>()} : KernelEntry{launch_m<4, false>, sym_m<4, false>()};
    if (K == 40) return reduced ? KernelEntry{launch_m<40, true>, sym_m<40, true>()} : KernelEntry{launch_m<40, false>, sym_m<40, false>()};
    if (K == 63) return reduced ? KernelEntry{launch_m<63, true>, sym_m<63, true>()} : KernelEntry{launch_m<63, false>, sym_m<63, false>()};
    return {nullptr, nullptr};
}

hipError_t launch_prologue(const LaunchDev *P, int n_rooms, hipStream_t st)
{
    const int n = n_rooms * 6 > 0 ? n_rooms * 6 : 1;
    hipLaunchKernelGGL(ism_prologue, dim3((n + 255) / 256), dim3(256), 0, st, P);
    return hipGetLastError();
}

}  // namespace ism
