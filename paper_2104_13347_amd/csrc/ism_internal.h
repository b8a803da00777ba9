// Internal layout shared by the HIP kernels and the host side of libism.so.
#pragma once
#include <stdint.h>

namespace ism {

// Work of one segment kernel launch lives in one device buffer: a LaunchDev
// header, the room table, microphone positions, work items and the wall-power
// tables.  Every scalar a kernel needs is read from the header, so a captured
// graph of the launch sequence stays valid for any batch that fits the buffer.

struct alignas(16) RoomDev {
    double L[3];
    double beta[6];
    double src[3];
    int32_t rir_len;
    int32_t max_order;
    int32_t n_mics;
    int32_t mic_offset;
    int64_t out_offset;
    int32_t pow_offset;  // wall-power tables at pow_tab[pow_offset + wall * pow_stride + e]
    int32_t pow_stride;  // exponents 0 .. pow_stride-1
    double inv_L[3];     // 1 / L (index bounds, which carry a margin of one)
};

// One work item: output samples [s0, s1) of the RIR of microphone `mic`
// (absolute index into the microphone table) of room `room`.
struct alignas(16) ItemDev {
    int32_t room;
    int32_t mic;
    int32_t s0;
    int32_t s1;
    int32_t pow_offset;  // the room's wall-power tables (copies of its RoomDev fields)
    int32_t pow_stride;
    int32_t pad[2];
};

enum Variant : int32_t { VAR_FX = 0, VAR_LUT = 1, VAR_F32ATOM = 2, VAR_LAG = 3 };

struct alignas(16) LaunchDev {
    double fs;
    double c;
    const RoomDev *rooms;
    const double *mics;
    const ItemDev *items;
    double *pow_tab;
    float *out;
    uint32_t *counter;  // persistent-kernel work counter, zeroed by the prologue
    unsigned long long *stats;  // [taps landing in outputs, records, images tested], zeroed by the prologue
    int32_t n_rooms;
    int32_t n_items;
    int32_t K;            // (fd_taps - 1) / 2
    int32_t order_mode;   // 0 index-L1, 1 reflections
    int32_t lagrange;     // 1: the 7th-order Lagrange filter (taps n0-3..n0+4, n0 = floor(tau)), K = 4
    int32_t split32;      // 1: distance and delay split in FP32 (ablation)
    int32_t seg_max;      // largest s1 - s0 of any item (sizes LDS)
    int32_t interleave;   // enumeration order inside a column chunk (1: strided over columns)
    int32_t coef_exp;     // moment kernel: the coefficients are scaled by 2^coef_exp (max <= 2^14)
    int32_t reserved1;
    const double *coef;   // moment kernel: Chebyshev filter coefficients [kMom][2K+1]
};

constexpr int kSegMaxLimit = 2048;  // largest supported segment (per-lane sums in registers)
constexpr int kKMax = 127;          // largest half-length (255 taps)
constexpr int kLagrangeTaps = 8;    // fd_taps value that selects the 7th-order Lagrange filter

// Half-length of the symmetric tap window that holds the filter: (fd_taps - 1) / 2 for the
// windowed sinc, 4 for the Lagrange filter (taps k = -3..4 about n0; tap -4 is zero).
constexpr int half_length(int fd_taps) { return fd_taps == kLagrangeTaps ? 4 : (fd_taps - 1) / 2; }
constexpr int kLutQ = 64;           // FP16 table steps per sample
constexpr int kBufCap = 256;        // record ring (power of two)
constexpr int kCols = 64;           // columns per enumeration chunk (one per lane)

// Moment kernel: Chebyshev moments per delay bin, waves per workgroup, largest segment.
constexpr int kMom = 9;
constexpr int kMomRed = 6;          // terms of the reduced-precision form
constexpr int kMomWaves = 16;       // waves per workgroup (one item per workgroup)
constexpr int kMomSetupWaves = 16;  // waves that set up a batch of image columns, 64 each
constexpr int kMomSegMax = 1024;
constexpr int kPowCap = 128;        // moment kernel: wall exponents below kPowCap (z powers in LDS)

// Moment kernel bins of one channel: delays n0 - (s0 - K) in [0, kMomSegMax + 2K).
constexpr int mom_ustride(int K) { return kMomSegMax + 2 * K; }
// The filter's K dimension per 16-sample output block (16 + 2K bins), rounded up to the
// 32 of one FP16 matrix-core step.
constexpr int mom_jp(int K) { return (16 + 2 * K + 31) / 32 * 32; }
// FP16 bins of one channel: every bin a step reads (1008 + JP), zeros past the last delay.
constexpr int mom_nbp(int K)
{
    return ((kMomSegMax + 2 * K > 1008 + mom_jp(K) ? kMomSegMax + 2 * K : 1008 + mom_jp(K)) + 7) / 8 * 8;
}
// FP16 coefficient row: reversed taps at offset 16, JP + 16 halves read, padded.
constexpr int mom_cl(int K) { return mom_jp(K) + 32; }

// Bytes of the moment kernel's int64 bins, rounded up to 128 so that the 16-byte column
// records after them stay aligned.
constexpr int mom_u_bytes(int K) { return (kMom * mom_ustride(K) * 8 + 127) & ~127; }

// LDS bytes that hold one work item's geometry (the kernel checks its struct fits).
constexpr int kMomGeomBytes = 256;

inline int mom_lds_bytes(int K)
{
    const int cols = 64 * kMomSetupWaves;
    int bytes = mom_u_bytes(K);
    bytes += cols * 48 + kMomSetupWaves * 4 + 32;                  // column records, slots
    bytes += kMomGeomBytes;                                        // the next item's geometry
    bytes += 2 * 4 * kPowCap * 8;                                  // z and x/y wall powers
    bytes += 4 * kMom * mom_cl(K) * 2;                             // FP16 coefficient rows
    return bytes;
}

// LDS bytes of the segment kernel for a given segment capacity, K and variant.
inline int seg_lds_bytes(int seg_max, int K, int variant)
{
    int acc = (seg_max + 4 * K + 63) / 64 * 64;         // int64 (FP32 in the atomic ablation)
    int clm = variant == VAR_F32ATOM ? (seg_max + 2 * K + 63) / 64 * 64 : 0;  // uint32
    int bytes = acc * 8 + clm * 4;
    bytes += kBufCap * 12;                              // f, g, n0rel
    bytes += (kCols + 4) * 4 + kCols * 8 * 2 + kCols * 4 + kCols * 4 * 3 * 4;  // column chunk
    bytes += (2 * K + 1) * 8;                           // generic-K trig table
    if (variant == VAR_LUT) bytes += (2 * K + 1) * kLutQ * 4;
    return bytes;
}

}  // namespace ism
