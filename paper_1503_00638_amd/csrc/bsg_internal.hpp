// Internal declarations shared by the bsg HIP translation units (gfx950).
//
// Masui et al., arXiv:1503.00638.  Stage 1 (Section 3): noise-relative
// rounding.  Stage 2 (Section 4.2): Bitshuffle = bit transpose within blocks
// followed by per-block LZ4.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "bsg.h"

namespace bsg {

constexpr int kWave = 64;
constexpr int kHeaderBytes = 24;
constexpr int kDefaultBlockBytes = 8192;

// Fixed LZ4 match rule (a format constant: changing any of these changes the
// compressed bytes).
constexpr int kHashBits = 9;
constexpr uint32_t kHashMult = 2654435761u;
constexpr int kChunk = 64;       // the candidate table is updated per 64 positions
constexpr int kMinMatch = 4;     // LZ4 codes match lengths as length - 4
constexpr int kMinTake = 12;     // the rule takes matches of >= 12 bytes only
constexpr int kMfLimit = 12;     // a match starts at p <= len - 12
constexpr int kLastLiterals = 5; // the last 5 bytes are literals
constexpr int kGroup = 512;      // positions hashed before each parse step (8 chunks)

__host__ __device__ inline int64_t lz4_bound(int64_t s) { return s + s / 255 + 16; }

// n elements cut into blocks of nb: n_full whole blocks, then one partial
// block of `last` = floor(rem / 8) * 8 elements, then `tail` = n mod 8 raw
// elements.
struct Layout {
    int64_t n, E, nb, n_full, last, n_blocks, tail;
    int64_t block_bytes() const { return nb * E; }
    int64_t elems(int64_t b) const { return b < n_full ? nb : last; }
};

int64_t block_elems(int64_t E, int64_t block_size);
bool make_layout(int64_t n, int64_t E, int64_t block_size, Layout *L);

// Elements one lane transposes in registers ("unit") for the fast paths:
// 128 bytes for E <= 4, 32 elements (one 32x32 bit matrix per 4-byte
// column) for E a multiple of 4.  0 = no fast path for this E.
__host__ __device__ inline int unit_elems(int64_t E)
{
    if (E == 1) return 128;
    if (E == 2) return 64;
    if (E % 4 == 0 && E <= 16) return 32;
    return 0;
}

// ---------------------------------------------------------------------------
// Register bit transpose.  a[i] bit j -> a[j] bit i for a 32x32 bit matrix.
// The 16- and 8-bit block swaps are byte permutes (v_perm_b32); the 4-, 2-
// and 1-bit swaps are shift + bitfield-insert pairs.  Its own inverse.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel)
{
    // result byte i = byte sel[i] of the 8-byte value {hi, lo} (lo = bytes 0..3)
    return __builtin_amdgcn_perm(hi, lo, sel);
}

template <int J>
__device__ __forceinline__ void swap_stage(uint32_t (&a)[32], uint32_t m)
{
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        if (k & J) continue;
        const uint32_t x = a[k], y = a[k + J];
        const uint32_t mh = m << J;
        a[k] = (x & ~mh) | ((y << J) & mh);
        a[k + J] = (y & ~m) | ((x >> J) & m);
    }
}

__device__ __forceinline__ void transpose32(uint32_t (&a)[32])
{
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t x = a[k], y = a[k + 16];
        a[k] = perm(y, x, 0x05040100u);
        a[k + 16] = perm(y, x, 0x07060302u);
    }
#pragma unroll
    for (int k0 = 0; k0 < 32; k0 += 16) {
#pragma unroll
        for (int k = k0; k < k0 + 8; ++k) {
            const uint32_t x = a[k], y = a[k + 8];
            a[k] = perm(y, x, 0x06020400u);
            a[k + 8] = perm(y, x, 0x07030501u);
        }
    }
    swap_stage<4>(a, 0x0F0F0F0Fu);
    swap_stage<2>(a, 0x33333333u);
    swap_stage<1>(a, 0x55555555u);
}

// Element packing around the transpose for narrow elements.  For E = 2 a
// unit is 64 elements held as 32 words w[m] = e[2m] | e[2m+1] << 16; the
// transpose wants d[k] = e[k] | e[k+32] << 16.  For E = 1 a unit is 128
// bytes, w[m] = bytes 4m..4m+3, and the transpose wants
// d[k] = b[k] | b[k+32] << 8 | b[k+64] << 16 | b[k+96] << 24.
// pack_* maps w -> d and unpack_* maps d -> w.
__device__ __forceinline__ void pack_e2(const uint32_t (&w)[32], uint32_t (&d)[32])
{
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        d[2 * m] = perm(w[m + 16], w[m], 0x05040100u);
        d[2 * m + 1] = perm(w[m + 16], w[m], 0x07060302u);
    }
}
__device__ __forceinline__ void unpack_e2(const uint32_t (&d)[32], uint32_t (&w)[32])
{
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        w[m] = perm(d[2 * m + 1], d[2 * m], 0x05040100u);
        w[m + 16] = perm(d[2 * m + 1], d[2 * m], 0x07060302u);
    }
}
// 4x4 byte transpose of (r0, r1, r2, r3): out[i] byte j = r[j] byte i.
__device__ __forceinline__ void byte_transpose4(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t r3,
                                                uint32_t &o0, uint32_t &o1, uint32_t &o2,
                                                uint32_t &o3)
{
    const uint32_t x0 = perm(r1, r0, 0x05010400u); // r0.b0 r1.b0 r0.b1 r1.b1
    const uint32_t x1 = perm(r1, r0, 0x07030602u); // r0.b2 r1.b2 r0.b3 r1.b3
    const uint32_t y0 = perm(r3, r2, 0x05010400u);
    const uint32_t y1 = perm(r3, r2, 0x07030602u);
    o0 = perm(y0, x0, 0x05040100u);
    o1 = perm(y0, x0, 0x07060302u);
    o2 = perm(y1, x1, 0x05040100u);
    o3 = perm(y1, x1, 0x07060302u);
}
__device__ __forceinline__ void pack_e1(const uint32_t (&w)[32], uint32_t (&d)[32])
{
#pragma unroll
    for (int q = 0; q < 8; ++q)
        byte_transpose4(w[q], w[q + 8], w[q + 16], w[q + 24], d[4 * q], d[4 * q + 1],
                        d[4 * q + 2], d[4 * q + 3]);
}
__device__ __forceinline__ void unpack_e1(const uint32_t (&d)[32], uint32_t (&w)[32])
{
#pragma unroll
    for (int q = 0; q < 8; ++q)
        byte_transpose4(d[4 * q], d[4 * q + 1], d[4 * q + 2], d[4 * q + 3], w[q], w[q + 8],
                        w[q + 16], w[q + 24]);
}

// ---------------------------------------------------------------------------
// Stage-1 parameters (fused into the compressor's load when requested).
// ---------------------------------------------------------------------------
struct RoundParams {
    const float *autos;     // [F][I][T] (float visibilities)
    const int32_t *autos_i32; // [F][I][T] (integer visibilities)
    const double *fscale;     // [F][T] factor on G2 (noise-model compensation) or nullptr
    const int32_t *prod_map; // [P][2] or nullptr (upper triangle row major)
    int64_t F, I, T, P;
    double c;      // (12 f) / (2 N): G2 = (V_ii V_jj) c for crosses
    double c_auto; // 2 c: G2 = V_ii^2 c_auto for autos
};

// ---------------------------------------------------------------------------
// Launchers (host, enqueue only; return hipError_t).
// ---------------------------------------------------------------------------
hipError_t launch_round(const float *vin, float *vout, const RoundParams &rp, hipStream_t s);
hipError_t launch_round_i32(const int32_t *vin, int32_t *vout, const RoundParams &rp, hipStream_t s);
hipError_t launch_noise_comp(const float *vis, const RoundParams &rp, double *scale, hipStream_t s);
int fullcov_max_inputs();
hipError_t launch_fullcov(const float *vis, const float *autos, int64_t F, int64_t I, int64_t T,
                          double c, float *vis_out, double *qdiag, hipStream_t s);
hipError_t launch_shuffle(const uint8_t *in, uint8_t *out, const Layout &L, bool inverse,
                          hipStream_t s);
hipError_t launch_byteshuffle(const uint8_t *in, uint8_t *out, const Layout &L, bool inverse,
                              hipStream_t s);
// may_segment: a large input may be encoded in segments over the library's
// own streams (off for callers that must not create anything).
hipError_t launch_compress(const uint8_t *in, uint8_t *out, const Layout &L, int64_t cap,
                           int64_t *d_nbytes, void *ws, int64_t ws_bytes,
                           const RoundParams *rp, hipStream_t s, int filter = BSG_FILTER_BIT,
                           bool may_segment = true);
int64_t compress_workspace(const Layout &L);

// Two streams of the library's own per device, an encode stream and a pack
// stream (default priority), with their events, made once.  Work split over
// them runs beside the caller's stream: side_streams_begin locks the
// current device's set (the lock stays held while the caller enqueues, so
// calls from several host threads do not interleave their use of the
// events) and makes both streams wait for the caller's work so far;
// side_streams_end makes the caller's stream wait for the pack stream and
// for event done[last_enc] of the encode stream.
constexpr int kSideEvents = 16;
struct SideStreams {
    bool made = false, ok = false;
    hipStream_t enc = nullptr, pack = nullptr;
    hipEvent_t fork = nullptr, join = nullptr, done[kSideEvents] = {};
};
hipError_t side_streams_begin(hipStream_t s, std::unique_lock<std::mutex> &lock,
                              SideStreams **out);
hipError_t side_streams_end(SideStreams *g, hipStream_t s, int last_enc);
hipError_t launch_decompress(const uint8_t *in, int64_t in_nbytes, uint8_t *out,
                             const Layout &L, int32_t *d_status, hipStream_t s, int filter = BSG_FILTER_BIT);

} // namespace bsg
