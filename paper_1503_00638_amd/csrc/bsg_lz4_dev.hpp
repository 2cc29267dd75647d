// Device code of the per-block LZ4 stage (Section 4.2 of Masui et al.:
// each block is bit-transposed and LZ4-compressed on its own, blocks are
// independent), shared by the single-stream and the batched kernels.  On
// gfx950 a block lives in LDS and one wavefront owns it.
#pragma once

#include "bsg_internal.hpp"
#include "bsg_round_dev.hpp"
#include "bsg_shuffle_dev.hpp"

namespace bsg {
namespace {


constexpr int kSmallBlock = 8192;     // LDS-resident block for the hot path
constexpr int kLargeBlock = 65536;
constexpr int kTile = 1024;           // blocks per scan tile

// DPP controls: lane i reads lane i + 1 of the wave; lane i reads lane i - n
// of its row of 16 (none: 0); lane 15 (31) feeds the next row (rows 2, 3).
typedef uint32_t u32x16 __attribute__((ext_vector_type(16)));

// The codec kernels run one wave per workgroup, and the lanes of a wave hand
// LDS data to each other between phases: a wavefront-scope fence orders those
// accesses in the memory model (on gfx950 it emits no instruction, since LDS
// accesses of one wave complete in order, but no access moves across it).  A
// workgroup barrier would also wait for every outstanding global load and
// store of the wave.
// The lane index, opaque to the optimiser, for the encoder: values derived
// from it are then not hoisted out of the persistent block loop, where they
// would stay live across the whole loop body and cost occupancy.
__device__ __forceinline__ int lane_id()
{
    int x = (int)threadIdx.x;
    asm volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

__device__ __forceinline__ uint32_t lds_le32(const uint32_t *b32, int pos)
{
    const uint32_t w0 = b32[pos >> 2], w1 = b32[(pos >> 2) + 1];
    return __builtin_amdgcn_alignbyte(w1, w0, (uint32_t)(pos & 3));
}

// ---- stage the block into LDS as bit planes -------------------------------
// Stage-1 rounding fused into the encoder's staging: none, plain, or with a
// per-(frequency, time) factor on the variance (separate instances, as the
// factors' registers would lower the occupancy of the plain one).
constexpr int kRoundNone = 0, kRoundPlain = 1, kRoundScaled = 2;

template <int E, int RM>
__device__ __forceinline__ void stage_fast(const uint8_t *__restrict__ src, int64_t elems,
                                           uint8_t *lds, const RoundParams &rp,
                                           int64_t first_elem)
{
    const int lane = lane_id();
    const int64_t units = elems / Unit<E>::G;
    for (int64_t u = lane; u < units; u += kWave) {
        uint32_t w[Unit<E>::IN_WORDS];
        load_unit<E>(src + u * (Unit<E>::G * E), w);
        if constexpr (RM != kRoundNone) {
            // E == 4: the unit is 32 float32 = 16 complex64 visibilities.
            VisCursor c = cursor_at(rp, (first_elem + u * 32) / 2);
            if (c.t + 16 <= rp.T) {
                // one product at one frequency: the autos (and factors) of
                // the 16 times are consecutive, read from one base each
                const float *pi = rp.autos + c.row_i + c.t;
                const float *pj = rp.autos + c.row_j + c.t;
                const bool is_auto = c.i == c.j;
                float ai[16], aj[16];
                double sc[RM == kRoundScaled ? 16 : 1];
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    ai[k] = pi[k];
                    aj[k] = pj[k];
                }
                if constexpr (RM == kRoundScaled) {
                    const double *fs = rp.fscale + c.fr * rp.T + c.t;
#pragma unroll
                    for (int k = 0; k < 16; ++k) sc[k] = fs[k];
                }
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    double G2 = ((double)ai[k] * (double)aj[k]) * (is_auto ? rp.c_auto : rp.c);
                    if constexpr (RM == kRoundScaled) G2 *= sc[k];
                    w[2 * k] = round_noise_bits_nb(w[2 * k], G2);
                    if (!is_auto) w[2 * k + 1] = round_noise_bits_nb(w[2 * k + 1], G2);
                }
            } else {
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const float2 o = round_at(make_float2(__uint_as_float(w[2 * k]),
                                                          __uint_as_float(w[2 * k + 1])),
                                              c, rp);
                    w[2 * k] = __float_as_uint(o.x);
                    w[2 * k + 1] = __float_as_uint(o.y);
                    if (k < 15) cursor_advance(rp, c, 1);
                }
            }
        }
        unit_forward<E>(w);
        store_planes<E>(lds, elems / 8, u, w);
    }
}

// Generic staging with the rounding fused in: element e of the buffer is
// component e & 1 of visibility e >> 1; each lane rounds its own element and
// the block is transposed with ballots.
__device__ __forceinline__ void block_forward_ballot_round(const uint8_t *__restrict__ in,
                                                           uint8_t *out, int64_t elems,
                                                           const RoundParams &rp,
                                                           int64_t first_elem)
{
    const int lane = lane_id();
    const int64_t pb = elems / 8;
    for (int64_t g = 0; g < elems; g += 64) {
        const int64_t i = g + lane;
        uint32_t v = 0;
        if (i < elems) {
            uint32_t x = 0;
            for (int k = 0; k < 4; ++k) x |= (uint32_t)in[i * 4 + k] << (8 * k);
            v = round_element(x, first_elem + i, rp);
        }
        const int64_t rem = (elems - g) / 8;
        const int nbytes = rem < 8 ? (int)rem : 8;
        for (int bit = 0; bit < 32; ++bit) {
            const uint64_t m = __ballot((v >> bit) & 1u);
            if (lane < nbytes) out[bit * pb + g / 8 + lane] = (uint8_t)(m >> (8 * lane));
        }
    }
}

// Element class of kernels that apply the byte shuffle instead of the bit
// transpose (the Blosc-style filter the paper compares against in Section
// 4.1 and Table t:performance): byte k of element i of a block goes to byte
// k * elems + i.
constexpr int kByteShuffle = -1;

// Lanes take 4 elements at a time, so every LDS access is one aligned dword
// (elems is a multiple of 8).
// Byte shuffle of elements whose size is a multiple of 4 (E <= 16), the
// input 16-byte aligned: each lane loads 4 elements (4E bytes) with 16-byte
// loads, and every 4 x 4 byte sub-matrix (dword kg of the 4 elements) is
// transposed in registers into dword g of planes 4kg .. 4kg + 3.
template <int E>
__device__ __forceinline__ void block_forward_bytes_fast(const uint8_t *__restrict__ in,
                                                         uint8_t *lds, int64_t elems)
{
    constexpr int W = E / 4; // dwords per element
    uint32_t *l32 = reinterpret_cast<uint32_t *>(lds);
    const int64_t pw = elems / 4; // dwords per plane
    for (int64_t g = lane_id(); g < elems / 4; g += kWave) {
        const uint4 *s4 = reinterpret_cast<const uint4 *>(in + 4 * g * E);
        uint32_t w[4 * W];
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const uint4 v = s4[q];
            w[4 * q] = v.x;
            w[4 * q + 1] = v.y;
            w[4 * q + 2] = v.z;
            w[4 * q + 3] = v.w;
        }
#pragma unroll
        for (int kg = 0; kg < W; ++kg) {
            uint32_t o0, o1, o2, o3;
            byte_transpose4(w[kg], w[W + kg], w[2 * W + kg], w[3 * W + kg], o0, o1, o2, o3);
            l32[(4 * kg) * pw + g] = o0;
            l32[(4 * kg + 1) * pw + g] = o1;
            l32[(4 * kg + 2) * pw + g] = o2;
            l32[(4 * kg + 3) * pw + g] = o3;
        }
    }
}

template <int E>
__device__ __forceinline__ void block_inverse_bytes_fast(const uint8_t *lds,
                                                         uint8_t *__restrict__ out, int64_t elems)
{
    constexpr int W = E / 4;
    const uint32_t *l32 = reinterpret_cast<const uint32_t *>(lds);
    const int64_t pw = elems / 4;
    for (int64_t g = threadIdx.x; g < elems / 4; g += kWave) {
        uint32_t w[4 * W];
#pragma unroll
        for (int kg = 0; kg < W; ++kg)
            byte_transpose4(l32[(4 * kg) * pw + g], l32[(4 * kg + 1) * pw + g],
                            l32[(4 * kg + 2) * pw + g], l32[(4 * kg + 3) * pw + g], w[kg],
                            w[W + kg], w[2 * W + kg], w[3 * W + kg]);
        uint4 *d4 = reinterpret_cast<uint4 *>(out + 4 * g * E);
#pragma unroll
        for (int q = 0; q < W; ++q)
            d4[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
    }
}

__device__ __forceinline__ void block_forward_bytes(const uint8_t *__restrict__ in, uint8_t *lds,
                                                    int64_t elems, int64_t E)
{
    if (((uintptr_t)in % 16) == 0) {
        switch (E) {
        case 4: block_forward_bytes_fast<4>(in, lds, elems); return;
        case 8: block_forward_bytes_fast<8>(in, lds, elems); return;
        case 12: block_forward_bytes_fast<12>(in, lds, elems); return;
        case 16: block_forward_bytes_fast<16>(in, lds, elems); return;
        default: break;
        }
    }
    uint32_t *l32 = reinterpret_cast<uint32_t *>(lds);
    for (int64_t g = lane_id(); g < elems / 4; g += kWave) {
        const uint8_t *src = in + 4 * g * E;
        for (int64_t k = 0; k < E; ++k)
            l32[(k * elems + 4 * g) >> 2] = (uint32_t)src[k] | ((uint32_t)src[E + k] << 8) |
                                           ((uint32_t)src[2 * E + k] << 16) |
                                           ((uint32_t)src[3 * E + k] << 24);
    }
}

__device__ __forceinline__ void block_inverse_bytes(const uint8_t *lds, uint8_t *__restrict__ out,
                                                    int64_t elems, int64_t E)
{
    if (((uintptr_t)out % 16) == 0) {
        switch (E) {
        case 4: block_inverse_bytes_fast<4>(lds, out, elems); return;
        case 8: block_inverse_bytes_fast<8>(lds, out, elems); return;
        case 12: block_inverse_bytes_fast<12>(lds, out, elems); return;
        case 16: block_inverse_bytes_fast<16>(lds, out, elems); return;
        default: break;
        }
    }
    const uint32_t *l32 = reinterpret_cast<const uint32_t *>(lds);
    for (int64_t g = threadIdx.x; g < elems / 4; g += kWave) {
        uint8_t *dst = out + 4 * g * E;
        for (int64_t k = 0; k < E; ++k) {
            const uint32_t v = l32[(k * elems + 4 * g) >> 2];
            dst[k] = (uint8_t)v;
            dst[E + k] = (uint8_t)(v >> 8);
            dst[2 * E + k] = (uint8_t)(v >> 16);
            dst[3 * E + k] = (uint8_t)(v >> 24);
        }
    }
}

// EC: the element size this kernel instance has a register fast path for
// (1, 2, 4, 8, 12, 16), 0 for the generic ballot path only, or kByteShuffle.
template <int EC, int RM>
__device__ __forceinline__ void stage_block(const uint8_t *__restrict__ src, int64_t elems,
                                            int64_t E, uint8_t *lds, const RoundParams &rp,
                                            int64_t first_elem)
{
    if constexpr (RM != kRoundNone) {
        static_assert(EC == 4 || EC == 0, "rounding is fused for float32 elements only");
        if (EC == 4 && elems % 32 == 0 && ((uintptr_t)src % 16) == 0)
            stage_fast<4, RM>(src, elems, lds, rp, first_elem);
        else
            block_forward_ballot_round(src, lds, elems, rp, first_elem);
    } else if constexpr (EC == kByteShuffle) {
        block_forward_bytes(src, lds, elems, E);
    } else {
        if constexpr (EC != 0) {
            if (elems % Unit<EC>::G == 0 && ((uintptr_t)src % 16) == 0) {
                stage_fast<EC, kRoundNone>(src, elems, lds, rp, first_elem);
                return;
            }
        }
        block_forward_ballot(src, lds, elems, E);
    }
}

// Elements of a full block of MAXB bytes for a register-path element class
// (the default block: MAXB / E rounded down to a multiple of 8), or 0 where
// the class has no register path or the block is not whole units.  With
// the count a constant the plane stride is one too, and every LDS read of
// the decoder's inverse transpose takes an immediate offset (pairs of plane
// words per instruction).  (Not for 16-byte elements, whose decoders would
// need more registers for it.)
template <int MAXB, int EC> constexpr int64_t full_block_elems()
{
    if constexpr (EC == 1 || EC == 2 || EC == 4 || EC == 8) {
        constexpr int64_t n = (MAXB / EC) / 8 * 8;
        return n % Unit<EC>::G == 0 ? n : 0;
    } else {
        return 0;
    }
}

// ---- LZ4 emission, one sequence per lane ------------------------------------
// Exclusive prefix sum of x over the wave's lanes; total = the sum of all.
// Inclusive sums within rows of 16 lanes by shifts of 1, 2, 4 and 8, then
// the row totals carried over by the broadcasts of lanes 15 and 31.
__device__ __forceinline__ int wave_excl_scan(int x, int &total)
{
    int s = x;
    s += __builtin_amdgcn_update_dpp(0, s, kDppRowShr1, 0xF, 0xF, true);
    s += __builtin_amdgcn_update_dpp(0, s, kDppRowShr2, 0xF, 0xF, true);
    s += __builtin_amdgcn_update_dpp(0, s, kDppRowShr4, 0xF, 0xF, true);
    s += __builtin_amdgcn_update_dpp(0, s, kDppRowShr8, 0xF, 0xF, true);
    s += __builtin_amdgcn_update_dpp(0, s, kDppRowBcast15, 0xA, 0xF, false);
    s += __builtin_amdgcn_update_dpp(0, s, kDppRowBcast31, 0xC, 0xF, false);
    total = __builtin_amdgcn_readlane(s, kWave - 1);
    return s - x;
}

// lds_le32 for a position as far as 3 bytes before the block: the bytes
// before it come out undefined.
__device__ __forceinline__ uint32_t lds_le32_head(const uint32_t *b32, int pos)
{
    const int wi = pos >> 2;
    const uint32_t w0 = b32[wi < 0 ? 0 : wi], w1 = b32[wi + 1];
    return __builtin_amdgcn_alignbyte(w1, w0, (uint32_t)(pos & 3));
}

// Write the ns (<= 64) sequences that lanes 0 .. ns-1 hold (lane j: the
// literals [lit, lit + ll) of the block at b32, then a match of ml bytes at
// distance off; ml == 0 marks the block's last sequence, literals only) from
// byte op of the 16-byte aligned slot dst; returns the byte after them.
// Each lane writes its own token, offset and length bytes; then the wave
// copies the literal runs, 16 output bytes per lane per step: whole dwords
// where a run covers them, single bytes at a run's ends.  The block must be
// readable 4 bytes past every run.
__device__ __forceinline__ int emit_sequences(uint8_t *__restrict__ dst, int op, const uint32_t *b32,
                                              int ns, int lit, int ll, int off, int ml)
{
    const int lane = lane_id();
    const bool act = lane < ns;
    const bool last = ml == 0;
    const int mlc = last ? 0 : ml - kMinMatch;
    const int lext = ll >= 15 ? (ll - 15) / 255 + 1 : 0;
    const int mext = mlc >= 15 ? (mlc - 15) / 255 + 1 : 0;
    const int hsz = 1 + lext, tsz = last ? 0 : 2 + mext;
    int total;
    const int start = op + wave_excl_scan(act ? hsz + ll + tsz : 0, total);

    // token, literal-length bytes; offset, match-length bytes
    const uint32_t tok = (uint32_t)(((ll < 15 ? ll : 15) << 4) | (mlc < 15 ? mlc : 15));
    const uint32_t lrem = (uint32_t)(ll - 15 - 255 * (lext - 1));
    const uint32_t mrem = (uint32_t)(mlc - 15 - 255 * (mext - 1));
    const int tpos = start + hsz + ll;
    const int fmax = act ? (hsz > tsz ? hsz : tsz) : 0;
    constexpr int kShort = 4; // field bytes each lane writes itself
    for (int k = 0; k < kShort && __ballot(k < fmax) != 0; ++k) {
        if (act && k < hsz) dst[start + k] = (uint8_t)(k == 0 ? tok : (k < lext ? 255u : lrem));
        if (act && k < tsz)
            dst[tpos + k] = (uint8_t)(k == 0 ? (uint32_t)off & 255u
                                             : (k == 1 ? (uint32_t)off >> 8 : (k < tsz - 1 ? 255u : mrem)));
    }
    // the rest of a long length field (a run of 255s, then the remainder):
    // the wave writes one such sequence at a time
    for (uint64_t longs = __ballot(fmax > kShort); longs; longs &= longs - 1) {
        const int j = __builtin_ctzll(longs);
        const int st_j = __builtin_amdgcn_readlane(start, j), h_j = __builtin_amdgcn_readlane(hsz, j);
        const int tp_j = __builtin_amdgcn_readlane(tpos, j), t_j = __builtin_amdgcn_readlane(tsz, j);
        const uint32_t lr_j = (uint32_t)__builtin_amdgcn_readlane((int)lrem, j);
        const uint32_t mr_j = (uint32_t)__builtin_amdgcn_readlane((int)mrem, j);
        for (int k = kShort + lane; k < h_j; k += kWave) dst[st_j + k] = (uint8_t)(k < h_j - 1 ? 255u : lr_j);
        for (int k = kShort + lane; k < t_j; k += kWave) dst[tp_j + k] = (uint8_t)(k < t_j - 1 ? 255u : mr_j);
    }

    // literal runs: task t of the wave is the 16 output bytes (ls_j / 16) +
    // t - first_j of the sequence j with first_j <= t < first_{j+1}
    const int ls = start + hsz;
    const int nd = act && ll > 0 ? ((ls + ll - 1) >> 4) - (ls >> 4) + 1 : 0;
    int ndt;
    const int first = wave_excl_scan(nd, ndt);
    uint32_t *dst32 = reinterpret_cast<uint32_t *>(dst);
    for (int t0 = 0; t0 < ndt; t0 += kWave) {
        const int t = t0 + lane;
        int j = 0; // the last sequence whose first task is <= t
#pragma unroll
        for (int st = kWave / 2; st >= 1; st >>= 1) {
            const int fj = __shfl(first, j + st);
            j = j + st < ns && fj <= t ? j + st : j;
        }
        const int ls_j = __shfl(ls, j), ll_j = __shfl(ll, j);
        const int lit_j = __shfl(lit, j), f_j = __shfl(first, j);
        if (t < ndt) {
            const int u = (ls_j >> 4) + t - f_j;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int w = 4 * u + k;
                const int b0 = ls_j - 4 * w, b1 = b0 + ll_j; // the run's bytes in dword w: [b0, b1)
                if (b1 > 0 && b0 < 4) {
                    const uint32_t val = lds_le32_head(b32, lit_j - b0);
                    if (b0 <= 0 && b1 >= 4) {
                        dst32[w] = val;
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (i >= b0 && i < b1) dst[4 * w + i] = (uint8_t)(val >> (8 * i));
                    }
                }
            }
        }
    }
    return op + total;
}

// ---- the fixed-rule LZ4 encoder of one LDS-resident block -----------------
// Length of the common prefix of b[q + L ...] and b[c + L ...] (c < q),
// capped at maxL: 256 bytes per step first, then 1 KiB per step.  Bytes at or
// beyond maxL count as mismatches.
template <int MAXB>
__device__ __forceinline__ int extend_match(const uint32_t *b32, int c, int q, int L, int maxL)
{
    const int lane = lane_id();
    if (L >= maxL) return maxL;
    if (L + 4 * kWave <= maxL) {
        // the whole first step lies inside the block and the limit
        const int o = L + 4 * lane;
        const uint32_t diff = lds_le32(b32, c + o) ^ lds_le32(b32, q + o);
        const uint64_t mm = __ballot(diff != 0);
        if (mm) {
            const int fl = __builtin_ctzll(mm);
            const uint32_t dd = (uint32_t)__builtin_amdgcn_readlane((int)diff, fl);
            return L + 4 * fl + (__builtin_ctz(dd) >> 3);
        }
        L += 4 * kWave;
    } else {
        const int o = L + 4 * lane;
        const int pa = c + o < MAXB ? c + o : MAXB;
        const int pb = q + o < MAXB ? q + o : MAXB;
        uint32_t diff = lds_le32(b32, pa) ^ lds_le32(b32, pb);
        const int vb = maxL - o;
        if (vb < 4) diff |= vb <= 0 ? 0xFFFFFFFFu : (0xFFFFFFFFu << (8 * vb));
        const uint64_t mm = __ballot(diff != 0);
        if (mm) {
            const int fl = __builtin_ctzll(mm);
            const uint32_t dd = (uint32_t)__builtin_amdgcn_readlane((int)diff, fl);
            return L + 4 * fl + (__builtin_ctz(dd) >> 3);
        }
        L += 4 * kWave;
    }
    while (L < maxL) {
        const int o = L + 16 * lane;
        int first = 16; // first differing byte of this lane's 16, 16 = none
#pragma unroll
        for (int j = 3; j >= 0; --j) {
            const int oj = o + 4 * j;
            const int pa = c + oj < MAXB ? c + oj : MAXB;
            const int pb = q + oj < MAXB ? q + oj : MAXB;
            uint32_t diff = lds_le32(b32, pa) ^ lds_le32(b32, pb);
            const int vb = maxL - oj;
            if (vb < 4) diff |= vb <= 0 ? 0xFFFFFFFFu : (0xFFFFFFFFu << (8 * vb));
            if (diff) first = 4 * j + (__builtin_ctz(diff) >> 3);
        }
        const uint64_t mm = __ballot(first < 16);
        if (mm) {
            const int fl = __builtin_ctzll(mm);
            return L + 16 * fl + __builtin_amdgcn_readlane(first, fl);
        }
        L += 16 * kWave;
    }
    return maxL;
}

// b32: block bytes (n <= MAXB) followed by >= 12 readable padding bytes.
// Per group of 512 positions: (1) read the 4 bytes at every position, (2)
// per 64-position chunk read the table entry of every position, then raise
// the entries to the chunk's positions (the wave's in-order LDS queue makes
// chunk c see exactly chunks < c), (3) verify 12 bytes at every candidate of
// a chunk the parse enters, (4) parse greedily with the candidates in VGPRs
// and the match masks in SGPRs.
// Hash and insert the kGroup positions from g0 (the fixed rule of the LZ4
// stage): per chunk cc of 64 positions, cand holds the table entry (position
// + 1, 0 = none) each lane's position found before the chunk's own inserts.
// FULL: the whole group lies at or below last_take, so the bound checks drop
// out, and as g0 is a multiple of 4 every chunk's loads share one base with
// immediate offsets.
template <int MAXB, bool FULL>
__device__ __forceinline__ void hash_group(const uint32_t *b32, uint32_t *table, int g0, int last_q,
                                           int last_ins, u32x16 &candv)
{
    constexpr int NC = kGroup / kChunk;
    const int lane = lane_id();
    uint32_t vv[NC];
    const uint32_t *dg = b32 + ((g0 + lane) >> 2);
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
        const int p = g0 + cc * kChunk + lane;
        const int pc = FULL || p < MAXB ? p : MAXB;
        const uint32_t *d = FULL ? dg + cc * (kChunk / 4) : b32 + (pc >> 2);
        vv[cc] = __builtin_amdgcn_alignbyte(d[1], d[0], (uint32_t)(pc & 3));
    }
    const auto chunk = [&](int cc) {
        // (chunks past last_q only insert positions that no lookup sees)
        const int c0 = g0 + cc * kChunk;
        const int p = c0 + lane;
        const uint32_t v = vv[cc];
        const uint32_t h = (v * kHashMult) >> (32 - kHashBits);
        const uint32_t t = table[h];
        candv[cc] = FULL || p <= last_q ? t : 0u;
        // In a run of equal 4-byte values (a constant bit plane) only the
        // run's last position writes: the entry takes the largest position
        // either way, and atomics of many lanes on one address would be
        // serialised.  The next lane's value comes from a DPP wave shift
        // (lane i reads lane i + 1).  The other lanes are masked off.
        const uint32_t vn = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppWaveShl1, 0xF, 0xF, true);
        const bool run_on = lane != kWave - 1 && (FULL || p + 1 <= last_ins) && vn == v;
        if ((FULL || p <= last_ins) && !run_on)
            atomicMax(&table[h], (uint32_t)(p + 1));
    };
    chunk(0);
    if constexpr (FULL) {
        // A group holding one 4-byte value at every position (half of the
        // groups of a rounded visibility block: its constant bit planes).
        // Chunk 0 went the usual way and left the entry at its last
        // position; chunk k > 0 would find the last position of chunk k - 1
        // and the entry would end at the group's last position, so the rest
        // takes one write instead of 7 reads and 7 inserts.  (The test runs
        // while chunk 0's table accesses are in flight.)
        const uint32_t v0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)vv[0]);
        uint32_t x = 0;
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) x |= vv[cc] ^ v0;
        if (__ballot(x != 0) == 0) {
#pragma unroll
            for (int cc = 1; cc < NC; ++cc) candv[cc] = (uint32_t)(g0 + cc * kChunk);
            if (lane == kWave - 1)
                table[(v0 * kHashMult) >> (32 - kHashBits)] = (uint32_t)(g0 + kGroup);
            return;
        }
    }
#pragma unroll
    for (int cc = 1; cc < NC; ++cc) chunk(cc);
}

// The mask of the chunk's positions (from c0, a multiple of 64) whose
// candidate matches for kMinTake = 12 bytes and may be taken (<= last_take).
// Branch-free: a lane without a candidate reads position 0 and is masked
// after.
__device__ __forceinline__ uint64_t verify_chunk(const uint32_t *b32, int c0, uint32_t cand,
                                                 int last_take)
{
    const int p = c0 + lane_id();
    const uint32_t cn = c0 + kChunk - 1 <= last_take || p <= last_take ? cand : 0u;
    const int c = cn != 0 ? (int)cn - 1 : 0;
    const uint32_t *o = b32 + (p >> 2);
    const uint32_t *d = b32 + (c >> 2);
    const uint32_t o0 = o[0], o1 = o[1], o2 = o[2], o3 = o[3];
    const uint32_t e0 = d[0], e1 = d[1], e2 = d[2], e3 = d[3];
    // zero when the candidate exists and its 12 bytes equal those at p
    const uint32_t x = (__builtin_amdgcn_alignbyte(e1, e0, (uint32_t)(c & 3)) ^
                        __builtin_amdgcn_alignbyte(o1, o0, (uint32_t)(p & 3))) |
                       (__builtin_amdgcn_alignbyte(e2, e1, (uint32_t)(c & 3)) ^
                        __builtin_amdgcn_alignbyte(o2, o1, (uint32_t)(p & 3))) |
                       (__builtin_amdgcn_alignbyte(e3, e2, (uint32_t)(c & 3)) ^
                        __builtin_amdgcn_alignbyte(o3, o2, (uint32_t)(p & 3))) |
                       ((cn - 1u) >> 31);
    return __ballot(x == 0);
}

// Greedy parse of one LDS-resident block of n bytes (n <= MAXB) into LZ4
// sequences written to dst; returns the compressed size.  Positions are
// hashed and inserted a group of 8 chunks at a time; a chunk's candidates
// are verified only when the parse reaches it, so chunks inside a long
// match are never verified.  Sequences are written 64 at a time.
// (The group's candidates sit in a 16-wide register vector: a uniform index
// into one compiles to a relative register move.)
template <int MAXB>
__device__ __forceinline__ int encode_block(const uint32_t *b32, int n, uint32_t *table,
                                            uint8_t *__restrict__ dst)
{
    constexpr int NC = kGroup / kChunk;
    static_assert(NC <= 16, "a group's candidates fit one vector");
    const int lane = lane_id();
    for (int i = lane; i < (1 << kHashBits) / 4; i += kWave)
        reinterpret_cast<uint4 *>(table)[i] = make_uint4(0, 0, 0, 0);
    wave_sync();

    const int last_q = n - kMfLimit;           // last position a match may start at
    const int last_take = last_q - (kMinTake - 7); // ... and still reach kMinTake bytes
                                                   // before the last 5 literals
    const int last_ins = n - kMinMatch;        // last position with a defined hash
    int anchor = 0, pnext = 0, op = 0;
    // sequences found and not yet written: lane j holds sequence j
    int ns = 0, s_lit = 0, s_ll = 0, s_off = 0, s_ml = 0;
    for (int g0 = 0; g0 <= last_q; g0 += kGroup) {
        u32x16 candv;
        // a group whose every position (and the one after it) may be
        // inserted, looked up and taken needs no bound checks
        if (g0 + kGroup <= last_take)
            hash_group<MAXB, true>(b32, table, g0, last_q, last_ins, candv);
        else
            hash_group<MAXB, false>(b32, table, g0, last_q, last_ins, candv);

        // chunk by chunk from the one holding the parse position
        for (int cc = (pnext > g0 ? pnext - g0 : 0) >> 6; cc < NC; ++cc) {
            const int c0 = g0 + cc * kChunk;
            if (c0 > last_take) break;
            const uint64_t mk = verify_chunk(b32, c0, candv[cc], last_take);
            for (;;) {
                const int rel = pnext - c0;
                const uint64_t mm = rel > 0 ? mk & (~0ull << rel) : mk;
                if (mm == 0) break;
                const int bit = __builtin_ctzll(mm);
                const int q = c0 + bit;
                const int c = __builtin_amdgcn_readlane((int)candv[cc], bit) - 1;
                const int L = __builtin_amdgcn_readfirstlane(
                    extend_match<MAXB>(b32, c, q, kMinTake, n - kLastLiterals - q));
                const bool me = lane == ns;
                s_lit = me ? anchor : s_lit;
                s_ll = me ? q - anchor : s_ll;
                s_off = me ? q - c : s_off;
                s_ml = me ? L : s_ml;
                if (++ns == kWave) {
                    op = emit_sequences(dst, op, b32, ns, s_lit, s_ll, s_off, s_ml);
                    ns = 0;
                }
                pnext = q + L;
                anchor = pnext;
                if (pnext >= c0 + kChunk) break;
            }
            // skip the chunks the match covers (the loop steps to the next)
            if (pnext >= c0 + kChunk) cc = (pnext - g0 - kChunk) >> 6;
        }
    }
    // the last literals
    const bool me = lane == ns;
    s_lit = me ? anchor : s_lit;
    s_ll = me ? n - anchor : s_ll;
    s_ml = me ? 0 : s_ml;
    return emit_sequences(dst, op, b32, ns + 1, s_lit, s_ll, s_off, s_ml);
}

// ---- sizes -> offsets -------------------------------------------------------
__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t *sh)
{
    // 256-thread inclusive scan helper storage: sh[256]
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int64_t x = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    return sh[t]; // inclusive
}

__device__ __forceinline__ void fail(int32_t *status)
{
    if (threadIdx.x == 0) atomicCAS(status, 0, BSG_ECORRUPT);
}

// Read an LZ4 length continuation (255-runs then a byte < 255) at ip, 64
// bytes per step.  Returns false when the input ends first.
__device__ __forceinline__ bool read_len_ext(const uint8_t *ci, int &ip, int iend, int &len)
{
    const int lane = threadIdx.x;
    for (;;) {
        // every lane reads (clamped into the input), so no lane branches
        const int pos = ip + lane;
        const uint32_t byte = ci[pos < iend ? pos : iend - 1];
        const uint32_t v = pos < iend ? byte : 0u;
        const uint64_t m = __ballot(v != 255u);
        if (m == 0) {
            len += 255 * kWave;
            ip += kWave;
            continue;
        }
        const int f = __builtin_ctzll(m);
        if (ip + f >= iend) return false;
        len = __builtin_amdgcn_readfirstlane(len + 255 * f + __shfl((int)v, f));
        ip += f + 1;
        return true;
    }
}

// Copies of the in-place decoder, aligned on the destination: the output
// bytes [op, op + len) are covered by whole dwords [op / 4, (op + len + 3) / 4),
// and each lane builds one dword per step from its source bytes and writes it
// with one aligned store.  Bytes of the first and last dword outside the
// range keep their old value (final output below, or input not yet read
// above: rewritten unchanged).  Every lane of a step takes part, no exec
// mask: a lane past the range (up to 63 dwords past it) reads its dword and
// sources and writes the dword back unchanged, so the buffer has 64 dwords
// of padding after it.  Sources may lie up to 3 bytes before b32[0], so the
// buffer has a padding dword in front.
//
// A byte mask takes three or four vector instructions: the bytes of the
// dword at byte d that lie at or past byte t are the low 32 bits of
// 0xFFFFFFFF shifted left by 8 (t - d), the shift clamped to [0, 32] (one
// med3; the 64-bit shift turns 32 into 0).
__device__ __forceinline__ uint32_t ge_mask(int d, int t)
{
    int s = 8 * (t - d);
    s = s < 0 ? 0 : (s > 32 ? 32 : s);
    return (uint32_t)(0xFFFFFFFFull << s);
}

// The bytes of the dword at byte d inside [op, end).
__device__ __forceinline__ uint32_t range_mask(int d, int op, int end)
{
    return ge_mask(d, op) & ~ge_mask(d, end);
}

// (every lane reads its destination dword together with its sources, so a
// partial dword costs no second round trip and no branch)
__device__ __forceinline__ void put_word(uint32_t *b32, int w, uint32_t v, uint32_t old, int op,
                                         int end)
{
    const uint32_t m = range_mask(4 * w, op, end);
    b32[w] = (v & m) | (old & ~m);
}

// out[op, op + len) = buf[src, src + len) for src >= op (literals: every step
// reads before it writes, and a later step never reads a dword an earlier
// step wrote) or src + len <= op (a match without overlap).
__device__ __forceinline__ void dcopy_step(uint32_t *b32, int w, int delta, uint32_t sh, int op,
                                           int end)
{
    const int a = w + (delta >> 2); // (4 w + delta) >> 2, no masking
    const uint32_t old = b32[w];
    put_word(b32, w, __builtin_amdgcn_alignbyte(b32[a + 1], b32[a], sh), old, op, end);
}

// (the first step is peeled: most runs fit one step of the wave, and the
// loop's per-lane induction updates would be wasted on it)
__device__ __forceinline__ void dcopy(uint32_t *b32, int op, int src, int len)
{
    if (len <= 0) return; // (a sequence without literals: a quarter of them)
    const int w0 = op >> 2, w1 = (op + len + 3) >> 2, end = op + len;
    const int delta = src - op;
    const uint32_t sh = (uint32_t)(delta & 3);
    dcopy_step(b32, w0 + (int)threadIdx.x, delta, sh, op, end);
    for (int b = w0 + kWave; b < w1; b += kWave)
        dcopy_step(b32, b + (int)threadIdx.x, delta, sh, op, end);
}

// Two adjacent copies in one pass: out[a, b) = buf[a + d1, b + d1) (a match
// whose source ends at or before a: d1 = -off, off >= b - a) and
// out[b, c) = buf[b + d2, c + d2) (literals, d2 >= 0).  Both are
// independent of each other's output, so each lane builds its dword from
// both sources and its old value with three byte masks (bytes from a, from
// b and from c on): old below a, match bytes in [a, b), literal bytes in
// [b, c), old from c on.  The masks are valid for every dword, so no lane
// branches.  Same padding and ordering rules as dcopy.
__device__ __forceinline__ void dcopy2_step(uint32_t *b32, int w, int d1, uint32_t sh1, int d2,
                                            uint32_t sh2, int a, int b, int c)
{
    const uint32_t old = b32[w];
    const int s1 = w + (d1 >> 2), s2 = w + (d2 >> 2); // (4 w + d) >> 2
    const uint32_t v1 = __builtin_amdgcn_alignbyte(b32[s1 + 1], b32[s1], sh1);
    const uint32_t v2 = __builtin_amdgcn_alignbyte(b32[s2 + 1], b32[s2], sh2);
    const uint32_t gb = ge_mask(4 * w, b), gc = ge_mask(4 * w, c), ga = ge_mask(4 * w, a);
    const uint32_t t = (v2 & gb) | (v1 & ~gb); // from b on the literals, below it the match
    const uint32_t u = (old & gc) | (t & ~gc); // from c on unchanged
    b32[w] = (u & ga) | (old & ~ga);           // below a unchanged
}

__device__ __forceinline__ void dcopy2(uint32_t *b32, int a, int d1, int b, int d2, int c)
{
    const int w0 = a >> 2, w1 = (c + 3) >> 2;
    const uint32_t sh1 = (uint32_t)(d1 & 3), sh2 = (uint32_t)(d2 & 3);
    dcopy2_step(b32, w0 + (int)threadIdx.x, d1, sh1, d2, sh2, a, b, c);
    for (int k = w0 + kWave; k < w1; k += kWave)
        dcopy2_step(b32, k + (int)threadIdx.x, d1, sh1, d2, sh2, a, b, c);
}

// One wave step of an overlapping match, for dword w (r: the byte offset of
// the dword's first byte from op, mod off).  Period 1..3: the dword is built
// from the period's bytes p0..p2.
__device__ __forceinline__ void dmatch_step_short(uint32_t *b32, int w, int r, int off, uint32_t p0,
                                                  uint32_t p1, uint32_t p2, int op, int end)
{
    const uint32_t old = b32[w];
    uint32_t v;
    if (off == 1) {
        v = p0 * 0x01010101u;
    } else if (off == 2) {
        v = (r == 0 ? (p0 | (p1 << 8)) : (p1 | (p0 << 8))) * 0x00010001u;
    } else {
        const uint32_t a = r == 0 ? p0 : (r == 1 ? p1 : p2);
        const uint32_t c1 = r == 0 ? p1 : (r == 1 ? p2 : p0);
        const uint32_t c2 = r == 0 ? p2 : (r == 1 ? p0 : p1);
        v = a | (c1 << 8) | (c2 << 16) | (a << 24);
    }
    put_word(b32, w, v, old, op, end);
}

// Period of 4 bytes or more starting at base: 4 bytes of it from r; where
// they run past its end (k = off - r < 4 of them), the rest comes from its
// start (head: its first dword).
__device__ __forceinline__ void dmatch_step(uint32_t *b32, int w, int r, int off, int base,
                                            uint32_t head, int op, int end)
{
    const uint32_t old = b32[w];
    const int sidx = base + r;
    uint32_t v = __builtin_amdgcn_alignbyte(b32[(sidx >> 2) + 1], b32[sidx >> 2],
                                            (uint32_t)(sidx & 3));
    const int k = off - r; // bytes from k on (none when k >= 4) wrap to the period's start
    const uint32_t gk = ge_mask(0, k);
    v = (v & ~gk) | ((head << (8 * (k & 3))) & gk);
    put_word(b32, w, v, old, op, end);
}

// LZ4 match: out[op + i] = out[op - off + (i mod off)] for i < len.  Every
// source byte lies in [op - off, op), final before the match starts, so all
// steps are independent.  Lane state r = (byte offset of its dword from op)
// mod off, advanced by 256 mod off per step.
__device__ __forceinline__ void dmatch(uint32_t *b32, int op, int off, int len)
{
    if (off >= len) {
        dcopy(b32, op, op - off, len);
        return;
    }
    const uint8_t *b8 = reinterpret_cast<const uint8_t *>(b32);
    const int w0 = op >> 2, w1 = (op + len + 3) >> 2, end = op + len;
    const int base = op - off;
    // Remainders by off without a division: with M = 2^32 / off rounded up
    // by less than 2^24 / off (an upward-biased hardware reciprocal is well
    // inside that), floor(x M / 2^32) = floor(x / off) for 0 <= x <= 256.
    // The lane's byte offset x = 4 (w0 + lane) - op lies in [-3, 252]; a
    // negative one (lane 0) is below off, so one or two periods lift it.
    // (For off = 1 the values are not used, and 2^32 / off does not fit.)
    const float mf = __builtin_amdgcn_rcpf((float)off) * 4294971392.0f;
    const uint32_t M =
        off > 1 ? (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)mf) + 1u : 0u;
    const int x = 4 * (w0 + (int)threadIdx.x) - op;
    int r = x >= 0 ? x - off * (int)__umulhi((uint32_t)x, M) : (x + off >= 0 ? x + off : x + 2 * off);
    const int step = 4 * kWave - off * (int)__umulhi(4u * kWave, M);
    if (off < 4) { // a period of 1..3 bytes, replicated from registers
        const uint32_t p0 = b8[base], p1 = b8[base + (off > 1 ? 1 : 0)],
                       p2 = b8[base + (off > 2 ? 2 : 0)];
        // the first step peeled (most matches fit one step of the wave)
        dmatch_step_short(b32, w0 + (int)threadIdx.x, r, off, p0, p1, p2, op, end);
        for (int b = w0 + kWave; b < w1; b += kWave) {
            r += step;
            if (r >= off) r -= off;
            dmatch_step_short(b32, b + (int)threadIdx.x, r, off, p0, p1, p2, op, end);
        }
        return;
    }
    const uint32_t head = __builtin_amdgcn_alignbyte(b32[(base >> 2) + 1], b32[base >> 2],
                                                     (uint32_t)(base & 3));
    dmatch_step(b32, w0 + (int)threadIdx.x, r, off, base, head, op, end);
    for (int b = w0 + kWave; b < w1; b += kWave) {
        r += step;
        if (r >= off) r -= off;
        dmatch_step(b32, b + (int)threadIdx.x, r, off, base, head, op, end);
    }
}

// Decode the LZ4 block held at buf[ip0, iend) into buf[0, ob) in place (the
// input sits at the tail of the buffer).  Returns false on malformed input:
// every length, offset and the input/output boundaries are checked once per
// sequence, and the output may never reach input not yet read.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// The bytes from position pos of the buffer as a wave-uniform little-endian
// 64-bit value (byte pos in bits 0-7): the two dwords holding pos, so at
// least the 5 bytes pos .. pos + 4 are valid.
__device__ __forceinline__ uint64_t lds_le64_uni(const uint32_t *b32, int pos)
{
    const int a = pos >> 2;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)b32[a]);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)b32[a + 1]);
    return ((uint64_t)hi << 32 | lo) >> (8 * (pos & 3));
}

// The head of a sequence from its token at ip (w: the token and the bytes
// after it): the literal length and the literals' position.  A length field
// whose continuation runs past the input gives a length that fails every
// check.
__device__ __forceinline__ void seq_head(const uint8_t *b8, int ip, uint64_t w, int iend, int &ll,
                                         int &lit)
{
    constexpr int kBadLength = 1 << 30;
    ll = (int)(((uint32_t)w & 255u) >> 4);
    lit = ip + 1;
    if (ll == 15) {
        const int e = (int)((uint32_t)(w >> 8) & 255u);
        if (e != 255) {
            ll += e;
            lit = ip + 2;
        } else {
            int q = ip + 1;
            if (!read_len_ext(b8, q, iend, ll)) ll = kBadLength;
            lit = uni(q);
            ll = uni(ll);
        }
    }
}

__device__ __forceinline__ bool decode_inplace(uint32_t *b32, int ip0, int iend, int ob)
{
    constexpr int kBadLength = 1 << 30;
    uint8_t *b8 = reinterpret_cast<uint8_t *>(b32);
    int ip = uni(ip0);
    iend = uni(iend);
    ob = uni(ob);
    if (ip >= iend) return false; // not even a token
    // Sequence j's match and sequence j + 1's literals are adjacent in the
    // output and independent of each other, so they are copied in one pass
    // (unless the match overlaps its own output).  The input past each
    // literal run is read once: offset, a match-length byte, the next token
    // and its first length byte.
    uint64_t w = lds_le64_uni(b32, ip);
    uint32_t tok = (uint32_t)w & 255u;
    int ll, lit;
    seq_head(b8, ip, w, iend, ll, lit);
    // literals (and so the length bytes) inside the input, output inside the
    // block.  All quantities are far below 2^31: a check fails iff its
    // difference is negative, so one sign test covers them all.
    if (((iend - lit - ll) | (ob - ll)) < 0) return false;
    int ip2 = lit + ll;
    uint32_t r0 = b32[ip2 >> 2], r1 = b32[(ip2 >> 2) + 1];
    dcopy(b32, 0, lit, ll);
    int op = ll;
    while (ip2 != iend) {
        const uint64_t ow = ((uint64_t)(uint32_t)uni((int)r1) << 32 | (uint32_t)uni((int)r0)) >>
                            (8 * (ip2 & 3));
        const int off = (int)((uint32_t)ow & 0xFFFFu);
        int ml = (int)(tok & 15u) + kMinMatch;
        int nip = ip2 + 2;
        uint64_t nw = ow >> 16;
        if ((tok & 15u) == 15u) {
            const int e = (int)((uint32_t)(ow >> 16) & 255u);
            if (e != 255) {
                ml += e;
                nip = ip2 + 3;
                nw = ow >> 24;
            } else {
                int q = ip2 + 2;
                if (!read_len_ext(b8, q, iend, ml)) ml = kBadLength;
                nip = uni(q);
                ml = uni(ml);
                nw = lds_le64_uni(b32, nip < iend ? nip : iend);
            }
        }
        // the next sequence's head (its input lies at or past nip, which the
        // match does not reach)
        const int op2 = op + ml;
        tok = (uint32_t)nw & 255u;
        int ll2, lit2;
        seq_head(b8, nip, nw, iend, ll2, lit2);
        // offset inside the output so far; the match ends at or before nip
        // (output never past unread input); the next literals inside the
        // input and the output inside the block.  These imply the rest:
        // lit2 > nip >= op2, nip < lit2 + ll2 <= iend, op2 <= op2 + ll2 <= ob.
        if (((off - 1) | (op - off) | (nip - op2) | (iend - lit2 - ll2) | (ob - op2 - ll2)) < 0)
            return false;
        ip2 = lit2 + ll2;
        r0 = b32[ip2 >> 2];
        r1 = b32[(ip2 >> 2) + 1];
        if (off >= ml) {
            dcopy2(b32, op, -off, op2, lit2 - op2, op2 + ll2);
        } else {
            dmatch(b32, op, off, ml);
            dcopy(b32, op2, lit2, ll2);
        }
        op = op2 + ll2;
    }
    return op == ob;
}

template <int E>
__device__ __forceinline__ void unstage_fast(const uint8_t *lds, int64_t elems,
                                             uint8_t *__restrict__ dst)
{
    const int64_t units = elems / Unit<E>::G;
    for (int64_t u = threadIdx.x; u < units; u += kWave) {
        uint32_t w[Unit<E>::IN_WORDS];
        load_planes<E>(lds, elems / 8, u, w);
        unit_inverse<E>(w);
        store_unit<E>(dst + u * (Unit<E>::G * E), w);
    }
}

template <int EC>
__device__ __forceinline__ void unstage_block(const uint8_t *lds, int64_t elems, int64_t E,
                                              uint8_t *__restrict__ dst, bool fast_out)
{
    if constexpr (EC == kByteShuffle) {
        block_inverse_bytes(lds, dst, elems, E);
        return;
    } else if constexpr (EC != 0) {
        if (fast_out && elems % Unit<EC>::G == 0) {
            unstage_fast<EC>(lds, elems, dst);
            return;
        }
    }
    block_inverse_bits(lds, dst, elems, E);
}

// Bytes of the in-place LDS buffer for blocks up to MAXB bytes: the block
// plus the slack a valid LZ4 block needs so that output never overtakes
// unread input (any suffix of a block codes its output with at most
// out/255 + 2 extra bytes), plus alignment.
template <int MAXB> constexpr int dec_buf_bytes() { return (MAXB + MAXB / 255 + 64 + 3) & ~3; }


// Copy sz bytes from a 16-byte aligned slot (readable for at least sz + 8
// bytes) to any byte address: head bytes until dst is 4-byte aligned, then
// aligned dwords assembled from two source dwords, then tail bytes.  Each
// lane takes 4 destination dwords per step: one 16-byte load of its source
// dwords plus the dword after them, and one 16-byte store.  All loads are
// issued before the first store.
__device__ __forceinline__ void copy_slot(uint8_t *__restrict__ dst, const uint8_t *__restrict__ src,
                                          int sz)
{
    constexpr int kSteps = 4; // 4 KiB per pass of the wave
    const int lane = lane_id();
    const int mis = (int)((4 - ((uintptr_t)dst & 3)) & 3);
    const int head = mis < sz ? mis : sz;
    if (lane < head) dst[lane] = src[lane];
    const int body = (sz - head) / 4;
    const uint32_t *s32 = reinterpret_cast<const uint32_t *>(src);
    const uint4 *s128 = reinterpret_cast<const uint4 *>(src);
    uint32_t *d32 = reinterpret_cast<uint32_t *>(dst + head);
    const uint32_t sh = (uint32_t)head;
    for (int b0 = 0; b0 < body; b0 += 4 * kWave * kSteps) {
        uint4 q[kSteps];
        uint32_t nx[kSteps];
#pragma unroll
        for (int k = 0; k < kSteps; ++k) {
            const int w = b0 + 4 * (kWave * k + lane); // first of the lane's 4 dwords
            q[k] = make_uint4(0, 0, 0, 0);
            nx[k] = 0;
            if (w + 4 <= body) {
                q[k] = s128[w >> 2];
                nx[k] = s32[w + 4];
            }
        }
#pragma unroll
        for (int k = 0; k < kSteps; ++k) {
            const int w = b0 + 4 * (kWave * k + lane);
            if (w + 4 <= body) {
                const uint4 o = make_uint4(__builtin_amdgcn_alignbyte(q[k].y, q[k].x, sh),
                                           __builtin_amdgcn_alignbyte(q[k].z, q[k].y, sh),
                                           __builtin_amdgcn_alignbyte(q[k].w, q[k].z, sh),
                                           __builtin_amdgcn_alignbyte(nx[k], q[k].w, sh));
                *reinterpret_cast<uint4 *>(d32 + w) = o;
            } else {
                for (int j = w; j < body && j < w + 4; ++j)
                    d32[j] = __builtin_amdgcn_alignbyte(s32[j + 1], s32[j], sh);
            }
        }
    }
    for (int i = head + 4 * body + lane; i < sz; i += kWave) dst[i] = src[i];
}

// ---- one block, start to end ----------------------------------------------
// 10 KiB for the 8 KiB block, exactly 20 of the 512-byte units LDS is
// allocated in (16 workgroups per CU).  Reads that run past the block land
// in the table and are masked out.
template <int MAXB> struct EncLds {
    uint32_t blk32[MAXB / 4];
    uint32_t table[1 << kHashBits];
};

// Transpose (and optionally round) the elems x E bytes at src into LDS, then
// LZ4-encode them into slot; returns the compressed size.  Leaves LDS free
// for the next block.
template <int MAXB, int EC, int RM>
__device__ __forceinline__ int encode_one(const uint8_t *__restrict__ src, int64_t elems, int64_t E,
                                          const RoundParams &rp, int64_t first_elem,
                                          uint8_t *__restrict__ slot, EncLds<MAXB> &L)
{
    stage_block<EC, RM>(src, elems, E, reinterpret_cast<uint8_t *>(L.blk32), rp, first_elem);
    wave_sync();
    const int sz = encode_block<MAXB>(L.blk32, (int)(elems * E), L.table, slot);
    wave_sync();
    return sz;
}

// Waves per SIMD the decoder kernels ask the register allocator for: 4
// (at most 128 VGPRs) for 8 KiB blocks of element classes up to 8 bytes,
// where LDS lets 18 blocks reside per CU and one more register would cost
// a quarter of them; 1 (no limit) where the transpose of 12- and 16-byte
// elements needs more registers or LDS already allows only a few blocks.
template <int MAXB, int EC> constexpr int dec_waves_per_eu()
{
    return MAXB <= kSmallBlock && EC != 12 && EC != 16 ? 4 : 1;
}

template <int MAXB> struct DecLds {
    // + 4 dwords in front (one readable padding dword before the buffer),
    // 4 over-read after, and 64 for the copy lanes past a range
    uint32_t buf32[dec_buf_bytes<MAXB>() / 4 + 8 + kWave];
};

// Stage the LZ4 bytes of block b of a stream (payload / off as laid out in
// the stream) at the tail of the in-place buffer B (B[-1] readable padding)
// with the same 4-byte phase as in HBM: the 16-byte lines holding them, one
// per lane and step (the dwords before the block land in the free output
// space, the last line's bytes past it in the padding; a line past in_end
// is read byte by byte).  Returns false when the block's offsets are not
// plausible; else base / len: where the bytes start in B and how many.
template <int MAXB>
__device__ __forceinline__ bool stage_lz4(const uint8_t *__restrict__ payload, int64_t payload_len,
                                          const uint64_t *__restrict__ off, int64_t b, int ob,
                                          const uint8_t *in_end, uint32_t *B, int &base, int &len)
{
    constexpr int kBuf = dec_buf_bytes<MAXB>();
    const int lane = threadIdx.x;
    const uint64_t o0 = off[b], o1 = off[b + 1];
    if (o0 > o1 || o1 > (uint64_t)payload_len || o1 - o0 > (uint64_t)lz4_bound(ob)) return false;
    len = (int)(o1 - o0);
    const uint8_t *src = payload + o0;
    const int s = (int)((uintptr_t)src & 3);
    base = ((kBuf - len - s) & ~3) + s;
    const int w0 = (base - s) >> 2;            // buffer dword of the stream dword holding src
    const int s16 = (int)((uintptr_t)src & 15);
    const uint4 *s128 = reinterpret_cast<const uint4 *>(src - s16);
    const int lines = (s16 + len + 15) >> 4;
    const int d0 = w0 - ((s16 - s) >> 2);      // buffer dword of the first line's first dword
    for (int k = lane; k < lines; k += kWave) {
        const uint8_t *lp = reinterpret_cast<const uint8_t *>(s128 + k);
        uint4 v;
        if (lp + 16 <= in_end) {
            v = s128[k];
        } else {
            uint32_t x[4] = {0, 0, 0, 0};
            for (int j = 0; j < 16; ++j)
                if (lp + j < in_end) x[j >> 2] |= (uint32_t)lp[j] << (8 * (j & 3));
            v = make_uint4(x[0], x[1], x[2], x[3]);
        }
        uint32_t *d = B + d0 + 4 * k;
        d[0] = v.x;
        d[1] = v.y;
        d[2] = v.z;
        d[3] = v.w;
    }
    return true;
}

// Decode block b of a stream into dst (elems x E bytes).  Returns false
// when the block is corrupt; then dst holds nothing meaningful.  Never
// reads past in_end.
template <int MAXB, int EC>
__device__ __forceinline__ bool decode_one(const uint8_t *__restrict__ payload, int64_t payload_len,
                                           const uint64_t *__restrict__ off, int64_t b,
                                           int64_t elems, int64_t E, const uint8_t *in_end,
                                           uint8_t *__restrict__ dst, bool fast_out,
                                           DecLds<MAXB> &L)
{
    const int ob = (int)(elems * E);
    uint32_t *B = L.buf32 + 4; // the decode buffer; B[-1] is readable padding
    int base, len;
    if (!stage_lz4<MAXB>(payload, payload_len, off, b, ob, in_end, B, base, len)) return false;
    wave_sync();
    // the serial token walk issues ahead of other waves' staging and
    // inverse transposes, which have independent work to fill the gaps
    __builtin_amdgcn_s_setprio(1);
    const bool ok = decode_inplace(B, base, base + len, ob);
    __builtin_amdgcn_s_setprio(0);
    wave_sync();
    if (ok) {
        constexpr int64_t kFull = full_block_elems<MAXB, EC>();
        bool done = false;
        if constexpr (kFull != 0) {
            if (fast_out && elems == kFull) {
                unstage_fast<EC>(reinterpret_cast<const uint8_t *>(B), kFull, dst);
                done = true;
            }
        }
        if (!done)
            unstage_block<EC>(reinterpret_cast<const uint8_t *>(B), elems, E, dst, fast_out);
    }
    wave_sync();
    return ok;
}

// Header fields and offsets table ends of a stream agree with the expected
// layout.  Called by one wavefront.
__device__ __forceinline__ bool header_ok(const uint8_t *in, int64_t payload_len, int64_t n,
                                          int64_t E, int64_t nb, int64_t n_blocks,
                                          uint32_t magic = BSG_MAGIC)
{
    const bsg_header *h = reinterpret_cast<const bsg_header *>(in);
    const uint64_t *off = reinterpret_cast<const uint64_t *>(in + kHeaderBytes);
    return h->magic == magic && h->elem_size == (uint32_t)E && h->n == (uint64_t)n &&
           h->block_elems == (uint32_t)nb && h->n_blocks == (uint32_t)n_blocks && off[0] == 0 &&
           off[n_blocks] == (uint64_t)payload_len;
}

// The element class with a register fast path, or 0.
inline int element_class(int64_t E) { return unit_elems(E) ? (int)E : 0; }

} // namespace
} // namespace bsg
