// Device-side bit transpose of one "unit" (Bitshuffle, Section 4.2 of
// Masui et al.).  A block of n_B elements is the (n_B x 8E) bit matrix of
// its elements; bit b of element i (b = 8 * byte + bit, LSB first) goes to
// plane b, byte i / 8, bit i % 8.
//
// A lane transposes one unit in registers:
//   E = 1  : 128 elements, output 16 bytes of each of the 8 planes
//   E = 2  : 64 elements,  output 8 bytes of each of the 16 planes
//   E = 4c : 32 elements,  per 4-byte column one 32x32 transpose, output 4
//            bytes of each of the 8E planes
// Plane bytes of unit u sit at plane * (n_B / 8) + u * (G / 8), so the
// block's units must tile it exactly (n_B a multiple of G).
#pragma once

#include "bsg_internal.hpp"

namespace bsg {

template <int E> struct Unit {
    static constexpr int G = E == 1 ? 128 : (E == 2 ? 64 : 32); // elements
    static constexpr int IN_WORDS = G * E / 4;                  // input dwords
    static constexpr int PB = G / 8;                            // plane bytes per unit
    static constexpr int NC = E >= 4 ? E / 4 : 1;               // 32x32 transposes
};

// In-register forward transform.  in: the unit's raw element dwords
// (IN_WORDS).  out (same array): plane words; plane pl of the unit is
//   E = 1 : out[pl], out[pl+8], out[pl+16], out[pl+24]   (16 bytes)
//   E = 2 : out[pl], out[pl+16]                           (8 bytes)
//   E = 4c: out[32 * (pl / 32) + pl % 32]                 (4 bytes)
template <int E>
__device__ __forceinline__ void unit_forward(uint32_t (&w)[Unit<E>::IN_WORDS])
{
    if constexpr (E == 1) {
        uint32_t d[32];
        pack_e1(w, d);
        transpose32(d);
#pragma unroll
        for (int k = 0; k < 32; ++k) w[k] = d[k];
    } else if constexpr (E == 2) {
        uint32_t d[32];
        pack_e2(w, d);
        transpose32(d);
#pragma unroll
        for (int k = 0; k < 32; ++k) w[k] = d[k];
    } else {
        constexpr int NC = Unit<E>::NC;
        uint32_t o[Unit<E>::IN_WORDS];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            uint32_t a[32];
#pragma unroll
            for (int i = 0; i < 32; ++i) a[i] = w[i * NC + c];
            transpose32(a);
#pragma unroll
            for (int b = 0; b < 32; ++b) o[32 * c + b] = a[b];
        }
#pragma unroll
        for (int k = 0; k < Unit<E>::IN_WORDS; ++k) w[k] = o[k];
    }
}

// Exact inverse of unit_forward (plane words in the layout above -> raw
// element dwords).
template <int E>
__device__ __forceinline__ void unit_inverse(uint32_t (&w)[Unit<E>::IN_WORDS])
{
    if constexpr (E == 1) {
        uint32_t d[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) d[k] = w[k];
        transpose32(d);
        unpack_e1(d, w);
    } else if constexpr (E == 2) {
        uint32_t d[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) d[k] = w[k];
        transpose32(d);
        unpack_e2(d, w);
    } else {
        constexpr int NC = Unit<E>::NC;
        uint32_t o[Unit<E>::IN_WORDS];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            uint32_t a[32];
#pragma unroll
            for (int b = 0; b < 32; ++b) a[b] = w[32 * c + b];
            transpose32(a);
#pragma unroll
            for (int i = 0; i < 32; ++i) o[i * NC + c] = a[i];
        }
#pragma unroll
        for (int k = 0; k < Unit<E>::IN_WORDS; ++k) w[k] = o[k];
    }
}

// Index of plane pl's first word within the unit's plane-word array, and
// the number of words per plane.
template <int E> struct PlaneWords {
    static constexpr int PER = Unit<E>::PB / 4; // 4, 2 or 1 words
    static constexpr int NPL = 8 * E;
    __device__ static constexpr int word(int pl, int q)
    {
        return E == 1 ? pl + 8 * q : (E == 2 ? pl + 16 * q : pl);
    }
};

// Load/store the unit's raw elements (16-byte aligned, IN_WORDS dwords).
template <int E>
__device__ __forceinline__ void load_unit(const uint8_t *p, uint32_t (&w)[Unit<E>::IN_WORDS])
{
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
#pragma unroll
    for (int k = 0; k < Unit<E>::IN_WORDS / 4; ++k) {
        const uint4 v = q[k];
        w[4 * k] = v.x;
        w[4 * k + 1] = v.y;
        w[4 * k + 2] = v.z;
        w[4 * k + 3] = v.w;
    }
}
template <int E>
__device__ __forceinline__ void store_unit(uint8_t *p, const uint32_t (&w)[Unit<E>::IN_WORDS])
{
    uint4 *q = reinterpret_cast<uint4 *>(p);
#pragma unroll
    for (int k = 0; k < Unit<E>::IN_WORDS / 4; ++k)
        q[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
}

// Store / load the unit's plane bytes into a block laid out as planes of
// plane_bytes each (global or LDS; aligned to the plane chunk size).
template <int E>
__device__ __forceinline__ void store_planes(uint8_t *blk, int64_t plane_bytes, int64_t u,
                                             const uint32_t (&w)[Unit<E>::IN_WORDS])
{
    using PW = PlaneWords<E>;
#pragma unroll
    for (int pl = 0; pl < PW::NPL; ++pl) {
        uint8_t *dst = blk + pl * plane_bytes + u * Unit<E>::PB;
        if constexpr (PW::PER == 4)
            *reinterpret_cast<uint4 *>(dst) =
                make_uint4(w[PW::word(pl, 0)], w[PW::word(pl, 1)], w[PW::word(pl, 2)],
                           w[PW::word(pl, 3)]);
        else if constexpr (PW::PER == 2)
            *reinterpret_cast<uint2 *>(dst) = make_uint2(w[PW::word(pl, 0)], w[PW::word(pl, 1)]);
        else
            *reinterpret_cast<uint32_t *>(dst) = w[PW::word(pl, 0)];
    }
}
template <int E>
__device__ __forceinline__ void load_planes(const uint8_t *blk, int64_t plane_bytes, int64_t u,
                                            uint32_t (&w)[Unit<E>::IN_WORDS])
{
    using PW = PlaneWords<E>;
#pragma unroll
    for (int pl = 0; pl < PW::NPL; ++pl) {
        const uint8_t *src = blk + pl * plane_bytes + u * Unit<E>::PB;
        if constexpr (PW::PER == 4) {
            const uint4 v = *reinterpret_cast<const uint4 *>(src);
            w[PW::word(pl, 0)] = v.x;
            w[PW::word(pl, 1)] = v.y;
            w[PW::word(pl, 2)] = v.z;
            w[PW::word(pl, 3)] = v.w;
        } else if constexpr (PW::PER == 2) {
            const uint2 v = *reinterpret_cast<const uint2 *>(src);
            w[PW::word(pl, 0)] = v.x;
            w[PW::word(pl, 1)] = v.y;
        } else {
            w[PW::word(pl, 0)] = *reinterpret_cast<const uint32_t *>(src);
        }
    }
}

// Generic transpose of one block by a whole wavefront, any E and any n_B
// (multiple of 8): lanes hold 64 consecutive elements; for every bit b one
// 64-lane ballot yields 8 bytes of plane b (ballot bit l = element 64g + l,
// which is exactly the LSB-first byte order of the plane).
__device__ __forceinline__ void block_forward_ballot(const uint8_t *in, uint8_t *out,
                                                     int64_t elems, int64_t E)
{
    const int lane = threadIdx.x & 63;
    const int64_t pb = elems / 8;
    for (int64_t g = 0; g < elems; g += 64) {
        const int64_t i = g + lane;
        const bool valid = i < elems;
        const int64_t rem = (elems - g) / 8;
        const int nbytes = rem < 8 ? (int)rem : 8;
        for (int64_t byte = 0; byte < E; ++byte) {
            const uint32_t v = valid ? in[i * E + byte] : 0u;
            for (int bit = 0; bit < 8; ++bit) {
                const uint64_t m = __ballot((v >> bit) & 1u);
                if (lane < nbytes) out[(8 * byte + bit) * pb + g / 8 + lane] = (uint8_t)(m >> (8 * lane));
            }
        }
    }
}

__device__ __forceinline__ void block_inverse_bits(const uint8_t *in, uint8_t *out,
                                                   int64_t elems, int64_t E)
{
    const int lane = threadIdx.x & 63;
    const int64_t pb = elems / 8;
    for (int64_t i = lane; i < elems; i += 64) {
        for (int64_t byte = 0; byte < E; ++byte) {
            uint32_t v = 0;
            for (int bit = 0; bit < 8; ++bit)
                v |= ((uint32_t)(in[(8 * byte + bit) * pb + i / 8] >> (i % 8)) & 1u) << bit;
            out[i * E + byte] = (uint8_t)v;
        }
    }
}

} // namespace bsg
