// Device helpers for the noise-relative rounding (Section 3.1 and 3.2 of
// Masui et al.), shared by the standalone kernel and the fused compressor.
#pragma once

#include "bsg_internal.hpp"

namespace bsg {

// (i, j) of product p.  Default order: upper triangle, row major,
// (0,0) (0,1) .. (0,I-1) (1,1) .. (I-1,I-1).  Counting from the end, q =
// P-1-p falls in reversed row r = floor((sqrt(8q+1)-1)/2), i.e. input
// i = I-1-r; the float estimate is corrected with exact integer checks.
__device__ __forceinline__ void product_pair(const RoundParams &rp, int64_t p, int32_t &i,
                                             int32_t &j)
{
    if (rp.prod_map) {
        i = rp.prod_map[2 * p];
        j = rp.prod_map[2 * p + 1];
        return;
    }
    const int64_t q = rp.P - 1 - p;
    int64_t r = (int64_t)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= q) ++r;
    while (r * (r + 1) / 2 > q) --r;
    const int64_t in_row = q - r * (r + 1) / 2; // 0 = last element of the row
    i = (int32_t)(rp.I - 1 - r);
    j = (int32_t)(rp.I - 1 - in_row);
}

// Largest integer k with 4^k < G2, for G2 > 0 and finite.  With G2 = m 2^e,
// 1/2 <= m < 1 (frexp, subnormals included): k = floor((e - 1) / 2), or
// floor((e - 2) / 2) when G2 is an exact power of two (4^k = G2 must not
// count).
__device__ __forceinline__ int granularity_k(double G2)
{
    const int e = __builtin_amdgcn_frexp_exp(G2);
    const double m = __builtin_amdgcn_frexp_mant(G2);
    return (m == 0.5 ? e - 2 : e - 1) >> 1; // >> on int is floor division
}

// Round float32 bits x to the nearest multiple of 2^k, ties to even: in
// double, x 2^-k and back are exact scalings (|k| stays far below the double
// exponent range for any finite float G2), rint rounds half to even and
// keeps the sign of zero, and the result is a float (a multiple of 2^k no
// larger than |x| + 2^k/2, or Inf past the float range).  NaN and Inf are
// returned as they are.
__device__ __forceinline__ uint32_t round_bits(uint32_t x, int k)
{
    if ((x & 0x7F800000u) == 0x7F800000u) return x;
    const double y = __builtin_ldexp((double)__uint_as_float(x), -k);
    return __float_as_uint((float)__builtin_ldexp(__builtin_rint(y), k));
}

__device__ __forceinline__ uint32_t round_noise_bits(uint32_t x, double G2)
{
    if (!(G2 > 0.0) || G2 == __builtin_inf()) return x;
    return round_bits(x, granularity_k(G2));
}

// round_noise_bits with both paths computed and one selected, for code
// that rounds many values back to back (no branch per value).
__device__ __forceinline__ uint32_t round_noise_bits_nb(uint32_t x, double G2)
{
    const int k = granularity_k(G2);
    const double y = __builtin_ldexp((double)__uint_as_float(x), -k);
    const uint32_t r = __float_as_uint((float)__builtin_ldexp(__builtin_rint(y), k));
    const bool keep = !(G2 > 0.0) || G2 == __builtin_inf() || (x & 0x7F800000u) == 0x7F800000u;
    return keep ? x : r;
}

// One complex visibility.  ai = V_ii, aj = V_jj at the same (f, t); sc is
// the factor on G2 at that (f, t) (1 without compensation).  Both
// components of a cross product share one G2 and one k.
__device__ __forceinline__ float2 round_complex(float2 v, float ai, float aj, bool is_auto,
                                                const RoundParams &rp, double sc = 1.0)
{
    double G2 = ((double)ai * (double)aj) * (is_auto ? rp.c_auto : rp.c);
    if (rp.fscale) G2 *= sc;
    if (!(G2 > 0.0) || G2 == __builtin_inf()) return v;
    const int k = granularity_k(G2);
    float2 o;
    o.x = __uint_as_float(round_bits(__float_as_uint(v.x), k));
    o.y = is_auto ? v.y : __uint_as_float(round_bits(__float_as_uint(v.y), k));
    return o;
}

// a / b and a % b for non-negative a, b > 0: 32-bit division when both fit.
__device__ __forceinline__ void divmod(int64_t a, int64_t b, int64_t &q, int64_t &r)
{
    if (((uint64_t)a | (uint64_t)b) >> 32 == 0) {
        const uint32_t q32 = (uint32_t)a / (uint32_t)b;
        q = q32;
        r = (int64_t)((uint32_t)a - q32 * (uint32_t)b);
    } else {
        q = a / b;
        r = a - q * b;
    }
}

// Position of a visibility in the [F][P][T] array with its product's inputs
// and the offsets of its two auto-correlation rows in [F][I][T]; stepping
// through time and products needs no division.
struct VisCursor {
    int64_t t, p, fr;
    int32_t i, j;
    int64_t row_i, row_j; // (fr I + i) T and (fr I + j) T
};

__device__ __forceinline__ void cursor_rows(const RoundParams &rp, VisCursor &c)
{
    c.row_i = (c.fr * rp.I + c.i) * rp.T;
    c.row_j = (c.fr * rp.I + c.j) * rp.T;
}

__device__ __forceinline__ VisCursor cursor_at(const RoundParams &rp, int64_t ci)
{
    VisCursor c;
    int64_t row;
    divmod(ci, rp.T, row, c.t);
    divmod(row, rp.P, c.fr, c.p);
    product_pair(rp, c.p, c.i, c.j);
    cursor_rows(rp, c);
    return c;
}

// The next product (upper-triangle order steps j, then i; past the last
// product the next frequency).
__device__ __forceinline__ void cursor_next_product(const RoundParams &rp, VisCursor &c)
{
    if (++c.p == rp.P) {
        c.p = 0;
        ++c.fr;
    }
    if (rp.prod_map) {
        c.i = rp.prod_map[2 * c.p];
        c.j = rp.prod_map[2 * c.p + 1];
    } else if (c.p == 0) {
        c.i = c.j = 0;
    } else if (++c.j == rp.I) {
        c.j = ++c.i;
    }
    cursor_rows(rp, c);
}

__device__ __forceinline__ void cursor_advance(const RoundParams &rp, VisCursor &c, int64_t dt)
{
    c.t += dt;
    while (c.t >= rp.T) {
        c.t -= rp.T;
        cursor_next_product(rp, c);
    }
}

__device__ __forceinline__ float2 round_at(float2 v, const VisCursor &c, const RoundParams &rp)
{
    const float ai = rp.autos[c.row_i + c.t];
    const float aj = rp.autos[c.row_j + c.t];
    const double sc = rp.fscale ? rp.fscale[c.fr * rp.T + c.t] : 1.0;
    return round_complex(v, ai, aj, c.i == c.j, rp, sc);
}

// Integer visibilities: the nearest multiple of 2^k, ties to the even
// multiple, in exact integer arithmetic; only k >= 1 changes an integer.  A
// result above INT32_MAX becomes the largest multiple of 2^k that fits (the
// negative side always fits: -2^31 is a multiple of every 2^k, k <= 31).
__device__ __forceinline__ int32_t round_int(int32_t x, int k)
{
    if (k <= 0) return x;
    if (k > 62) k = 62; // |x| <= 2^31 < g/2
    const int64_t g = (int64_t)1 << k;
    int64_t q = (int64_t)x >> k; // floor division
    const int64_t rem = (int64_t)x - q * g;
    if (rem > (g >> 1) || (rem == (g >> 1) && (q & 1))) ++q;
    int64_t r = q * g;
    if (r > 2147483647ll) r = (2147483647ll >> k) * g;
    return (int32_t)r;
}

// One integer visibility (re, im); G2 from the exact int64 product of the
// two autos rounded once to double.
__device__ __forceinline__ int2 round_at_i32(int2 v, const VisCursor &c, const RoundParams &rp)
{
    const int64_t ai = rp.autos_i32[c.row_i + c.t];
    const int64_t aj = rp.autos_i32[c.row_j + c.t];
    const bool is_auto = c.i == c.j;
    const double G2 = (double)(ai * aj) * (is_auto ? rp.c_auto : rp.c);
    if (!(G2 > 0.0) || G2 == __builtin_inf()) return v;
    const int k = granularity_k(G2);
    return make_int2(round_int(v.x, k), is_auto ? v.y : round_int(v.y, k));
}

// Element e of the visibility array viewed as float32 (component e & 1 of
// visibility e >> 1), rounded.  Used where elements are visited one by one.
__device__ __forceinline__ uint32_t round_element(uint32_t x, int64_t e, const RoundParams &rp)
{
    const VisCursor c = cursor_at(rp, e >> 1);
    const float ai = rp.autos[c.row_i + c.t];
    const float aj = rp.autos[c.row_j + c.t];
    const double sc = rp.fscale ? rp.fscale[c.fr * rp.T + c.t] : 1.0;
    if (c.i != c.j) {
        double G2 = ((double)ai * (double)aj) * rp.c;
        if (rp.fscale) G2 *= sc;
        return round_noise_bits(x, G2);
    }
    if ((e & 1) == 0) {
        double G2 = ((double)ai * (double)ai) * rp.c_auto;
        if (rp.fscale) G2 *= sc;
        return round_noise_bits(x, G2);
    }
    return x;
}

} // namespace bsg
