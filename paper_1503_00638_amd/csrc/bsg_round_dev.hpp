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

// Largest integer k with 4^k < G2, for G2 > 0 and finite, from the bits of
// G2 = m 2^E (1 <= m < 2): k = floor(E/2) when m > 1, floor((E-1)/2) when
// G2 is an exact power of two.
__device__ __forceinline__ int granularity_k(double G2)
{
    const uint64_t u = (uint64_t)__double_as_longlong(G2);
    const int ex = (int)(u >> 52);
    uint64_t mant = u & 0xFFFFFFFFFFFFFull;
    int E;
    if (ex == 0) { // subnormal double: value = mant * 2^-1074
        const int top = 63 - __clzll((long long)mant);
        E = top - 1074;
        mant &= ~(1ull << top);
    } else {
        E = ex - 1023;
    }
    return mant == 0 ? ((E - 1) >> 1) : (E >> 1); // >> on int is floor division
}

// Round float32 bits x to the nearest multiple of 2^k, ties to even, keeping
// the sign (a result of zero keeps the sign of x); NaN and Inf unchanged.
// With ulp(x) = 2^(max(exp,1) - 150), d = k - log2 ulp low magnitude bits
// are cleared after adding the round-half-even increment; a carry into the
// exponent field is the correct next binade (and 0x7f800000 = Inf on
// overflow).
__device__ __forceinline__ uint32_t round_bits(uint32_t x, int k)
{
    const uint32_t mag = x & 0x7FFFFFFFu;
    const int ex = (int)(mag >> 23);
    if (ex == 255) return x;
    const int d = k - ((ex == 0 ? 1 : ex) - 150);
    if (d <= 0) return x;
    const uint32_t sign = x & 0x80000000u;
    if (d >= 25 || (d == 24 && ex == 0)) return sign; // |x| < g/2
    if (d == 24) // g/2 <= |x| < g: the tie g/2 goes to 0 (even), else to g
        return sign | (((mag & 0x7FFFFFu) == 0) ? 0u : ((uint32_t)(ex + 1) << 23));
    // parity of floor(|x| / g): bit d of the significand (1.m or 0.m); for
    // a normal x with d == 23 that is the implicit leading 1, not bit 23 of
    // the stored magnitude (the exponent's lowest bit)
    const uint32_t odd = (d == 23 && ex != 0) ? 1u : ((mag >> d) & 1u);
    const uint32_t inc = (1u << (d - 1)) - 1u + odd;
    return sign | ((mag + inc) & ~((1u << d) - 1u));
}

__device__ __forceinline__ uint32_t round_noise_bits(uint32_t x, double G2)
{
    if (!(G2 > 0.0) || G2 == __builtin_inf()) return x;
    return round_bits(x, granularity_k(G2));
}

// One complex visibility.  ai = V_ii, aj = V_jj at the same (f, t).
__device__ __forceinline__ float2 round_complex(float2 v, float ai, float aj, bool is_auto,
                                                const RoundParams &rp)
{
    float2 o;
    if (!is_auto) {
        const double G2 = ((double)ai * (double)aj) * rp.c;
        o.x = __uint_as_float(round_noise_bits(__float_as_uint(v.x), G2));
        o.y = __uint_as_float(round_noise_bits(__float_as_uint(v.y), G2));
    } else {
        const double G2 = ((double)ai * (double)ai) * rp.c_auto;
        o.x = __uint_as_float(round_noise_bits(__float_as_uint(v.x), G2));
        o.y = v.y;
    }
    return o;
}

// Element e of the visibility array viewed as float32 (component e & 1 of
// visibility e >> 1), rounded.  Used where elements are visited one by one.
__device__ __forceinline__ uint32_t round_element(uint32_t x, int64_t e, const RoundParams &rp)
{
    const int64_t ci = e >> 1;
    const int64_t row = ci / rp.T, t = ci - row * rp.T;
    const int64_t fr = row / rp.P, p = row - fr * rp.P;
    int32_t i, j;
    product_pair(rp, p, i, j);
    const float ai = rp.autos[(fr * rp.I + i) * rp.T + t];
    const float aj = rp.autos[(fr * rp.I + j) * rp.T + t];
    if (i != j) return round_noise_bits(x, ((double)ai * (double)aj) * rp.c);
    if ((e & 1) == 0) return round_noise_bits(x, ((double)ai * (double)ai) * rp.c_auto);
    return x;
}

} // namespace bsg
