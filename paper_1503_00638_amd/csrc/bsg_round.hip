// Stage 1: noise-relative precision reduction (Masui et al., Section 3).
//
// Per visibility (freq f, product p = (i, j), time t):
//   G2 = 12 f s^2 with s from the diagonal radiometer equation (Section 3.1):
//        s^2 = V_ii V_jj / (2N) for i != j, s^2 = V_ii^2 / N for autos,
//   g  = the largest power of two with g^2 < G2 (Eq. trunc_error, strict),
//   re and im are rounded to the nearest multiple of g, ties to even (the
//   tie-breaking footnote of Section 3.2); Im of an auto carries no noise
//   and is left alone.
//
// The value is scaled by 2^-k in double, rounded half to even there and
// scaled back (both scalings exact); k comes from the exponent and mantissa
// of the double G2 (frexp): no log, sqrt or division.
#include "bsg_internal.hpp"
#include "bsg_round_dev.hpp"

namespace bsg {

namespace {

constexpr int kComplexPerThread = 4;

// Lane i of the grid rounds the kComplexPerThread consecutive visibilities
// from e0 = i * kComplexPerThread.  When they lie in one product row at one
// frequency (times t .. t + 3, the case whenever T is a multiple of 4), the
// values and their autos are read with 16-byte loads from one base each and
// every value is rounded without a branch; otherwise a cursor steps through
// them one by one.
__global__ __launch_bounds__(256) void k_round(const float2 *__restrict__ vin,
                                               float2 *__restrict__ vout, RoundParams rp,
                                               int64_t n_complex, int aligned16)
{
    constexpr int K = kComplexPerThread;
    const int64_t e0 = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) * K;
    if (e0 >= n_complex) return;
    VisCursor c = cursor_at(rp, e0);
    if (aligned16 && e0 + K <= n_complex && c.t + K <= rp.T) {
        const float4 *v4 = reinterpret_cast<const float4 *>(vin + e0);
        float4 v[K / 2];
#pragma unroll
        for (int k = 0; k < K / 2; ++k) v[k] = v4[k];
        const float *pi = rp.autos + c.row_i + c.t;
        const float *pj = rp.autos + c.row_j + c.t;
        float ai[K], aj[K];
        double sc[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            ai[k] = pi[k];
            aj[k] = pj[k];
            sc[k] = 1.0;
        }
        if (rp.fscale) {
            const double *fs = rp.fscale + c.fr * rp.T + c.t;
#pragma unroll
            for (int k = 0; k < K; ++k) sc[k] = fs[k];
        }
        const bool is_auto = c.i == c.j;
        float4 *o4 = reinterpret_cast<float4 *>(vout + e0);
#pragma unroll
        for (int k = 0; k < K / 2; ++k) {
            uint32_t x[4] = {__float_as_uint(v[k].x), __float_as_uint(v[k].y), __float_as_uint(v[k].z),
                             __float_as_uint(v[k].w)};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int j = 2 * k + h;
                double G2 = ((double)ai[j] * (double)aj[j]) * (is_auto ? rp.c_auto : rp.c);
                if (rp.fscale) G2 *= sc[j];
                x[2 * h] = round_noise_bits_nb(x[2 * h], G2);
                if (!is_auto) x[2 * h + 1] = round_noise_bits_nb(x[2 * h + 1], G2);
            }
            o4[k] = make_float4(__uint_as_float(x[0]), __uint_as_float(x[1]), __uint_as_float(x[2]),
                                __uint_as_float(x[3]));
        }
        return;
    }
    for (int k = 0; k < K && e0 + k < n_complex; ++k) {
        if (k) cursor_advance(rp, c, 1);
        vout[e0 + k] = round_at(vin[e0 + k], c, rp);
    }
}

// As k_round, for int32 visibilities and autos (exact int64 products).
__global__ __launch_bounds__(256) void k_round_i32(const int2 *__restrict__ vin,
                                                   int2 *__restrict__ vout, RoundParams rp,
                                                   int64_t n_complex, int aligned16)
{
    constexpr int K = kComplexPerThread;
    const int64_t e0 = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) * K;
    if (e0 >= n_complex) return;
    VisCursor c = cursor_at(rp, e0);
    if (aligned16 && e0 + K <= n_complex && c.t + K <= rp.T) {
        const int4 *v4 = reinterpret_cast<const int4 *>(vin + e0);
        int4 v[K / 2];
#pragma unroll
        for (int k = 0; k < K / 2; ++k) v[k] = v4[k];
        const int32_t *pi = rp.autos_i32 + c.row_i + c.t;
        const int32_t *pj = rp.autos_i32 + c.row_j + c.t;
        int64_t ai[K], aj[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            ai[k] = pi[k];
            aj[k] = pj[k];
        }
        const bool is_auto = c.i == c.j;
        int4 *o4 = reinterpret_cast<int4 *>(vout + e0);
#pragma unroll
        for (int k = 0; k < K / 2; ++k) {
            int32_t x[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int j = 2 * k + h;
                const double G2 = (double)(ai[j] * aj[j]) * (is_auto ? rp.c_auto : rp.c);
                if (G2 > 0.0 && G2 != __builtin_inf()) {
                    const int kk = granularity_k(G2);
                    x[2 * h] = round_int(x[2 * h], kk);
                    if (!is_auto) x[2 * h + 1] = round_int(x[2 * h + 1], kk);
                }
            }
            o4[k] = make_int4(x[0], x[1], x[2], x[3]);
        }
        return;
    }
    for (int k = 0; k < K && e0 + k < n_complex; ++k) {
        if (k) cursor_advance(rp, c, 1);
        vout[e0 + k] = round_at_i32(vin[e0 + k], c, rp);
    }
}

// Compensation of the diagonal noise model (Section 3.2): per (frequency,
// time) the minimum over cross products of 1 - |V_ij|^2 / (V_ii V_jj), in
// double and in that order (products with V_ii V_jj not positive and finite
// skipped, 1 when none is left).  A workgroup takes one frequency and 64
// times; its 4 wavefronts walk a quarter of the products each (lanes =
// times, so every load is coalesced) and the 4 partial minima meet in LDS.
__global__ __launch_bounds__(256) void k_noise_comp(const float2 *__restrict__ vis, RoundParams rp,
                                                    double *__restrict__ scale)
{
    __shared__ double part[4][kWave];
    const int tl = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t fr = blockIdx.x;
    const int64_t t = int64_t(blockIdx.y) * kWave + tl;
    double m = 1.0;
    const int64_t p0 = rp.P * q / 4, p1 = rp.P * (q + 1) / 4;
    if (t < rp.T && p0 < p1) {
        VisCursor c = cursor_at(rp, (fr * rp.P + p0) * rp.T + t);
        for (int64_t p = p0;;) {
            if (c.i != c.j) {
                const double ab = (double)rp.autos[c.row_i + c.t] * (double)rp.autos[c.row_j + c.t];
                if (ab > 0.0 && ab != __builtin_inf()) {
                    const float2 v = vis[(fr * rp.P + p) * rp.T + t];
                    const double term =
                        1.0 - ((double)v.x * (double)v.x + (double)v.y * (double)v.y) / ab;
                    if (term < m) m = term; // a NaN term never wins
                }
            }
            if (++p == p1) break;
            cursor_next_product(rp, c);
        }
    }
    part[q][tl] = m;
    __syncthreads();
    if (q == 0 && t < rp.T) {
        for (int k = 1; k < 4; ++k)
            if (part[k][tl] < m) m = part[k][tl];
        scale[fr * rp.T + t] = m;
    }
}

// T a power of two up to 1024: one workgroup of 1024 threads per frequency.
// Thread k takes time t = k mod T and the products p = k / T, k / T + R, ...
// (R = 1024 / T), so each step of the workgroup reads 8 KiB of the
// contiguous [P][T] block of that frequency; the thread's inputs (i, j) are
// stepped along with p.  The per-thread minima are then reduced over the R
// threads of each time in LDS.  The minimum does not depend on the order of
// the terms (no term is -0, NaN terms are skipped).
constexpr int kCompThreads = 1024;

__global__ __launch_bounds__(kCompThreads) void k_noise_comp_rows(const float2 *__restrict__ vis,
                                                                 RoundParams rp,
                                                                 double *__restrict__ scale)
{
    __shared__ double part[kCompThreads];
    const int k = threadIdx.x;
    const int T = (int)rp.T, R = kCompThreads / T;
    const int t = k & (T - 1), r = k / T;
    const int64_t fr = blockIdx.x;
    const float2 *vrow = vis + fr * rp.P * rp.T + t;
    const float *arow = rp.autos + fr * rp.I * rp.T + t;
    double m = 1.0;
    int32_t i = 0, j = 0;
    if (r < rp.P) product_pair(rp, r, i, j);
#pragma unroll 4
    for (int64_t p = r; p < rp.P; p += R) {
        const float2 v = vrow[p * T];
        const double ab = (double)arow[(int64_t)i * T] * (double)arow[(int64_t)j * T];
        const double term = 1.0 - ((double)v.x * (double)v.x + (double)v.y * (double)v.y) / ab;
        if (i != j && ab > 0.0 && ab != __builtin_inf() && term < m) m = term; // a NaN term never wins
        // the inputs of product p + R
        if (rp.prod_map) {
            if (p + R < rp.P) {
                i = rp.prod_map[2 * (p + R)];
                j = rp.prod_map[2 * (p + R) + 1];
            }
        } else {
            j += R;
            while (j >= rp.I && i < rp.I) {
                j += i + 1 - (int32_t)rp.I; // the next row starts at j = i + 1
                ++i;
            }
        }
    }
    part[k] = m;
    __syncthreads();
    for (int st = R / 2; st >= 1; st >>= 1) {
        if (r < st && part[k + st * T] < part[k]) part[k] = part[k + st * T];
        __syncthreads();
    }
    if (r == 0) scale[fr * T + t] = part[t];
}

} // namespace

hipError_t launch_round(const float *vin, float *vout, const RoundParams &rp, hipStream_t s)
{
    const int64_t n_complex = rp.F * rp.P * rp.T;
    if (n_complex == 0) return hipSuccess;
    const int64_t waves = (n_complex + kWave * kComplexPerThread - 1) / (kWave * kComplexPerThread);
    const int64_t blocks = (waves * kWave + 255) / 256;
    const int aligned16 = (((uintptr_t)vin | (uintptr_t)vout) & 15) == 0;
    hipLaunchKernelGGL(k_round, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<const float2 *>(vin), reinterpret_cast<float2 *>(vout),
                       rp, n_complex, aligned16);
    return hipGetLastError();
}

hipError_t launch_round_i32(const int32_t *vin, int32_t *vout, const RoundParams &rp, hipStream_t s)
{
    const int64_t n_complex = rp.F * rp.P * rp.T;
    if (n_complex == 0) return hipSuccess;
    const int64_t waves = (n_complex + kWave * kComplexPerThread - 1) / (kWave * kComplexPerThread);
    const int64_t blocks = (waves * kWave + 255) / 256;
    const int aligned16 = (((uintptr_t)vin | (uintptr_t)vout) & 15) == 0;
    hipLaunchKernelGGL(k_round_i32, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<const int2 *>(vin), reinterpret_cast<int2 *>(vout), rp,
                       n_complex, aligned16);
    return hipGetLastError();
}

hipError_t launch_noise_comp(const float *vis, const RoundParams &rp, double *scale, hipStream_t s)
{
    if (rp.F * rp.T == 0) return hipSuccess;
    if (rp.T <= kCompThreads && (rp.T & (rp.T - 1)) == 0) {
        hipLaunchKernelGGL(k_noise_comp_rows, dim3((unsigned)rp.F), dim3(kCompThreads), 0, s,
                           reinterpret_cast<const float2 *>(vis), rp, scale);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)rp.F, (unsigned)((rp.T + kWave - 1) / kWave));
    hipLaunchKernelGGL(k_noise_comp, grid, dim3(256), 0, s, reinterpret_cast<const float2 *>(vis),
                       rp, scale);
    return hipGetLastError();
}

} // namespace bsg
