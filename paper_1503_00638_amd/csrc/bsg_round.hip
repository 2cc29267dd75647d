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
// The rounding is done on the float32 bit pattern with integer arithmetic
// (round-half-even on the magnitude bits), the exponent k of g is read off
// the bits of the double G2: no log, sqrt or division.
#include "bsg_internal.hpp"
#include "bsg_round_dev.hpp"

namespace bsg {

namespace {

constexpr int kComplexPerThread = 8;

// A wavefront rounds 512 consecutive visibilities; lane l takes elements
// l, l + 64, ..., l + 448 of them, so every load and store instruction of the
// wave touches 512 contiguous bytes.  The position (time, product, inputs,
// auto rows) is found once per lane and then stepped.
__global__ __launch_bounds__(256) void k_round(const float2 *__restrict__ vin,
                                               float2 *__restrict__ vout, RoundParams rp,
                                               int64_t n_complex)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    int64_t e = wave * (kWave * kComplexPerThread) + lane;
    if (e >= n_complex) return;
    VisCursor c = cursor_at(rp, e);
    for (int k = 0;;) {
        vout[e] = round_at(vin[e], c, rp);
        e += kWave;
        if (++k == kComplexPerThread || e >= n_complex) break;
        cursor_advance(rp, c, kWave);
    }
}

// The same walk over integer visibilities (int32 re, im).
__global__ __launch_bounds__(256) void k_round_i32(const int2 *__restrict__ vin,
                                                   int2 *__restrict__ vout, RoundParams rp,
                                                   int64_t n_complex)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    int64_t e = wave * (kWave * kComplexPerThread) + lane;
    if (e >= n_complex) return;
    VisCursor c = cursor_at(rp, e);
    for (int k = 0;;) {
        vout[e] = round_at_i32(vin[e], c, rp);
        e += kWave;
        if (++k == kComplexPerThread || e >= n_complex) break;
        cursor_advance(rp, c, kWave);
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

} // namespace

hipError_t launch_round(const float *vin, float *vout, const RoundParams &rp, hipStream_t s)
{
    const int64_t n_complex = rp.F * rp.P * rp.T;
    if (n_complex == 0) return hipSuccess;
    const int64_t waves = (n_complex + kWave * kComplexPerThread - 1) / (kWave * kComplexPerThread);
    const int64_t blocks = (waves * kWave + 255) / 256;
    hipLaunchKernelGGL(k_round, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<const float2 *>(vin), reinterpret_cast<float2 *>(vout),
                       rp, n_complex);
    return hipGetLastError();
}

hipError_t launch_round_i32(const int32_t *vin, int32_t *vout, const RoundParams &rp, hipStream_t s)
{
    const int64_t n_complex = rp.F * rp.P * rp.T;
    if (n_complex == 0) return hipSuccess;
    const int64_t waves = (n_complex + kWave * kComplexPerThread - 1) / (kWave * kComplexPerThread);
    const int64_t blocks = (waves * kWave + 255) / 256;
    hipLaunchKernelGGL(k_round_i32, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<const int2 *>(vin), reinterpret_cast<int2 *>(vout), rp,
                       n_complex);
    return hipGetLastError();
}

hipError_t launch_noise_comp(const float *vis, const RoundParams &rp, double *scale, hipStream_t s)
{
    if (rp.F * rp.T == 0) return hipSuccess;
    const dim3 grid((unsigned)rp.F, (unsigned)((rp.T + kWave - 1) / kWave));
    hipLaunchKernelGGL(k_noise_comp, grid, dim3(256), 0, s, reinterpret_cast<const float2 *>(vis),
                       rp, scale);
    return hipGetLastError();
}

} // namespace bsg
