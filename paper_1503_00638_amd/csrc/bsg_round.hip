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

constexpr int kComplexPerThread = 4;

// A wavefront rounds 256 consecutive visibilities; lane l takes elements
// l, l + 64, l + 128, l + 192 of them, so every load and store instruction
// of the wave touches 512 contiguous bytes.
__global__ __launch_bounds__(256) void k_round(const float2 *__restrict__ vin,
                                               float2 *__restrict__ vout, RoundParams rp,
                                               int64_t n_complex)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    int64_t e = wave * (kWave * kComplexPerThread) + lane;
    if (e >= n_complex) return;
    int64_t row = e / rp.T;
    int64_t t = e - row * rp.T;
    int64_t fr = row / rp.P;
    int64_t p = row - fr * rp.P;
    int32_t i, j;
    product_pair(rp, p, i, j);
    for (int k = 0; k < kComplexPerThread && e < n_complex; ++k) {
        const float2 v = vin[e];
        const float ai = rp.autos[(fr * rp.I + i) * rp.T + t];
        const float aj = rp.autos[(fr * rp.I + j) * rp.T + t];
        vout[e] = round_complex(v, ai, aj, i == j, rp);
        // advance by one wave width (64 visibilities)
        e += kWave;
        t += kWave;
        if (t >= rp.T) {
            while (t >= rp.T) {
                t -= rp.T;
                if (++p == rp.P) {
                    p = 0;
                    ++fr;
                }
            }
            product_pair(rp, p, i, j);
        }
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

} // namespace bsg
