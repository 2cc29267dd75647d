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

__global__ __launch_bounds__(256) void k_round(const float2 *__restrict__ vin,
                                               float2 *__restrict__ vout, RoundParams rp,
                                               int64_t n_complex)
{
    const int64_t e0 = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) * kComplexPerThread;
    if (e0 >= n_complex) return;
    int64_t row = e0 / rp.T;
    int64_t t = e0 - row * rp.T;
    int64_t fr = row / rp.P;
    int64_t p = row - fr * rp.P;
    int32_t i, j;
    product_pair(rp, p, i, j);
    const int64_t cnt = n_complex - e0 < kComplexPerThread ? n_complex - e0 : kComplexPerThread;
    for (int k = 0; k < cnt; ++k) {
        const int64_t e = e0 + k;
        const float2 v = vin[e];
        const float ai = rp.autos[(fr * rp.I + i) * rp.T + t];
        const float aj = rp.autos[(fr * rp.I + j) * rp.T + t];
        vout[e] = round_complex(v, ai, aj, i == j, rp);
        if (++t == rp.T) {
            t = 0;
            if (++p == rp.P) {
                p = 0;
                ++fr;
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
    const int64_t threads = (n_complex + kComplexPerThread - 1) / kComplexPerThread;
    const int64_t blocks = (threads + 255) / 256;
    hipLaunchKernelGGL(k_round, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<const float2 *>(vin), reinterpret_cast<float2 *>(vout),
                       rp, n_complex);
    return hipGetLastError();
}

} // namespace bsg
