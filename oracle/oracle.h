/*
 * CPU oracle for the two-stage radio-data compression scheme of
 * Masui et al., "A compression scheme for radio data in high performance
 * computing" (arXiv:1503.00638).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * statement of what the GPU path must compute.  It shares no code, header,
 * table or helper with the GPU library.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the product path
 * never does.
 *
 * All buffers are host memory owned by the caller.  Return codes:
 *   0 (or a byte count >= 0)  success
 *  -1  invalid argument
 *  -2  output capacity too small
 *  -3  corrupt or inconsistent compressed stream
 */
#ifndef BSHUF_ORACLE_H
#define BSHUF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Section 3.1 (diagonal radiometer equation) and 3.2 (rounding granularity,
 * Eq. trunc_error; ties-to-even footnote).  vis is complex64 laid out as
 * float pairs [F][P][T][2]; autos float32 [F][I][T]; P = I(I+1)/2 with the
 * products in upper-triangle row-major order unless prod_map ([P][2] int32
 * (i, j) pairs) is given.  vis_out may equal vis_in.  nthreads <= 0 means
 * the OpenMP default. */
int oracle_round_to_noise(const float *vis_in, float *vis_out, const float *autos,
                          int64_t F, int64_t I, int64_t T, const int32_t *prod_map,
                          double n_samples, double f, int nthreads);

/* The granularity exponent: largest integer k with 4^k < G2 (G2 > 0, finite). */
int oracle_granularity_exponent(double G2);

/* Round one float to the nearest multiple of 2^k, ties to the even multiple. */
float oracle_round_to_multiple(float x, int k);

/* Section 3.2, compensation of the diagonal noise model: scale[F][T]
 * (double) = per (frequency, time) the minimum over cross products of
 * 1 - |V_ij|^2 / (V_ii V_jj), computed in double in that order; products
 * with V_ii V_jj not positive and finite are skipped; 1 when none is left. */
int oracle_noise_compensation(const float *vis, const float *autos, int64_t F, int64_t I,
                              int64_t T, const int32_t *prod_map, double *scale);
/* oracle_round_to_noise with G2 multiplied by scale[f][t] last. */
int oracle_round_to_noise_scaled(const float *vis_in, float *vis_out, const float *autos,
                                 int64_t F, int64_t I, int64_t T, const int32_t *prod_map,
                                 double n_samples, double f, const double *scale, int nthreads);

/* Full-covariance noise for small arrays (Section 3.1, Eqs. rad_full1-3,
 * Eq. noise; I <= 64).  Per (frequency, time), the I^2 real degrees of
 * freedom in product order (Re of each product, then Im if it is a cross
 * product); qdiag[F][T][I^2] receives (Q^-1)_kk with Q = 2N C from a
 * Cholesky factor and its inverse, every sum in increasing index order, or
 * NaN for the whole sample when Q is not positive definite. */
int oracle_fullcov_inverse_diag(const float *vis, const float *autos, int64_t F, int64_t I,
                                int64_t T, double *qdiag);
/* Rounding with G2 = c / (Q^-1)_kk for each degree of freedom (c =
 * (12 f) / (2N)); a sample without a valid estimate is left unchanged; Im
 * of autos is copied.  Default product order only. */
int oracle_round_to_noise_fullcov(const float *vis_in, float *vis_out, const float *autos,
                                  int64_t F, int64_t I, int64_t T, double n_samples, double f);

/* Integer visibilities (Section 5 data type): int32 [F][P][T][2] and int32
 * autos [F][I][T]; G2 from the exact int64 product rounded once to double;
 * rounding to a multiple of 2^k only for k >= 1, ties to even in integer
 * arithmetic, a result above INT32_MAX saturating to the largest multiple
 * that fits. */
int32_t oracle_round_int_to_multiple(int32_t x, int k);
int oracle_round_to_noise_i32(const int32_t *vis_in, int32_t *vis_out, const int32_t *autos,
                              int64_t F, int64_t I, int64_t T, const int32_t *prod_map,
                              double n_samples, double f, int nthreads);

/* Section 4.2: bit transpose of each block of block_size elements (a multiple
 * of 8; 0 = 8192 bytes' worth); the last partial block keeps floor(rem/8)*8
 * elements and the final n mod 8 elements are copied verbatim. */
int oracle_bitshuffle(const uint8_t *in, uint8_t *out, int64_t n, int64_t elem_size,
                      int64_t block_size, int nthreads);
int oracle_bitunshuffle(const uint8_t *in, uint8_t *out, int64_t n, int64_t elem_size,
                        int64_t block_size, int nthreads);

/* One LZ4 block with the fixed greedy rule: 9-bit multiplicative hash of
 * 4 bytes, candidate = the last earlier position with that hash in an
 * earlier 64-position chunk, forward extension only (the last 5 bytes stay
 * literal), a match taken when it covers at least 12 bytes and starts at
 * p <= n - 12.  Returns the compressed size, or -2 when cap is too small. */
int64_t oracle_lz4_compress_block(const uint8_t *src, int64_t n, uint8_t *dst, int64_t cap);

/* General safe LZ4 block decoder: returns n_out when src decodes to exactly
 * n_out bytes, -3 otherwise. */
int64_t oracle_lz4_decompress_block(const uint8_t *src, int64_t n_in, uint8_t *dst,
                                    int64_t n_out);

/* Blocked stream (header, offsets, LZ4 payloads, raw tail). */
int64_t oracle_block_elems(int64_t elem_size, int64_t block_size);
int64_t oracle_compress_bound(int64_t n, int64_t elem_size, int64_t block_size);
int64_t oracle_compress(const uint8_t *in, uint8_t *out, int64_t n, int64_t elem_size,
                        int64_t block_size, int64_t cap, int nthreads);
int64_t oracle_decompress(const uint8_t *in, int64_t in_nbytes, uint8_t *out, int64_t n,
                          int64_t elem_size, int64_t block_size, int nthreads);

/* The comparison filter (Section 4.1, Table t:performance): Blosc-style
 * byte shuffle within the same blocks (byte k of element i -> k * nb + i),
 * and streams whose blocks are byte-shuffled (filter 1, magic "BSB1")
 * instead of bit-transposed (filter 0, identical to oracle_compress). */
int oracle_byteshuffle(const uint8_t *in, uint8_t *out, int64_t n, int64_t elem_size,
                       int64_t block_size, int nthreads);
int oracle_byteunshuffle(const uint8_t *in, uint8_t *out, int64_t n, int64_t elem_size,
                         int64_t block_size, int nthreads);
int64_t oracle_compress_filter(const uint8_t *in, uint8_t *out, int64_t n, int64_t elem_size,
                               int64_t block_size, int filter, int64_t cap, int nthreads);
int64_t oracle_decompress_filter(const uint8_t *in, int64_t in_nbytes, uint8_t *out, int64_t n,
                                 int64_t elem_size, int64_t block_size, int filter, int nthreads);

int oracle_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
