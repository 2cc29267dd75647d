/* Drives every oracle entry point, on valid inputs and on the error paths,
 * so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * checks the oracle's memory accesses and integer arithmetic.  Exits 0 when
 * every round trip holds and every bad input is refused; the sanitizers
 * abort on any invalid access or undefined operation. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void)
{ /* xorshift64* */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return rng_state * 0x2545F4914F6CDD1Dull;
}
static double uniform(void) { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }
static double gauss(void)
{
    double u = uniform(), v = uniform();
    if (u < 1e-300) u = 1e-300;
    return sqrt(-2.0 * log(u)) * cos(6.283185307179586 * v);
}

#define CHECK(c)                                                                \
    do {                                                                        \
        if (!(c)) {                                                             \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);    \
            exit(1);                                                            \
        }                                                                       \
    } while (0)

static void fill_bytes(uint8_t *p, int64_t n, int kind)
{
    for (int64_t i = 0; i < n; i++) {
        switch (kind) {
        case 0: p[i] = (uint8_t)next_u64(); break;                 /* random */
        case 1: p[i] = (uint8_t)(next_u64() % 3); break;           /* low entropy */
        case 2: p[i] = (uint8_t)((i / 7) * 13); break;             /* structured */
        default: p[i] = (uint8_t)(i % 251 == 0 ? next_u64() : 0); /* mostly zero */
        }
    }
}

static void streams(void)
{
    static const int64_t es[] = {1, 2, 3, 4, 8, 16};
    static const int64_t bs[] = {0, 8, 64, 2048};
    for (int t = 0; t < 60; t++) {
        const int64_t E = es[t % 6], B = bs[(t / 6) % 4];
        const int64_t n = (int64_t)(next_u64() % 9000);
        const int kind = t % 4;
        uint8_t *x = malloc((size_t)(n * E) + 1), *y = malloc((size_t)(n * E) + 1);
        fill_bytes(x, n * E, kind);
        /* transposes */
        CHECK(oracle_bitshuffle(x, y, n, E, B, 1) == 0);
        uint8_t *z = malloc((size_t)(n * E) + 1);
        CHECK(oracle_bitunshuffle(y, z, n, E, B, 4) == 0);
        CHECK(memcmp(x, z, (size_t)(n * E)) == 0);
        CHECK(oracle_byteshuffle(x, y, n, E, B, 1) == 0);
        CHECK(oracle_byteunshuffle(y, z, n, E, B, 1) == 0);
        CHECK(memcmp(x, z, (size_t)(n * E)) == 0);
        /* stream round trip, both filters */
        for (int filter = 0; filter < 2; filter++) {
            const int64_t cap = oracle_compress_bound(n, E, B);
            CHECK(cap > 0);
            uint8_t *s = malloc((size_t)cap);
            const int64_t m = oracle_compress_filter(x, s, n, E, B, filter, cap, 1 + t % 3);
            CHECK(m > 0 && m <= cap);
            memset(z, 0xA5, (size_t)(n * E) + 1);
            CHECK(oracle_decompress_filter(s, m, z, n, E, B, filter, 2) == 0);
            CHECK(memcmp(x, z, (size_t)(n * E)) == 0);
            /* too little room is refused */
            if (m > 24)
                CHECK(oracle_compress_filter(x, s, n, E, B, filter, m - 1, 1) == -2);
            /* corrupt streams: flipped bytes, truncation, trailing bytes */
            for (int k = 0; k < 20 && m > 0; k++) {
                uint8_t *c = malloc((size_t)m + 8);
                memcpy(c, s, (size_t)m);
                const int64_t at = (int64_t)(next_u64() % (uint64_t)m);
                c[at] ^= (uint8_t)(1 + next_u64() % 255);
                (void)oracle_decompress_filter(c, m, z, n, E, B, filter, 1);
                CHECK(oracle_decompress_filter(c, m - 1 - at % (m > 1 ? m - 1 : 1), z, n, E, B,
                                               filter, 1) != 0 || n == 0);
                memcpy(c, s, (size_t)m);
                c[m] = 0;
                CHECK(oracle_decompress_filter(c, m + 1, z, n, E, B, filter, 1) == -3);
                free(c);
            }
            free(s);
        }
        free(x);
        free(y);
        free(z);
    }
    /* single blocks: every block length, a decoder fed random bytes */
    uint8_t blk[700], out[2000], dec[700];
    for (int n = 0; n <= 700; n += 7) {
        fill_bytes(blk, n, n % 4);
        const int64_t m = oracle_lz4_compress_block(blk, n, out, sizeof out);
        CHECK(m > 0);
        CHECK(oracle_lz4_decompress_block(out, m, dec, n) == n);
        CHECK(memcmp(blk, dec, (size_t)n) == 0);
        CHECK(oracle_lz4_compress_block(blk, n, out, m - 1) == -2);
    }
    for (int k = 0; k < 2000; k++) {
        const int64_t m = 1 + (int64_t)(next_u64() % 64);
        fill_bytes(out, m, k % 4);
        (void)oracle_lz4_decompress_block(out, m, dec, (int64_t)(next_u64() % 700));
    }
    /* bad arguments */
    CHECK(oracle_compress_bound(10, 0, 0) < 0);
    CHECK(oracle_compress_bound(10, 4, 12) < 0);
    CHECK(oracle_bitshuffle(blk, out, -1, 4, 0, 1) != 0);
}

static void rounding(void)
{
    const int64_t F = 3, I = 5, T = 9, P = I * (I + 1) / 2;
    float *vis = malloc(sizeof(float) * 2 * F * P * T), *out = malloc(sizeof(float) * 2 * F * P * T);
    float *autos = malloc(sizeof(float) * F * I * T);
    int32_t *vi = malloc(sizeof(int32_t) * 2 * F * P * T), *vo = malloc(sizeof(int32_t) * 2 * F * P * T);
    int32_t *ai = malloc(sizeof(int32_t) * F * I * T);
    double *scale = malloc(sizeof(double) * F * T);
    double *qdiag = malloc(sizeof(double) * F * T * I * I);
    int32_t pm[2 * 15];
    for (int64_t k = 0, i = 0; i < I; i++)
        for (int64_t j = i; j < I; j++, k++) {
            pm[2 * k] = (int32_t)j; /* a permuted but valid map */
            pm[2 * k + 1] = (int32_t)i;
        }
    for (int rep = 0; rep < 20; rep++) {
        for (int64_t k = 0; k < F * I * T; k++) {
            autos[k] = (float)(1000.0 * (1.0 + 0.2 * gauss()));
            ai[k] = (int32_t)(autos[k] * 64);
        }
        if (rep % 5 == 1) autos[3] = 0.0f;
        if (rep % 5 == 2) autos[4] = NAN;
        if (rep % 5 == 3) autos[5] = -5.0f;
        for (int64_t k = 0; k < 2 * F * P * T; k++) {
            vis[k] = (float)(gauss() * (rep % 2 ? 1e-3 : 30.0));
            vi[k] = (int32_t)(gauss() * 4096);
        }
        if (rep == 7) {
            vis[0] = INFINITY;
            vis[1] = -0.0f;
            vis[2] = NAN;
            vis[3] = 3.4e38f;
            vi[0] = INT32_MAX;
            vi[1] = INT32_MIN;
        }
        const double f = rep % 4 == 0 ? 0.0 : pow(10.0, -1 - rep % 4);
        CHECK(oracle_round_to_noise(vis, out, autos, F, I, T, NULL, 3.9e6, f, 1 + rep % 3) == 0);
        CHECK(oracle_round_to_noise(vis, out, autos, F, I, T, pm, 3.9e6, f, 2) == 0);
        CHECK(oracle_round_to_noise_i32(vi, vo, ai, F, I, T, rep % 2 ? pm : NULL, 3.9e6, f, 2) == 0);
        CHECK(oracle_noise_compensation(vis, autos, F, I, T, NULL, scale) == 0);
        CHECK(oracle_round_to_noise_scaled(vis, out, autos, F, I, T, NULL, 3.9e6, f, scale, 2) == 0);
        CHECK(oracle_fullcov_inverse_diag(vis, autos, F, I, T, qdiag) == 0);
        CHECK(oracle_round_to_noise_fullcov(vis, out, autos, F, I, T, 3.9e6, f) == 0);
        memcpy(out, vis, sizeof(float) * 2 * F * P * T); /* in place */
        CHECK(oracle_round_to_noise(out, out, autos, F, I, T, NULL, 3.9e6, f, 1) == 0);
    }
    for (int k = -160; k <= 160; k += 3) {
        (void)oracle_round_to_multiple((float)gauss() * 1e20f, k);
        (void)oracle_round_int_to_multiple((int32_t)next_u64(), k < 0 ? -k / 5 : k / 5);
    }
    for (int k = 0; k < 200; k++) (void)oracle_granularity_exponent(ldexp(uniform() + 0.5, (int)(next_u64() % 400) - 200));
    CHECK(oracle_round_to_noise(vis, out, autos, F, I, T, NULL, 0.0, 0.01, 1) != 0);
    CHECK(oracle_round_to_noise(vis, out, autos, F, I, T, NULL, 3.9e6, -1.0, 1) != 0);
    free(vis); free(out); free(autos); free(vi); free(vo); free(ai); free(scale); free(qdiag);
}

int main(void)
{
    streams();
    rounding();
    printf("oracle sanitizer driver ok\n");
    return 0;
}
