/*
 * CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Masui et al., arXiv:1503.00638.  Every function below is the plain
 * definition of one step of the scheme, written for a reader to check
 * against the paper by eye: no blocking, fusion or reordering beyond what
 * the definition states.  Floating point is IEEE double with the default
 * round-to-nearest-even mode; build without -ffast-math and with
 * -ffp-contract=off.  OpenMP only distributes independent rows / blocks
 * over threads, which is the paper's own threading model (Section 4.2,
 * "Implementation": blocks are distributed among threads).
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ---- constants of the stream format and of the fixed LZ4 match rule ---- */
#define STREAM_MAGIC 0x31475342u /* bytes "BSG1" */
#define STREAM_MAGIC_BYTE 0x31425342u /* bytes "BSB1": byte-shuffled blocks */
#define HEADER_BYTES 24
#define DEFAULT_BLOCK_BYTES 8192
#define MAX_BLOCK_BYTES 65536 /* LZ4 offsets are 16-bit */
#define HASH_BITS 9
#define HASH_MULT 2654435761u /* Knuth's multiplicative constant */
#define CHUNK 64             /* candidate table is updated every 64 positions */
#define MINMATCH 4       /* LZ4 format: match lengths are coded as length - 4 */
#define MINTAKE 12       /* the rule only takes matches of at least 12 bytes */
#define MFLIMIT 12       /* a match may start only at p <= n - 12 */
#define LASTLITERALS 5   /* the last 5 bytes of a block are literals */

int oracle_max_threads(void) { return omp_get_max_threads(); }

static int pick_threads(int nthreads) { return nthreads > 0 ? nthreads : omp_get_max_threads(); }

/* ======================================================================
 * Stage 1: noise-relative precision reduction (Section 3)
 * ====================================================================== */

/* Eq. trunc_error: g < sqrt(12 f s^2), g a power of two.  With
 * G2 = 12 f s^2 this is g^2 < G2, i.e. the largest k with 4^k < G2
 * (strict).  frexp gives G2 < 2^e, so any k with 2k >= e fails the test
 * and is a safe starting point; the loop then walks down to the first k
 * that satisfies it (at most a few steps). */
int oracle_granularity_exponent(double G2)
{
    int e;
    (void)frexp(G2, &e);
    int k = e / 2 + 1; /* 2k >= e + 1 > e */
    while (ldexp(1.0, 2 * k) >= G2)
        k--;
    return k;
}

/* Round to the nearest multiple of g = 2^k, ties to the even multiple
 * (Section 3.2, tie-breaking footnote: IEEE round-half-even, unbiased).
 * Evaluated in double: x * 2^-k is exact for the k range kept here, rint
 * rounds half to even in the default mode, and the result is a float
 * value (or overflows to +-inf, the IEEE outcome). */
float oracle_round_to_multiple(float x, int k)
{
    if (isnan(x) || isinf(x))
        return x;
    if (k < -149) /* every float is already a multiple of 2^-149 */
        return x;
    if (k > 200) /* |x| < 2^128 <= g/2: nearest multiple is zero */
        return copysignf(0.0f, x);
    double r = rint(ldexp((double)x, -k));
    return (float)ldexp(r, k);
}

static float round_to_noise_1(float x, double G2)
{
    /* No positive finite noise estimate (f = 0, a dead or negative auto,
     * NaN): nothing is discarded. */
    if (!(G2 > 0.0) || isinf(G2))
        return x;
    return oracle_round_to_multiple(x, oracle_granularity_exponent(G2));
}

int oracle_round_to_noise(const float *vis_in, float *vis_out, const float *autos,
                          int64_t F, int64_t I, int64_t T, const int32_t *prod_map,
                          double n_samples, double f, int nthreads)
{
    if (F < 0 || I < 0 || T < 0)
        return -1;
    if (!(n_samples > 0.0) || isinf(n_samples) || !(f >= 0.0) || isinf(f))
        return -1;
    const int64_t P = I * (I + 1) / 2;
    if (F * P * T > 0 && (!vis_in || !vis_out || !autos))
        return -1;
    int32_t *pairs = (int32_t *)malloc((size_t)(P > 0 ? P : 1) * 2 * sizeof(int32_t));
    if (!pairs)
        return -1;
    if (prod_map) {
        for (int64_t p = 0; p < P; p++) {
            if (prod_map[2 * p] < 0 || prod_map[2 * p] >= I || prod_map[2 * p + 1] < 0 ||
                prod_map[2 * p + 1] >= I) {
                free(pairs);
                return -1;
            }
            pairs[2 * p] = prod_map[2 * p];
            pairs[2 * p + 1] = prod_map[2 * p + 1];
        }
    } else {
        /* upper triangle, row major: (0,0) (0,1) ... (0,I-1) (1,1) ... */
        int64_t p = 0;
        for (int64_t i = 0; i < I; i++)
            for (int64_t j = i; j < I; j++) {
                pairs[2 * p] = (int32_t)i;
                pairs[2 * p + 1] = (int32_t)j;
                p++;
            }
    }

    /* Section 3.1 diagonal radiometer equation, with G2 = 12 f s^2:
     *   i != j:  s^2 = V_ii V_jj / (2N)  ->  G2 = (V_ii V_jj) * c
     *   i == j:  s^2 = V_ii^2 / N        ->  G2 = (V_ii V_ii) * (2c)
     * and the imaginary part of an auto carries no noise and is left alone.
     * The product of two floats is exact in double; only "* c" rounds. */
    const double c = (12.0 * f) / (2.0 * n_samples);
    const double c_auto = 2.0 * c;

    const int64_t rows = F * P;
#pragma omp parallel for num_threads(pick_threads(nthreads)) schedule(static)
    for (int64_t row = 0; row < rows; row++) {
        const int64_t fr = row / P, p = row % P;
        const int64_t i = pairs[2 * p], j = pairs[2 * p + 1];
        const float *Ai = autos + (fr * I + i) * T;
        const float *Aj = autos + (fr * I + j) * T;
        for (int64_t t = 0; t < T; t++) {
            const int64_t e = 2 * (row * T + t);
            const float re = vis_in[e], im = vis_in[e + 1];
            if (i != j) {
                const double G2 = ((double)Ai[t] * (double)Aj[t]) * c;
                vis_out[e] = round_to_noise_1(re, G2);
                vis_out[e + 1] = round_to_noise_1(im, G2);
            } else {
                const double G2 = ((double)Ai[t] * (double)Ai[t]) * c_auto;
                vis_out[e] = round_to_noise_1(re, G2);
                vis_out[e + 1] = im;
            }
        }
    }
    free(pairs);
    return 0;
}

/* ----------------------------------------------------------------------
 * Compensation of the diagonal noise model (Section 3.2): the diagonal
 * radiometer equation neglects the correlation between products; multiplying
 * f by the minimum over cross products of 1 - |V_ij|^2 / (V_ii V_jj) roughly
 * makes up for it.  The paper suggests doing so per frequency and time; here
 * scale[f][t] is that minimum (1 when no cross product has V_ii V_jj > 0).
 * ---------------------------------------------------------------------- */
static int make_pairs(int64_t I, const int32_t *prod_map, int32_t **out)
{
    const int64_t P = I * (I + 1) / 2;
    int32_t *pairs = (int32_t *)malloc((size_t)(P > 0 ? P : 1) * 2 * sizeof(int32_t));
    if (!pairs)
        return -1;
    if (prod_map) {
        for (int64_t p = 0; p < P; p++) {
            if (prod_map[2 * p] < 0 || prod_map[2 * p] >= I || prod_map[2 * p + 1] < 0 ||
                prod_map[2 * p + 1] >= I) {
                free(pairs);
                return -1;
            }
            pairs[2 * p] = prod_map[2 * p];
            pairs[2 * p + 1] = prod_map[2 * p + 1];
        }
    } else {
        int64_t p = 0;
        for (int64_t i = 0; i < I; i++)
            for (int64_t j = i; j < I; j++) {
                pairs[2 * p] = (int32_t)i;
                pairs[2 * p + 1] = (int32_t)j;
                p++;
            }
    }
    *out = pairs;
    return 0;
}

int oracle_noise_compensation(const float *vis, const float *autos, int64_t F, int64_t I,
                              int64_t T, const int32_t *prod_map, double *scale)
{
    if (F < 0 || I < 0 || T < 0)
        return -1;
    const int64_t P = I * (I + 1) / 2;
    if (F * T > 0 && !scale)
        return -1;
    if (F * P * T > 0 && (!vis || !autos))
        return -1;
    int32_t *pairs;
    if (make_pairs(I, prod_map, &pairs))
        return -1;
    for (int64_t fr = 0; fr < F; fr++)
        for (int64_t t = 0; t < T; t++) {
            double m = 1.0;
            for (int64_t p = 0; p < P; p++) {
                const int64_t i = pairs[2 * p], j = pairs[2 * p + 1];
                if (i == j)
                    continue;
                const double a = autos[(fr * I + i) * T + t], b = autos[(fr * I + j) * T + t];
                const double ab = a * b;
                if (!(ab > 0.0) || isinf(ab))
                    continue;
                const int64_t e = 2 * ((fr * P + p) * T + t);
                const double re = vis[e], im = vis[e + 1];
                const double term = 1.0 - (re * re + im * im) / ab;
                if (term < m) /* a NaN term never wins */
                    m = term;
            }
            scale[fr * T + t] = m;
        }
    free(pairs);
    return 0;
}

/* oracle_round_to_noise with G2 multiplied by scale[f][t] (the compensation
 * factor, or any per-sample factor on f): G2 = ((V_ii V_jj) c) scale for
 * crosses and ((V_ii V_ii) 2c) scale for autos. */
int oracle_round_to_noise_scaled(const float *vis_in, float *vis_out, const float *autos,
                                 int64_t F, int64_t I, int64_t T, const int32_t *prod_map,
                                 double n_samples, double f, const double *scale, int nthreads)
{
    if (F < 0 || I < 0 || T < 0)
        return -1;
    if (!(n_samples > 0.0) || isinf(n_samples) || !(f >= 0.0) || isinf(f))
        return -1;
    const int64_t P = I * (I + 1) / 2;
    if (F * P * T > 0 && (!vis_in || !vis_out || !autos || !scale))
        return -1;
    int32_t *pairs;
    if (make_pairs(I, prod_map, &pairs))
        return -1;
    const double c = (12.0 * f) / (2.0 * n_samples);
    const double c_auto = 2.0 * c;
    const int64_t rows = F * P;
#pragma omp parallel for num_threads(pick_threads(nthreads)) schedule(static)
    for (int64_t row = 0; row < rows; row++) {
        const int64_t fr = row / P, p = row % P;
        const int64_t i = pairs[2 * p], j = pairs[2 * p + 1];
        const float *Ai = autos + (fr * I + i) * T;
        const float *Aj = autos + (fr * I + j) * T;
        for (int64_t t = 0; t < T; t++) {
            const int64_t e = 2 * (row * T + t);
            const double sc = scale[fr * T + t];
            if (i != j) {
                const double G2 = (((double)Ai[t] * (double)Aj[t]) * c) * sc;
                vis_out[e] = round_to_noise_1(vis_in[e], G2);
                vis_out[e + 1] = round_to_noise_1(vis_in[e + 1], G2);
            } else {
                const double G2 = (((double)Ai[t] * (double)Ai[t]) * c_auto) * sc;
                vis_out[e] = round_to_noise_1(vis_in[e], G2);
                vis_out[e + 1] = vis_in[e + 1];
            }
        }
    }
    free(pairs);
    return 0;
}

/* ----------------------------------------------------------------------
 * Full-covariance noise for small arrays (Section 3.1, Eqs. rad_full1-3 and
 * Eq. noise).  Per (frequency, time) the real degrees of freedom are, in
 * product order, Re of every product and Im of every cross product (the Im
 * of an auto is identically zero and carries no noise): D = I^2 of them.
 * With V_ab = conj(V_ba) and V_aa = the measured auto, 2N times the
 * covariance between (x, ij) and (y, gh) is
 *   Re Re:  Re[V_ig conj(V_jh) + V_ih conj(V_jg)]
 *   Im Im:  Re[V_ig conj(V_jh) - V_ih conj(V_jg)]
 *   Re Im:  Im[-V_ig conj(V_jh) + V_ih conj(V_jg)]     (Im Re by symmetry)
 * and the noise of a degree of freedom k is s_k^2 = 1 / (C^-1)_kk, the
 * variance not marginalised over the others.  With Q = 2N C,
 * G2 = 12 f s_k^2 = c / (Q^-1)_kk, c = (12 f) / (2N) as in the diagonal case.
 * (Q^-1)_kk comes from the Cholesky factor Q = L L^T and M = L^-1:
 * (Q^-1)_kk = sum over i >= k of M_ik^2.  Every sum runs in increasing
 * index order.  A (frequency, time) whose Q is not positive definite (a
 * pivot not > 0, NaN data) is left unchanged.
 * ---------------------------------------------------------------------- */
typedef struct {
    double re, im;
} cplx;

static cplx cmul_conj(cplx a, cplx b) /* a * conj(b) */
{
    cplx r = {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
    return r;
}

int oracle_fullcov_inverse_diag(const float *vis, const float *autos, int64_t F, int64_t I,
                                int64_t T, double *qdiag)
{
    if (F < 0 || I < 0 || T < 0 || I > 64)
        return -1;
    const int64_t P = I * (I + 1) / 2, D = I * I;
    if (F * T * D > 0 && (!vis || !autos || !qdiag))
        return -1;
    /* degree of freedom k -> (product p, 0 = Re / 1 = Im), and product -> (i, j) */
    int64_t *dof_p = (int64_t *)malloc((size_t)(D > 0 ? D : 1) * sizeof(int64_t));
    int *dof_im = (int *)malloc((size_t)(D > 0 ? D : 1) * sizeof(int));
    int64_t *pi = (int64_t *)malloc((size_t)(P > 0 ? P : 1) * sizeof(int64_t));
    int64_t *pj = (int64_t *)malloc((size_t)(P > 0 ? P : 1) * sizeof(int64_t));
    int64_t *pidx = (int64_t *)malloc((size_t)(I > 0 ? I * I : 1) * sizeof(int64_t));
    double *Q = (double *)malloc((size_t)(D > 0 ? D * D : 1) * sizeof(double));
    double *M = (double *)malloc((size_t)(D > 0 ? D * D : 1) * sizeof(double));
    cplx *V = (cplx *)malloc((size_t)(I > 0 ? I * I : 1) * sizeof(cplx));
    if (!dof_p || !dof_im || !pi || !pj || !pidx || !Q || !M || !V) {
        free(dof_p); free(dof_im); free(pi); free(pj); free(pidx); free(Q); free(M); free(V);
        return -1;
    }
    {
        int64_t p = 0, k = 0;
        for (int64_t i = 0; i < I; i++)
            for (int64_t j = i; j < I; j++) {
                pi[p] = i;
                pj[p] = j;
                pidx[i * I + j] = p;
                p++;
            }
        for (p = 0; p < P; p++) {
            dof_p[k] = p;
            dof_im[k] = 0;
            k++;
            if (pi[p] != pj[p]) {
                dof_p[k] = p;
                dof_im[k] = 1;
                k++;
            }
        }
    }
    for (int64_t fr = 0; fr < F; fr++)
        for (int64_t t = 0; t < T; t++) {
            /* the Hermitian matrix V of this sample */
            for (int64_t a = 0; a < I; a++)
                for (int64_t b = 0; b < I; b++) {
                    cplx v;
                    if (a == b) {
                        v.re = autos[(fr * I + a) * T + t];
                        v.im = 0.0;
                    } else {
                        const int64_t lo = a < b ? a : b, hi = a < b ? b : a;
                        const int64_t e = 2 * ((fr * P + pidx[lo * I + hi]) * T + t);
                        v.re = vis[e];
                        v.im = a < b ? (double)vis[e + 1] : -(double)vis[e + 1];
                    }
                    V[a * I + b] = v;
                }
            /* Q = 2N C */
            for (int64_t x = 0; x < D; x++)
                for (int64_t y = 0; y < D; y++) {
                    const int64_t i = pi[dof_p[x]], j = pj[dof_p[x]];
                    const int64_t g = pi[dof_p[y]], h = pj[dof_p[y]];
                    const cplx A = cmul_conj(V[i * I + g], V[j * I + h]);
                    const cplx B = cmul_conj(V[i * I + h], V[j * I + g]);
                    double q;
                    if (!dof_im[x] && !dof_im[y])
                        q = A.re + B.re;
                    else if (dof_im[x] && dof_im[y])
                        q = A.re - B.re;
                    else if (!dof_im[x]) /* Re ij, Im gh */
                        q = -A.im + B.im;
                    else { /* Im ij, Re gh = Re gh, Im ij */
                        const cplx A2 = cmul_conj(V[g * I + i], V[h * I + j]);
                        const cplx B2 = cmul_conj(V[g * I + j], V[h * I + i]);
                        q = -A2.im + B2.im;
                    }
                    Q[x * D + y] = q;
                }
            /* Cholesky, right-looking: after step k the trailing block holds
             * Q_ij - sum_{m <= k} L_im L_jm, subtracted in increasing m */
            int ok = 1;
            for (int64_t k = 0; k < D && ok; k++) {
                const double d = Q[k * D + k];
                if (!(d > 0.0) || isinf(d)) {
                    ok = 0;
                    break;
                }
                const double lkk = sqrt(d);
                Q[k * D + k] = lkk;
                for (int64_t i = k + 1; i < D; i++)
                    Q[i * D + k] = Q[i * D + k] / lkk;
                for (int64_t i = k + 1; i < D; i++)
                    for (int64_t j = k + 1; j <= i; j++)
                        Q[i * D + j] = Q[i * D + j] - Q[i * D + k] * Q[j * D + k];
            }
            double *out = qdiag + (fr * T + t) * D;
            if (!ok) {
                for (int64_t k = 0; k < D; k++)
                    out[k] = NAN; /* no valid noise estimate */
                continue;
            }
            /* M = L^-1 column by column: M_jj = 1 / L_jj, and for i > j
             * M_ij = -(sum_{m=j}^{i-1} L_im M_mj) / L_ii */
            for (int64_t j = 0; j < D; j++) {
                M[j * D + j] = 1.0 / Q[j * D + j];
                for (int64_t i = j + 1; i < D; i++) {
                    double acc = Q[i * D + j] * M[j * D + j];
                    for (int64_t m = j + 1; m < i; m++)
                        acc = acc + Q[i * D + m] * M[m * D + j];
                    M[i * D + j] = -acc / Q[i * D + i];
                }
                double q = 0.0;
                for (int64_t i = j; i < D; i++)
                    q = q + M[i * D + j] * M[i * D + j];
                out[j] = q;
            }
        }
    free(dof_p); free(dof_im); free(pi); free(pj); free(pidx); free(Q); free(M); free(V);
    return 0;
}

int oracle_round_to_noise_fullcov(const float *vis_in, float *vis_out, const float *autos,
                                  int64_t F, int64_t I, int64_t T, double n_samples, double f)
{
    if (!(n_samples > 0.0) || isinf(n_samples) || !(f >= 0.0) || isinf(f))
        return -1;
    if (F < 0 || I < 0 || T < 0 || I > 64)
        return -1;
    const int64_t P = I * (I + 1) / 2, D = I * I;
    if (F * P * T == 0)
        return 0;
    if (!vis_in || !vis_out || !autos)
        return -1;
    double *qd = (double *)malloc((size_t)(F * T * D) * sizeof(double));
    if (!qd)
        return -1;
    if (oracle_fullcov_inverse_diag(vis_in, autos, F, I, T, qd)) {
        free(qd);
        return -1;
    }
    const double c = (12.0 * f) / (2.0 * n_samples);
    for (int64_t fr = 0; fr < F; fr++)
        for (int64_t t = 0; t < T; t++) {
            const double *q = qd + (fr * T + t) * D;
            int64_t k = 0;
            for (int64_t i = 0; i < I; i++)
                for (int64_t j = i; j < I; j++) {
                    const int64_t prod = (i * I - i * (i - 1) / 2) + (j - i);
                    const int64_t e = 2 * ((fr * P + prod) * T + t);
                    /* Re: G2 = c / (Q^-1)_kk; NaN (no estimate) leaves it */
                    vis_out[e] = round_to_noise_1(vis_in[e], c / q[k]);
                    k++;
                    if (i != j) {
                        vis_out[e + 1] = round_to_noise_1(vis_in[e + 1], c / q[k]);
                        k++;
                    } else {
                        vis_out[e + 1] = vis_in[e + 1];
                    }
                }
        }
    free(qd);
    return 0;
}

/* ----------------------------------------------------------------------
 * Integer visibilities (the data type of the paper's own evaluation,
 * Section 5): re and im are int32.  Every integer is already a multiple of
 * g = 1, so only k >= 1 changes anything (g <= 1 means no rounding).
 * ---------------------------------------------------------------------- */

/* Nearest multiple of 2^k to x, ties to the even multiple, in exact integer
 * arithmetic.  A result above INT32_MAX (only x near INT32_MAX rounding up)
 * becomes the largest multiple of 2^k that fits; the negative side always
 * fits because -2^31 is a multiple of every 2^k with k <= 31. */
int32_t oracle_round_int_to_multiple(int32_t x, int k)
{
    if (k <= 0)
        return x;
    if (k > 62) /* |x| <= 2^31 < g/2: the nearest multiple is zero */
        k = 62;
    const int64_t g = (int64_t)1 << k;
    int64_t q = (int64_t)x / g, rem = (int64_t)x % g; /* C truncates toward zero */
    if (rem < 0) {                                      /* make it floor division */
        q -= 1;
        rem += g;
    }
    const int64_t half = g / 2;
    if (rem > half || (rem == half && (q % 2 != 0)))
        q += 1;
    int64_t r = q * g;
    if (r > INT32_MAX)
        r = ((int64_t)INT32_MAX / g) * g;
    return (int32_t)r;
}

static int32_t round_int_to_noise_1(int32_t x, double G2)
{
    if (!(G2 > 0.0) || isinf(G2))
        return x;
    return oracle_round_int_to_multiple(x, oracle_granularity_exponent(G2));
}

/* As oracle_round_to_noise for int32 visibilities [F][P][T][2] and int32
 * autos [F][I][T].  The product V_ii V_jj is exact in int64 and is rounded
 * once to double; G2 = that * c (crosses) or * 2c (autos). */
int oracle_round_to_noise_i32(const int32_t *vis_in, int32_t *vis_out, const int32_t *autos,
                              int64_t F, int64_t I, int64_t T, const int32_t *prod_map,
                              double n_samples, double f, int nthreads)
{
    if (F < 0 || I < 0 || T < 0)
        return -1;
    if (!(n_samples > 0.0) || isinf(n_samples) || !(f >= 0.0) || isinf(f))
        return -1;
    const int64_t P = I * (I + 1) / 2;
    if (F * P * T > 0 && (!vis_in || !vis_out || !autos))
        return -1;
    int32_t *pairs = (int32_t *)malloc((size_t)(P > 0 ? P : 1) * 2 * sizeof(int32_t));
    if (!pairs)
        return -1;
    if (prod_map) {
        for (int64_t p = 0; p < P; p++) {
            if (prod_map[2 * p] < 0 || prod_map[2 * p] >= I || prod_map[2 * p + 1] < 0 ||
                prod_map[2 * p + 1] >= I) {
                free(pairs);
                return -1;
            }
            pairs[2 * p] = prod_map[2 * p];
            pairs[2 * p + 1] = prod_map[2 * p + 1];
        }
    } else {
        int64_t p = 0;
        for (int64_t i = 0; i < I; i++)
            for (int64_t j = i; j < I; j++) {
                pairs[2 * p] = (int32_t)i;
                pairs[2 * p + 1] = (int32_t)j;
                p++;
            }
    }
    const double c = (12.0 * f) / (2.0 * n_samples);
    const double c_auto = 2.0 * c;
    const int64_t rows = F * P;
#pragma omp parallel for num_threads(pick_threads(nthreads)) schedule(static)
    for (int64_t row = 0; row < rows; row++) {
        const int64_t fr = row / P, p = row % P;
        const int64_t i = pairs[2 * p], j = pairs[2 * p + 1];
        const int32_t *Ai = autos + (fr * I + i) * T;
        const int32_t *Aj = autos + (fr * I + j) * T;
        for (int64_t t = 0; t < T; t++) {
            const int64_t e = 2 * (row * T + t);
            const int32_t re = vis_in[e], im = vis_in[e + 1];
            if (i != j) {
                const double G2 = (double)((int64_t)Ai[t] * (int64_t)Aj[t]) * c;
                vis_out[e] = round_int_to_noise_1(re, G2);
                vis_out[e + 1] = round_int_to_noise_1(im, G2);
            } else {
                const double G2 = (double)((int64_t)Ai[t] * (int64_t)Ai[t]) * c_auto;
                vis_out[e] = round_int_to_noise_1(re, G2);
                vis_out[e + 1] = im;
            }
        }
    }
    free(pairs);
    return 0;
}

/* ======================================================================
 * Stage 2a: bit transpose within blocks (Section 4.2)
 * ====================================================================== */

int64_t oracle_block_elems(int64_t elem_size, int64_t block_size)
{
    if (elem_size <= 0)
        return -1;
    if (block_size == 0) {
        block_size = (DEFAULT_BLOCK_BYTES / elem_size) / 8 * 8;
        if (block_size < 8)
            block_size = 8;
    }
    if (block_size < 8 || block_size % 8 != 0)
        return -1;
    return block_size;
}

/* n elements in blocks of nb: full blocks, then one partial block of
 * floor(rem/8)*8 elements, then rem mod 8 = n mod 8 raw tail elements. */
static void block_layout(int64_t n, int64_t nb, int64_t *n_full, int64_t *last_elems,
                         int64_t *n_blocks, int64_t *tail)
{
    *n_full = n / nb;
    const int64_t rem = n - *n_full * nb;
    *last_elems = rem - rem % 8;
    *tail = rem % 8;
    *n_blocks = *n_full + (*last_elems > 0 ? 1 : 0);
}

/* The (nb x 8E) bit matrix of a block, rows = elements, columns = bit
 * significance b = 8 * (byte in element) + (bit in byte, LSB first),
 * transposed into 8E rows ("planes") of nb bits, LSB plane first, each
 * packed LSB-first into bytes (Fig. bits: bytes unpack LSB to MSB). */
static void bitshuffle_block(const uint8_t *in, uint8_t *out, int64_t nb, int64_t E)
{
    const int64_t plane_bytes = nb / 8;
    memset(out, 0, (size_t)(nb * E));
    for (int64_t i = 0; i < nb; i++)
        for (int64_t b = 0; b < 8 * E; b++) {
            const unsigned bit = (in[i * E + b / 8] >> (b % 8)) & 1u;
            out[b * plane_bytes + i / 8] |= (uint8_t)(bit << (i % 8));
        }
}

static void bitunshuffle_block(const uint8_t *in, uint8_t *out, int64_t nb, int64_t E)
{
    const int64_t plane_bytes = nb / 8;
    memset(out, 0, (size_t)(nb * E));
    for (int64_t i = 0; i < nb; i++)
        for (int64_t b = 0; b < 8 * E; b++) {
            const unsigned bit = (in[b * plane_bytes + i / 8] >> (i % 8)) & 1u;
            out[i * E + b / 8] |= (uint8_t)(bit << (b % 8));
        }
}

/* The byte shuffle of Blosc-style compressors (the comparison of Section
 * 4.1 / Table t:performance): the (nb x E) byte matrix of a block is
 * transposed, byte k of element i going to byte k * nb + i. */
static void byteshuffle_block(const uint8_t *in, uint8_t *out, int64_t nb, int64_t E)
{
    for (int64_t i = 0; i < nb; i++)
        for (int64_t k = 0; k < E; k++)
            out[k * nb + i] = in[i * E + k];
}

static void byteunshuffle_block(const uint8_t *in, uint8_t *out, int64_t nb, int64_t E)
{
    for (int64_t i = 0; i < nb; i++)
        for (int64_t k = 0; k < E; k++)
            out[i * E + k] = in[k * nb + i];
}

/* filter 0: bit transpose (the method); 1: byte shuffle (the comparison) */
static void filter_block(const uint8_t *in, uint8_t *out, int64_t nb, int64_t E, int filter,
                         int inverse)
{
    if (filter == 1) {
        if (inverse)
            byteunshuffle_block(in, out, nb, E);
        else
            byteshuffle_block(in, out, nb, E);
    } else {
        if (inverse)
            bitunshuffle_block(in, out, nb, E);
        else
            bitshuffle_block(in, out, nb, E);
    }
}

static int transpose_blocks(const uint8_t *in, uint8_t *out, int64_t n, int64_t E,
                            int64_t block_size, int nthreads, int inverse, int filter)
{
    const int64_t nb = oracle_block_elems(E, block_size);
    if (nb < 0 || n < 0)
        return -1;
    if (n > 0 && (!in || !out))
        return -1;
    int64_t n_full, last, n_blocks, tail;
    block_layout(n, nb, &n_full, &last, &n_blocks, &tail);
#pragma omp parallel for num_threads(pick_threads(nthreads)) schedule(static)
    for (int64_t blk = 0; blk < n_blocks; blk++) {
        const int64_t elems = blk < n_full ? nb : last;
        const int64_t off = blk * nb * E;
        filter_block(in + off, out + off, elems, E, filter, inverse);
    }
    if (tail)
        memcpy(out + (n - tail) * E, in + (n - tail) * E, (size_t)(tail * E));
    return 0;
}

int oracle_bitshuffle(const uint8_t *in, uint8_t *out, int64_t n, int64_t elem_size,
                      int64_t block_size, int nthreads)
{
    return transpose_blocks(in, out, n, elem_size, block_size, nthreads, 0, 0);
}

int oracle_bitunshuffle(const uint8_t *in, uint8_t *out, int64_t n, int64_t elem_size,
                        int64_t block_size, int nthreads)
{
    return transpose_blocks(in, out, n, elem_size, block_size, nthreads, 1, 0);
}

int oracle_byteshuffle(const uint8_t *in, uint8_t *out, int64_t n, int64_t elem_size,
                       int64_t block_size, int nthreads)
{
    return transpose_blocks(in, out, n, elem_size, block_size, nthreads, 0, 1);
}

int oracle_byteunshuffle(const uint8_t *in, uint8_t *out, int64_t n, int64_t elem_size,
                         int64_t block_size, int nthreads)
{
    return transpose_blocks(in, out, n, elem_size, block_size, nthreads, 1, 1);
}

/* ======================================================================
 * Stage 2b: LZ4 block compression with a fixed greedy rule (Section 4.2:
 * each bit-transposed block is LZ4-compressed on its own)
 * ====================================================================== */

static uint32_t le32(const uint8_t *p)
{
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) |
           ((uint32_t)p[3] << 24);
}

static uint32_t hash4(uint32_t v) { return (uint32_t)(v * HASH_MULT) >> (32 - HASH_BITS); }

/* LZ4 length field continuation: a run of 255s then one byte < 255. */
static int put_length_ext(uint8_t *dst, int64_t *op, int64_t cap, int64_t r)
{
    while (r >= 255) {
        if (*op >= cap)
            return -2;
        dst[(*op)++] = 255;
        r -= 255;
    }
    if (*op >= cap)
        return -2;
    dst[(*op)++] = (uint8_t)r;
    return 0;
}

static int put_literals(uint8_t *dst, int64_t *op, int64_t cap, const uint8_t *lit,
                        int64_t ll, int ml_nibble)
{
    if (*op >= cap)
        return -2;
    dst[(*op)++] = (uint8_t)(((ll < 15 ? ll : 15) << 4) | ml_nibble);
    if (ll >= 15 && put_length_ext(dst, op, cap, ll - 15))
        return -2;
    if (ll > cap - *op)
        return -2;
    memcpy(dst + *op, lit, (size_t)ll);
    *op += ll;
    return 0;
}

int64_t oracle_lz4_compress_block(const uint8_t *x, int64_t n, uint8_t *dst, int64_t cap)
{
    if (n < 0 || cap < 0 || (n > 0 && !x) || (cap > 0 && !dst) || n > MAX_BLOCK_BYTES)
        return -1;

    /* Candidates: cand(p) = the largest q <= n-4 in an earlier 64-position
     * chunk than p with the same hash, or none.  Per chunk: every position
     * first reads the table, then every position is written in increasing
     * order, so the largest q of each hash value survives. */
    const int64_t last_start = n - MFLIMIT; /* matches start at p <= n - 12 */
    int32_t *cand = (int32_t *)malloc((size_t)(last_start >= 0 ? last_start + 1 : 1) * sizeof(int32_t));
    int32_t table[1 << HASH_BITS];
    if (!cand)
        return -1;
    for (int h = 0; h < (1 << HASH_BITS); h++)
        table[h] = -1;
    for (int64_t c0 = 0; c0 <= n - 4; c0 += CHUNK) {
        const int64_t c1 = (c0 + CHUNK <= n - 3) ? c0 + CHUNK : n - 3; /* q <= n-4 */
        for (int64_t q = c0; q < c1; q++)
            if (q <= last_start)
                cand[q] = table[hash4(le32(x + q))];
        for (int64_t q = c0; q < c1; q++)
            table[hash4(le32(x + q))] = (int32_t)q;
    }

    /* Greedy parse: at p, extend the candidate forward only (no backward
     * extension, no lazy evaluation) while keeping the last 5 bytes as
     * literals; the match is taken when it covers at least 12 bytes, else p
     * moves on by one byte. */
    int64_t op = 0, anchor = 0, p = 0;
    while (p <= last_start) {
        const int64_t c = cand[p];
        int64_t L = 0;
        if (c >= 0)
            while (p + L < n - LASTLITERALS && x[c + L] == x[p + L])
                L++;
        if (L >= MINTAKE) {
            const int64_t ml4 = L - MINMATCH;
            const int64_t off = p - c;
            if (put_literals(dst, &op, cap, x + anchor, p - anchor, ml4 < 15 ? (int)ml4 : 15) ||
                cap - op < 2) {
                free(cand);
                return -2;
            }
            dst[op++] = (uint8_t)(off & 255);
            dst[op++] = (uint8_t)(off >> 8);
            if (ml4 >= 15 && put_length_ext(dst, &op, cap, ml4 - 15)) {
                free(cand);
                return -2;
            }
            p += L;
            anchor = p;
        } else {
            p++;
        }
    }
    free(cand);
    if (put_literals(dst, &op, cap, x + anchor, n - anchor, 0))
        return -2;
    return op;
}

/* Any valid LZ4 block: sequences of (token, literal length extension,
 * literals, 16-bit offset, match length extension); the last sequence is
 * literals only.  A match may overlap its own output (offset < length). */
int64_t oracle_lz4_decompress_block(const uint8_t *src, int64_t n_in, uint8_t *dst,
                                    int64_t n_out)
{
    if (n_in < 0 || n_out < 0 || (n_in > 0 && !src) || (n_out > 0 && !dst))
        return -1;
    int64_t ip = 0, op = 0;
    for (;;) {
        if (ip >= n_in)
            return -3;
        const unsigned token = src[ip++];
        int64_t ll = token >> 4;
        if (ll == 15) {
            unsigned b;
            do {
                if (ip >= n_in)
                    return -3;
                b = src[ip++];
                ll += b;
            } while (b == 255);
        }
        if (ll > n_in - ip || ll > n_out - op)
            return -3;
        memcpy(dst + op, src + ip, (size_t)ll);
        ip += ll;
        op += ll;
        if (ip == n_in)
            break;
        if (n_in - ip < 2)
            return -3;
        const int64_t off = (int64_t)src[ip] | ((int64_t)src[ip + 1] << 8);
        ip += 2;
        if (off == 0 || off > op)
            return -3;
        int64_t ml = (token & 15) + MINMATCH;
        if ((token & 15) == 15) {
            unsigned b;
            do {
                if (ip >= n_in)
                    return -3;
                b = src[ip++];
                ml += b;
            } while (b == 255);
        }
        if (ml > n_out - op)
            return -3;
        for (int64_t i = 0; i < ml; i++) /* byte by byte: overlap replicates */
            dst[op + i] = dst[op - off + i];
        op += ml;
    }
    return op == n_out ? n_out : -3;
}

/* ======================================================================
 * The blocked stream.  Layout (little-endian):
 *   u32 magic "BSG1", u32 elem_size, u64 n, u32 block elements, u32 n_blocks
 *   u64 off[n_blocks + 1]   (relative to the payload start, off[0] = 0)
 *   LZ4 block payloads, concatenated
 *   raw tail: the last n mod 8 elements
 * ====================================================================== */

static void put_u32(uint8_t *p, uint32_t v)
{
    for (int i = 0; i < 4; i++)
        p[i] = (uint8_t)(v >> (8 * i));
}
static void put_u64(uint8_t *p, uint64_t v)
{
    for (int i = 0; i < 8; i++)
        p[i] = (uint8_t)(v >> (8 * i));
}
static uint32_t get_u32(const uint8_t *p)
{
    uint32_t v = 0;
    for (int i = 0; i < 4; i++)
        v |= (uint32_t)p[i] << (8 * i);
    return v;
}
static uint64_t get_u64(const uint8_t *p)
{
    uint64_t v = 0;
    for (int i = 0; i < 8; i++)
        v |= (uint64_t)p[i] << (8 * i);
    return v;
}

static int64_t lz4_block_bound(int64_t s) { return s + s / 255 + 16; }

int64_t oracle_compress_bound(int64_t n, int64_t elem_size, int64_t block_size)
{
    const int64_t nb = oracle_block_elems(elem_size, block_size);
    if (nb < 0 || n < 0 || nb * elem_size > MAX_BLOCK_BYTES)
        return -1;
    int64_t n_full, last, n_blocks, tail;
    block_layout(n, nb, &n_full, &last, &n_blocks, &tail);
    int64_t bound = HEADER_BYTES + 8 * (n_blocks + 1) + tail * elem_size;
    bound += n_full * lz4_block_bound(nb * elem_size);
    if (last)
        bound += lz4_block_bound(last * elem_size);
    return bound;
}

int64_t oracle_compress_filter(const uint8_t *in, uint8_t *out, int64_t n, int64_t elem_size,
                               int64_t block_size, int filter, int64_t cap, int nthreads)
{
    if (filter != 0 && filter != 1)
        return -1;
    const int64_t bound = oracle_compress_bound(n, elem_size, block_size);
    if (bound < 0 || (n > 0 && !in) || !out)
        return -1;
    const int64_t E = elem_size, nb = oracle_block_elems(E, block_size);
    int64_t n_full, last, n_blocks, tail;
    block_layout(n, nb, &n_full, &last, &n_blocks, &tail);
    const int64_t slot = lz4_block_bound(nb * E);
    uint8_t *slots = (uint8_t *)malloc((size_t)(n_blocks > 0 ? n_blocks * slot : 1));
    int64_t *size = (int64_t *)malloc((size_t)(n_blocks + 1) * sizeof(int64_t));
    if (!slots || !size) {
        free(slots);
        free(size);
        return -1;
    }
    /* each block: bit transpose, then LZ4 (Section 4.2) */
#pragma omp parallel num_threads(pick_threads(nthreads))
    {
        uint8_t *tmp = (uint8_t *)malloc((size_t)(nb * E));
#pragma omp for schedule(dynamic, 64)
        for (int64_t blk = 0; blk < n_blocks; blk++) {
            const int64_t elems = blk < n_full ? nb : last;
            filter_block(in + blk * nb * E, tmp, elems, E, filter, 0);
            size[blk] = oracle_lz4_compress_block(tmp, elems * E, slots + blk * slot, slot);
        }
        free(tmp);
    }
    int64_t total = HEADER_BYTES + 8 * (n_blocks + 1);
    for (int64_t blk = 0; blk < n_blocks; blk++) {
        if (size[blk] < 0) { /* cannot happen: a slot holds the LZ4 bound */
            free(slots);
            free(size);
            return -1;
        }
        total += size[blk];
    }
    total += tail * E;
    if (total > cap) {
        free(slots);
        free(size);
        return -2;
    }
    put_u32(out, filter == 1 ? STREAM_MAGIC_BYTE : STREAM_MAGIC);
    put_u32(out + 4, (uint32_t)E);
    put_u64(out + 8, (uint64_t)n);
    put_u32(out + 16, (uint32_t)nb);
    put_u32(out + 20, (uint32_t)n_blocks);
    uint8_t *payload = out + HEADER_BYTES + 8 * (n_blocks + 1);
    int64_t off = 0;
    for (int64_t blk = 0; blk < n_blocks; blk++) {
        put_u64(out + HEADER_BYTES + 8 * blk, (uint64_t)off);
        memcpy(payload + off, slots + blk * slot, (size_t)size[blk]);
        off += size[blk];
    }
    put_u64(out + HEADER_BYTES + 8 * n_blocks, (uint64_t)off);
    if (tail)
        memcpy(payload + off, in + (n - tail) * E, (size_t)(tail * E));
    free(slots);
    free(size);
    return total;
}

int64_t oracle_compress(const uint8_t *in, uint8_t *out, int64_t n, int64_t elem_size,
                        int64_t block_size, int64_t cap, int nthreads)
{
    return oracle_compress_filter(in, out, n, elem_size, block_size, 0, cap, nthreads);
}

int64_t oracle_decompress_filter(const uint8_t *in, int64_t in_nbytes, uint8_t *out, int64_t n,
                                 int64_t elem_size, int64_t block_size, int filter, int nthreads)
{
    if (filter != 0 && filter != 1)
        return -1;
    const int64_t nb = oracle_block_elems(elem_size, block_size);
    if (nb < 0 || n < 0 || !in || (n > 0 && !out) || nb * elem_size > MAX_BLOCK_BYTES)
        return -1;
    const int64_t E = elem_size;
    int64_t n_full, last, n_blocks, tail;
    block_layout(n, nb, &n_full, &last, &n_blocks, &tail);
    const int64_t table_end = HEADER_BYTES + 8 * (n_blocks + 1);
    if (in_nbytes < table_end)
        return -3;
    if (get_u32(in) != (filter == 1 ? STREAM_MAGIC_BYTE : STREAM_MAGIC) ||
        get_u32(in + 4) != (uint32_t)E ||
        get_u64(in + 8) != (uint64_t)n || get_u32(in + 16) != (uint32_t)nb ||
        get_u32(in + 20) != (uint32_t)n_blocks)
        return -3;
    const int64_t payload_len = in_nbytes - table_end - tail * E;
    if (payload_len < 0 || get_u64(in + HEADER_BYTES) != 0 ||
        get_u64(in + HEADER_BYTES + 8 * n_blocks) != (uint64_t)payload_len)
        return -3;
    for (int64_t blk = 0; blk < n_blocks; blk++)
        if (get_u64(in + HEADER_BYTES + 8 * (blk + 1)) < get_u64(in + HEADER_BYTES + 8 * blk))
            return -3;
    const uint8_t *payload = in + table_end;
    int bad = 0;
#pragma omp parallel num_threads(pick_threads(nthreads))
    {
        uint8_t *tmp = (uint8_t *)malloc((size_t)(nb * E));
#pragma omp for schedule(dynamic, 64)
        for (int64_t blk = 0; blk < n_blocks; blk++) {
            const int64_t elems = blk < n_full ? nb : last;
            const int64_t o0 = (int64_t)get_u64(in + HEADER_BYTES + 8 * blk);
            const int64_t o1 = (int64_t)get_u64(in + HEADER_BYTES + 8 * (blk + 1));
            if (oracle_lz4_decompress_block(payload + o0, o1 - o0, tmp, elems * E) != elems * E) {
#pragma omp atomic write
                bad = 1;
                continue;
            }
            filter_block(tmp, out + blk * nb * E, elems, E, filter, 1);
        }
        free(tmp);
    }
    if (bad)
        return -3;
    if (tail)
        memcpy(out + (n - tail) * E, payload + payload_len, (size_t)(tail * E));
    return 0;
}

int64_t oracle_decompress(const uint8_t *in, int64_t in_nbytes, uint8_t *out, int64_t n,
                          int64_t elem_size, int64_t block_size, int nthreads)
{
    return oracle_decompress_filter(in, in_nbytes, out, n, elem_size, block_size, 0, nthreads);
}
