// Full-covariance noise for small arrays (Masui et al., Section 3.1, Eqs.
// rad_full1-3 and Eq. noise): per (frequency, time) the covariance of the
// I^2 real degrees of freedom of the visibilities (Re of every product, Im
// of every cross product, in product order), the noise of each degree of
// freedom s_k^2 = 1 / (C^-1)_kk, and the rounding of Section 3.2 with
// G2 = 12 f s_k^2.  With Q = 2N C this is G2 = c / (Q^-1)_kk, c = (12 f)/(2N).
//
// One workgroup per sample holds Q in LDS (D = I^2 <= 121, so at most
// 120 KiB): the Hermitian V of the sample, the lower triangle of Q from it,
// a right-looking Cholesky factorisation Q = L L^T in place (a step per
// column, the trailing update spread over the workgroup), then M = L^-1 one
// column per thread, a few rows per pass (stored transposed in the free
// upper triangle) and (Q^-1)_kk = sum_i M_ik^2.  Every element sees its
// operations in the same order as a plain serial implementation (sums in
// increasing index order), so the results are reproducible bit for bit.  A
// sample whose Q is not positive definite gets no estimate and is left
// unchanged.
#include <cmath>

#include "bsg_internal.hpp"
#include "bsg_round_dev.hpp"

namespace bsg {

namespace {

constexpr int kMaxInputs = 11; // D = 121 degrees of freedom, 120 KiB of LDS
static_assert(kMaxInputs * kMaxInputs <= 128, "the trailing update keeps 8 columns per thread");
// Up to this many degrees of freedom (8 inputs, four samples per CU) the
// instance has 256 threads and its inverse forms ROWS = 8 rows of a column
// per pass (16 would cost occupancy); above it (one sample per CU) 512
// threads hide more latency in the factorisation, and 2 rows per pass were
// faster than 4.
constexpr int kFourRowMaxD = 64;

struct Cplx {
    double re, im;
};

__device__ __forceinline__ Cplx mul_conj(Cplx a, Cplx b) // a * conj(b)
{
    return Cplx{a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

// inputs (i, j) of product p in upper-triangle row-major order
__device__ __forceinline__ void pair_of(int I, int p, int &i, int &j)
{
    i = 0;
    while (p >= I - i) {
        p -= I - i;
        ++i;
    }
    j = i + p;
}

struct FullcovArgs {
    const float2 *vis;
    const float *autos;
    int64_t F, T;
    int I, P, D;
    double c;
    float2 *vis_out;  // nullptr: only the inverse diagonal
    double *qdiag;    // [F][T][D] or nullptr
};

template <int ROWS, int THREADS>
__global__ __launch_bounds__(THREADS) void k_fullcov(FullcovArgs a)
{
    extern __shared__ double smem[];
    const int D = a.D, I = a.I, P = a.P;
    // Q: D x D, row major with rows of LD doubles, LD even: the inverse's
    // lanes walk rows LD + 1 doubles apart (an odd stride spreads them over
    // the LDS banks); the factorisation reads column k from its copy colk
    const int LD = D + (D & 1);
    double *Q = smem;
    double *colk = Q + D * LD;            // D: column k of L during step k
    Cplx *V = reinterpret_cast<Cplx *>(colk + D); // I x I
    int *dof = reinterpret_cast<int *>(V + I * I);  // D: product * 2 + (Im ? 1 : 0)
    int *dij = dof + D;                             // D: the product's inputs, i | j << 8
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int64_t s = blockIdx.x; // sample (fr, t)
    const int64_t fr = s / a.T, t = s - fr * a.T;

    if (tid == 0) {
        bad = 0;
        int k = 0;
        for (int p = 0; p < P; ++p) {
            int i, j;
            pair_of(I, p, i, j);
            dij[k] = i | j << 8;
            dof[k++] = 2 * p;
            if (i != j) {
                dij[k] = i | j << 8;
                dof[k++] = 2 * p + 1;
            }
        }
    }
    for (int e = tid; e < I * I; e += blockDim.x) {
        const int x = e / I, y = e - x * I;
        Cplx v;
        if (x == y) {
            v.re = a.autos[(fr * I + x) * a.T + t];
            v.im = 0.0;
        } else {
            const int lo = x < y ? x : y, hi = x < y ? y : x;
            const int p = lo * I - lo * (lo - 1) / 2 + (hi - lo);
            const float2 w = a.vis[(fr * P + p) * a.T + t];
            v.re = w.x;
            v.im = x < y ? (double)w.y : -(double)w.y;
        }
        V[e] = v;
    }
    __syncthreads();

    // Q = 2N C (Eqs. rad_full1-3), its lower triangle only (the factorisation
    // reads nothing else, and the inverse writes the upper half before it
    // reads it); element e of the triangle in row-major order is (x, y),
    // y <= x, from a float estimate of the row corrected by exact checks.
    // Each degree of freedom's inputs come from the table built above.
    for (int e = tid; e < D * (D + 1) / 2; e += blockDim.x) {
        int x = (int)((__builtin_sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
        while (x * (x + 1) / 2 > e) --x;
        while ((x + 1) * (x + 2) / 2 <= e) ++x;
        const int y = e - x * (x + 1) / 2;
        const int i = dij[x] & 255, j = dij[x] >> 8, g = dij[y] & 255, h = dij[y] >> 8;
        const bool ix = dof[x] & 1, iy = dof[y] & 1;
        const Cplx A = mul_conj(V[i * I + g], V[j * I + h]);
        const Cplx B = mul_conj(V[i * I + h], V[j * I + g]);
        double q;
        if (!ix && !iy) {
            q = A.re + B.re;
        } else if (ix && iy) {
            q = A.re - B.re;
        } else if (!ix) {
            q = -A.im + B.im;
        } else { // (Im ij, Re gh) is the (Re gh, Im ij) element
            const Cplx A2 = mul_conj(V[g * I + i], V[h * I + j]);
            const Cplx B2 = mul_conj(V[g * I + j], V[h * I + i]);
            q = -A2.im + B2.im;
        }
        Q[x * LD + y] = q;
    }
    __syncthreads();

    // Cholesky, right-looking, in place in the lower triangle
    for (int k = 0; k < D; ++k) {
        const double d = Q[k * LD + k];
        if (!(d > 0.0) || d == __builtin_inf()) { // uniform: every thread reads the same d
            if (tid == 0) bad = 1;
            break;
        }
        // (only the threads that scale the column, and thread 0, need L_kk:
        // a wave with none of them skips the square root)
        double lkk = 0.0;
        if (k + 1 + tid < D || tid == 0) lkk = sqrt(d);
        for (int i = k + 1 + tid; i < D; i += blockDim.x) {
            const double lik = Q[i * LD + k] / lkk;
            Q[i * LD + k] = lik;
            colk[i] = lik;
        }
        __syncthreads();
        // every thread has read Q[k][k] before the barrier, and the trailing
        // update below does not touch it
        if (tid == 0) Q[k * LD + k] = lkk;
        // trailing lower triangle, rows and columns k+1 .. D-1, on a
        // (THREADS / 16) x 16 grid of threads; a thread's columns j0 + 16 b
        // are the same for all its rows, so their column-k values stay in
        // registers (D <= 128)
        const int j0 = k + 1 + (tid & 15);
        double cj[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) cj[b] = j0 + 16 * b < D ? colk[j0 + 16 * b] : 0.0;
        for (int i = k + 1 + (tid >> 4); i < D; i += THREADS / 16) {
            const double lik = colk[i];
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int j = j0 + 16 * b;
                if (j > i) break;
                Q[i * LD + j] = Q[i * LD + j] - lik * cj[b];
            }
        }
        __syncthreads();
    }
    __syncthreads();
    const bool failed = bad != 0;

    // M = L^-1, column j by thread j; M_ij (i > j) kept at Q[j][i]
    double qk = __builtin_nan("");
    if (!failed) {
        for (int j = tid; j < D; j += blockDim.x) {
            const double mjj = 1.0 / Q[j * LD + j];
            // (Q^-1)_jj = sum_{i >= j} M_ij^2 in increasing i, added as each
            // M_ij is formed (its own chain, beside the next row's sum)
            double q = 0.0;
            q = q + mjj * mjj;
            const double *Mj = Q + j * LD; // M_mj at Mj[m]
            int i = j + 1;
            // ROWS rows per pass: their sums share the terms m < i, so each
            // M_mj is read once for all of them, and the sums are independent
            // chains; every sum still adds its terms one by one in increasing m
            for (; ROWS > 1 && i + ROWS - 1 < D; i += ROWS) {
                const double *Lr[ROWS];
                double acc[ROWS], mv[ROWS];
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    Lr[r] = Q + (i + r) * LD;
                    acc[r] = Lr[r][j] * mjj;
                }
#pragma unroll 4
                for (int m = j + 1; m < i; ++m) {
                    const double mm = Mj[m];
#pragma unroll
                    for (int r = 0; r < ROWS; ++r) acc[r] = acc[r] + Lr[r][m] * mm;
                }
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
#pragma unroll
                    for (int t = 0; t < r; ++t) acc[r] = acc[r] + Lr[r][i + t] * mv[t];
                    mv[r] = -acc[r] / Lr[r][i + r];
                    Q[j * LD + i + r] = mv[r];
                    q = q + mv[r] * mv[r];
                }
            }
            for (; i < D; ++i) {
                double acc = Q[i * LD + j] * mjj;
#pragma unroll 8
                for (int m = j + 1; m < i; ++m) acc = acc + Q[i * LD + m] * Mj[m];
                const double mij = -acc / Q[i * LD + i];
                Q[j * LD + i] = mij;
                q = q + mij * mij;
            }
            if (j == tid) qk = q;
            if (a.qdiag) a.qdiag[s * D + j] = q;
        }
    } else if (a.qdiag) {
        for (int j = tid; j < D; j += blockDim.x) a.qdiag[s * D + j] = __builtin_nan("");
    }
    if (!a.vis_out) return;
    // round degree of freedom k = tid (D <= 121 < 256 threads)
    if (tid < D) {
        const int p = dof[tid] >> 1;
        const bool im = dof[tid] & 1;
        const int64_t e = (fr * P + p) * a.T + t;
        const float x = im ? a.vis[e].y : a.vis[e].x;
        const uint32_t r = round_noise_bits(__float_as_uint(x), a.c / qk);
        float *o = reinterpret_cast<float *>(a.vis_out + e);
        o[im ? 1 : 0] = __uint_as_float(r);
        int i, j;
        pair_of(I, p, i, j);
        if (i == j) o[1] = a.vis[e].y; // Im of an auto is copied
    }
}

} // namespace

int fullcov_max_inputs() { return kMaxInputs; }

hipError_t launch_fullcov(const float *vis, const float *autos, int64_t F, int64_t I, int64_t T,
                          double c, float *vis_out, double *qdiag, hipStream_t s)
{
    const int D = (int)(I * I), P = (int)(I * (I + 1) / 2);
    if (F * T == 0 || D == 0) return hipSuccess;
    FullcovArgs a{reinterpret_cast<const float2 *>(vis), autos, F, T, (int)I, P, D, c,
                  reinterpret_cast<float2 *>(vis_out), qdiag};
    const size_t lds = sizeof(double) * ((size_t)D * (D + (D & 1)) + D) +
                       sizeof(Cplx) * (size_t)(I * I) +
                       sizeof(int) * (size_t)(2 * D);
    if (D <= kFourRowMaxD)
        hipLaunchKernelGGL((k_fullcov<8, 256>), dim3((unsigned)(F * T)), dim3(256), lds, s, a);
    else
        hipLaunchKernelGGL((k_fullcov<2, 512>), dim3((unsigned)(F * T)), dim3(512), lds, s, a);
    return hipGetLastError();
}

} // namespace bsg
