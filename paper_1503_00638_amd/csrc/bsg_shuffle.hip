// Stage 2a: the Bitshuffle bit transpose within blocks (Section 4.2 of
// Masui et al.), standalone (no LZ4).  One lane per unit on the fast path;
// one wavefront per block with ballots on the generic path.
#include "bsg_internal.hpp"
#include "bsg_shuffle_dev.hpp"

namespace bsg {

namespace {

// units_per_block units tile each block; unit t of the launch belongs to
// block t / units_per_block.  in/out point at the first block.
template <int E, bool INV>
__global__ __launch_bounds__(256) void k_shuffle_fast(const uint8_t *__restrict__ in,
                                                      uint8_t *__restrict__ out,
                                                      int64_t units_total,
                                                      int64_t units_per_block, int64_t nb)
{
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= units_total) return;
    const int64_t blk = t / units_per_block;
    const int64_t u = t - blk * units_per_block;
    const int64_t blk_off = blk * nb * E;
    uint32_t w[Unit<E>::IN_WORDS];
    if constexpr (!INV) {
        load_unit<E>(in + blk_off + u * (Unit<E>::G * E), w);
        unit_forward<E>(w);
        store_planes<E>(out + blk_off, nb / 8, u, w);
    } else {
        load_planes<E>(in + blk_off, nb / 8, u, w);
        unit_inverse<E>(w);
        store_unit<E>(out + blk_off + u * (Unit<E>::G * E), w);
    }
}

template <bool INV>
__global__ __launch_bounds__(64) void k_shuffle_generic(const uint8_t *__restrict__ in,
                                                        uint8_t *__restrict__ out, int64_t nb,
                                                        int64_t E)
{
    const int64_t off = int64_t(blockIdx.x) * nb * E;
    if (!INV)
        block_forward_ballot(in + off, out + off, nb, E);
    else
        block_inverse_bits(in + off, out + off, nb, E);
}

__global__ __launch_bounds__(64) void k_copy_bytes(const uint8_t *__restrict__ in,
                                                   uint8_t *__restrict__ out, int64_t nbytes)
{
    for (int64_t i = threadIdx.x; i < nbytes; i += 64) out[i] = in[i];
}

template <int E, bool INV>
hipError_t fast_launch(const uint8_t *in, uint8_t *out, int64_t nblocks, int64_t nb,
                       hipStream_t s)
{
    const int64_t upb = nb / Unit<E>::G;
    const int64_t total = nblocks * upb;
    const int64_t grid = (total + 255) / 256;
    hipLaunchKernelGGL((k_shuffle_fast<E, INV>), dim3((unsigned)grid), dim3(256), 0, s, in, out,
                       total, upb, nb);
    return hipGetLastError();
}

template <bool INV>
hipError_t blocks_launch(const uint8_t *in, uint8_t *out, int64_t nblocks, int64_t nb,
                         int64_t E, hipStream_t s)
{
    if (nblocks == 0) return hipSuccess;
    const int G = unit_elems(E);
    const bool aligned = ((uintptr_t)in % 16 == 0) && ((uintptr_t)out % 16 == 0);
    if (G && nb % G == 0 && aligned) {
        switch (E) {
        case 1: return fast_launch<1, INV>(in, out, nblocks, nb, s);
        case 2: return fast_launch<2, INV>(in, out, nblocks, nb, s);
        case 4: return fast_launch<4, INV>(in, out, nblocks, nb, s);
        case 8: return fast_launch<8, INV>(in, out, nblocks, nb, s);
        case 12: return fast_launch<12, INV>(in, out, nblocks, nb, s);
        case 16: return fast_launch<16, INV>(in, out, nblocks, nb, s);
        default: break;
        }
    }
    hipLaunchKernelGGL((k_shuffle_generic<INV>), dim3((unsigned)nblocks), dim3(64), 0, s, in, out,
                       nb, E);
    return hipGetLastError();
}

} // namespace

hipError_t launch_shuffle(const uint8_t *in, uint8_t *out, const Layout &L, bool inverse,
                          hipStream_t s)
{
    hipError_t e;
    if (inverse) {
        e = blocks_launch<true>(in, out, L.n_full, L.nb, L.E, s);
        if (e == hipSuccess && L.last)
            e = blocks_launch<true>(in + L.n_full * L.nb * L.E, out + L.n_full * L.nb * L.E, 1,
                                    L.last, L.E, s);
    } else {
        e = blocks_launch<false>(in, out, L.n_full, L.nb, L.E, s);
        if (e == hipSuccess && L.last)
            e = blocks_launch<false>(in + L.n_full * L.nb * L.E, out + L.n_full * L.nb * L.E, 1,
                                     L.last, L.E, s);
    }
    if (e == hipSuccess && L.tail) {
        const int64_t off = (L.n - L.tail) * L.E;
        hipLaunchKernelGGL(k_copy_bytes, dim3(1), dim3(64), 0, s, in + off, out + off,
                           L.tail * L.E);
        e = hipGetLastError();
    }
    return e;
}

} // namespace bsg
