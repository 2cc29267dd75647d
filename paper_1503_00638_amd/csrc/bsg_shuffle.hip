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

namespace {

// Byte shuffle of whole blocks, one thread per output dword: forward, output
// byte k * nb + i of a block is input byte i * E + k; inverse, output byte
// i * E + k is input byte k * nb + i.  Block bytes are a multiple of 8, so
// dwords never straddle blocks.
template <bool INV>
__global__ __launch_bounds__(256) void k_byteshuffle(const uint8_t *__restrict__ in,
                                                     uint8_t *__restrict__ out, int64_t n_blocks,
                                                     int64_t nb, int64_t E)
{
    const int64_t words_per_block = nb * E / 4;
    const int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (d >= n_blocks * words_per_block) return;
    const int64_t b = d / words_per_block, w = d - b * words_per_block;
    const uint8_t *src = in + b * nb * E;
    uint32_t v = 0;
    for (int q = 0; q < 4; ++q) {
        const int64_t o = 4 * w + q; // output byte within the block
        int64_t i, k;
        if (INV) {
            i = o / E;
            k = o - i * E;
        } else {
            k = o / nb;
            i = o - k * nb;
        }
        v |= (uint32_t)src[INV ? k * nb + i : i * E + k] << (8 * q);
    }
    reinterpret_cast<uint32_t *>(out + b * nb * E)[w] = v;
}

// The byte shuffle for element sizes that are multiples of 4, both buffers
// 16-byte aligned: a thread takes 4 elements of a block (4E bytes, 16-byte
// accesses) and transposes each 4 x 4 byte sub-matrix (dword kg of the 4
// elements) in registers into dword g of planes 4kg .. 4kg + 3.
template <int E, bool INV>
__global__ __launch_bounds__(256) void k_byteshuffle_fast(const uint8_t *__restrict__ in,
                                                          uint8_t *__restrict__ out,
                                                          int64_t n_blocks, int64_t nb)
{
    constexpr int W = E / 4;
    const int64_t per = nb / 4; // groups of 4 elements per block
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n_blocks * per) return;
    const int64_t b = t / per, g = t - b * per;
    const int64_t base = b * nb * E;
    uint32_t w[4 * W];
    if constexpr (!INV) {
        const uint4 *s4 = reinterpret_cast<const uint4 *>(in + base + 4 * g * E);
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const uint4 v = s4[q];
            w[4 * q] = v.x;
            w[4 * q + 1] = v.y;
            w[4 * q + 2] = v.z;
            w[4 * q + 3] = v.w;
        }
        uint32_t *o32 = reinterpret_cast<uint32_t *>(out + base);
#pragma unroll
        for (int kg = 0; kg < W; ++kg) {
            uint32_t o0, o1, o2, o3;
            byte_transpose4(w[kg], w[W + kg], w[2 * W + kg], w[3 * W + kg], o0, o1, o2, o3);
            o32[(4 * kg) * per + g] = o0;
            o32[(4 * kg + 1) * per + g] = o1;
            o32[(4 * kg + 2) * per + g] = o2;
            o32[(4 * kg + 3) * per + g] = o3;
        }
    } else {
        const uint32_t *i32 = reinterpret_cast<const uint32_t *>(in + base);
#pragma unroll
        for (int kg = 0; kg < W; ++kg)
            byte_transpose4(i32[(4 * kg) * per + g], i32[(4 * kg + 1) * per + g],
                            i32[(4 * kg + 2) * per + g], i32[(4 * kg + 3) * per + g], w[kg],
                            w[W + kg], w[2 * W + kg], w[3 * W + kg]);
        uint4 *d4 = reinterpret_cast<uint4 *>(out + base + 4 * g * E);
#pragma unroll
        for (int q = 0; q < W; ++q)
            d4[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
    }
}

template <bool INV>
hipError_t bytes_launch(const uint8_t *in, uint8_t *out, int64_t n_blocks, int64_t nb, int64_t E,
                        hipStream_t s)
{
    const int64_t words = n_blocks * nb * E / 4;
    if (words == 0) return hipSuccess;
    if (((uintptr_t)in | (uintptr_t)out) % 16 == 0 && E % 4 == 0 && E <= 16) {
        const unsigned grid = (unsigned)((n_blocks * (nb / 4) + 255) / 256);
        switch (E) {
        case 4: hipLaunchKernelGGL((k_byteshuffle_fast<4, INV>), dim3(grid), dim3(256), 0, s, in, out, n_blocks, nb); break;
        case 8: hipLaunchKernelGGL((k_byteshuffle_fast<8, INV>), dim3(grid), dim3(256), 0, s, in, out, n_blocks, nb); break;
        case 12: hipLaunchKernelGGL((k_byteshuffle_fast<12, INV>), dim3(grid), dim3(256), 0, s, in, out, n_blocks, nb); break;
        default: hipLaunchKernelGGL((k_byteshuffle_fast<16, INV>), dim3(grid), dim3(256), 0, s, in, out, n_blocks, nb); break;
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_byteshuffle<INV>), dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s,
                       in, out, n_blocks, nb, E);
    return hipGetLastError();
}

} // namespace

hipError_t launch_byteshuffle(const uint8_t *in, uint8_t *out, const Layout &L, bool inverse,
                              hipStream_t s)
{
    hipError_t e = inverse ? bytes_launch<true>(in, out, L.n_full, L.nb, L.E, s)
                           : bytes_launch<false>(in, out, L.n_full, L.nb, L.E, s);
    const int64_t off = L.n_full * L.nb * L.E;
    if (e == hipSuccess && L.last)
        e = inverse ? bytes_launch<true>(in + off, out + off, 1, L.last, L.E, s)
                    : bytes_launch<false>(in + off, out + off, 1, L.last, L.E, s);
    if (e == hipSuccess && L.tail) {
        const int64_t t0 = (L.n - L.tail) * L.E;
        hipLaunchKernelGGL(k_copy_bytes, dim3(1), dim3(64), 0, s, in + t0, out + t0, L.tail * L.E);
        e = hipGetLastError();
    }
    return e;
}

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
