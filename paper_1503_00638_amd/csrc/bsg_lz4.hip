// Stage 2b: per-block LZ4 after the bit transpose (Section 4.2 of Masui et
// al.: each block is transposed and compressed while it is still on chip;
// blocks are independent).  On gfx950 a block lives in LDS and one
// wavefront owns it.
//
// Compression = k_encode (transpose into LDS [+ fused rounding], LDS hash
// table, greedy parse, write to a bound-sized slot) -> k_tile_sum ->
// k_tile_offsets (one workgroup) -> k_write_offsets -> k_pack (copy slots to
// their final place, header, raw tail).
// Decompression = k_decode (stage the LZ4 block in LDS, decode into LDS,
// inverse transpose on the way out to HBM).
#include "bsg_lz4_dev.hpp"

namespace bsg {

namespace {

struct EncArgs {
    const uint8_t *in; // first element of the buffer
    int64_t nb, E, n_full, last;
    uint8_t *slots;
    int64_t slot_bytes;
    int32_t *sizes;
    int64_t block0; // index of the first block of this launch
};

template <int MAXB, int EC, bool ROUND>
__global__ __launch_bounds__(64) void k_encode(EncArgs a, RoundParams rp)
{
    __shared__ EncLds<MAXB> L;
    const int64_t b = a.block0 + blockIdx.x;
    const int64_t elems = b < a.n_full ? a.nb : a.last;
    const int64_t first = b * a.nb;
    const int sz = encode_one<MAXB, EC, ROUND>(a.in + first * a.E, elems, a.E, rp, first,
                                               a.slots + b * a.slot_bytes, L);
    if (threadIdx.x == 0) a.sizes[b] = sz;
}

// tile_sum[k] = sum of sizes over blocks [k * kTile, (k + 1) * kTile)
__global__ __launch_bounds__(256) void k_tile_sum(const int32_t *__restrict__ sizes,
                                                  int64_t n_blocks, int64_t *__restrict__ tile_sum)
{
    __shared__ int64_t sh[256];
    const int64_t base = int64_t(blockIdx.x) * kTile;
    int64_t s = 0;
    for (int k = threadIdx.x; k < kTile; k += 256)
        if (base + k < n_blocks) s += sizes[base + k];
    const int64_t inc = block_sum_i64(s, sh);
    if (threadIdx.x == 255) tile_sum[blockIdx.x] = inc;
}

// One workgroup: exclusive scan of the tile sums (in place), stream total,
// capacity verdict, stream header.
__global__ __launch_bounds__(256) void k_tile_offsets(int64_t *__restrict__ tile_sum,
                                                      int64_t n_tiles, int64_t fixed_bytes,
                                                      int64_t cap, int64_t *__restrict__ d_nbytes,
                                                      uint8_t *__restrict__ out, bsg_header hdr)
{
    __shared__ int64_t sh[256];
    int64_t carry = 0;
    for (int64_t base = 0; base < n_tiles; base += 256) {
        const int64_t k = base + threadIdx.x;
        const int64_t v = k < n_tiles ? tile_sum[k] : 0;
        const int64_t inc = block_sum_i64(v, sh);
        if (k < n_tiles) tile_sum[k] = carry + inc - v;
        carry += sh[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t total = fixed_bytes + carry;
        *d_nbytes = total <= cap ? total : (int64_t)BSG_ECAPACITY;
        *reinterpret_cast<bsg_header *>(out) = hdr;
        // payload length at the end of the offset table
        reinterpret_cast<uint64_t *>(out + kHeaderBytes)[hdr.n_blocks] = (uint64_t)carry;
    }
}

// off[b] for every block of a tile (written straight into the stream).
__global__ __launch_bounds__(256) void k_write_offsets(const int32_t *__restrict__ sizes,
                                                       int64_t n_blocks,
                                                       const int64_t *__restrict__ tile_off,
                                                       uint8_t *__restrict__ out)
{
    __shared__ int64_t sh[256];
    constexpr int PER = kTile / 256;
    const int64_t base = int64_t(blockIdx.x) * kTile + threadIdx.x * PER;
    int64_t v[PER];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = base + k < n_blocks ? sizes[base + k] : 0;
        s += v[k];
    }
    const int64_t inc = block_sum_i64(s, sh);
    int64_t o = tile_off[blockIdx.x] + inc - s;
    uint64_t *off = reinterpret_cast<uint64_t *>(out + kHeaderBytes);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (base + k < n_blocks) off[base + k] = (uint64_t)o;
        o += v[k];
    }
}

// Copy each block's LZ4 bytes from its slot to the payload; the extra last
// workgroup copies the raw tail.  Nothing is written when the stream does
// not fit (d_nbytes < 0).
__global__ __launch_bounds__(64) void k_pack(const uint8_t *__restrict__ slots, int64_t slot_bytes,
                                             const int32_t *__restrict__ sizes, int64_t n_blocks,
                                             uint8_t *__restrict__ out,
                                             const int64_t *__restrict__ d_nbytes,
                                             const uint8_t *__restrict__ tail_src,
                                             int64_t tail_bytes, RoundParams rp, int round_tail,
                                             int64_t tail_first_elem)
{
    const int64_t b = blockIdx.x;
    const uint64_t *off = reinterpret_cast<const uint64_t *>(out + kHeaderBytes);
    // (the three loads issue together)
    const int64_t nbytes = *d_nbytes;
    const uint64_t ob = off[b];
    const int sz = b < n_blocks ? sizes[b] : 0;
    if (nbytes < 0) return;
    uint8_t *payload = out + kHeaderBytes + 8 * (n_blocks + 1);
    const int lane = threadIdx.x;
    if (b == n_blocks) {
        uint8_t *dst = payload + off[n_blocks];
        if (round_tail) { // the raw tail of the fused path is rounded too (float32 elements)
            for (int64_t k = lane; k < tail_bytes / 4; k += kWave) {
                uint32_t x = 0;
                for (int q = 0; q < 4; ++q) x |= (uint32_t)tail_src[4 * k + q] << (8 * q);
                x = round_element(x, tail_first_elem + k, rp);
                for (int q = 0; q < 4; ++q) dst[4 * k + q] = (uint8_t)(x >> (8 * q));
            }
            return;
        }
        for (int64_t i = lane; i < tail_bytes; i += kWave) dst[i] = tail_src[i];
        return;
    }
    copy_slot(payload + ob, slots + b * slot_bytes, sz);
}

struct DecArgs {
    const uint8_t *in;
    int64_t in_nbytes;
    uint8_t *out;
    int64_t n, E, nb, n_full, last, n_blocks, tail;
    int32_t *status;
    int fast_out; // out is 16-byte aligned
    uint32_t magic; // the stream's filter: bit transpose or byte shuffle
};

template <int MAXB, int EC>
__global__ __launch_bounds__(64) void k_decode(DecArgs a)
{
    __shared__ DecLds<MAXB> L;
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int64_t table_end = kHeaderBytes + 8 * (a.n_blocks + 1);
    const int64_t tail_bytes = a.tail * a.E;
    const int64_t payload_len = a.in_nbytes - table_end - tail_bytes; // >= 0 (host-checked)
    const uint8_t *payload = a.in + table_end;
    if (b == a.n_blocks) { // header check and raw tail
        if (!header_ok(a.in, payload_len, a.n, a.E, a.nb, a.n_blocks, a.magic)) {
            fail(a.status);
            return;
        }
        uint8_t *dst = a.out + (a.n - a.tail) * a.E;
        for (int64_t i = lane; i < tail_bytes; i += kWave) dst[i] = payload[payload_len + i];
        return;
    }
    const int64_t elems = b < a.n_full ? a.nb : a.last;
    const uint64_t *off = reinterpret_cast<const uint64_t *>(a.in + kHeaderBytes);
    if (!decode_one<MAXB, EC>(payload, payload_len, off, b, elems, a.E, a.in + a.in_nbytes,
                              a.out + b * a.nb * a.E, a.fast_out != 0, L))
        fail(a.status);
}

template <int MAXB, int EC, bool ROUND>
hipError_t encode_launch(const EncArgs &ea, int64_t nblocks, const RoundParams &rp,
                         hipStream_t s)
{
    if (nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL((k_encode<MAXB, EC, ROUND>), dim3((unsigned)nblocks), dim3(kWave), 0, s, ea,
                       rp);
    return hipGetLastError();
}

template <int MAXB>
hipError_t encode_dispatch(const EncArgs &ea, int64_t nblocks, const RoundParams *rp, int ec,
                           hipStream_t s)
{
    const RoundParams none{};
    if (rp) return ec == 4 ? encode_launch<MAXB, 4, true>(ea, nblocks, *rp, s)
                           : encode_launch<MAXB, 0, true>(ea, nblocks, *rp, s);
    switch (ec) {
    case kByteShuffle: return encode_launch<MAXB, kByteShuffle, false>(ea, nblocks, none, s);
    case 1: return encode_launch<MAXB, 1, false>(ea, nblocks, none, s);
    case 2: return encode_launch<MAXB, 2, false>(ea, nblocks, none, s);
    case 4: return encode_launch<MAXB, 4, false>(ea, nblocks, none, s);
    case 8: return encode_launch<MAXB, 8, false>(ea, nblocks, none, s);
    case 12: return encode_launch<MAXB, 12, false>(ea, nblocks, none, s);
    case 16: return encode_launch<MAXB, 16, false>(ea, nblocks, none, s);
    default: return encode_launch<MAXB, 0, false>(ea, nblocks, none, s);
    }
}

template <int MAXB, int EC>
hipError_t decode_launch(const DecArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_decode<MAXB, EC>), dim3((unsigned)(a.n_blocks + 1)), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

template <int MAXB>
hipError_t decode_dispatch(const DecArgs &a, int ec, hipStream_t s)
{
    switch (ec) {
    case kByteShuffle: return decode_launch<MAXB, kByteShuffle>(a, s);
    case 1: return decode_launch<MAXB, 1>(a, s);
    case 2: return decode_launch<MAXB, 2>(a, s);
    case 4: return decode_launch<MAXB, 4>(a, s);
    case 8: return decode_launch<MAXB, 8>(a, s);
    case 12: return decode_launch<MAXB, 12>(a, s);
    case 16: return decode_launch<MAXB, 16>(a, s);
    default: return decode_launch<MAXB, 0>(a, s);
    }
}

} // namespace

int64_t compress_workspace(const Layout &L)
{
    const int64_t slot = (lz4_bound(L.block_bytes()) + 15) / 16 * 16;
    const int64_t n_tiles = (L.n_blocks + kTile - 1) / kTile;
    int64_t ws = L.n_blocks * slot;
    ws = (ws + 255) / 256 * 256 + ((L.n_blocks * 4 + 255) / 256) * 256;
    ws += ((n_tiles * 8 + 255) / 256) * 256;
    return ws > 0 ? ws : 256;
}

hipError_t launch_compress(const uint8_t *in, uint8_t *out, const Layout &L, int64_t cap,
                           int64_t *d_nbytes, void *ws, int64_t ws_bytes, const RoundParams *rp,
                           hipStream_t s, int filter)
{
    (void)ws_bytes;
    const int64_t slot = (lz4_bound(L.block_bytes()) + 15) / 16 * 16;
    const int64_t n_tiles = (L.n_blocks + kTile - 1) / kTile;
    uint8_t *w = static_cast<uint8_t *>(ws);
    uint8_t *slots = w;
    int64_t pos = (L.n_blocks * slot + 255) / 256 * 256;
    int32_t *sizes = reinterpret_cast<int32_t *>(w + pos);
    pos += ((L.n_blocks * 4 + 255) / 256) * 256;
    int64_t *tile_sum = reinterpret_cast<int64_t *>(w + pos);

    EncArgs ea{in, L.nb, L.E, L.n_full, L.last, slots, slot, sizes, 0};
    RoundParams none{};
    const int ec = filter == BSG_FILTER_BYTE ? kByteShuffle : element_class(L.E);
    hipError_t e = L.block_bytes() <= kSmallBlock
                       ? encode_dispatch<kSmallBlock>(ea, L.n_blocks, rp, ec, s)
                       : encode_dispatch<kLargeBlock>(ea, L.n_blocks, rp, ec, s);
    if (e != hipSuccess) return e;

    bsg_header hdr{filter == BSG_FILTER_BYTE ? BSG_MAGIC_BYTE : BSG_MAGIC, (uint32_t)L.E, (uint64_t)L.n, (uint32_t)L.nb, (uint32_t)L.n_blocks};
    const int64_t fixed = kHeaderBytes + 8 * (L.n_blocks + 1) + L.tail * L.E;
    if (n_tiles > 0) {
        hipLaunchKernelGGL(k_tile_sum, dim3((unsigned)n_tiles), dim3(256), 0, s, sizes, L.n_blocks,
                           tile_sum);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_tile_offsets, dim3(1), dim3(256), 0, s, tile_sum, n_tiles, fixed, cap,
                       d_nbytes, out, hdr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n_tiles > 0) {
        hipLaunchKernelGGL(k_write_offsets, dim3((unsigned)n_tiles), dim3(256), 0, s, sizes,
                           L.n_blocks, tile_sum, out);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const uint8_t *tail_src = in + (L.n - L.tail) * L.E;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)(L.n_blocks + 1)), dim3(kWave), 0, s, slots, slot,
                       sizes, L.n_blocks, out, d_nbytes, tail_src, L.tail * L.E,
                       rp ? *rp : none, rp ? 1 : 0, L.n - L.tail);
    return hipGetLastError();
}

hipError_t launch_decompress(const uint8_t *in, int64_t in_nbytes, uint8_t *out, const Layout &L,
                             int32_t *d_status, hipStream_t s, int filter)
{
    DecArgs a{in,     in_nbytes,  out,    L.n,        L.E,    L.nb, L.n_full,
              L.last, L.n_blocks, L.tail, d_status, ((uintptr_t)out % 16) == 0,
              filter == BSG_FILTER_BYTE ? BSG_MAGIC_BYTE : BSG_MAGIC};
    const int ec = filter == BSG_FILTER_BYTE ? kByteShuffle : element_class(L.E);
    return L.block_bytes() <= kSmallBlock ? decode_dispatch<kSmallBlock>(a, ec, s)
                                          : decode_dispatch<kLargeBlock>(a, ec, s);
}

} // namespace bsg
