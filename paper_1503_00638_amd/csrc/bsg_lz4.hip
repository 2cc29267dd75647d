// Stage 2b: per-block LZ4 after the bit transpose (Section 4.2 of Masui et
// al.: each block is transposed and compressed while it is still on chip;
// blocks are independent).  On gfx950 a block lives in LDS and one
// wavefront owns it.
//
// Compression = k_encode (transpose into LDS [+ fused rounding], LDS hash
// table, greedy parse, write to a bound-sized slot) -> k_tile_sum ->
// k_tile_offsets (one workgroup) -> k_write_offsets -> k_pack (copy slots to
// their final place, header, raw tail).  A large input is encoded in
// segments on two streams while a third stream scans and packs each
// finished segment, so the copy out of the slots runs under the encoding
// of the next segments (the encoder is bound by instruction issue, the
// copy by HBM).
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

template <int MAXB, int EC, int RM>
__global__ __launch_bounds__(64) void k_encode(EncArgs a, RoundParams rp)
{
    __shared__ EncLds<MAXB> L;
    const int64_t b = a.block0 + blockIdx.x;
    const int64_t elems = b < a.n_full ? a.nb : a.last;
    const int64_t first = b * a.nb;
    const int sz = encode_one<MAXB, EC, RM>(a.in + first * a.E, elems, a.E, rp, first,
                                               a.slots + b * a.slot_bytes, L);
    if (threadIdx.x == 0) a.sizes[b] = sz;
}

// tile_sum[k] = sum of sizes over blocks [k * kTile, (k + 1) * kTile)
__global__ __launch_bounds__(256) void k_tile_sum(const int32_t *__restrict__ sizes,
                                                  int64_t n_blocks, int64_t tile0,
                                                  int64_t *__restrict__ tile_sum)
{
    __shared__ int64_t sh[256];
    const int64_t tile = tile0 + blockIdx.x;
    const int64_t base = tile * kTile;
    int64_t s = 0;
    for (int k = threadIdx.x; k < kTile; k += 256)
        if (base + k < n_blocks) s += sizes[base + k];
    const int64_t inc = block_sum_i64(s, sh);
    if (threadIdx.x == 255) tile_sum[tile] = inc;
}

// One workgroup: exclusive scan of the tile sums of tiles [t0, t1) (in
// place) after the payload bytes of the tiles before t0 (*carry, 0 when t0 =
// 0); leaves the payload bytes up to t1 in *carry.  With last set: stream
// total, capacity verdict, stream header.
__global__ __launch_bounds__(256) void k_tile_offsets(int64_t *__restrict__ tile_sum,
                                                      int64_t t0, int64_t t1,
                                                      int64_t *__restrict__ carry_io, int last,
                                                      int64_t fixed_bytes, int64_t cap,
                                                      int64_t *__restrict__ d_nbytes,
                                                      uint8_t *__restrict__ out, bsg_header hdr)
{
    __shared__ int64_t sh[256];
    int64_t carry = t0 > 0 ? *carry_io : 0;
    for (int64_t base = t0; base < t1; base += 256) {
        const int64_t k = base + threadIdx.x;
        const int64_t v = k < t1 ? tile_sum[k] : 0;
        const int64_t inc = block_sum_i64(v, sh);
        if (k < t1) tile_sum[k] = carry + inc - v;
        carry += sh[255];
        __syncthreads();
    }
    if (threadIdx.x == 0 && !last) *carry_io = carry;
    if (threadIdx.x == 0 && last) {
        const int64_t total = fixed_bytes + carry;
        *d_nbytes = total <= cap ? total : (int64_t)BSG_ECAPACITY;
        *reinterpret_cast<bsg_header *>(out) = hdr;
        // payload length at the end of the offset table
        reinterpret_cast<uint64_t *>(out + kHeaderBytes)[hdr.n_blocks] = (uint64_t)carry;
    }
}

// off[b] for every block of a tile (written straight into the stream).
__global__ __launch_bounds__(256) void k_write_offsets(const int32_t *__restrict__ sizes,
                                                       int64_t n_blocks, int64_t tile0,
                                                       const int64_t *__restrict__ tile_off,
                                                       uint8_t *__restrict__ out)
{
    __shared__ int64_t sh[256];
    constexpr int PER = kTile / 256;
    const int64_t tile = tile0 + blockIdx.x;
    const int64_t base = tile * kTile + threadIdx.x * PER;
    int64_t v[PER];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = base + k < n_blocks ? sizes[base + k] : 0;
        s += v[k];
    }
    const int64_t inc = block_sum_i64(s, sh);
    int64_t o = tile_off[tile] + inc - s;
    uint64_t *off = reinterpret_cast<uint64_t *>(out + kHeaderBytes);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (base + k < n_blocks) off[base + k] = (uint64_t)o;
        o += v[k];
    }
}

// Copy the LZ4 bytes of blocks block0, block0 + 1, ... from their slots to
// the payload; block n_blocks (in the last launch) stands for the raw tail.
// Nothing is written past the output's capacity: a block whose bytes would
// end past payload_cap is skipped (the stream then does not fit and the
// call reports so), and the tail is written only when the stream fits
// (d_nbytes >= 0, known by the time the last launch runs).
__global__ __launch_bounds__(64) void k_pack(const uint8_t *__restrict__ slots, int64_t slot_bytes,
                                             const int32_t *__restrict__ sizes, int64_t n_blocks,
                                             int64_t block0, int64_t payload_cap,
                                             uint8_t *__restrict__ out,
                                             const int64_t *__restrict__ d_nbytes,
                                             const uint8_t *__restrict__ tail_src,
                                             int64_t tail_bytes, RoundParams rp, int round_tail,
                                             int64_t tail_first_elem)
{
    const int64_t b = block0 + blockIdx.x;
    const uint64_t *off = reinterpret_cast<const uint64_t *>(out + kHeaderBytes);
    uint8_t *payload = out + kHeaderBytes + 8 * (n_blocks + 1);
    const int lane = threadIdx.x;
    if (b == n_blocks) {
        if (*d_nbytes < 0) return;
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
    const uint64_t ob = off[b];
    const int sz = sizes[b];
    if ((int64_t)(ob + sz) > payload_cap) return;
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
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(dec_waves_per_eu<MAXB, EC>()))) void k_decode(DecArgs a)
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

template <int MAXB, int EC, int RM>
hipError_t encode_launch(const EncArgs &ea, int64_t nblocks, const RoundParams &rp,
                         hipStream_t s)
{
    if (nblocks == 0) return hipSuccess;
    hipLaunchKernelGGL((k_encode<MAXB, EC, RM>), dim3((unsigned)nblocks), dim3(kWave), 0, s, ea,
                       rp);
    return hipGetLastError();
}

template <int MAXB>
hipError_t encode_dispatch(const EncArgs &ea, int64_t nblocks, const RoundParams *rp, int ec,
                           hipStream_t s)
{
    const RoundParams none{};
    if (rp) {
        if (ec != 4) return encode_launch<MAXB, 0, kRoundPlain>(ea, nblocks, *rp, s);
        return rp->fscale ? encode_launch<MAXB, 4, kRoundScaled>(ea, nblocks, *rp, s)
                          : encode_launch<MAXB, 4, kRoundPlain>(ea, nblocks, *rp, s);
    }
    switch (ec) {
    case kByteShuffle: return encode_launch<MAXB, kByteShuffle, kRoundNone>(ea, nblocks, none, s);
    case 1: return encode_launch<MAXB, 1, kRoundNone>(ea, nblocks, none, s);
    case 2: return encode_launch<MAXB, 2, kRoundNone>(ea, nblocks, none, s);
    case 4: return encode_launch<MAXB, 4, kRoundNone>(ea, nblocks, none, s);
    case 8: return encode_launch<MAXB, 8, kRoundNone>(ea, nblocks, none, s);
    case 12: return encode_launch<MAXB, 12, kRoundNone>(ea, nblocks, none, s);
    case 16: return encode_launch<MAXB, 16, kRoundNone>(ea, nblocks, none, s);
    default: return encode_launch<MAXB, 0, kRoundNone>(ea, nblocks, none, s);
    }
}

// VGPRs of an encoder instance (from its kernel attributes, read once).
template <int MAXB, int EC, int RM> int encoder_vgprs()
{
    static const int regs = [] {
        hipFuncAttributes a{};
        return hipFuncGetAttributes(&a, reinterpret_cast<const void *>(&k_encode<MAXB, EC, RM>)) ==
                       hipSuccess
                   ? a.numRegs
                   : 1 << 20;
    }();
    return regs;
}

// The VGPRs of the instance encode_dispatch picks.
template <int MAXB> int encoder_vgprs_for(const RoundParams *rp, int ec)
{
    if (rp) {
        if (ec != 4) return encoder_vgprs<MAXB, 0, kRoundPlain>();
        return rp->fscale ? encoder_vgprs<MAXB, 4, kRoundScaled>()
                          : encoder_vgprs<MAXB, 4, kRoundPlain>();
    }
    switch (ec) {
    case kByteShuffle: return encoder_vgprs<MAXB, kByteShuffle, kRoundNone>();
    case 1: return encoder_vgprs<MAXB, 1, kRoundNone>();
    case 2: return encoder_vgprs<MAXB, 2, kRoundNone>();
    case 4: return encoder_vgprs<MAXB, 4, kRoundNone>();
    case 8: return encoder_vgprs<MAXB, 8, kRoundNone>();
    case 12: return encoder_vgprs<MAXB, 12, kRoundNone>();
    case 16: return encoder_vgprs<MAXB, 16, kRoundNone>();
    default: return encoder_vgprs<MAXB, 0, kRoundNone>();
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
    ws += 256; // the payload bytes carried from one segment to the next
    return ws;
}

constexpr int kMaxSeg = kSideEvents;     // segments of a large input
constexpr int64_t kSegMinBlocks = 8192; // ... of at least this many blocks
// Segments pay only when the encoder leaves registers for the pack waves
// beside its 4 resident waves per SIMD (LDS allows 16 per CU): at 112 VGPRs
// or fewer.  An encoder that fills the register file (125 VGPRs for 8-byte
// elements) lost 14 % to them, one at 84 gained 4 %.
constexpr int kSegMaxVgprs = 112;

namespace {
constexpr int kMaxSideDevices = 64;
std::mutex side_mu;
SideStreams side_dev[kMaxSideDevices]; // guarded by side_mu
} // namespace

hipError_t side_streams_begin(hipStream_t s, std::unique_lock<std::mutex> &lock,
                              SideStreams **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxSideDevices) return hipErrorInvalidDevice;
    lock = std::unique_lock<std::mutex>(side_mu);
    SideStreams &g = side_dev[dev];
    if (!g.made) {
        g.made = true;
        bool ok = hipStreamCreateWithFlags(&g.enc, hipStreamNonBlocking) == hipSuccess &&
                  hipStreamCreateWithFlags(&g.pack, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&g.fork, hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&g.join, hipEventDisableTiming) == hipSuccess;
        for (int i = 0; ok && i < kSideEvents; ++i)
            ok = hipEventCreateWithFlags(&g.done[i], hipEventDisableTiming) == hipSuccess;
        g.ok = ok;
    }
    if (!g.ok) return hipErrorOutOfMemory;
    if ((e = hipEventRecord(g.fork, s)) != hipSuccess ||
        (e = hipStreamWaitEvent(g.enc, g.fork, 0)) != hipSuccess ||
        (e = hipStreamWaitEvent(g.pack, g.fork, 0)) != hipSuccess)
        return e;
    *out = &g;
    return hipSuccess;
}

// (the encode stream is also joined directly, so that a stream capture sees
// it joined)
hipError_t side_streams_end(SideStreams *g, hipStream_t s, int last_enc)
{
    hipError_t e;
    if ((e = hipEventRecord(g->join, g->pack)) != hipSuccess ||
        (e = hipStreamWaitEvent(s, g->join, 0)) != hipSuccess)
        return e;
    if (last_enc >= 0 && (e = hipStreamWaitEvent(s, g->done[last_enc], 0)) != hipSuccess) return e;
    return hipSuccess;
}

hipError_t launch_compress(const uint8_t *in, uint8_t *out, const Layout &L, int64_t cap,
                           int64_t *d_nbytes, void *ws, int64_t ws_bytes, const RoundParams *rp,
                           hipStream_t s, int filter, bool may_segment)
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
    pos += ((n_tiles * 8 + 255) / 256) * 256;
    int64_t *carry = reinterpret_cast<int64_t *>(w + pos);

    RoundParams none{};
    const int ec = filter == BSG_FILTER_BYTE ? kByteShuffle : element_class(L.E);
    bsg_header hdr{filter == BSG_FILTER_BYTE ? BSG_MAGIC_BYTE : BSG_MAGIC, (uint32_t)L.E,
                   (uint64_t)L.n, (uint32_t)L.nb, (uint32_t)L.n_blocks};
    const int64_t fixed = kHeaderBytes + 8 * (L.n_blocks + 1) + L.tail * L.E;
    const uint8_t *tail_src = in + (L.n - L.tail) * L.E;

    // segments of whole tiles
    int nseg = (int)std::min<int64_t>(kMaxSeg, L.n_blocks / kSegMinBlocks);
    if (nseg > 1 && may_segment) {
        const int regs = L.block_bytes() <= kSmallBlock ? encoder_vgprs_for<kSmallBlock>(rp, ec)
                                                        : encoder_vgprs_for<kLargeBlock>(rp, ec);
        if (regs > kSegMaxVgprs) nseg = 1;
    }
    if (nseg < 1 || !may_segment) nseg = 1;
    std::unique_lock<std::mutex> lock;
    SideStreams *g = nullptr;
    hipError_t e;
    if (nseg > 1 && (e = side_streams_begin(s, lock, &g)) != hipSuccess) return e;
    hipStream_t ps = g ? g->pack : s;
    for (int i = 0; i < nseg; ++i) {
        const int64_t t0 = n_tiles * i / nseg, t1 = n_tiles * (i + 1) / nseg;
        const int64_t b0 = t0 * kTile, b1 = std::min(t1 * kTile, L.n_blocks);
        const bool last = i == nseg - 1;
        hipStream_t es = (g && (i & 1)) ? g->enc : s;
        EncArgs ea{in, L.nb, L.E, L.n_full, L.last, slots, slot, sizes, b0};
        e = L.block_bytes() <= kSmallBlock ? encode_dispatch<kSmallBlock>(ea, b1 - b0, rp, ec, es)
                                           : encode_dispatch<kLargeBlock>(ea, b1 - b0, rp, ec, es);
        if (e != hipSuccess) return e;
        if (g && ((e = hipEventRecord(g->done[i], es)) != hipSuccess ||
                  (e = hipStreamWaitEvent(ps, g->done[i], 0)) != hipSuccess))
            return e;
        if (t1 > t0) {
            hipLaunchKernelGGL(k_tile_sum, dim3((unsigned)(t1 - t0)), dim3(256), 0, ps, sizes,
                               L.n_blocks, t0, tile_sum);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_tile_offsets, dim3(1), dim3(256), 0, ps, tile_sum, t0, t1, carry,
                           last ? 1 : 0, fixed, cap, d_nbytes, out, hdr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (t1 > t0) {
            hipLaunchKernelGGL(k_write_offsets, dim3((unsigned)(t1 - t0)), dim3(256), 0, ps,
                               sizes, L.n_blocks, t0, tile_sum, out);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        const int64_t npack = b1 - b0 + (last ? 1 : 0);
        if (npack > 0) {
            hipLaunchKernelGGL(k_pack, dim3((unsigned)npack), dim3(kWave), 0, ps, slots, slot,
                               sizes, L.n_blocks, b0, cap - fixed, out, d_nbytes, tail_src,
                               L.tail * L.E, rp ? *rp : none, rp ? 1 : 0, L.n - L.tail);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    // (odd segments went to the encode stream)
    if (g) return side_streams_end(g, s, (nseg & 1) ? nseg - 2 : nseg - 1);
    return hipSuccess;
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
