// Batched compression / decompression of many independent chunks (each its
// own stream of the format in bsg.h) in a handful of launches: one
// persistent kernel per element-size class walks every block of every chunk
// of that class (chunks are independent units, like the blocks inside them,
// Section 4.2 of Masui et al.), then one global scan of the block sizes, a
// per-chunk finish (header, offsets, capacity verdict, raw tail) and one
// pack pass.  Nothing is allocated and nothing is synchronised with the
// host, so the whole sequence can be captured into a hipGraph.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "bsg_lz4_dev.hpp"

namespace bsg {

namespace {

constexpr int kMaxClasses = kSideEvents; // (one encode event per class)
// a batch of at least this many blocks splits its classes over two streams
constexpr int64_t kBatchSideMinBlocks = 16384;

struct BatchHeader {
    int32_t count, n_classes;
    int64_t total_blocks, slot_total;
};

struct BatchClass {
    int32_t ec, small, first_chunk, n_chunks; // ec: element class (0 = generic)
    int64_t first_block, n_blocks;
};

struct BatchChunk {
    const uint8_t *in;
    uint8_t *out;
    int64_t n, in_nbytes, out_capacity;
    int64_t nb, n_full, last, tail, n_blocks;
    int64_t block_start; // global index of the chunk's first block
    int64_t slot_start;  // byte offset of its first slot in the slot area
    int64_t slot_bytes;
    int32_t E, orig;     // element size, index in the caller's array
};

constexpr int64_t table_bytes(int64_t count)
{
    return (int64_t)sizeof(BatchHeader) + kMaxClasses * (int64_t)sizeof(BatchClass) +
           count * (int64_t)sizeof(BatchChunk);
}

struct TableView {
    const BatchHeader *h;
    const BatchClass *cls;
    const BatchChunk *ch;
    __host__ __device__ explicit TableView(const void *t)
        : h(reinterpret_cast<const BatchHeader *>(t)),
          cls(reinterpret_cast<const BatchClass *>(reinterpret_cast<const uint8_t *>(t) +
                                                    sizeof(BatchHeader))),
          ch(reinterpret_cast<const BatchChunk *>(reinterpret_cast<const uint8_t *>(t) +
                                                  sizeof(BatchHeader) +
                                                  kMaxClasses * sizeof(BatchClass)))
    {
    }
};

// The chunk (in table order, within [lo, hi]) that owns global block g: the
// last one whose first block is <= g.  A chunk without blocks shares its
// first-block index with the chunk after it, which the search prefers, so it
// is never chosen.
__device__ __forceinline__ int find_chunk(const BatchChunk *ch, int lo, int hi, int64_t g)
{
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ch[mid].block_start <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The blocks of a class that one workgroup of a persistent launch takes, in
// increasing order: every gridDim.x-th block from blockIdx.x
// (BSG_SCHED_STRIDED), or one contiguous range of ceil(n / gridDim.x) blocks
// (BSG_SCHED_RANGES).  Either way every block is taken by exactly one
// workgroup, so the output does not depend on the schedule.
struct BlockWalk {
    int64_t first, end, step;
    __device__ BlockWalk(const BatchClass &C, int schedule)
    {
        const int64_t n = C.n_blocks;
        if (schedule == BSG_SCHED_RANGES) {
            const int64_t per = (n + gridDim.x - 1) / gridDim.x;
            const int64_t lo = (int64_t)blockIdx.x * per < n ? (int64_t)blockIdx.x * per : n;
            first = C.first_block + lo;
            end = C.first_block + (lo + per < n ? lo + per : n);
            step = 1;
        } else {
            first = C.first_block + blockIdx.x;
            end = C.first_block + n;
            step = gridDim.x;
        }
    }
};

// The chunk owning block g, given the chunk c of an earlier block of the
// same walk (blocks only grow): under the range schedule the walk steps
// through the table, one read per block; under the strided one it searches
// the rest of the table.
__device__ __forceinline__ int next_chunk(const BatchChunk *ch, int c, int last, int64_t g,
                                          int64_t step)
{
    if (step == 1) {
        while (c < last && ch[c + 1].block_start <= g) ++c;
        return c;
    }
    return find_chunk(ch, c, last, g);
}

template <int MAXB, int EC>
__global__ __launch_bounds__(64) void k_batch_encode(const uint8_t *__restrict__ table, int cls,
                                                     uint8_t *__restrict__ slots,
                                                     int32_t *__restrict__ sizes, int schedule)
{
    __shared__ EncLds<MAXB> L;
    const TableView T(table);
    const BatchClass C = T.cls[cls];
    const RoundParams none{};
    const BlockWalk W(C, schedule);
    const int last = C.first_chunk + C.n_chunks - 1;
    int c = W.first < W.end ? find_chunk(T.ch, C.first_chunk, last, W.first) : C.first_chunk;
    for (int64_t g = W.first; g < W.end; g += W.step) {
        c = next_chunk(T.ch, c, last, g, W.step);
        const BatchChunk &ch = T.ch[c];
        const int64_t local = g - ch.block_start;
        const int64_t elems = local < ch.n_full ? ch.nb : ch.last;
        const int sz = encode_one<MAXB, EC, kRoundNone>(ch.in + local * ch.nb * ch.E, elems, ch.E, none, 0,
                                                   slots + ch.slot_start + local * ch.slot_bytes, L);
        if (threadIdx.x == 0) sizes[g] = sz;
    }
}

template <int MAXB, int EC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(dec_waves_per_eu<MAXB, EC>()))) void k_batch_decode(const uint8_t *__restrict__ table, int cls,
                                                     int32_t *__restrict__ status, int schedule)
{
    __shared__ DecLds<MAXB> L;
    const TableView T(table);
    const BatchClass C = T.cls[cls];
    const BlockWalk W(C, schedule);
    const int last = C.first_chunk + C.n_chunks - 1;
    int c = W.first < W.end ? find_chunk(T.ch, C.first_chunk, last, W.first) : C.first_chunk;
    for (int64_t g = W.first; g < W.end; g += W.step) {
        c = next_chunk(T.ch, c, last, g, W.step);
        const BatchChunk &ch = T.ch[c];
        const int64_t local = g - ch.block_start;
        const int64_t elems = local < ch.n_full ? ch.nb : ch.last;
        const int64_t table_end = kHeaderBytes + 8 * (ch.n_blocks + 1);
        const int64_t payload_len = ch.in_nbytes - table_end - ch.tail * ch.E;
        bool ok = payload_len >= 0;
        if (ok) {
            uint8_t *dst = ch.out + local * ch.nb * ch.E;
            ok = decode_one<MAXB, EC>(ch.in + table_end, payload_len,
                                      reinterpret_cast<const uint64_t *>(ch.in + kHeaderBytes),
                                      local, elems, ch.E, ch.in + ch.in_nbytes, dst,
                                      ((uintptr_t)ch.out % 16) == 0, L);
        }
        if (!ok && threadIdx.x == 0) atomicCAS(&status[ch.orig], 0, BSG_ECORRUPT);
    }
}

// One wavefront per chunk: header check and raw tail of each stream.
__global__ __launch_bounds__(64) void k_batch_dec_tail(const uint8_t *__restrict__ table,
                                                       int32_t *__restrict__ status)
{
    const TableView T(table);
    const BatchChunk &ch = T.ch[blockIdx.x];
    const int64_t table_end = kHeaderBytes + 8 * (ch.n_blocks + 1);
    const int64_t tail_bytes = ch.tail * ch.E;
    const int64_t payload_len = ch.in_nbytes - table_end - tail_bytes;
    if (payload_len < 0 || !header_ok(ch.in, payload_len, ch.n, ch.E, ch.nb, ch.n_blocks)) {
        if (threadIdx.x == 0) atomicCAS(&status[ch.orig], 0, BSG_ECORRUPT);
        return;
    }
    uint8_t *dst = ch.out + (ch.n - ch.tail) * ch.E;
    for (int64_t i = threadIdx.x; i < tail_bytes; i += kWave) dst[i] = ch.in[table_end + payload_len + i];
}

// ---- exclusive prefix of the block sizes, one element class at a time ----
// Blocks [b0, b0 + n) (a class); tile k holds blocks b0 + k kTile .. .
__global__ __launch_bounds__(256) void k_btile_sum(const int32_t *__restrict__ sizes, int64_t b0,
                                                   int64_t n, int64_t *__restrict__ tile_sum)
{
    __shared__ int64_t sh[256];
    const int64_t base = int64_t(blockIdx.x) * kTile;
    int64_t s = 0;
    for (int k = threadIdx.x; k < kTile; k += 256)
        if (base + k < n) s += sizes[b0 + base + k];
    const int64_t inc = block_sum_i64(s, sh);
    if (threadIdx.x == 255) tile_sum[blockIdx.x] = inc;
}

// In place, after the bytes of the classes before (*carry, 0 for the
// first); leaves the bytes up to the end of this class in *carry.
__global__ __launch_bounds__(256) void k_btile_scan(int64_t *__restrict__ tile_sum, int64_t n_tiles,
                                                    int64_t *__restrict__ carry_io, int first)
{
    __shared__ int64_t sh[256];
    int64_t carry = first ? 0 : *carry_io;
    for (int64_t base = 0; base < n_tiles; base += 256) {
        const int64_t k = base + threadIdx.x;
        const int64_t v = k < n_tiles ? tile_sum[k] : 0;
        const int64_t inc = block_sum_i64(v, sh);
        if (k < n_tiles) tile_sum[k] = carry + inc - v;
        carry += sh[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) *carry_io = carry;
}

__global__ __launch_bounds__(256) void k_bprefix(const int32_t *__restrict__ sizes, int64_t b0,
                                                 int64_t n, const int64_t *__restrict__ tile_off,
                                                 int64_t *__restrict__ prefix)
{
    __shared__ int64_t sh[256];
    constexpr int PER = kTile / 256;
    const int64_t base = int64_t(blockIdx.x) * kTile + threadIdx.x * PER;
    int64_t v[PER];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = base + k < n ? sizes[b0 + base + k] : 0;
        s += v[k];
    }
    const int64_t inc = block_sum_i64(s, sh);
    int64_t o = tile_off[blockIdx.x] + inc - s;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (base + k <= n) prefix[b0 + base + k] = o; // prefix[b0 + n] = end of the class
        o += v[k];
    }
}

// One wavefront per chunk: stream length and capacity verdict, header,
// offsets table and raw tail.
__global__ __launch_bounds__(64) void k_batch_finish(const uint8_t *__restrict__ table, int chunk0,
                                                     const int64_t *__restrict__ prefix,
                                                     int64_t *__restrict__ d_nbytes)
{
    const TableView T(table);
    const BatchChunk &ch = T.ch[chunk0 + blockIdx.x];
    const int lane = threadIdx.x;
    const int64_t base = prefix[ch.block_start];
    const int64_t pay = prefix[ch.block_start + ch.n_blocks] - base;
    const int64_t table_end = kHeaderBytes + 8 * (ch.n_blocks + 1);
    const int64_t tail_bytes = ch.tail * ch.E;
    const int64_t total = table_end + pay + tail_bytes;
    const bool fits = total <= ch.out_capacity;
    if (lane == 0) d_nbytes[ch.orig] = fits ? total : (int64_t)BSG_ECAPACITY;
    if (!fits) return;
    if (lane == 0) {
        bsg_header hdr{BSG_MAGIC, (uint32_t)ch.E, (uint64_t)ch.n, (uint32_t)ch.nb,
                       (uint32_t)ch.n_blocks};
        *reinterpret_cast<bsg_header *>(ch.out) = hdr;
    }
    uint64_t *off = reinterpret_cast<uint64_t *>(ch.out + kHeaderBytes);
    for (int64_t k = lane; k <= ch.n_blocks; k += kWave)
        off[k] = (uint64_t)(prefix[ch.block_start + k] - base);
    const uint8_t *tsrc = ch.in + (ch.n - ch.tail) * ch.E;
    uint8_t *tdst = ch.out + table_end + pay;
    for (int64_t i = lane; i < tail_bytes; i += kWave) tdst[i] = tsrc[i];
}

// The LZ4 bytes of a class's blocks from their slots to their places in
// their chunks' streams.
__global__ __launch_bounds__(64) void k_batch_pack(const uint8_t *__restrict__ table, int cls,
                                                   const uint8_t *__restrict__ slots,
                                                   const int32_t *__restrict__ sizes,
                                                   const int64_t *__restrict__ prefix,
                                                   const int64_t *__restrict__ d_nbytes)
{
    const TableView T(table);
    const BatchClass C = T.cls[cls];
    const int last = C.first_chunk + C.n_chunks - 1;
    for (int64_t g = C.first_block + blockIdx.x; g < C.first_block + C.n_blocks; g += gridDim.x) {
        const int c = find_chunk(T.ch, C.first_chunk, last, g);
        const BatchChunk &ch = T.ch[c];
        if (d_nbytes[ch.orig] < 0) continue;
        const int64_t local = g - ch.block_start;
        copy_slot(ch.out + kHeaderBytes + 8 * (ch.n_blocks + 1) + (prefix[g] - prefix[ch.block_start]),
                  slots + ch.slot_start + local * ch.slot_bytes, sizes[g]);
    }
}

int cu_count()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        return 256;
    return n;
}

int64_t persistent_grid(int64_t n_blocks, int waves_per_cu)
{
    const int64_t g = (int64_t)cu_count() * (waves_per_cu > 0 ? waves_per_cu : 16);
    return n_blocks < g ? n_blocks : g;
}

template <int MAXB, int EC>
hipError_t launch_benc(const uint8_t *d_table, int cls, int64_t nblk, int wpc, int sched,
                       uint8_t *slots, int32_t *sizes, hipStream_t s)
{
    hipLaunchKernelGGL((k_batch_encode<MAXB, EC>), dim3((unsigned)persistent_grid(nblk, wpc)),
                       dim3(kWave), 0, s, d_table, cls, slots, sizes, sched);
    return hipGetLastError();
}

template <int MAXB, int EC>
hipError_t launch_bdec(const uint8_t *d_table, int cls, int64_t nblk, int wpc, int sched,
                       int32_t *status, hipStream_t s)
{
    hipLaunchKernelGGL((k_batch_decode<MAXB, EC>), dim3((unsigned)persistent_grid(nblk, wpc)),
                       dim3(kWave), 0, s, d_table, cls, status, sched);
    return hipGetLastError();
}

template <int MAXB>
hipError_t benc_dispatch(int ec, const uint8_t *t, int cls, int64_t nblk, int wpc, int sched,
                         uint8_t *slots, int32_t *sizes, hipStream_t s)
{
    switch (ec) {
    case 1: return launch_benc<MAXB, 1>(t, cls, nblk, wpc, sched, slots, sizes, s);
    case 2: return launch_benc<MAXB, 2>(t, cls, nblk, wpc, sched, slots, sizes, s);
    case 4: return launch_benc<MAXB, 4>(t, cls, nblk, wpc, sched, slots, sizes, s);
    case 8: return launch_benc<MAXB, 8>(t, cls, nblk, wpc, sched, slots, sizes, s);
    case 12: return launch_benc<MAXB, 12>(t, cls, nblk, wpc, sched, slots, sizes, s);
    case 16: return launch_benc<MAXB, 16>(t, cls, nblk, wpc, sched, slots, sizes, s);
    default: return launch_benc<MAXB, 0>(t, cls, nblk, wpc, sched, slots, sizes, s);
    }
}

template <int MAXB>
hipError_t bdec_dispatch(int ec, const uint8_t *t, int cls, int64_t nblk, int wpc, int sched,
                         int32_t *status, hipStream_t s)
{
    switch (ec) {
    case 1: return launch_bdec<MAXB, 1>(t, cls, nblk, wpc, sched, status, s);
    case 2: return launch_bdec<MAXB, 2>(t, cls, nblk, wpc, sched, status, s);
    case 4: return launch_bdec<MAXB, 4>(t, cls, nblk, wpc, sched, status, s);
    case 8: return launch_bdec<MAXB, 8>(t, cls, nblk, wpc, sched, status, s);
    case 12: return launch_bdec<MAXB, 12>(t, cls, nblk, wpc, sched, status, s);
    case 16: return launch_bdec<MAXB, 16>(t, cls, nblk, wpc, sched, status, s);
    default: return launch_bdec<MAXB, 0>(t, cls, nblk, wpc, sched, status, s);
    }
}

struct WsLayout {
    int64_t slots, sizes, prefix, tiles, carry, total;
};

WsLayout ws_layout(const BatchHeader &h)
{
    auto up = [](int64_t x) { return (x + 255) / 256 * 256; };
    const int64_t n_tiles = (h.total_blocks + kTile - 1) / kTile;
    WsLayout w;
    w.slots = 0;
    w.sizes = up(h.slot_total);
    w.prefix = w.sizes + up(4 * h.total_blocks);
    w.tiles = w.prefix + up(8 * (h.total_blocks + 1 + kTile));
    w.carry = w.tiles + up(8 * (n_tiles + 1));
    w.total = w.carry + 256;
    return w;
}

inline int hip_status(hipError_t e) { return e == hipSuccess ? BSG_OK : BSG_EHIP; }

} // namespace
} // namespace bsg

using namespace bsg;

extern "C" {

int64_t bsg_batch_table_bytes(int32_t count)
{
    return count < 0 ? BSG_EINVAL : table_bytes(count);
}

int bsg_batch_build_table(const bsg_chunk *chunks, int32_t count, void *host_table,
                          int64_t host_table_bytes)
{
    if (count < 0 || (count > 0 && !chunks) || !host_table ||
        host_table_bytes < table_bytes(count))
        return BSG_EINVAL;
    std::vector<BatchChunk> rows(count);
    std::vector<int> key(count);
    for (int i = 0; i < count; ++i) {
        const bsg_chunk &c = chunks[i];
        Layout L;
        if (!make_layout(c.n, c.elem_size, c.block_size, &L)) return BSG_EINVAL;
        if (L.block_bytes() > BSG_MAX_BLOCK_BYTES) return BSG_EINVAL;
        BatchChunk &r = rows[i];
        std::memset(&r, 0, sizeof(r));
        r.in = static_cast<const uint8_t *>(c.in);
        r.out = static_cast<uint8_t *>(c.out);
        r.n = c.n;
        r.in_nbytes = c.in_nbytes;
        r.out_capacity = c.out_capacity;
        r.nb = L.nb;
        r.n_full = L.n_full;
        r.last = L.last;
        r.tail = L.tail;
        r.n_blocks = L.n_blocks;
        r.slot_bytes = (lz4_bound(L.block_bytes()) + 15) / 16 * 16;
        r.E = (int32_t)c.elem_size;
        r.orig = i;
        // class key: element class, and whether blocks fit the 8 KiB LDS kernel
        key[i] = element_class(c.elem_size) * 2 + (L.block_bytes() <= kSmallBlock ? 0 : 1);
    }
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
    uint8_t *t = static_cast<uint8_t *>(host_table);
    std::memset(t, 0, (size_t)table_bytes(count));
    BatchHeader &h = *reinterpret_cast<BatchHeader *>(t);
    BatchClass *cls = reinterpret_cast<BatchClass *>(t + sizeof(BatchHeader));
    BatchChunk *ch = reinterpret_cast<BatchChunk *>(t + sizeof(BatchHeader) +
                                                    kMaxClasses * sizeof(BatchClass));
    int64_t blk = 0, slot = 0;
    int nc = 0;
    for (int k = 0; k < count; ++k) {
        BatchChunk r = rows[order[k]];
        if (k == 0 || key[order[k]] != key[order[k - 1]]) {
            BatchClass &C = cls[nc++]; // at most 7 element classes x 2 sizes
            C.ec = key[order[k]] / 2;
            C.small = key[order[k]] % 2 == 0;
            C.first_chunk = k;
            C.first_block = blk;
        }
        BatchClass &C = cls[nc - 1];
        C.n_chunks = k - C.first_chunk + 1;
        r.block_start = blk;
        r.slot_start = slot;
        blk += r.n_blocks;
        slot += r.n_blocks * r.slot_bytes;
        C.n_blocks = blk - C.first_block;
        ch[k] = r;
    }
    h.count = count;
    h.n_classes = nc;
    h.total_blocks = blk;
    h.slot_total = slot;
    return BSG_OK;
}

int64_t bsg_batch_workspace_size(const void *host_table)
{
    if (!host_table) return BSG_EINVAL;
    return ws_layout(*reinterpret_cast<const BatchHeader *>(host_table)).total;
}

int bsg_batch_compress(const void *host_table, const void *d_table, int64_t *d_nbytes,
                       void *workspace, int64_t workspace_bytes, int32_t waves_per_cu,
                       int32_t schedule, void *stream)
{
    if (!host_table || !d_table || !d_nbytes || !workspace) return BSG_EINVAL;
    if (schedule != BSG_SCHED_STRIDED && schedule != BSG_SCHED_RANGES) return BSG_EINVAL;
    if ((uintptr_t)workspace % 256 || (uintptr_t)d_table % 16 || (uintptr_t)d_nbytes % 8)
        return BSG_EINVAL;
    const TableView T(host_table);
    const BatchHeader &h = *T.h;
    const WsLayout w = ws_layout(h);
    if (workspace_bytes < w.total) return BSG_ECAPACITY;
    for (int i = 0; i < h.count; ++i)
        if ((T.ch[i].n > 0 && !T.ch[i].in) || !T.ch[i].out || (uintptr_t)T.ch[i].out % 8)
            return BSG_EINVAL;
    if (h.count == 0) return BSG_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint8_t *t = static_cast<const uint8_t *>(d_table);
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    uint8_t *slots = ws + w.slots;
    int32_t *sizes = reinterpret_cast<int32_t *>(ws + w.sizes);
    int64_t *prefix = reinterpret_cast<int64_t *>(ws + w.prefix);
    int64_t *tiles = reinterpret_cast<int64_t *>(ws + w.tiles);
    int64_t *carry = reinterpret_cast<int64_t *>(ws + w.carry);
    // Class by class: the encode on the caller's stream or (every other
    // class) the library's encode stream; then on the pack stream the
    // class's scan (after the bytes of the classes before), finish and pack,
    // which run beside the next classes' encodes.
    int nonempty = 0;
    for (int c = 0; c < h.n_classes; ++c) nonempty += T.cls[c].n_blocks > 0;
    std::unique_lock<std::mutex> lock;
    SideStreams *g = nullptr;
    if (nonempty >= 2 && h.total_blocks >= kBatchSideMinBlocks &&
        side_streams_begin(s, lock, &g) != hipSuccess)
        return BSG_EHIP;
    hipStream_t ps = g ? g->pack : s;
    int i = 0, last_enc = -1;
    for (int c = 0; c < h.n_classes; ++c) {
        const BatchClass &C = T.cls[c];
        if (C.n_blocks > 0) {
            hipStream_t es = (g && (i & 1)) ? g->enc : s;
            const hipError_t e =
                C.small ? benc_dispatch<kSmallBlock>(C.ec, t, c, C.n_blocks, waves_per_cu,
                                                     schedule, slots, sizes, es)
                        : benc_dispatch<kLargeBlock>(C.ec, t, c, C.n_blocks, waves_per_cu,
                                                     schedule, slots, sizes, es);
            if (e != hipSuccess) return BSG_EHIP;
            if (g) {
                if (hipEventRecord(g->done[i], es) != hipSuccess ||
                    hipStreamWaitEvent(ps, g->done[i], 0) != hipSuccess)
                    return BSG_EHIP;
                if (i & 1) last_enc = i;
            }
            ++i;
        }
        const int64_t nt = (C.n_blocks + kTile - 1) / kTile + 1; // + room for the class's end
        hipLaunchKernelGGL(k_btile_sum, dim3((unsigned)nt), dim3(256), 0, ps, sizes, C.first_block,
                           C.n_blocks, tiles);
        hipLaunchKernelGGL(k_btile_scan, dim3(1), dim3(256), 0, ps, tiles, nt, carry, c == 0 ? 1 : 0);
        hipLaunchKernelGGL(k_bprefix, dim3((unsigned)nt), dim3(256), 0, ps, sizes, C.first_block,
                           C.n_blocks, tiles, prefix);
        if (C.n_chunks > 0)
            hipLaunchKernelGGL(k_batch_finish, dim3((unsigned)C.n_chunks), dim3(kWave), 0, ps, t,
                               C.first_chunk, prefix, d_nbytes);
        if (C.n_blocks > 0)
            hipLaunchKernelGGL(k_batch_pack, dim3((unsigned)persistent_grid(C.n_blocks, waves_per_cu)),
                               dim3(kWave), 0, ps, t, c, slots, sizes, prefix, d_nbytes);
        if (hipGetLastError() != hipSuccess) return BSG_EHIP;
    }
    if (g && side_streams_end(g, s, last_enc) != hipSuccess) return BSG_EHIP;
    return BSG_OK;
}

int bsg_batch_decompress(const void *host_table, const void *d_table, int32_t *d_status,
                         int32_t waves_per_cu, int32_t schedule, void *stream)
{
    if (!host_table || !d_table || !d_status || (uintptr_t)d_table % 16 || (uintptr_t)d_status % 4)
        return BSG_EINVAL;
    if (schedule != BSG_SCHED_STRIDED && schedule != BSG_SCHED_RANGES) return BSG_EINVAL;
    const TableView T(host_table);
    const BatchHeader &h = *T.h;
    for (int i = 0; i < h.count; ++i)
        if (!T.ch[i].in || (uintptr_t)T.ch[i].in % 8 || (T.ch[i].n > 0 && !T.ch[i].out))
            return BSG_EINVAL;
    if (h.count == 0) return BSG_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint8_t *t = static_cast<const uint8_t *>(d_table);
    hipError_t e = hipSuccess;
    for (int c = 0; c < h.n_classes && e == hipSuccess; ++c) {
        const BatchClass &C = T.cls[c];
        if (C.n_blocks == 0) continue;
        e = C.small ? bdec_dispatch<kSmallBlock>(C.ec, t, c, C.n_blocks, waves_per_cu, schedule,
                                                 d_status, s)
                    : bdec_dispatch<kLargeBlock>(C.ec, t, c, C.n_blocks, waves_per_cu, schedule,
                                                 d_status, s);
    }
    if (e != hipSuccess) return BSG_EHIP;
    hipLaunchKernelGGL(k_batch_dec_tail, dim3((unsigned)h.count), dim3(kWave), 0, s, t, d_status);
    return hip_status(hipGetLastError());
}

} // extern "C"
