// The C-ABI of the bsg library: argument checks on the host, then kernel
// launches on the caller's stream.  Nothing here allocates device memory.
#include <cmath>
#include <cstring>
#include <mutex>

#include "bsg_internal.hpp"

namespace bsg {

int64_t block_elems(int64_t E, int64_t block_size)
{
    if (E <= 0) return BSG_EINVAL;
    if (block_size == 0) {
        block_size = (kDefaultBlockBytes / E) / 8 * 8;
        if (block_size < 8) block_size = 8;
    }
    if (block_size < 8 || block_size % 8 != 0 || block_size > (int64_t)UINT32_MAX)
        return BSG_EINVAL;
    return block_size;
}

bool make_layout(int64_t n, int64_t E, int64_t block_size, Layout *L)
{
    const int64_t nb = block_elems(E, block_size);
    if (nb < 0 || n < 0) return false;
    L->n = n;
    L->E = E;
    L->nb = nb;
    L->n_full = n / nb;
    const int64_t rem = n - L->n_full * nb;
    L->last = rem - rem % 8;
    L->tail = rem % 8;
    L->n_blocks = L->n_full + (L->last > 0 ? 1 : 0);
    return true;
}

} // namespace bsg

using namespace bsg;

namespace {

inline int hip_status(hipError_t e) { return e == hipSuccess ? BSG_OK : BSG_EHIP; }

inline bool round_args_ok(int64_t F, int64_t I, int64_t T, double n_samples, double f)
{
    return F >= 0 && I >= 0 && T >= 0 && n_samples > 0.0 && std::isfinite(n_samples) &&
           f >= 0.0 && std::isfinite(f);
}

inline RoundParams make_round(const float *autos, const int32_t *prod_map, int64_t F, int64_t I,
                              int64_t T, double n_samples, double f)
{
    RoundParams rp;
    rp.autos = autos;
    rp.autos_i32 = nullptr;
    rp.fscale = nullptr;
    rp.prod_map = prod_map;
    rp.F = F;
    rp.I = I;
    rp.T = T;
    rp.P = I * (I + 1) / 2;
    // G2 = 12 f s^2: s^2 = V_ii V_jj / (2N) for crosses, V_ii^2 / N for autos
    rp.c = (12.0 * f) / (2.0 * n_samples);
    rp.c_auto = 2.0 * rp.c;
    return rp;
}

inline int64_t fixed_stream_bytes(const Layout &L)
{
    return kHeaderBytes + 8 * (L.n_blocks + 1) + L.tail * L.E;
}

// Compression scratch space for callers that cannot allocate: one array of
// fixed size in every GPU's copy of the code object.  In host code its name
// only stands for the symbol; the device address of each GPU's copy comes
// from hipGetSymbolAddress, made once per device with that device current.
__device__ __align__(256) uint8_t scratch[BSG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices]; // guarded by scratch_mu

// Device address of the current device's scratch array.
int scratch_for_current_device(void **ptr)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return BSG_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return BSG_EINVAL;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BSG_EHIP;
        scratch_ptr[dev] = p;
    }
    *ptr = scratch_ptr[dev];
    return BSG_OK;
}

} // namespace

extern "C" {

const char *bsg_strerror(int code)
{
    switch (code) {
    case BSG_OK: return "ok";
    case BSG_EINVAL: return "invalid argument";
    case BSG_ECAPACITY: return "output buffer or workspace too small";
    case BSG_ECORRUPT: return "corrupt or mismatched compressed stream";
    case BSG_EHIP: return "HIP runtime error";
    default: return "unknown error";
    }
}

int64_t bsg_block_elems(int64_t elem_size, int64_t block_size)
{
    return block_elems(elem_size, block_size);
}

int bsg_round_to_noise(const void *vis_in, void *vis_out, const float *autos, int64_t F,
                       int64_t I, int64_t T, const int32_t *prod_map, double n_samples, double f,
                       void *stream)
{
    if (!round_args_ok(F, I, T, n_samples, f)) return BSG_EINVAL;
    const int64_t P = I * (I + 1) / 2;
    if (F * P * T == 0) return BSG_OK;
    if (!vis_in || !vis_out || !autos) return BSG_EINVAL;
    if ((uintptr_t)vis_in % 8 || (uintptr_t)vis_out % 8 || (uintptr_t)autos % 4) return BSG_EINVAL;
    const RoundParams rp = make_round(autos, prod_map, F, I, T, n_samples, f);
    return hip_status(launch_round(static_cast<const float *>(vis_in), static_cast<float *>(vis_out),
                                   rp, static_cast<hipStream_t>(stream)));
}

int bsg_noise_compensation(const void *vis, const float *autos, int64_t F, int64_t I, int64_t T,
                           const int32_t *prod_map, double *scale, void *stream)
{
    if (F < 0 || I < 0 || T < 0) return BSG_EINVAL;
    if (F * T == 0) return BSG_OK;
    if (!scale || (uintptr_t)scale % 8) return BSG_EINVAL;
    const int64_t P = I * (I + 1) / 2;
    if (P > 0 && (!vis || !autos || (uintptr_t)vis % 8 || (uintptr_t)autos % 4)) return BSG_EINVAL;
    if (F > (int64_t)UINT32_MAX || (T + 63) / 64 > 65535) return BSG_EINVAL;
    const RoundParams rp = make_round(autos, prod_map, F, I, T, 1.0, 0.0);
    return hip_status(launch_noise_comp(static_cast<const float *>(vis), rp, scale,
                                        static_cast<hipStream_t>(stream)));
}

int bsg_round_to_noise_scaled(const void *vis_in, void *vis_out, const float *autos, int64_t F,
                              int64_t I, int64_t T, const int32_t *prod_map, double n_samples,
                              double f, const double *scale, void *stream)
{
    if (!round_args_ok(F, I, T, n_samples, f)) return BSG_EINVAL;
    const int64_t P = I * (I + 1) / 2;
    if (F * P * T == 0) return BSG_OK;
    if (!vis_in || !vis_out || !autos || !scale) return BSG_EINVAL;
    if ((uintptr_t)vis_in % 8 || (uintptr_t)vis_out % 8 || (uintptr_t)autos % 4 ||
        (uintptr_t)scale % 8)
        return BSG_EINVAL;
    RoundParams rp = make_round(autos, prod_map, F, I, T, n_samples, f);
    rp.fscale = scale;
    return hip_status(launch_round(static_cast<const float *>(vis_in), static_cast<float *>(vis_out),
                                   rp, static_cast<hipStream_t>(stream)));
}

int bsg_fullcov_inverse_diag(const void *vis, const float *autos, int64_t F, int64_t I,
                             int64_t T, double *qdiag, void *stream)
{
    if (F < 0 || I < 0 || T < 0 || I > fullcov_max_inputs()) return BSG_EINVAL;
    if (F * T * I == 0) return BSG_OK;
    if (!vis || !autos || !qdiag || (uintptr_t)vis % 8 || (uintptr_t)autos % 4 ||
        (uintptr_t)qdiag % 8 || F * T > (int64_t)INT32_MAX)
        return BSG_EINVAL;
    return hip_status(launch_fullcov(static_cast<const float *>(vis), autos, F, I, T, 0.0, nullptr,
                                     qdiag, static_cast<hipStream_t>(stream)));
}

int bsg_round_to_noise_fullcov(const void *vis_in, void *vis_out, const float *autos, int64_t F,
                               int64_t I, int64_t T, double n_samples, double f, void *stream)
{
    if (!round_args_ok(F, I, T, n_samples, f) || I > fullcov_max_inputs()) return BSG_EINVAL;
    if (F * T * I == 0) return BSG_OK;
    if (!vis_in || !vis_out || !autos || (uintptr_t)vis_in % 8 || (uintptr_t)vis_out % 8 ||
        (uintptr_t)autos % 4 || F * T > (int64_t)INT32_MAX)
        return BSG_EINVAL;
    const double c = (12.0 * f) / (2.0 * n_samples);
    return hip_status(launch_fullcov(static_cast<const float *>(vis_in), autos, F, I, T, c,
                                     static_cast<float *>(vis_out), nullptr,
                                     static_cast<hipStream_t>(stream)));
}

int bsg_round_to_noise_i32(const void *vis_in, void *vis_out, const int32_t *autos, int64_t F,
                           int64_t I, int64_t T, const int32_t *prod_map, double n_samples,
                           double f, void *stream)
{
    if (!round_args_ok(F, I, T, n_samples, f)) return BSG_EINVAL;
    const int64_t P = I * (I + 1) / 2;
    if (F * P * T == 0) return BSG_OK;
    if (!vis_in || !vis_out || !autos) return BSG_EINVAL;
    if ((uintptr_t)vis_in % 8 || (uintptr_t)vis_out % 8 || (uintptr_t)autos % 4) return BSG_EINVAL;
    RoundParams rp = make_round(nullptr, prod_map, F, I, T, n_samples, f);
    rp.autos_i32 = autos;
    return hip_status(launch_round_i32(static_cast<const int32_t *>(vis_in),
                                       static_cast<int32_t *>(vis_out), rp,
                                       static_cast<hipStream_t>(stream)));
}

static int shuffle_common(const void *in, void *out, int64_t n, int64_t E, int64_t block_size,
                          void *stream, bool inverse)
{
    Layout L;
    if (!make_layout(n, E, block_size, &L)) return BSG_EINVAL;
    if (n == 0) return BSG_OK;
    if (!in || !out) return BSG_EINVAL;
    return hip_status(launch_shuffle(static_cast<const uint8_t *>(in), static_cast<uint8_t *>(out),
                                     L, inverse, static_cast<hipStream_t>(stream)));
}

int bsg_byteshuffle(const void *in, void *out, int64_t n, int64_t elem_size, int64_t block_size,
                    void *stream)
{
    Layout L;
    if (!make_layout(n, elem_size, block_size, &L)) return BSG_EINVAL;
    if (n == 0) return BSG_OK;
    if (!in || !out || (uintptr_t)out % 4) return BSG_EINVAL;
    return hip_status(launch_byteshuffle(static_cast<const uint8_t *>(in),
                                         static_cast<uint8_t *>(out), L, false,
                                         static_cast<hipStream_t>(stream)));
}

int bsg_byteunshuffle(const void *in, void *out, int64_t n, int64_t elem_size,
                      int64_t block_size, void *stream)
{
    Layout L;
    if (!make_layout(n, elem_size, block_size, &L)) return BSG_EINVAL;
    if (n == 0) return BSG_OK;
    if (!in || !out || (uintptr_t)out % 4) return BSG_EINVAL;
    return hip_status(launch_byteshuffle(static_cast<const uint8_t *>(in),
                                         static_cast<uint8_t *>(out), L, true,
                                         static_cast<hipStream_t>(stream)));
}

int bsg_bitshuffle(const void *in, void *out, int64_t n, int64_t elem_size, int64_t block_size,
                   void *stream)
{
    return shuffle_common(in, out, n, elem_size, block_size, stream, false);
}

int bsg_bitunshuffle(const void *in, void *out, int64_t n, int64_t elem_size, int64_t block_size,
                     void *stream)
{
    return shuffle_common(in, out, n, elem_size, block_size, stream, true);
}

int64_t bsg_compress_bound(int64_t n, int64_t elem_size, int64_t block_size)
{
    Layout L;
    if (!make_layout(n, elem_size, block_size, &L)) return BSG_EINVAL;
    if (L.block_bytes() > BSG_MAX_BLOCK_BYTES) return BSG_EINVAL;
    int64_t b = fixed_stream_bytes(L) + L.n_full * lz4_bound(L.block_bytes());
    if (L.last) b += lz4_bound(L.last * L.E);
    return b;
}

int64_t bsg_compress_workspace_size(int64_t n, int64_t elem_size, int64_t block_size)
{
    Layout L;
    if (!make_layout(n, elem_size, block_size, &L)) return BSG_EINVAL;
    if (L.block_bytes() > BSG_MAX_BLOCK_BYTES) return BSG_EINVAL;
    return compress_workspace(L);
}

static int compress_common(const void *in, void *out, const Layout &L, int64_t out_capacity,
                           int64_t *d_out_nbytes, void *workspace, int64_t workspace_bytes,
                           const RoundParams *rp, void *stream, int filter = BSG_FILTER_BIT,
                           bool may_segment = true)
{
    if (filter != BSG_FILTER_BIT && filter != BSG_FILTER_BYTE) return BSG_EINVAL;
    if (L.block_bytes() > BSG_MAX_BLOCK_BYTES) return BSG_EINVAL;
    if (!out || !d_out_nbytes || !workspace || (L.n > 0 && !in)) return BSG_EINVAL;
    if ((uintptr_t)out % 8 || (uintptr_t)workspace % 256 || (uintptr_t)d_out_nbytes % 8)
        return BSG_EINVAL;
    if (workspace_bytes < compress_workspace(L)) return BSG_ECAPACITY;
    if (out_capacity < fixed_stream_bytes(L)) return BSG_ECAPACITY;
    return hip_status(launch_compress(static_cast<const uint8_t *>(in), static_cast<uint8_t *>(out),
                                      L, out_capacity, d_out_nbytes, workspace, workspace_bytes, rp,
                                      static_cast<hipStream_t>(stream), filter, may_segment));
}

int bsg_compress_lz4(const void *in, void *out, int64_t n, int64_t elem_size, int64_t block_size,
                     int64_t out_capacity, int64_t *d_out_nbytes, void *workspace,
                     int64_t workspace_bytes, void *stream)
{
    Layout L;
    if (!make_layout(n, elem_size, block_size, &L)) return BSG_EINVAL;
    return compress_common(in, out, L, out_capacity, d_out_nbytes, workspace, workspace_bytes,
                           nullptr, stream);
}

int bsg_compress_lz4_noalloc(const void *in, void *out, int64_t n, int64_t elem_size,
                             int64_t block_size, int64_t out_capacity, int64_t *d_out_nbytes,
                             void *stream)
{
    Layout L;
    if (!make_layout(n, elem_size, block_size, &L)) return BSG_EINVAL;
    if (L.block_bytes() > BSG_MAX_BLOCK_BYTES) return BSG_EINVAL;
    // every part of the scratch space is written before it is read, so the
    // previous call's contents need no clearing
    if (compress_workspace(L) > (int64_t)BSG_NOALLOC_SCRATCH_BYTES) return BSG_ECAPACITY;
    if (!out || !d_out_nbytes || (L.n > 0 && !in)) return BSG_EINVAL;
    void *ws = nullptr;
    const int st = scratch_for_current_device(&ws);
    if (st != BSG_OK) return st;
    return compress_common(in, out, L, out_capacity, d_out_nbytes, ws,
                           (int64_t)BSG_NOALLOC_SCRATCH_BYTES, nullptr, stream, BSG_FILTER_BIT,
                           false);
}

int bsg_compress_lz4_filter(const void *in, void *out, int64_t n, int64_t elem_size,
                            int64_t block_size, int32_t filter, int64_t out_capacity,
                            int64_t *d_out_nbytes, void *workspace, int64_t workspace_bytes,
                            void *stream)
{
    Layout L;
    if (!make_layout(n, elem_size, block_size, &L)) return BSG_EINVAL;
    return compress_common(in, out, L, out_capacity, d_out_nbytes, workspace, workspace_bytes,
                           nullptr, stream, filter);
}

int bsg_round_compress_lz4(const void *vis_in, const float *autos, int64_t F, int64_t I,
                           int64_t T, const int32_t *prod_map, double n_samples, double f,
                           int64_t block_size, void *out, int64_t out_capacity,
                           int64_t *d_out_nbytes, void *workspace, int64_t workspace_bytes,
                           void *stream)
{
    if (!round_args_ok(F, I, T, n_samples, f)) return BSG_EINVAL;
    const int64_t P = I * (I + 1) / 2;
    Layout L;
    if (!make_layout(2 * F * P * T, 4, block_size, &L)) return BSG_EINVAL;
    if (L.n > 0 && (!autos || (uintptr_t)vis_in % 8 || (uintptr_t)autos % 4)) return BSG_EINVAL;
    const RoundParams rp = make_round(autos, prod_map, F, I, T, n_samples, f);
    return compress_common(vis_in, out, L, out_capacity, d_out_nbytes, workspace,
                           workspace_bytes, &rp, stream);
}

static int decompress_common(const void *in, int64_t in_nbytes, void *out, int64_t n,
                             int64_t elem_size, int64_t block_size, int32_t *d_status,
                             void *stream, int filter)
{
    if (filter != BSG_FILTER_BIT && filter != BSG_FILTER_BYTE) return BSG_EINVAL;
    Layout L;
    if (!make_layout(n, elem_size, block_size, &L)) return BSG_EINVAL;
    if (L.block_bytes() > BSG_MAX_BLOCK_BYTES) return BSG_EINVAL;
    if (!in || !d_status || (n > 0 && !out)) return BSG_EINVAL;
    if ((uintptr_t)in % 8 || (uintptr_t)d_status % 4) return BSG_EINVAL;
    if (in_nbytes < fixed_stream_bytes(L)) return BSG_ECORRUPT;
    return hip_status(launch_decompress(static_cast<const uint8_t *>(in), in_nbytes,
                                        static_cast<uint8_t *>(out), L, d_status,
                                        static_cast<hipStream_t>(stream), filter));
}

int bsg_decompress_lz4(const void *in, int64_t in_nbytes, void *out, int64_t n, int64_t elem_size,
                       int64_t block_size, int32_t *d_status, void *stream)
{
    return decompress_common(in, in_nbytes, out, n, elem_size, block_size, d_status, stream,
                             BSG_FILTER_BIT);
}

int bsg_decompress_lz4_filter(const void *in, int64_t in_nbytes, void *out, int64_t n,
                              int64_t elem_size, int64_t block_size, int32_t filter,
                              int32_t *d_status, void *stream)
{
    return decompress_common(in, in_nbytes, out, n, elem_size, block_size, d_status, stream,
                             filter);
}

int bsg_read_header(const void *host_bytes, int64_t nbytes, bsg_header *hdr)
{
    if (!host_bytes || !hdr) return BSG_EINVAL;
    if (nbytes < kHeaderBytes) return BSG_ECORRUPT;
    std::memcpy(hdr, host_bytes, sizeof(bsg_header));
    if (hdr->magic != BSG_MAGIC && hdr->magic != BSG_MAGIC_BYTE) return BSG_ECORRUPT;
    return BSG_OK;
}

} // extern "C"
