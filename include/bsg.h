/*
 * bsg: GPU (gfx950) implementation of the two-stage compression scheme for
 * radio visibilities of Masui et al., "A compression scheme for radio data in
 * high performance computing", arXiv:1503.00638:
 *
 *   1. noise-relative precision reduction (Section 3): every visibility is
 *      rounded to a multiple of the largest power of two g with
 *      g^2 < 12 f s^2, s from the diagonal radiometer equation (Section 3.1);
 *   2. Bitshuffle (Section 4.2): the bits of each fixed-size block of typed
 *      elements are transposed (element x bit matrix -> bit planes), then each
 *      block is compressed on its own with LZ4.
 *
 * Conventions for every entry point:
 *  - Data pointers are DEVICE pointers.  The caller allocates and owns every
 *    buffer; the library never allocates on these paths.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *    enqueues work on it and returns; results are ready when the stream is.
 *  - The int return value reports argument and launch checks made on the host
 *    (BSG_OK or a negative BSG_E* code).  Results that depend on the data
 *    (compressed size, decode status) are written to caller-provided device
 *    words.
 *  - Calls on different streams may run concurrently (the paper's
 *    thread-safety requirement, Section 2 and Section 4.2).  The only state
 *    the library keeps is made once per device and guarded by locks: the
 *    two streams and their events of the segmented compression
 *    (bsg_compress_lz4) and the scratch array of bsg_compress_lz4_noalloc.
 *  - block_size is counted in ELEMENTS and must be a multiple of 8; 0 selects
 *    the default, 8192 bytes' worth of elements rounded down to a multiple of 8.
 *    A block of n_B elements is transposed as an (n_B x 8E) bit matrix.  The
 *    buffer is cut into floor(n / n_B) full blocks, one partial block of
 *    floor(rem / 8) * 8 elements when that is non-zero, and a raw tail of the
 *    last n mod 8 elements which is copied verbatim.
 */
#ifndef BSG_H
#define BSG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BSG_OK 0
#define BSG_EINVAL (-1)    /* invalid argument */
#define BSG_ECAPACITY (-2) /* output buffer or workspace too small */
#define BSG_ECORRUPT (-3)  /* compressed stream is corrupt or does not match */
#define BSG_EHIP (-4)      /* a HIP runtime call failed */

#define BSG_MAX_BLOCK_BYTES 65536 /* LZ4 offsets are 16-bit */

/* Compressed stream layout (all little-endian):
 *   bsg_header (24 bytes)
 *   uint64 off[n_blocks + 1]   LZ4 block k occupies payload[off[k], off[k+1])
 *   payload: the LZ4 blocks, concatenated, off[0] = 0
 *   raw tail: the last (n mod 8) elements, verbatim                       */
#define BSG_MAGIC 0x31475342u /* bytes "BSG1" */
#define BSG_MAGIC_BYTE 0x31425342u /* bytes "BSB1": byte-shuffled stream */

/* Block filters applied before LZ4: the bit transpose of Section 4.2 (the
 * method), or the byte shuffle of Blosc-style compressors (the comparison
 * of Section 4.1 and Table t:performance): byte k of element i of a block
 * goes to byte k * n_B + i. */
#define BSG_FILTER_BIT 0
#define BSG_FILTER_BYTE 1
typedef struct bsg_header {
    uint32_t magic;
    uint32_t elem_size;
    uint64_t n;          /* elements */
    uint32_t block_elems;
    uint32_t n_blocks;
} bsg_header;

const char *bsg_strerror(int code);

/* Elements per block for a given block_size argument (0 = default), or
 * BSG_EINVAL. Host only. */
int64_t bsg_block_elems(int64_t elem_size, int64_t block_size);

/* ---- Stage 1: precision reduction (Section 3.1, Section 3.2) ----------
 * vis_in / vis_out: complex64 [F][P][T] (re, im float32 pairs), C order,
 *   time fastest; vis_out may equal vis_in (in place).  8-byte aligned.
 * autos: float32 [F][I][T], the measured auto-correlations V_ii (the real
 *   parts of the auto products BEFORE rounding); must not overlap vis_out.
 * P = I (I + 1) / 2 products.  prod_map: NULL for upper-triangle row-major
 *   order ((0,0), (0,1), ..., (0,I-1), (1,1), ...), else a device int32
 *   [P][2] table of (i, j) with 0 <= i, j < I (i == j marks an auto).
 * n_samples: N = bandwidth x integration time (> 0).  f: the tolerated
 *   fractional increase of the noise variance (>= 0; 0 leaves data as is).
 * Per element: G2 = (V_ii V_jj) c for i != j and (V_ii V_ii) 2c for autos,
 *   c = (12 f) / (2 N) in IEEE double (the product of two floats is exact);
 *   k = the largest integer with 4^k < G2; re and im are rounded to the
 *   nearest multiple of 2^k, ties to even; the imaginary part of an auto is
 *   copied.  G2 not positive and finite (f = 0, a zero or NaN auto, autos
 *   of opposite sign) leaves the element unchanged; NaN and Inf values pass through; the sign
 *   of zero is kept.
 * Errors: BSG_EINVAL for negative sizes, NULL pointers with a non-empty
 *   array, n_samples <= 0 or f < 0 or non-finite; BSG_EHIP on launch failure.
 *   Entries of prod_map outside [0, I) are not checked here (that would
 *   need a device read); the kernels index autos with them, so such a map
 *   reads out of bounds and can fault.  The caller validates the map (the
 *   Python binding does, before every call that takes one). */
int bsg_round_to_noise(const void *vis_in, void *vis_out, const float *autos, int64_t F,
                       int64_t I, int64_t T, const int32_t *prod_map, double n_samples,
                       double f, void *stream);

/* Compensation of the diagonal noise model (Section 3.2): the diagonal
 * radiometer equation ignores how correlated the products are; multiplying
 * f by the minimum over cross products of 1 - |V_ij|^2 / (V_ii V_jj) makes
 * up for it, here per frequency and time.
 * vis: complex64 [F][P][T]; autos: float32 [F][I][T] (as bsg_round_to_noise).
 * scale: device float64 [F][T], 8-byte aligned, receives per (f, t) the
 *   minimum over products with i != j of 1 - (re^2 + im^2) / (V_ii V_jj),
 *   each term in double in that order; products with V_ii V_jj not positive
 *   and finite, and NaN terms, are skipped; 1 when no product is left.
 * Errors: BSG_EINVAL (negative sizes, NULL or misaligned pointers, more
 *   than 2^32 - 1 frequencies); BSG_EHIP. */
int bsg_noise_compensation(const void *vis, const float *autos, int64_t F, int64_t I, int64_t T,
                           const int32_t *prod_map, double *scale, void *stream);

/* bsg_round_to_noise with a per-(f, t) factor on G2: G2 = ((V_ii V_jj) c)
 * scale[f][t] for crosses and ((V_ii V_ii) 2c) scale[f][t] for autos (scale
 * from bsg_noise_compensation, or any factor on f; scale = 1 gives exactly
 * bsg_round_to_noise).  scale: device float64 [F][T], 8-byte aligned. */
int bsg_round_to_noise_scaled(const void *vis_in, void *vis_out, const float *autos, int64_t F,
                              int64_t I, int64_t T, const int32_t *prod_map, double n_samples,
                              double f, const double *scale, void *stream);

/* Full-covariance noise for small arrays (Section 3.1, Eqs. rad_full1-3 and
 * Eq. noise; I <= 11 inputs).  Per (frequency, time) the covariance C of
 * the I^2 real degrees of freedom (in product order: Re of each product,
 * then Im if it is a cross product) is built from the sample's visibilities
 * (V_ab = conj(V_ba), V_aa = the measured auto), and each degree of freedom
 * gets the noise s_k^2 = 1 / (C^-1)_kk (not marginalised over the others).
 * With Q = 2N C, (Q^-1)_kk is computed from the Cholesky factor of Q and
 * its inverse with every sum in increasing index order.
 * bsg_fullcov_inverse_diag: qdiag = device float64 [F][T][I^2] receives
 *   (Q^-1)_kk, or NaN for every k of a sample whose Q is not positive
 *   definite.
 * bsg_round_to_noise_fullcov: rounding of Section 3.2 with G2 = c /
 *   (Q^-1)_kk, c = (12 f) / (2N), each degree of freedom with its own k;
 *   samples without an estimate are left unchanged; Im of autos copied;
 *   vis_out may equal vis_in.  Default product order only.
 * Layouts and errors as bsg_round_to_noise (BSG_EINVAL also for I > 11). */
int bsg_fullcov_inverse_diag(const void *vis, const float *autos, int64_t F, int64_t I,
                             int64_t T, double *qdiag, void *stream);
int bsg_round_to_noise_fullcov(const void *vis_in, void *vis_out, const float *autos, int64_t F,
                               int64_t I, int64_t T, double n_samples, double f, void *stream);

/* Integer visibilities, the correlator's own data type (Section 5): the
 * same noise-relative rounding on int32 values.
 * vis_in / vis_out: int32 [F][P][T][2] (re, im), 8-byte aligned; may alias.
 * autos: int32 [F][I][T], the measured auto-correlations (real parts of
 *   the auto products before rounding); must not overlap vis_out.
 * G2 = (V_ii V_jj as an exact int64, rounded once to double) c for crosses,
 *   (V_ii^2 likewise) 2c for autos, c = (12 f) / (2 N); k = the largest
 *   integer with 4^k < G2.  Every integer is a multiple of 2^k for k <= 0,
 *   so only k >= 1 changes a value: re and im go to the nearest multiple of
 *   2^k, ties to the even multiple, computed in exact integer arithmetic; a
 *   result above INT32_MAX becomes the largest multiple of 2^k that fits.
 *   The imaginary part of an auto is copied; G2 not positive and finite
 *   leaves the element unchanged.
 * Errors as bsg_round_to_noise.  A stream of the rounded values is made by
 * bsg_compress_lz4 with elem_size 8 (one complex value per element). */
int bsg_round_to_noise_i32(const void *vis_in, void *vis_out, const int32_t *autos, int64_t F,
                           int64_t I, int64_t T, const int32_t *prod_map, double n_samples,
                           double f, void *stream);

/* ---- Stage 2a: bit transpose within blocks (Section 4.2) --------------
 * in, out: n elements of elem_size bytes; must not overlap.
 * Bit b = 8 * (byte within element) + (bit within byte, LSB = 0) of element
 * i of a block goes to output byte  b * (n_B / 8) + i / 8,  bit i mod 8, i.e.
 * 8E planes, least-significant plane first, each packed LSB-first.
 * bitunshuffle is the exact inverse.
 * Errors: BSG_EINVAL (elem_size < 1, bad block_size, n < 0, NULL). */
int bsg_bitshuffle(const void *in, void *out, int64_t n, int64_t elem_size, int64_t block_size,
                   void *stream);
int bsg_bitunshuffle(const void *in, void *out, int64_t n, int64_t elem_size,
                     int64_t block_size, void *stream);

/* The byte shuffle within blocks (same blocks, partial block and raw tail
 * as bsg_bitshuffle), and its inverse. */
int bsg_byteshuffle(const void *in, void *out, int64_t n, int64_t elem_size, int64_t block_size,
                    void *stream);
int bsg_byteunshuffle(const void *in, void *out, int64_t n, int64_t elem_size,
                      int64_t block_size, void *stream);

/* ---- Stage 2b: bit transpose + per-block LZ4 (Section 4.2) ------------
 * Exact worst-case size of the compressed stream (host, no device work). */
int64_t bsg_compress_bound(int64_t n, int64_t elem_size, int64_t block_size);

/* Device workspace bytes bsg_compress_lz4 needs for these sizes. */
int64_t bsg_compress_workspace_size(int64_t n, int64_t elem_size, int64_t block_size);

/* Compress n elements into the stream format above.  Every block is
 * bit-transposed and LZ4-encoded with one fixed, deterministic greedy rule
 * (hash of 4 bytes, 9 bits, Knuth's multiplier 2654435761; candidate = the
 * last earlier position with that hash in an earlier 64-position chunk; the
 * candidate is extended forward only, keeping the last 5 bytes literal, and
 * taken when it covers at least 12 bytes starting at p <= len - 12), so the
 * output bytes are a pure function of the input.  The result is a standard
 * LZ4 block that any LZ4 decoder reads.
 * out: out_capacity bytes.  *d_out_nbytes (device int64) receives the
 *   stream length, or BSG_ECAPACITY when it would exceed out_capacity (then
 *   out holds nothing meaningful).  Pass out_capacity >= bsg_compress_bound
 *   to never see that.
 * workspace: device memory of bsg_compress_workspace_size bytes, 256-byte
 *   aligned; workspace_bytes is its size.  Blocks above 65536 bytes are
 *   rejected (BSG_EINVAL).
 * stream: an input of 16384 blocks or more is encoded in up to 16 segments
 *   on this stream and one of the library's own, while a third stream (also
 *   the library's: both made once per device, default priority) copies each
 *   finished segment's blocks to their place; both are joined back into
 *   this stream, so the call orders like one operation on it, also under
 *   stream capture.  Host threads enqueueing such calls take turns. */
int bsg_compress_lz4(const void *in, void *out, int64_t n, int64_t elem_size,
                     int64_t block_size, int64_t out_capacity, int64_t *d_out_nbytes,
                     void *workspace, int64_t workspace_bytes, void *stream);

/* bsg_compress_lz4 for callers that cannot allocate device memory (code
 * under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no workspace argument; the scratch space (block slots, block
 * sizes, scan tiles) is a fixed array of BSG_NOALLOC_SCRATCH_BYTES inside the
 * library, one per GPU, held from the library's load until the process
 * ends.  The call allocates nothing (it never uses the library's own
 * streams: a large input is encoded in one pass on `stream`).  It uses the device current on the
 * calling thread (the stream must belong to it).  Same stream format, bytes,
 * bounds and errors as bsg_compress_lz4, plus BSG_ECAPACITY when
 * bsg_compress_workspace_size(n, elem_size, block_size) exceeds
 * BSG_NOALLOC_SCRATCH_BYTES (at 8192-byte blocks, inputs above about 63 MiB).
 * Every call on a GPU shares that GPU's array: calls whose work overlaps in
 * time on one GPU (different streams, or different host threads) race and
 * must be serialised by the caller. */
#define BSG_NOALLOC_SCRATCH_BYTES (64ll << 20)
int bsg_compress_lz4_noalloc(const void *in, void *out, int64_t n, int64_t elem_size,
                             int64_t block_size, int64_t out_capacity, int64_t *d_out_nbytes,
                             void *stream);

/* The two stages fused: round_to_noise on complex64 visibilities (arguments
 * as bsg_round_to_noise, vis_in is not modified), then bitshuffle + LZ4 of
 * the rounded values viewed as float32 elements (elem_size 4, n = 2 F P T),
 * without writing the rounded array.  The stream is byte-identical to
 * bsg_round_to_noise followed by bsg_compress_lz4 with elem_size 4. */
int bsg_round_compress_lz4(const void *vis_in, const float *autos, int64_t F, int64_t I,
                           int64_t T, const int32_t *prod_map, double n_samples, double f,
                           int64_t block_size, void *out, int64_t out_capacity,
                           int64_t *d_out_nbytes, void *workspace, int64_t workspace_bytes,
                           void *stream);

/* Decompress a stream made by bsg_compress_lz4 (any valid LZ4 encoding of
 * the blocks is accepted, not only this library's).  n, elem_size and
 * block_size must equal the header's.  in_nbytes is the stream length.
 * *d_status (device int32) must be 0 on entry; it stays 0 on success and
 * receives BSG_ECORRUPT when the header, offsets or any block is invalid
 * (bad offset, overrun, short or long output, trailing bytes).  Reads and
 * writes stay inside in[0, in_nbytes) and out[0, n * elem_size) whatever
 * the input holds. */
int bsg_decompress_lz4(const void *in, int64_t in_nbytes, void *out, int64_t n,
                       int64_t elem_size, int64_t block_size, int32_t *d_status, void *stream);

/* ---- Many independent streams in one pass (Section 4.2) ---------------
 * A batch is a set of chunks, each compressed into (or decompressed from) a
 * stream of its own, exactly the stream bsg_compress_lz4 makes for that
 * chunk alone.  Chunks are independent units like the blocks inside them,
 * so one persistent kernel per element-size class walks every block of
 * every chunk; the launches neither allocate nor synchronise with the host,
 * so a hipGraph can capture them.
 *
 * For compression: in = n elements of elem_size bytes (device), out = the
 *   stream buffer (device, 8-byte aligned) of out_capacity bytes; in_nbytes
 *   is ignored.
 * For decompression: in = the stream (device, 8-byte aligned) of in_nbytes
 *   bytes, out = room for n elements (device); out_capacity is ignored.
 * block_size: elements per block as for bsg_compress_lz4 (0 = default);
 *   blocks above 65536 bytes are rejected. */
typedef struct bsg_chunk {
    const void *in;
    int64_t in_nbytes;
    void *out;
    int64_t out_capacity;
    int64_t n;
    int64_t elem_size;
    int64_t block_size;
} bsg_chunk;

/* Bytes of the descriptor table for count chunks, or BSG_EINVAL. */
int64_t bsg_batch_table_bytes(int32_t count);

/* Fill host_table (host memory, host_table_bytes >= bsg_batch_table_bytes)
 * from chunks[0..count).  The caller copies the same bytes to a 16-byte
 * aligned device buffer (d_table below) before the batch call and keeps
 * both alive, unchanged, until the work has run; a table may be reused for
 * any number of calls on the same buffers.  The chunk pointers are stored,
 * not dereferenced.  Errors: BSG_EINVAL for a bad size or block size. */
int bsg_batch_build_table(const bsg_chunk *chunks, int32_t count, void *host_table,
                          int64_t host_table_bytes);

/* Device workspace bytes bsg_batch_compress needs for this table. */
int64_t bsg_batch_workspace_size(const void *host_table);

/* Launch shape of the persistent batch kernels (it never changes the
 * output): waves_per_cu = workgroups per compute unit in the grid (<= 0:
 * 16; one wavefront per workgroup, one block at a time); schedule = how the
 * blocks of a class are dealt to the workgroups: BSG_SCHED_STRIDED, every
 * grid-th block from the workgroup's index, or BSG_SCHED_RANGES, one
 * contiguous range of blocks per workgroup. */
#define BSG_SCHED_STRIDED 0
#define BSG_SCHED_RANGES 1

/* Compress every chunk of the table.  d_nbytes: device int64[count],
 * entry i (the caller's chunk order) receives chunk i's stream length, or
 * BSG_ECAPACITY when it would exceed that chunk's out_capacity (then its
 * out holds nothing meaningful; the other chunks are unaffected).
 * workspace: 256-byte aligned, workspace_bytes >= bsg_batch_workspace_size.
 * waves_per_cu, schedule: the launch shape (above).
 * stream: a batch of 16384 blocks or more in two or more element classes
 *   encodes its classes alternately on this stream and on the library's
 *   encode stream, while the library's pack stream scans, finishes and packs
 *   each class (the streams of bsg_compress_lz4, joined back into this one).
 * Errors: BSG_EINVAL (NULL pointers, misaligned buffers, unknown schedule),
 *   BSG_ECAPACITY (workspace too small), BSG_EHIP (launch failure). */
int bsg_batch_compress(const void *host_table, const void *d_table, int64_t *d_nbytes,
                       void *workspace, int64_t workspace_bytes, int32_t waves_per_cu,
                       int32_t schedule, void *stream);

/* Decompress every chunk of the table (streams from bsg_compress_lz4 or
 * bsg_batch_compress, or any valid LZ4 encoding of their blocks).
 * d_status: device int32[count], zero on entry; entry i stays 0 on success
 * and receives BSG_ECORRUPT when chunk i's stream is invalid, with the same
 * checks and the same memory bounds as bsg_decompress_lz4. */
int bsg_batch_decompress(const void *host_table, const void *d_table, int32_t *d_status,
                         int32_t waves_per_cu, int32_t schedule, void *stream);

/* bsg_compress_lz4 / bsg_decompress_lz4 with the block filter chosen by
 * `filter` (BSG_FILTER_BIT gives exactly those calls; BSG_FILTER_BYTE
 * byte-shuffles each block instead and marks the stream with
 * BSG_MAGIC_BYTE).  Same workspace, bounds and errors; decompression
 * rejects a stream whose magic does not match the filter. */
int bsg_compress_lz4_filter(const void *in, void *out, int64_t n, int64_t elem_size,
                            int64_t block_size, int32_t filter, int64_t out_capacity,
                            int64_t *d_out_nbytes, void *workspace, int64_t workspace_bytes,
                            void *stream);
int bsg_decompress_lz4_filter(const void *in, int64_t in_nbytes, void *out, int64_t n,
                              int64_t elem_size, int64_t block_size, int32_t filter,
                              int32_t *d_status, void *stream);

/* Parse a stream header from HOST memory (no device work). */
int bsg_read_header(const void *host_bytes, int64_t nbytes, bsg_header *hdr);

#ifdef __cplusplus
}
#endif
#endif
