// Drives the host-side logic of the C-ABI (layouts, bounds, workspace
// sizes, stream headers, batch descriptor tables, and every argument check
// that returns before any device work) so that a build with the host pass
// under AddressSanitizer and UndefinedBehaviorSanitizer checks it.  No call
// here reaches the GPU.  Exits 0 when every result is as documented.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "bsg.h"

#define CHECK(c)                                                                \
    do {                                                                        \
        if (!(c)) {                                                             \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            std::exit(1);                                                       \
        }                                                                       \
    } while (0)

static void *P(uintptr_t a) { return reinterpret_cast<void *>(a); }

int main()
{
    // sizes and layouts over a sweep of element sizes, block sizes, lengths
    const int64_t es[] = {1, 2, 3, 4, 5, 8, 12, 16, 1000};
    const int64_t bs[] = {0, 8, 16, 24, 1024, 2048, 8192, 65536, 12, -8};
    const int64_t ns[] = {0, 1, 7, 8, 9, 12345, 1 << 20, (int64_t)1 << 40};
    for (int64_t e : es)
        for (int64_t b : bs) {
            const int64_t nb = bsg_block_elems(e, b);
            CHECK(nb == BSG_EINVAL || (nb >= 8 && nb % 8 == 0));
            for (int64_t n : ns) {
                const int64_t bound = bsg_compress_bound(n, e, b);
                const int64_t ws = bsg_compress_workspace_size(n, e, b);
                if (nb == BSG_EINVAL || nb * e > BSG_MAX_BLOCK_BYTES) {
                    CHECK(bound == BSG_EINVAL && ws == BSG_EINVAL);
                } else {
                    CHECK(bound >= 24 + 8 && ws > 0);
                }
            }
        }
    // argument checks that need no device
    CHECK(bsg_bitshuffle(P(16), P(32), -1, 4, 0, nullptr) == BSG_EINVAL);
    CHECK(bsg_bitshuffle(nullptr, nullptr, 64, 4, 0, nullptr) == BSG_EINVAL);
    CHECK(bsg_bitunshuffle(P(16), P(32), 64, 0, 0, nullptr) == BSG_EINVAL);
    CHECK(bsg_byteshuffle(P(16), P(33), 64, 4, 0, nullptr) == BSG_EINVAL);
    CHECK(bsg_round_to_noise(P(16), P(16), (const float *)P(16), 1, 2, 3, nullptr, 3.9e6, -1.0,
                             nullptr) == BSG_EINVAL);
    CHECK(bsg_round_to_noise(P(16), P(16), (const float *)P(16), 1, 2, 3, nullptr, 0.0, 0.01,
                             nullptr) == BSG_EINVAL);
    CHECK(bsg_round_to_noise(P(16), P(17), (const float *)P(16), 1, 2, 3, nullptr, 3.9e6, 0.01,
                             nullptr) == BSG_EINVAL);
    CHECK(bsg_round_to_noise(nullptr, nullptr, nullptr, 0, 2, 3, nullptr, 3.9e6, 0.01, nullptr) ==
          BSG_OK);
    CHECK(bsg_round_to_noise_i32(P(16), P(16), (const int32_t *)P(16), -1, 2, 3, nullptr, 3.9e6,
                                 0.01, nullptr) == BSG_EINVAL);
    CHECK(bsg_noise_compensation(P(16), (const float *)P(16), 1, 2, 3, nullptr, (double *)P(12),
                                 nullptr) == BSG_EINVAL);
    CHECK(bsg_round_to_noise_fullcov(P(16), P(16), (const float *)P(16), 1, 12, 3, 3.9e6, 0.01,
                                     nullptr) == BSG_EINVAL);
    CHECK(bsg_fullcov_inverse_diag(P(16), (const float *)P(16), 1, 2, 3, nullptr, nullptr) ==
          BSG_EINVAL);
    int64_t *d_nb = (int64_t *)P(64);
    CHECK(bsg_compress_lz4(P(16), P(64), 2048, 4, 0, 1 << 20, d_nb, P(256), 0, nullptr) ==
          BSG_ECAPACITY);
    CHECK(bsg_compress_lz4(P(16), P(64), 2048, 4, 12, 1 << 20, d_nb, P(256), 1 << 20, nullptr) ==
          BSG_EINVAL);
    CHECK(bsg_compress_lz4(P(16), P(64), 2048, 4, 0, 8, d_nb, P(256), 1 << 20, nullptr) ==
          BSG_ECAPACITY);
    CHECK(bsg_compress_lz4(P(16), P(64), 2048, 4, 0, 1 << 20, d_nb, P(257), 1 << 20, nullptr) ==
          BSG_EINVAL);
    CHECK(bsg_compress_lz4_filter(P(16), P(64), 2048, 4, 0, 7, 1 << 20, d_nb, P(256), 1 << 20,
                                  nullptr) == BSG_EINVAL);
    CHECK(bsg_compress_lz4_noalloc(P(16), P(64), (int64_t)1 << 30, 4, 0, (int64_t)1 << 40, d_nb,
                                   nullptr) == BSG_ECAPACITY);
    CHECK(bsg_round_compress_lz4(P(16), (const float *)P(16), 4, 3, 8, nullptr, 3.9e6, 0.01, 12,
                                 P(64), 1 << 20, d_nb, P(256), 1 << 20, nullptr) == BSG_EINVAL);
    CHECK(bsg_decompress_lz4(P(16), 10, P(64), 2048, 4, 0, (int32_t *)P(64), nullptr) ==
          BSG_ECORRUPT);
    CHECK(bsg_decompress_lz4(P(17), 1 << 20, P(64), 2048, 4, 0, (int32_t *)P(64), nullptr) ==
          BSG_EINVAL);
    CHECK(bsg_decompress_lz4_filter(P(16), 1 << 20, P(64), 2048, 4, 0, 5, (int32_t *)P(64),
                                    nullptr) == BSG_EINVAL);
    // stream headers from host memory
    bsg_header h;
    uint8_t hb[32] = {0};
    CHECK(bsg_read_header(hb, 10, &h) == BSG_ECORRUPT);
    CHECK(bsg_read_header(hb, 32, &h) == BSG_ECORRUPT);
    const uint32_t magic = BSG_MAGIC;
    std::memcpy(hb, &magic, 4);
    CHECK(bsg_read_header(hb, 24, &h) == BSG_OK && h.magic == BSG_MAGIC);
    CHECK(bsg_read_header(nullptr, 24, &h) == BSG_EINVAL);
    CHECK(std::strlen(bsg_strerror(BSG_ECORRUPT)) > 0 && std::strlen(bsg_strerror(12345)) > 0);
    // batch descriptor tables
    CHECK(bsg_batch_table_bytes(-1) == BSG_EINVAL);
    for (int count : {0, 1, 5, 300}) {
        std::vector<bsg_chunk> ch(count);
        for (int i = 0; i < count; ++i) {
            const int64_t e = es[i % 8];
            ch[i] = bsg_chunk{P(4096), 0, P(8192), 1 << 20, (int64_t)(i * 977 % 50000), e,
                              (i % 3) ? 0 : 64};
        }
        const int64_t tb = bsg_batch_table_bytes(count);
        CHECK(tb > 0);
        std::vector<uint8_t> table((size_t)tb + 1);
        CHECK(bsg_batch_build_table(count ? ch.data() : nullptr, count, table.data(), tb) == BSG_OK);
        CHECK(bsg_batch_build_table(ch.data(), count, table.data(), tb - 1) == BSG_EINVAL);
        CHECK(bsg_batch_workspace_size(table.data()) > 0);
        CHECK(bsg_batch_compress(table.data(), nullptr, d_nb, P(256), 1 << 20, 0, 0, nullptr) ==
              BSG_EINVAL);
        CHECK(bsg_batch_compress(table.data(), P(4096), d_nb, P(256), 1 << 30, 0, 2, nullptr) ==
              BSG_EINVAL);
        CHECK(bsg_batch_decompress(table.data(), P(4096), (int32_t *)P(64), 0, -1, nullptr) ==
              BSG_EINVAL);
        if (count) {
            ch[count - 1].block_size = 12; // not a multiple of 8
            CHECK(bsg_batch_build_table(ch.data(), count, table.data(), tb) == BSG_EINVAL);
            ch[count - 1].block_size = 65536; // 64 KiB blocks of >= 2-byte elements: too large
            ch[count - 1].elem_size = 2;
            CHECK(bsg_batch_build_table(ch.data(), count, table.data(), tb) == BSG_EINVAL);
        }
    }
    std::printf("abi sanitizer driver ok\n");
    return 0;
}
