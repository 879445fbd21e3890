// Host check of the per-order walk's block order (block_stride and
// scatter_block): for pool sizes with and without a partial last block, every
// item of [0, total) is handed out exactly once, each 64-item block stays
// whole.  Prints "ok <sizes checked>".
#include <cstdio>
#include <cstdint>
#include <vector>

#include "qrt_wave.h"

int main()
{
    const uint64_t sizes[] = {0, 1, 63, 64, 65, 127, 128, 129, 4096, 4097, 64 * 1000 + 17, 64 * 65536,
                              3 * 64 * 65536 + 4194304, (1ull << 26) + 5};
    int checked = 0;
    for (uint64_t total : sizes) {
        const uint64_t stride = qrt::block_stride(total >> 6);
        std::vector<uint8_t> seen(total, 0);
        for (uint64_t i = 0; i < total; ++i) {
            const uint64_t j = qrt::scatter_block(i, total, stride);
            if (j >= total || seen[j]) {
                printf("bad map: total %llu item %llu -> %llu\n", (unsigned long long)total,
                       (unsigned long long)i, (unsigned long long)j);
                return 1;
            }
            seen[j] = 1;
            if ((j & 63) != (i & 63) || (j >> 6) != (qrt::scatter_block(i & ~63ull, total, stride) >> 6)) {
                printf("block split: total %llu item %llu\n", (unsigned long long)total, (unsigned long long)i);
                return 1;
            }
        }
        ++checked;
    }
    printf("ok %d\n", checked);
    return 0;
}
