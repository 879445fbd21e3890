// Host check of the per-order walk's block order (block_stride and
// scatter_block): for pool sizes with and without a partial last block, every
// item of [0, total) is handed out exactly once, each block of kOrderBlock
// items stays whole.  Prints "ok <sizes checked>".
#include <cstdio>
#include <cstdint>
#include <vector>

#include "qrt_wave.h"

int main()
{
    const uint64_t B = qrt::kOrderBlock;
    const uint64_t sizes[] = {0, 1, B - 1, B, B + 1, 2 * B - 1, 2 * B, 2 * B + 1, 64 * B, 64 * B + 1,
                              1000 * B + 17, 8192 * B, 3 * 64 * 65536 + 4194304, (1ull << 26) + 5};
    int checked = 0;
    for (uint64_t total : sizes) {
        const uint64_t stride = qrt::block_stride(total >> qrt::kOrderBlockLog2);
        std::vector<uint8_t> seen(total, 0);
        for (uint64_t i = 0; i < total; ++i) {
            const uint64_t j = qrt::scatter_block(i, total, stride);
            if (j >= total || seen[j]) {
                printf("bad map: total %llu item %llu -> %llu\n", (unsigned long long)total,
                       (unsigned long long)i, (unsigned long long)j);
                return 1;
            }
            seen[j] = 1;
            const uint64_t head = qrt::scatter_block(i & ~(B - 1), total, stride);
            if ((j & (B - 1)) != (i & (B - 1)) || (j & ~(B - 1)) != (head & ~(B - 1))) {
                printf("block split: total %llu item %llu\n", (unsigned long long)total, (unsigned long long)i);
                return 1;
            }
        }
        ++checked;
    }
    printf("ok %d\n", checked);
    return 0;
}
