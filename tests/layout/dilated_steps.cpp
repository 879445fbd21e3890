// Host check of the bricked mesh layout and the walk's dilated-integer steps:
// for random meshes (brick counts along x and y padded to powers of two), every
// cell's element index is the OR of its three axis parts, and a step of one
// cell along any axis, up or down, done as the walk does it on the byte-offset
// parts, lands on the brick_index of the moved cell.  Prints "ok" or the first
// mismatch.
#include <cstdio>
#include <cstdint>
#include <random>

#include "qrt_walk.h"

using namespace qrt;

int main()
{
    std::mt19937 rng(2406);
    int checked = 0;
    for (int trial = 0; trial < 200; ++trial) {
        const int n[3] = {1 + (int)(rng() % 300), 1 + (int)(rng() % 300), 1 + (int)(rng() % 300)};
        int nb[3];
        mesh_bricks(n[0], n[1], n[2], nb);
        if ((nb[0] & (nb[0] - 1)) || (nb[1] & (nb[1] - 1)) || nb[0] * 4 < n[0] || nb[1] * 4 < n[1] || nb[2] * 4 < n[2]) {
            std::printf("bad brick counts %d %d %d for %d %d %d\n", nb[0], nb[1], nb[2], n[0], n[1], n[2]);
            return 1;
        }
        uint32_t m[3];
        axis_masks(nb[0], nb[1], m);
        for (int k = 0; k < 2000; ++k) {
            const int c[3] = {(int)(rng() % n[0]), (int)(rng() % n[1]), (int)(rng() % n[2])};
            const uint32_t part[3] = {(uint32_t)brick_index(c[0], 0, 0, nb[0], nb[1]) << 2,
                                      (uint32_t)brick_index(0, c[1], 0, nb[0], nb[1]) << 2,
                                      (uint32_t)brick_index(0, 0, c[2], nb[0], nb[1]) << 2};
            const uint32_t whole = (uint32_t)brick_index(c[0], c[1], c[2], nb[0], nb[1]) << 2;
            if ((part[0] | part[1] | part[2]) != whole || (part[0] & ~m[0]) || (part[1] & ~m[1]) || (part[2] & ~m[2])) {
                std::printf("parts of (%d %d %d) in %d %d %d\n", c[0], c[1], c[2], n[0], n[1], n[2]);
                return 1;
            }
            for (int a = 0; a < 3; ++a)
                for (int s = -1; s <= 1; s += 2) {
                    const int to = c[a] + s;
                    if (to < 0 || to >= n[a]) continue;
                    const uint32_t up = s > 0 ? ~m[a] : 0u;
                    const uint32_t moved = ((part[a] | up) + (uint32_t)(4 * s)) & m[a];
                    int d[3] = {c[0], c[1], c[2]};
                    d[a] = to;
                    uint32_t p2[3] = {part[0], part[1], part[2]};
                    p2[a] = moved;
                    const uint32_t want = (uint32_t)brick_index(d[0], d[1], d[2], nb[0], nb[1]) << 2;
                    if ((p2[0] | p2[1] | p2[2]) != want) {
                        std::printf("step %d along %d from (%d %d %d) in %d %d %d\n", s, a, c[0], c[1], c[2], n[0],
                                    n[1], n[2]);
                        return 1;
                    }
                    ++checked;
                }
        }
    }
    std::printf("ok %d\n", checked);
    return 0;
}
