// Stress test of the serving loop's host copy pool (copy_pool.h): batches of
// copies of random sizes (empty, tiny, below and above the inline and chunk
// thresholds, ragged last chunks) through pools with and without worker
// threads, several pool lifetimes; every destination byte and the guard
// bytes around it are checked.  Built with -fsanitize=thread by the test
// that runs it, so a data race in the pool fails the test too.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "copy_pool.h"

int main(int argc, char **argv)
{
    const int rounds = argc > 1 ? std::atoi(argv[1]) : 150;
    const size_t sizes[] = {0, 1, 7, 4096, 262143, 262144, 262145, 524287, 524288, 1 << 20, 3 * (1 << 20) + 5};
    const size_t kGuard = 32;
    for (int life = 0; life < 4; ++life) {
        spk::CopyPool pool;
        pool.start(life == 0 ? 0 : 3);
        std::mt19937_64 rng(1234 + life);
        for (int r = 0; r < rounds; ++r) {
            const int nitems = 1 + (int)(rng() % 12);
            std::vector<std::vector<unsigned char>> src(nitems), dst(nitems);
            std::vector<spk::CopyPool::Chunk> items;
            for (int i = 0; i < nitems; ++i) {
                const size_t n = (rng() % 3 == 0) ? (size_t)(rng() % (3u << 20))
                                                  : sizes[rng() % (sizeof sizes / sizeof sizes[0])];
                // a fill byte per item and a distinct marker every 4 KiB, so
                // a chunk landing at the wrong offset shows
                src[i].resize(n);
                if (n) std::memset(src[i].data(), (unsigned char)(i * 7 + r + 1), n);
                for (size_t k = 0; k < n; k += 4096) src[i][k] = (unsigned char)(k / 4096 * 13 + i);
                if (n) src[i][n - 1] = (unsigned char)(0x5A + i);
                dst[i].assign(n + 2 * kGuard, 0xAB);
                items.push_back({dst[i].data() + kGuard, src[i].data(), n});
            }
            pool.copy(items);
            for (int i = 0; i < nitems; ++i) {
                const size_t n = src[i].size();
                for (size_t k = 0; k < kGuard; ++k)
                    if (dst[i][k] != 0xAB || dst[i][kGuard + n + k] != 0xAB) {
                        std::printf("life %d round %d item %d: guard overwritten\n", life, r, i);
                        return 1;
                    }
                if (n && std::memcmp(dst[i].data() + kGuard, src[i].data(), n) != 0) {
                    std::printf("life %d round %d item %d (%zu bytes): wrong bytes\n", life, r, i, n);
                    return 1;
                }
            }
        }
        pool.finish();
    }
    std::printf("ok\n");
    return 0;
}
