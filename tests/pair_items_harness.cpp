// Host check of the tile-pair work items of a paired set (rici_pairs.h):
// for each grid size T on the command line, every item k < T (T + 1) / 2 is
// mapped with pair_coords and compared with the band order written out as
// plain nested loops (bands of kPairBand tile rows; inside a band, its own
// triangle column by column, then the columns beyond it, rows fastest).  A
// leading "-p" prints the items of the (single) grid instead.
#define __host__
#define __device__
#include "rici_pairs.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>

int main(int argc, char** argv)
{
    using rici::kPairBand;
    const bool print = argc > 1 && std::strcmp(argv[1], "-p") == 0;
    long bad = 0, checked = 0;
    for (int a = print ? 2 : 1; a < argc; ++a) {
        const uint32_t T = (uint32_t)std::strtoul(argv[a], nullptr, 10);
        uint32_t k = 0;
        for (uint32_t b0 = 0; b0 < T; b0 += kPairBand) {
            const uint32_t bw = T - b0 < kPairBand ? T - b0 : kPairBand;
            auto expect = [&](uint32_t i, uint32_t j) {
                uint32_t I = ~0u, J = ~0u;
                rici::pair_coords(k, T, I, J);
                if (print) std::printf("%u %u\n", I, J);
                if (I != i || J != j) {
                    if (bad < 5) std::fprintf(stderr, "T %u item %u: (%u, %u), expected (%u, %u)\n", T, k, I, J, i, j);
                    ++bad;
                }
                ++k;
                ++checked;
            };
            for (uint32_t c = 0; c < bw; ++c)
                for (uint32_t r = 0; r <= c; ++r) expect(b0 + r, b0 + c);
            for (uint32_t c = b0 + bw; c < T; ++c)
                for (uint32_t r = 0; r < bw; ++r) expect(b0 + r, c);
        }
        if (k != rici::pair_items(T)) {
            std::fprintf(stderr, "T %u: %u items enumerated, pair_items says %u\n", T, k, rici::pair_items(T));
            ++bad;
        }
    }
    if (!print) std::printf("checked %ld items, %ld wrong\n", checked, bad);
    return bad ? 1 : 0;
}
