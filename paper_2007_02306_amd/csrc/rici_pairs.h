// Work items of a set ranked against itself (a paired set): the search
// visits each pair of tiles (I, J), I <= J, once, for both directions of the
// ranks of Sec. 4.1 step 6c.  Host and device code; the device search kernels
// and a host test of the mapping include it.
#pragma once

#include <cmath>
#include <cstdint>

namespace rici {

// Item k of a T x T tile grid is the tile pair (I, J), I <= J.  Items come in
// bands of kPairBand = 8 consecutive I; within a band J-major, so the items
// running at the same time share their I tiles and a few J tiles.  (On the
// 256-mesh workload 8 measured 1.4 % faster than 4, whose bands stream every J
// tile twice as often, and 12 and 16 slower; on a single set of 92 tiles 4 and
// 8 are within 1.4 %.)
// Items before full band b: b (BW T - BW (BW - 1) / 2) - BW^2 b (b - 1) / 2
// = b (BW T + BW / 2) - (BW^2 / 2) b^2; the band of item k is the largest b
// with that count <= k, found from the quadratic's smaller root and settled
// by integer comparisons (O(1) per item: a large mesh has hundreds of bands).
constexpr uint32_t kPairBand = 8;

__host__ __device__ inline void pair_coords(uint32_t k, uint32_t T, uint32_t& I, uint32_t& J)
{
    constexpr uint32_t BW = kPairBand;
    const uint64_t nfull = T / BW;
    auto before = [&](uint64_t b) { return b * ((uint64_t)BW * T + BW / 2) - (uint64_t)(BW * BW / 2) * b * b; };
    const double p = (double)BW * T + BW / 2, disc = p * p - 2.0 * BW * BW * (double)k;
    uint64_t b = disc > 0.0 ? (uint64_t)((p - sqrt(disc)) / (double)(BW * BW)) : nfull;
    if (b > nfull) b = nfull;
    while (b > 0 && before(b) > k) --b;
    while (b < nfull && before(b + 1) <= k) ++b;
    const uint32_t b0 = (uint32_t)(BW * b);
    const uint32_t bw = T - b0 < BW ? T - b0 : BW;        // the last band may be narrower
    const uint32_t r = k - (uint32_t)before(b);
    const uint32_t tri = bw * (bw + 1) / 2;               // J inside the band
    if (r < tri) {
        uint32_t a = 0;
        while ((a + 1) * (a + 2) / 2 <= r) ++a;
        J = b0 + a;
        I = b0 + (r - a * (a + 1) / 2);
    } else {
        const uint32_t q = r - tri;                       // J beyond the band
        J = b0 + bw + q / bw;
        I = b0 + q % bw;
    }
}

// number of items: T (T + 1) / 2
__host__ __device__ inline uint32_t pair_items(uint32_t T) { return T * (T + 1) / 2; }

}  // namespace rici
