// Clutter-resistant distance (CRD) search for gfx950 (Sec. 3.2, Eq. 6-7) and
// the rank of the true match (Sec. 4.1 step 6c, ties to the best rank).
//
// The masked sum of Eq. 7 is split into contractions (exact, because the
// needle mask m = [D_n != 0] times D_n is D_n):
//     CRD(n, h) = |D_n|^2 - 2 <D_n, D_h> + <m_n, D_h^2>.
// |D_n|^2 is one number per needle, so a (needle, haystack) pair costs two
// length-4096 int8 dot products -- a dense int8 x int8 -> int32 GEMM over all
// pairs, which is what MFMA does best.  Operands stay exact int8 under a range
// check: needles with |D| <= 127 use planes (D_n, m_n); haystack images with
// |D| <= 127 use (D_h, r, q) with D_h^2 = 256 q + r + 128, i.e.
// r = (D_h^2 mod 256) - 128 in [-128, 127] and q = D_h^2 div 256 in [0, 63].
// The accumulator is scaled between phases so a single int32 accumulator holds
//     <m, q> ... (x -128) ... + <D_n, D_h> ... (x -2) ... + <m, r>
//   = <m, D_h^2> - 2 <D_n, D_h> - 128 |m|,
// and the needle's constant |D_n|^2 + 128 |m| (|m| = its non-zero deltas) is
// added outside.  The q phase is skipped for haystack tiles where every
// |D_h| <= 15 (then q = 0).  All partial sums stay far below 2^31
// (4032 * 63 * 256 + 2 * 4032 * 127^2 + 4032 * 128 < 2^31).  Any image outside
// the int8 range goes to an exact int64 VALU path instead.
//
// Ranking never sorts: rank_i = #{ h : CRD(n_i, h) < CRD(n_i, h_true) } is a
// sum of per-tile counts, so tiles add their counts with integer atomics and
// the result is exact and independent of the order of tiles.
#include "rici_internal.h"
#include "rici_pairs.h"

#include <limits.h>
#include <type_traits>

namespace rici {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr uint32_t kSlow = 127;     // largest |D| an int8 operand holds
constexpr uint32_t kSmallD = 15;    // |D| <= 15  =>  D^2 <= 225: q = 0, r = D^2 - 128 fits int8
constexpr uint32_t kPad = 0xFFFFFFFFu;
// paired sets keep one flag word per tile of this many slots (the paired
// search's tile width)
constexpr uint32_t kFlagTile = 256;
// word 3 of a gfx9 buffer resource for untyped (raw) dword accesses
constexpr int kBufferWord3 = 0x00020000;
// cache policy of a buffer access: sc1 (device scope; a load misses in the
// CU's vector L1)
constexpr int kDeviceScope = 16;

// ------------------------------------------------------------------ delta prep

constexpr int kDeltaWaves = 8;   // wavefronts per delta-prep workgroup (rows split among them; 8 measured best)

// One block per group of 16 images; thread (row-in-step, lane) with
// lane = 16 * q + i writes columns 16 q .. 16 q + 15 of image i.
// needle_side: 1 needle planes (D, mask) into `planes`; 0 haystack planes
// (D, r, q) into `planes`; 2 both, in slot order (a set ranked against
// itself): the mask plane into `planes` and the haystack planes into
// `hplanes`, whose D plane serves as the needles' D plane too.  With
// `qflags` (the set's tile flags) the q plane is written only in tiles whose
// bit 1 is set: no other tile runs the q phase, so none reads it.
__device__ void delta_group(const uint32_t* __restrict__ images, uint32_t n, int needle_side,
                            int8_t* __restrict__ planes, uint32_t ngroups, int64_t* __restrict__ sumsq,
                            uint32_t* __restrict__ maxabs, const uint32_t* __restrict__ perm, uint32_t grp,
                            int8_t* __restrict__ hplanes = nullptr, const uint32_t* __restrict__ qflags = nullptr)
{
    __shared__ uint32_t smax[kDeltaWaves][kGroup];
    __shared__ int64_t ssum[kDeltaWaves][kGroup];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i = lane & 15, q = lane >> 4;
    const uint32_t slot = grp * kGroup + i;
    const uint32_t img = perm ? perm[slot] : slot;
    const bool live = perm ? img != kPad : slot < n;
    const size_t plane_stride = (size_t)ngroups * kPlaneGroupBytes;
    const bool write_q = !qflags || (qflags[grp / (kFlagTile / kGroup)] & 2u);

    uint32_t mx = 0;
    int64_t ss = 0;
    for (int r = wave; r < NB; r += kDeltaWaves) {
        int32_t d[16];
        if (live) {
            const uint32_t* row = images + (size_t)img * NPIX + r * NB + 16 * q;
            const uint4* row4 = reinterpret_cast<const uint4*>(row);
            uint32_t v[17];
            v[0] = q > 0 ? row[-1] : 0u;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                uint4 u = row4[k];
                v[1 + 4 * k] = u.x; v[2 + 4 * k] = u.y; v[3 + 4 * k] = u.z; v[4 + 4 * k] = u.w;
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                // Eq. 6 in signed 64-bit; column 0 has no left neighbour and no term
                int64_t dd = (q == 0 && k == 0) ? 0 : (int64_t)v[k + 1] - (int64_t)v[k];
                uint64_t a = dd < 0 ? (uint64_t)(-dd) : (uint64_t)dd;
                mx = (uint32_t)max((uint64_t)mx, min(a, (uint64_t)0xFFFFFFFEu));
                ss += dd * dd + (dd != 0 ? 128 : 0);   // |D|^2 + 128 |m|
                d[k] = (int32_t)max(min(dd, (int64_t)127), (int64_t)-127);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) d[k] = 0;
        }
        // pack into the fragment-major planes: D (both sides), needle mask,
        // haystack r = (D^2 mod 256) - 128 and q = D^2 div 256 (int8 bytes)
        const size_t frag = ((size_t)grp * NB + r) * kFragBytes + (size_t)lane * 16;
        uint32_t nm[4], hd[4], hr[4], hq[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint32_t a1 = 0, b0 = 0, b1 = 0, b2 = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int32_t x = d[4 * k + b];
                const uint32_t sq = (uint32_t)(x * x);
                a1 |= (x != 0 ? 1u : 0u) << (8 * b);
                b0 |= (uint32_t)(uint8_t)(int8_t)x << (8 * b);
                b1 |= ((sq & 255u) ^ 0x80u) << (8 * b);
                b2 |= (sq >> 8) << (8 * b);
            }
            nm[k] = a1; hd[k] = b0; hr[k] = b1; hq[k] = b2;
        }
        if (needle_side == 1)
            *reinterpret_cast<uint4*>(planes + frag) = make_uint4(hd[0], hd[1], hd[2], hd[3]);
        if (needle_side)
            *reinterpret_cast<uint4*>(planes + plane_stride + frag) = make_uint4(nm[0], nm[1], nm[2], nm[3]);
        if (needle_side != 1) {
            int8_t* hp = needle_side == 2 ? hplanes : planes;
            *reinterpret_cast<uint4*>(hp + frag) = make_uint4(hd[0], hd[1], hd[2], hd[3]);
            *reinterpret_cast<uint4*>(hp + plane_stride + frag) = make_uint4(hr[0], hr[1], hr[2], hr[3]);
            if (write_q)
                *reinterpret_cast<uint4*>(hp + 2 * plane_stride + frag) = make_uint4(hq[0], hq[1], hq[2], hq[3]);
        }
    }
    // the haystack's statistics come from k_hay_stats; a paired set's
    // needle constants from k_stats_true (sumsq == nullptr)
    if (perm && (!needle_side || !sumsq)) return;
    // per-image reductions: 4 lanes (q) per wave and kDeltaWaves waves share image i
#pragma unroll
    for (int o = 16; o < 64; o <<= 1) {
        mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
        ss += __shfl_xor(ss, o, 64);
    }
    if (q == 0) { smax[wave][i] = mx; ssum[wave][i] = ss; }
    __syncthreads();
    if (tid < kGroup) {
        const uint32_t im = grp * kGroup + tid;
        uint32_t m = 0;
        int64_t s = 0;
#pragma unroll
        for (int w = 0; w < kDeltaWaves; ++w) { m = max(m, smax[w][tid]); s += ssum[w][tid]; }
        if (perm) {
            // needles in the haystack's slot order (paired sets): the constant
            // is kept per image; max |D| per slot and per image come from the
            // haystack statistics
            const uint32_t img = perm[im];
            if (img != kPad && sumsq) sumsq[img] = s;
        } else {
            maxabs[im] = im < n ? m : kPad;
            if (sumsq) sumsq[im] = im < n ? s : 0;
        }
    }
}

__global__ void __launch_bounds__(kDeltaWaves * 64)
k_delta_prep(const uint32_t* __restrict__ images, uint32_t n, int needle_side,
             int8_t* __restrict__ planes, uint32_t ngroups, int64_t* __restrict__ sumsq,
             uint32_t* __restrict__ maxabs, const uint32_t* __restrict__ perm, int8_t* __restrict__ hplanes,
             const uint32_t* __restrict__ qflags)
{
    delta_group(images, n, needle_side, planes, ngroups, sumsq, maxabs, perm, blockIdx.x, hplanes, qflags);
}

// Haystack slot assignment.  k_hay_init marks every slot as padding;
// k_hay_stats (one wavefront per image) finds max |D|; k_hay_assign (one
// workgroup, prefix sums) gives images with |D| <= 15 the front slots and the
// others the back slots, both in image order, so the layout is deterministic.
__global__ void __launch_bounds__(256)
k_hay_init(uint32_t* __restrict__ perm, uint32_t* __restrict__ maxabs, int32_t* __restrict__ thr, uint32_t nslots)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nslots) {
        perm[s] = kPad;
        maxabs[s] = kPad;
        if (thr) thr[s] = INT_MIN;   // paired sets: thresholds per slot, none for padding
    }
}

__device__ void hay_stats_one(const uint32_t* __restrict__ images, uint32_t* __restrict__ maxabs_img,
                              uint32_t img, int lane)
{
    // each load instruction covers four rows: lane l holds columns
    // 4 (l % 16) .. 4 (l % 16) + 3 of row 4 it + l / 16
    const uint4* im = reinterpret_cast<const uint4*>(images + (size_t)img * NPIX);
    const bool first = (lane & 15) == 0;
    uint32_t mx = 0;
#pragma unroll 4
    for (int it = 0; it < NB / 4; ++it) {
        const uint4 v = im[it * 64 + lane];
        const uint32_t left = __shfl_up(v.w, 1, 64);   // column 4 (l % 16) - 1 of the same row
        const int64_t d0 = first ? 0 : (int64_t)v.x - (int64_t)left;
        const int64_t d1 = (int64_t)v.y - (int64_t)v.x;
        const int64_t d2 = (int64_t)v.z - (int64_t)v.y;
        const int64_t d3 = (int64_t)v.w - (int64_t)v.z;
        const uint64_t m01 = max((uint64_t)(d0 < 0 ? -d0 : d0), (uint64_t)(d1 < 0 ? -d1 : d1));
        const uint64_t m23 = max((uint64_t)(d2 < 0 ? -d2 : d2), (uint64_t)(d3 < 0 ? -d3 : d3));
        mx = (uint32_t)max((uint64_t)mx, min(max(m01, m23), (uint64_t)0xFFFFFFFEu));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    if (lane == 0) maxabs_img[img] = mx;
}

__global__ void __launch_bounds__(256)
k_hay_stats(const uint32_t* __restrict__ images, uint32_t n, uint32_t* __restrict__ maxabs_img)
{
    const uint32_t img = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (img < n) hay_stats_one(images, maxabs_img, img, threadIdx.x & 63);
}

__global__ void __launch_bounds__(256)
k_copy_u32(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// One workgroup of 1024 threads walks the images in rounds of 1024
// consecutive ones (coalesced loads, the next round prefetched); a workgroup
// scan of the small/other flags gives each image its slot in image order.
// A set ranked against itself (thr != nullptr) also gets, per image, its
// threshold in its slot, CRD(i, t(i)) minus the needle constant (none when
// t(i) is outside the set or max |D| > 127), and its rank's start value
// (0, or n for a true index outside the set: Sec. 4.1 step 6c).
__device__ void hay_assign_block(const uint32_t* __restrict__ maxabs_img, uint32_t n, uint32_t nslots,
                                 uint32_t* __restrict__ perm, uint32_t* __restrict__ maxabs,
                                 uint32_t* __restrict__ inv, const uint32_t* __restrict__ true_idx = nullptr,
                                 const int64_t* __restrict__ dstar = nullptr,
                                 const int64_t* __restrict__ sumsq = nullptr, int32_t* __restrict__ thr = nullptr,
                                 uint32_t* __restrict__ rank = nullptr)
{
    __shared__ uint32_t wsum[2][16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t base_s = 0, base_o = 0;   // small / other images of the earlier rounds
    uint32_t m_next = (uint32_t)tid < n ? maxabs_img[tid] : 0u;
    int par = 0;
    for (uint32_t r0 = 0; r0 < n; r0 += 1024, par ^= 1) {
        const uint32_t i = r0 + (uint32_t)tid;
        const bool live = i < n;
        const uint32_t m = m_next;
        if (i + 1024 < n) m_next = maxabs_img[i + 1024];
        const bool small = live && m <= kSmallD;
        const uint64_t bs = __ballot(small);
        if (lane == 0) wsum[par][wave] = (uint32_t)__popcll(bs);
        __syncthreads();   // one barrier a round: the two halves of wsum alternate
        uint32_t ps = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const uint32_t x = wsum[par][w];
            ps += w < wave ? x : 0u;
            tot += x;
        }
        const uint32_t small_before = ps + (uint32_t)__popcll(bs & below);   // in this round
        if (live) {
            const uint32_t slot = small ? base_s + small_before
                                        : nslots - 1 - (base_o + (uint32_t)tid - small_before);
            perm[slot] = i;
            maxabs[slot] = m;
            if (inv) inv[i] = slot;
            if (thr) {
                const bool in_set = true_idx[i] < n;
                int64_t th = dstar[i] - sumsq[i];
                th = min(max(th, (int64_t)INT_MIN + 1), (int64_t)INT_MAX);
                thr[slot] = (in_set && m <= kSlow) ? (int32_t)th : INT_MIN;
                rank[i] = in_set ? 0u : n;
            }
        }
        const uint32_t cnt = min(1024u, n - r0);
        base_s += tot;
        base_o += cnt - tot;
    }
}

__global__ void __launch_bounds__(1024)
k_hay_assign(const uint32_t* __restrict__ maxabs_img, uint32_t n, uint32_t nslots,
             uint32_t* __restrict__ perm, uint32_t* __restrict__ maxabs, uint32_t* __restrict__ inv,
             const uint32_t* __restrict__ true_idx, const int64_t* __restrict__ dstar,
             const int64_t* __restrict__ sumsq, int32_t* __restrict__ thr, uint32_t* __restrict__ rank)
{
    hay_assign_block(maxabs_img, n, nslots, perm, maxabs, inv, true_idx, dstar, sumsq, thr, rank);
}

// Paired sets: per tile of kFlagTile slots, bit 0 = some image with |D| <= 127 (the
// tile takes part in the contraction), bit 1 = some such image with |D| > 15
// (the tile needs the q phase).  One wavefront per tile.
__device__ void tile_flags_one(const uint32_t* __restrict__ maxabs, uint32_t* __restrict__ flags, uint32_t t,
                               int lane)
{
    static_assert(kFlagTile == 4 * 64, "one wavefront of uint4 loads per tile");
    const uint4 m = reinterpret_cast<const uint4*>(maxabs + (size_t)t * kFlagTile)[lane];
    const uint32_t mx[4] = {m.x, m.y, m.z, m.w};
    bool use = false, big = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        use |= mx[k] <= kSlow;
        big |= mx[k] > kSmallD && mx[k] <= kSlow;
    }
    const uint64_t bu = __ballot(use), bb = __ballot(big);
    if (lane == 0) flags[t] = (bu ? 1u : 0u) | (bb ? 2u : 0u);
}

__global__ void __launch_bounds__(256)
k_tile_flags(const uint32_t* __restrict__ maxabs, uint32_t tiles, uint32_t* __restrict__ flags)
{
    const uint32_t t = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t < tiles) tile_flags_one(maxabs, flags, t, threadIdx.x & 63);
}

// ------------------------------------------------------------ exact int64 CRD

// CRD(n, h) by Eq. 7 for one pair, summed by one wavefront in int64.  Each
// load instruction covers four rows: lane l holds columns 4 (l % 16) ..
// 4 (l % 16) + 3 of row 4 it + l / 16, and takes the column to their left from
// lane l - 1 (column 0 of a row has no delta and no term).
__device__ __forceinline__ int64_t crd_wave(const uint32_t* __restrict__ nimg, const uint32_t* __restrict__ himg,
                                            int lane)
{
    const uint4* a4 = reinterpret_cast<const uint4*>(nimg);
    const uint4* b4 = reinterpret_cast<const uint4*>(himg);
    const bool first = (lane & 15) == 0;
    auto term = [](uint32_t n1, uint32_t n0, uint32_t h1, uint32_t h0) -> int64_t {
        const int64_t dn = (int64_t)n1 - (int64_t)n0, dh = (int64_t)h1 - (int64_t)h0;
        return dn != 0 ? (dn - dh) * (dn - dh) : 0;   // only the needle's non-zero deltas count
    };
    int64_t s = 0;
#pragma unroll 4
    for (int it = 0; it < NB / 4; ++it) {
        const uint4 a = a4[it * 64 + lane], b = b4[it * 64 + lane];
        const uint32_t al = __shfl_up(a.w, 1, 64), bl = __shfl_up(b.w, 1, 64);
        if (!first) s += term(a.x, al, b.x, bl);
        s += term(a.y, a.x, b.y, b.x) + term(a.z, a.y, b.z, b.y) + term(a.w, a.z, b.w, b.z);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

// thr is indexed by needle, or by the needle's slot (inv) for paired sets.
__device__ void true_distance_one(const uint32_t* __restrict__ needles, const uint32_t* __restrict__ hay,
                                  uint32_t nh, const uint32_t* __restrict__ true_idx,
                                  const int64_t* __restrict__ sumsq, const uint32_t* __restrict__ nmax,
                                  int64_t* __restrict__ dstar, int32_t* __restrict__ thr, uint32_t* __restrict__ rank,
                                  const uint32_t* __restrict__ inv, uint32_t i, int lane)
{
    const uint32_t t = true_idx[i];
    const uint32_t ti = inv ? inv[i] : i;
    if (t >= nh) {
        if (lane == 0) { dstar[i] = -1; thr[ti] = INT_MIN; rank[i] = nh; }
        return;
    }
    const int64_t d = crd_wave(needles + (size_t)i * NPIX, hay + (size_t)t * NPIX, lane);
    if (lane == 0) {
        dstar[i] = d;
        int64_t th = d - sumsq[i];
        th = min(max(th, (int64_t)INT_MIN + 1), (int64_t)INT_MAX);
        thr[ti] = nmax[i] <= kSlow ? (int32_t)th : INT_MIN;
        rank[i] = 0;
    }
}

// A set ranked against itself: one wavefront reads image i and its true
// match t(i) once and finds max |D| of image i (saturating as k_hay_stats),
// its constant |D|^2 + 128 #(D != 0) and CRD(i, t(i)) (Eq. 6-7; -1 for a true
// index outside the set), with the bits of the int64 sums.  The slot
// assignment, which needs max |D| of every image first, turns them into
// thresholds.  Lane layout as crd_wave.  Per pixel the work is 32-bit: |D| is
// an unsigned absolute difference, squares are 32 x 32 -> 64-bit products,
// and D_n - D_h is exact in 32 bits while both deltas are below 2^30 in
// magnitude; a wavefront that meets a wider delta takes the distance from
// crd_wave instead.
__device__ void stats_true_one(const uint32_t* __restrict__ images, uint32_t n,
                               const uint32_t* __restrict__ true_idx, uint32_t* __restrict__ maxabs_img,
                               int64_t* __restrict__ sumsq, int64_t* __restrict__ dstar, uint32_t i, int lane)
{
    const uint32_t t = true_idx[i];
    const bool in_set = t < n;   // one needle per wavefront: uniform
    const uint32_t* nimg = images + (size_t)i * NPIX;
    const uint32_t* himg = images + (size_t)(in_set ? t : i) * NPIX;
    const uint4* a4 = reinterpret_cast<const uint4*>(nimg);
    const uint4* b4 = reinterpret_cast<const uint4*>(himg);
    const bool first = (lane & 15) == 0;
    uint32_t mx = 0, nz = 0, wide = 0;
    uint64_t sq = 0, s = 0;
#pragma unroll 4
    for (int it = 0; it < NB / 4; ++it) {
        const uint4 a = a4[it * 64 + lane];
        const uint4 b = b4[it * 64 + lane];
        const uint32_t al = __shfl_up(a.w, 1, 64), bl = __shfl_up(b.w, 1, 64);
        const uint32_t an[5] = {al, a.x, a.y, a.z, a.w}, bn[5] = {bl, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // column 0 of a row has no delta: no term, no statistic
            const bool none = k == 0 && first;
            const uint32_t ad = none ? 0u : __usad(an[k + 1], an[k], 0u);
            const uint32_t bd = none ? 0u : __usad(bn[k + 1], bn[k], 0u);
            mx = max(mx, ad);
            nz += min(ad, 1u);
            sq += (uint64_t)ad * ad;
            wide |= ad | bd;
            const int32_t e = (int32_t)((an[k + 1] - an[k]) - (bn[k + 1] - bn[k]));
            const uint32_t ae = ad ? (uint32_t)(e < 0 ? -e : e) : 0u;
            s += (uint64_t)ae * ae;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
        nz += (uint32_t)__shfl_xor((int)nz, o, 64);
        wide |= (uint32_t)__shfl_xor((int)wide, o, 64);
        sq += (uint64_t)__shfl_xor((long long)sq, o, 64);
        s += (uint64_t)__shfl_xor((long long)s, o, 64);
    }
    int64_t d = (int64_t)s;
    if (in_set && wide >= (1u << 30)) d = crd_wave(nimg, himg, lane);
    if (lane == 0) {
        maxabs_img[i] = min(mx, 0xFFFFFFFEu);
        sumsq[i] = (int64_t)(sq + 128ull * nz);
        dstar[i] = in_set ? d : -1;
    }
}

__global__ void __launch_bounds__(256)
k_stats_true(const uint32_t* __restrict__ images, uint32_t n, const uint32_t* __restrict__ true_idx,
             uint32_t* __restrict__ maxabs_img, int64_t* __restrict__ sumsq, int64_t* __restrict__ dstar)
{
    const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i < n) stats_true_one(images, n, true_idx, maxabs_img, sumsq, dstar, i, threadIdx.x & 63);
}

__global__ void __launch_bounds__(256)
k_true_distance(const uint32_t* __restrict__ needles, uint32_t nn, const uint32_t* __restrict__ hay, uint32_t nh,
                const uint32_t* __restrict__ true_idx, const int64_t* __restrict__ sumsq,
                const uint32_t* __restrict__ nmax, int64_t* __restrict__ dstar, int32_t* __restrict__ thr,
                uint32_t* __restrict__ rank, const uint32_t* __restrict__ inv)
{
    const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i < nn)
        true_distance_one(needles, hay, nh, true_idx, sumsq, nmax, dstar, thr, rank, inv, i, threadIdx.x & 63);
}

// ----------------------------------------------------------------- MFMA search

template <int WM, int WN, int MB, int NBK, int NS>
struct SearchCfg {
    static constexpr int kWM = WM, kWN = WN, kMB = MB, kNBK = NBK, kNS = NS;
    static constexpr int kWaves = WM * WN;
    static constexpr int kThreads = kWaves * 64;
    static constexpr int BM = WM * MB * 16;          // needles per tile
    static constexpr int BN = WN * NBK * 16;         // haystack images per tile
    static constexpr int GA = BM / 16, GB = BN / 16; // fragment groups per tile
    static constexpr int kFrags = GA + GB;           // 1 KiB fragments per stage (one image row)
    static constexpr int kStage = kFrags * (int)kFragBytes;
    static constexpr int kLPW = kFrags / kWaves;     // fragment loads per wave per stage
    // after the ring: early-exit votes (one word per wave), the tile's needle
    // thresholds (BM int32), haystack usability flags (BN bytes) and per-row
    // hit counts of the rank epilogue (BM uint32)
    static constexpr int kVote = NS * kStage;
    static constexpr int kThr = kVote + 64;
    static constexpr int kCol = kThr + BM * 4;
    static constexpr int kRow = kCol + ((BN + 15) & ~15);
    // tile pairs of a paired set also count the mirrored direction: the
    // column tile's thresholds (BN int32), the row tile's usability flags (BM
    // bytes) and per-column hit counts (BN uint32)
    static constexpr int kThrC = kRow + BM * 4;
    static constexpr int kRowOk = kThrC + BN * 4;
    static constexpr int kColCnt = kRowOk + ((BM + 15) & ~15);
    // ... and the original image ids of both tiles, for the final atomics
    static constexpr int kPermR = kColCnt + BN * 4;
    static constexpr int kPermC = kPermR + BM * 4;
    static constexpr int kLds = kPermC + BN * 4;
    static_assert(kFrags % kWaves == 0, "fragments must split evenly over the waves");
};

// 256 x 256 (needle x haystack) tile, 8 waves of 128 x 64, a 4-deep ring of
// one-row stages (4 x 32 KiB) filled by direct global -> LDS loads two stages
// ahead of their use (measured on MI355X: 3- and 5-deep rings are slower)
using Cfg = SearchCfg<2, 4, 8, 4, 4>;
static_assert(Cfg::BM == kFlagTile && Cfg::BN == kFlagTile, "paired tiles are the flag tiles");
// 128 x 256 tile (8 waves of 64 x 64, 4-deep ring of 24 KiB stages): less
// padding for needle sets of at most 128 images
using CfgS = SearchCfg<2, 4, 4, 4, 4>;

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding)
template <int V>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(V >= 0 && V < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((V & 15) | (7 << 4) | (15 << 8) | ((V >> 4) << 14));
}

// Workgroup barrier without a memory fence: the LDS data of a stage is
// published by each wave's own vmcnt wait on its direct-to-LDS loads (a
// fence would also drain the prefetches of later stages).  The empty asm
// statements keep the compiler from moving LDS accesses across it.
__device__ __forceinline__ void stage_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Tile `logical` of a tiles_m x tiles_n grid in an L2-friendly order: groups
// of 8 needle tiles are walked haystack tile by haystack tile.
__device__ __forceinline__ void tile_coords(uint32_t logical, uint32_t tiles_m, uint32_t tiles_n,
                                            uint32_t& tm, uint32_t& tn)
{
    constexpr uint32_t GM = 8;
    const uint32_t in_group = GM * tiles_n;
    const uint32_t first_m = (logical / in_group) * GM;
    const uint32_t gsz = min(tiles_m - first_m, GM);
    tm = first_m + (logical % in_group) % gsz;
    tn = (logical % in_group) / gsz;
}

// Inclusive prefix sum of x over the lane's row of 16 lanes (DPP row shifts,
// zero shifted in): lane 15 of each row ends with the row's total.
__device__ __forceinline__ uint32_t row16_prefix_sum(uint32_t x)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);   // row_shr:8
    return x;
}

// Global memory through the global address space: a generic (flat) access
// also counts in the LDS counter, so that every LDS wait issued after it
// (a barrier's, for one) would also wait for it.
template <class T>
__device__ __forceinline__ T ldg(const T* p)
{
    return *(const __attribute__((address_space(1))) T*)p;
}

// A workgroup-uniform word through the constant address space (a scalar
// load): for data that no kernel running at the same time writes
__device__ __forceinline__ uint32_t ldc(const uint32_t* p)
{
    return *(const __attribute__((address_space(4))) uint32_t*)p;
}

__device__ __forceinline__ void red_add(uint32_t* p, uint32_t v)
{
    __hip_atomic_fetch_add((__attribute__((address_space(1))) uint32_t*)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// LDS add without a result, in asm: written through the builtin, the
// compiler waits for every direct-to-LDS load in flight before it (it cannot
// tell that the ring slots and the count words are disjoint), which would
// drain the ring where the count runs between two phases.  LDS operations
// retire in order, so the compiler's own LDS waits stay correct (only
// stricter) with this one among them; a workgroup barrier with its fence
// orders it before the counts are read.
__device__ __forceinline__ void lds_add_u32(uint32_t* p, uint32_t v)
{
    const uint32_t a = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint32_t*)p;
    asm volatile("ds_add_u32 %0, %1" ::"v"(a), "v"(v) : "memory");
}

// Thresholds as the counts use them: limited to +-2^30, which changes no
// comparison (an accumulator of the int8 path stays below 2^28 in
// magnitude; INT_MIN, no count, becomes -2^30), so that below() cannot
// overflow.
__device__ __forceinline__ int32_t clamp_thr(int32_t t)
{
    return min(max(t, -(1 << 30)), 1 << 30);
}

// [acc < t] as the sign bit of the difference: plain vector arithmetic, no
// compare mask (whose readers need wait states after each compare)
__device__ __forceinline__ uint32_t below(int32_t acc, int32_t t)
{
    return ((uint32_t)acc - (uint32_t)t) >> 31;   // (unsigned: kept as arithmetic)
}

// Row bases of the planes a tile streams in each phase.
struct StageSrc { const int8_t *a0, *a1, *a2, *b0, *b1, *b2; };

// Direct global -> LDS loads of stage t into ring slot `slot`: this wave's
// kLPW fragments, fragment j being fragment wv + j * kWaves of the stage (the
// GA needle fragments first, then the GB haystack fragments); voff[j] is its
// group offset plus the lane's 16 bytes.  Values only (no references into the
// caller), so the selects below stay scalar.
template <class C>
__device__ __forceinline__ void issue_stage(int8_t* lds, int slot, int t, int wv, StageSrc src,
                                            const uint32_t (&voff)[C::kLPW])
{
    constexpr int kJA = C::GA / C::kWaves;
    const int p = t / NB;
    const size_t roff = (size_t)(t % NB) * kFragBytes;
    const int8_t* sa = (p == 0 ? src.a0 : (p == 1 ? src.a1 : src.a2)) + roff;
    const int8_t* sb = (p == 0 ? src.b0 : (p == 1 ? src.b1 : src.b2)) + roff;
    int8_t* dst = lds + slot * C::kStage;
#pragma unroll
    for (int j = 0; j < C::kLPW; ++j) {
        // the offset is re-read here (opaque), so that its zero extension is
        // formed next to the load and the load takes the scalar-base form
        // (a 32-bit offset register instead of a 64-bit address per fragment)
        uint32_t o = voff[j];
        asm volatile("" : "+v"(o));
        const int8_t* g = (j < kJA ? sa : sb) + o;
        __builtin_amdgcn_global_load_lds(
            (const void __attribute__((address_space(1)))*)g,
            (void __attribute__((address_space(3)))*)(dst + (wv + j * C::kWaves) * (int)kFragBytes), 16, 0, 0);
    }
}

// Passes over one tile: kModePlain, the whole tile (rows needles, columns
// haystack images); kModePair, both directions of the tile pair (I, J) =
// (tm, tn) of a paired set whose images all have |D| <= 15, in one pass of
// three phases: the cross term -<D_I, D_J> (the same for both directions),
// doubled and kept in `cslot`; then <m_I, r_J>, after which the rows (needles
// of tile I against the haystack images of tile J) are counted; then
// <r_I, m_J> from zero, to which the kept cross term is added, after which
// the columns (needles of tile J against the haystack images of tile I) are
// counted.
// kModeRank is kModePlain known to be in rank mode (no distance matrix):
// the kernels that only rank (the persistent and the scan kernels) carry no
// matrix epilogue.
enum { kModePlain = 0, kModePair = 1, kModeRank = 2 };

// One BM x BN (needle x haystack) tile, or tile pair: every workgroup thread
// takes part.  EXIT compiles in the early exit of rank mode (taken when
// A.early_exit is set).  cslot (pair mode): this workgroup's BM x BN int32
// slot.
template <class C, bool EXIT, int MODE = kModePlain>
__device__ void search_tile(const SearchArgs& A, uint32_t tm, uint32_t tn, int8_t* lds, int32_t* cslot = nullptr)
{
    static_assert(MODE != kModePair || (!EXIT && C::BM == C::BN), "tile pairs: square tiles, no early exit");
    // the thread index is made opaque here so that nothing derived from it is
    // hoisted out of a persistent kernel's item loop (register pressure)
    int tid_ = threadIdx.x;
    asm volatile("" : "+v"(tid_));
    const int tid = tid_, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / C::kWN, wn = wave % C::kWN;
    const uint32_t ga0 = tm * C::GA, gb0 = tn * C::GB;

    // q phase needed iff some usable haystack image of the tile has
    // 15 < |D| <= 127; a tile without any usable haystack image is skipped.
    // The same loads fill the tile's usable-column flags and (rank mode) its
    // needle thresholds in LDS past the ring, for the epilogue and the early
    // exit votes: issued together, they cost one load latency per tile, and
    // the epilogue reads no global memory in rank mode.
    int32_t* thr_l = reinterpret_cast<int32_t*>(lds + C::kThr);
    uint8_t* col_l = reinterpret_cast<uint8_t*>(lds + C::kCol);
    uint32_t* rowcnt = reinterpret_cast<uint32_t*>(lds + C::kRow);
    int32_t* thrc_l = reinterpret_cast<int32_t*>(lds + C::kThrC);      // pair: tile J's thresholds
    uint8_t* rowok_l = reinterpret_cast<uint8_t*>(lds + C::kRowOk);    // pair: tile I's usable flags
    uint32_t* colcnt = reinterpret_cast<uint32_t*>(lds + C::kColCnt);  // pair: tile J's counts
    uint32_t* permr_l = reinterpret_cast<uint32_t*>(lds + C::kPermR);  // pair: image ids of tile I
    uint32_t* permc_l = reinterpret_cast<uint32_t*>(lds + C::kPermC);  // pair: image ids of tile J
    const bool ranks = MODE != kModePlain || A.matrix == nullptr;
    // needle rows with a threshold: the needles, or every slot of a paired set
    const uint32_t nrows = A.paired ? A.a_groups * kGroup : A.nn;

    // Block (mb, nb) of wave (wm, wn) in `cslot`: the tile's 16 x 16 blocks,
    // row-block major, each as the 64 lanes hold it (16 bytes per lane), so a
    // lane reads back exactly what it wrote; as int16, blocks nb and nb + 1
    // share block nb's 16 bytes.  Buffer accesses: the lane's 16 bytes are
    // the only per-lane offset, the block's offset is a scalar, and the
    // resource's size (one slot) bounds every access.
    static_assert(C::kNBK % 2 == 0, "int16 cross terms pack pairs of blocks");
    const int cwave = (__builtin_amdgcn_readfirstlane(wm) * C::kMB * (C::kWN * C::kNBK) +
                       __builtin_amdgcn_readfirstlane(wn) * C::kNBK) * 1024;
    auto cslot_soff = [&](int mb, int nb) { return cwave + (mb * (C::kWN * C::kNBK) + nb) * 1024; };
    // the lane's 16-byte offset, computed where it is used (nothing to keep
    // live, or to spill, across the stage loop)
    auto cslot_voff = []() {
        uint32_t v;
        asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0\n\tv_lshlrev_b32 %0, 4, %0"
                     : "=v"(v));
        return v;
    };
    // the lane index, recomputed where it is used (likewise)
    auto lane_here = []() {
        int v;
        asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(v));
        return v;
    };
    // (the slot address is workgroup-uniform: scalar registers, so that the
    // compiler needs no per-lane loop over resource values)
    // (readfirstlane returns a signed int: each half is taken back as
    // uint32_t before widening, so bit 31 of the low half is not sign-extended)
    const uint64_t caddr = reinterpret_cast<uint64_t>(MODE == kModePair ? cslot : nullptr);
    const uint32_t c_hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(caddr >> 32));
    const uint32_t c_lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)caddr);
    int32_t* const cslot_u = reinterpret_cast<int32_t*>(((uint64_t)c_hi << 32) | (uint64_t)c_lo);
    const __amdgpu_buffer_rsrc_t crsrc = __builtin_amdgcn_make_buffer_rsrc(cslot_u, 0, C::BM * C::BN * 4, kBufferWord3);
    v4i acc[C::kMB][C::kNBK];
    bool c16 = false;   // pair mode: the wave's cross term fits int16 (wave-uniform)

    int flags = 0;
    constexpr int kPro = C::BM > C::BN ? C::BM : C::BN;
    if constexpr (MODE == kModePair) {
        // Both tiles are needles and haystack images: six loads before any
        // use (every slot of a paired set has a threshold word).  (Issuing
        // the ring's first stages between the loads and their uses, to
        // overlap the two latencies, pushed the stage loops into scratch.)
        static_assert(C::BM == C::BN && C::BM <= C::kThreads, "one prologue slot per thread");
        const int j = tid < C::BM ? tid : 0;
        const uint32_t mi = ldg(A.hmax + ga0 * 16 + j), mj = ldg(A.hmax + gb0 * 16 + j);
        const int32_t ti = ldg(A.thr + ga0 * 16 + j), tj = ldg(A.thr + gb0 * 16 + j);
        const uint32_t pi = ldg(A.nperm + ga0 * 16 + j), pj = ldg(A.nperm + gb0 * 16 + j);
        if (tid < C::BM) {
            flags |= (mi <= kSlow || mj <= kSlow) ? 2 : 0;
            flags |= (ti != INT_MIN || tj != INT_MIN) ? 4 : 0;
            flags |= (mj > kSlow) ? 8 : 0;    // a column (tile J image) is not usable
            flags |= (mi > kSlow) ? 16 : 0;   // a row (tile I image) is not usable
            col_l[j] = mj <= kSlow ? 1 : 0;
            rowok_l[j] = mi <= kSlow ? 1 : 0;
            thr_l[j] = clamp_thr(ti);
            thrc_l[j] = clamp_thr(tj);
            rowcnt[j] = 0u;
            colcnt[j] = 0u;
            permr_l[j] = pi;
            permc_l[j] = pj;
        }
    }
    for (int j = tid; j < kPro; j += C::kThreads) {
        if constexpr (MODE == kModePair) {
            break;
        } else {
            // both loads before either value is used
            const uint32_t m = j < C::BN ? ldg(A.hmax + gb0 * 16 + j) : kPad;
            const uint32_t row = ga0 * 16 + j;
            const int32_t t = (ranks && j < C::BM && row < nrows) ? ldg(A.thr + row) : INT_MIN;
            if (j < C::BN) {
                flags |= (m > kSmallD && m <= kSlow) ? 1 : 0;
                flags |= (m <= kSlow) ? 2 : 0;
                flags |= (m > kSlow) ? 8 : 0;                // a column is not usable
                col_l[j] = m <= kSlow ? 1 : 0;               // padding and |D| > 127 excluded
            }
            if (j < C::BM) {
                flags |= (t != INT_MIN) ? 4 : 0;
                thr_l[j] = clamp_thr(t);
                rowcnt[j] = 0u;
            }
        }
    }
    // workgroup OR of the flags through the words after the early-exit vote
    // words (all of the LDS is the kernel's dynamic block: no static shared
    // array is allocated); they stay for the epilogue, which reads them again
    // rather than keep the flags in registers through the stage loop
    static_assert(C::kWaves <= 8, "16 words hold the votes and the flags");
    volatile __attribute__((address_space(3))) uint32_t* red =
        (volatile __attribute__((address_space(3))) uint32_t*)(lds + C::kVote) + 8;
    auto tile_flags_lds = [&]() {
        int all = 0;
#pragma unroll
        for (int w = 0; w < C::kWaves; ++w) all |= (int)red[w];
        return __builtin_amdgcn_readfirstlane(all);   // uniform: scalar control flow
    };
    {
        uint32_t w = 0;
#pragma unroll
        for (int b = 0; b < 5; ++b) w |= __ballot(flags & (1 << b)) ? 1u << b : 0u;
        if (lane == 0) red[wave] = w;
        __syncthreads();
        flags = tile_flags_lds();
    }
    const bool hq = MODE != kModePair && (flags & 1) != 0;
    // no usable haystack image, or no needle that can count
    if (!(flags & 2) || (ranks && !(flags & 4))) return;
    // Stage s = phase s / 64, image row s % 64.  Phase -> planes: needle planes
    // 0 = D, 1 = mask; haystack planes 0 = D, 1 = r, 2 = q (D^2 = 256 q + r + 128).
    // Each wave moves kLPW whole fragments (1 KiB, one instruction each) from
    // global memory straight into the stage's LDS slot.  Fragment j of wave w
    // is fragment w + j * kWaves of the stage (the GA needle groups, then the
    // GB haystack groups), so whether it comes from the needle or the haystack
    // planes is known at compile time; its group offset and the lane's 16
    // bytes are a per-tile 32-bit offset, and per stage only the two
    // wave-uniform plane-row bases change.
    static_assert(C::GA % C::kWaves == 0, "needle fragments must split evenly over the waves");
    constexpr int kJA = C::GA / C::kWaves;             // fragments per wave from the needle planes
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const size_t a_ps = (size_t)A.a_groups * kPlaneGroupBytes, b_ps = (size_t)A.b_groups * kPlaneGroupBytes;
    const int8_t* a_base = A.a_planes + (size_t)ga0 * kPlaneGroupBytes;
    const int8_t* b_base = A.b_planes + (size_t)gb0 * kPlaneGroupBytes;
    uint32_t voff[C::kLPW];
#pragma unroll
    for (int j = 0; j < C::kLPW; ++j) {
        const int g = wv + j * C::kWaves - (j < kJA ? 0 : C::GA);
        voff[j] = (uint32_t)g * (uint32_t)kPlaneGroupBytes + (uint32_t)lane * 16;
    }
    // planes of phases 0, 1: needles D, mask; haystack D, r.  With the q
    // phase first (hq): needles mask, D, mask; haystack q, D, r.  Pair mode:
    // needles D, mask of tile I against haystack D, r of tile J, then the r
    // plane of tile I (haystack planes) against the mask of tile J (needle
    // planes).  A paired set keeps one D plane, the haystack's (same slot
    // order).
    auto plane_src = [&](bool hq) {
        const int8_t* a_d = (MODE == kModePair || A.paired) ? A.b_planes + (size_t)ga0 * kPlaneGroupBytes : a_base;
        const int8_t* a_p0 = hq ? a_base + a_ps : a_d;
        const int8_t* a_p1 = hq ? a_d : a_base + a_ps;
        const int8_t* a_p2 = MODE == kModePair ? A.b_planes + (size_t)ga0 * kPlaneGroupBytes + b_ps : a_p0;
        const int8_t* b_p0 = b_base + (hq ? 2 * b_ps : 0);
        const int8_t* b_p1 = b_base + (hq ? 0 : b_ps);
        const int8_t* b_p2 = MODE == kModePair ? A.a_planes + (size_t)gb0 * kPlaneGroupBytes + a_ps : b_base + b_ps;
        return StageSrc{a_p0, a_p1, a_p2, b_p0, b_p1, b_p2};
    };

    const int nstage = (MODE == kModePair || hq ? 3 : 2) * NB;
    const int last = nstage - 1;
    const StageSrc src = plane_src(hq);
    auto issue = [&](int slot, int t) { issue_stage<C>(lds, slot, min(t, last), wv, src, voff); };

    auto zero_acc = [&]() {
#pragma unroll
        for (int mb = 0; mb < C::kMB; ++mb)
#pragma unroll
            for (int nb = 0; nb < C::kNBK; ++nb) acc[mb][nb] = v4i{0, 0, 0, 0};
    };
    zero_acc();

    struct Frags { v4i a[C::kMB]; v4i b[C::kNBK]; };
    auto read_frags = [&](int slot, Frags& F) {
        const int8_t* sA = lds + slot * C::kStage + lane * 16;
        const int8_t* sB = sA + C::GA * (int)kFragBytes;
#pragma unroll
        for (int nb = 0; nb < C::kNBK; ++nb)
            F.b[nb] = *reinterpret_cast<const v4i*>(sB + (wn * C::kNBK + nb) * (int)kFragBytes);
#pragma unroll
        for (int mb = 0; mb < C::kMB; ++mb)
            F.a[mb] = *reinterpret_cast<const v4i*>(sA + (wm * C::kMB + mb) * (int)kFragBytes);
    };
    // One pipeline step: make stage s+1 visible, refill the slot of stage s-1
    // with stage s+NS-1, then run stage s's MFMAs (fragments fetched one step
    // earlier) interleaved with the LDS reads of stage s+1's fragments, so
    // the reads of one stage overlap the matrix work of the previous one.  The
    // loop is unrolled NS times, so every ring slot is a compile-time
    // constant.  Loads and reads are issued on every step (past the last
    // stage the loads repeat the last row into a dead slot and the reads take
    // a stale slot that is never used), which keeps them in the MFMAs' basic
    // block; the loads go out after the first MFMA and the reads after the
    // next ones, so that the wait in front of the MFMAs covers only the
    // previous step's reads.
    // Early exit (rank mode): the last phase adds <m, r> with r >= -128, so
    // after k of its 64 rows no partial sum can fall by more than
    // 128 * 63 * (64 - k) (all remaining deltas of the needle non-zero).  Once
    // no pair of the tile is below its needle's threshold by that margin none
    // will end below it, and the tile adds nothing to any rank.  Checked every
    // 16 rows of that phase: each wave votes through LDS, the next stage
    // barrier publishes the votes.
    // (the votes read the tile's thresholds and usable columns from LDS:
    // global loads there would drain the stage loads in flight)
    const bool exit_ok = EXIT && A.early_exit && A.thr && ranks;
    volatile __attribute__((address_space(3))) uint32_t* votes =
        (volatile __attribute__((address_space(3))) uint32_t*)(lds + C::kVote);
    const int last_phase = nstage - NB;
    auto vote = [&](int32_t slack) {
        bool alive = false;
        const int cl = lane & 15, rq = lane >> 4;
        bool colok[C::kNBK];
#pragma unroll
        for (int nb = 0; nb < C::kNBK; ++nb) colok[nb] = col_l[(wn * C::kNBK + nb) * 16 + cl] != 0;
#pragma unroll
        for (int mb = 0; mb < C::kMB; ++mb) {
            // one block row at a time (four thresholds live), in program order
            const v4i t = *reinterpret_cast<const v4i*>(thr_l + (wm * C::kMB + mb) * 16 + 4 * rq);
#pragma unroll
            for (int nb = 0; nb < C::kNBK; ++nb)   // |acc| + slack stays far from the int32 limits
                alive |= colok[nb] && (acc[mb][nb].x - slack < t.x || acc[mb][nb].y - slack < t.y ||
                                       acc[mb][nb].z - slack < t.z || acc[mb][nb].w - slack < t.w);
            __builtin_amdgcn_sched_barrier(0);
        }
        const uint64_t any_alive = __ballot(alive);   // every lane takes part
        if (lane == 0) votes[wave] = any_alive != 0 ? 1u : 0u;
    };
    auto all_done = [&]() -> bool {
        uint32_t any = 0;
#pragma unroll
        for (int w = 0; w < C::kWaves; ++w) any |= votes[w];
        return __builtin_amdgcn_readfirstlane(any) == 0;
    };

    // Rank epilogue of the rows.  16x16 accumulator layout: lane l holds
    // column l % 16 and rows 4 * (l / 16) + v of its block, v = 0..3.  Per
    // lane, the counts of its four rows of block mb (each at most kNBK)
    // packed one per byte; a DPP prefix sum over the lane's row of 16 lanes
    // (the lanes holding those rows' 16 columns) leaves the block rows'
    // counts in lane 15 of it, at most 16 * kNBK < 256 per byte.  The kWN
    // waves sharing a needle row add them in LDS (zeroed in the prologue);
    // one global atomic per row of the tile follows at the end.
    auto count_rows = [&]() {
        static_assert(16 * C::kNBK < 256, "row counts must fit a byte");
        // (two copies: without the per-column test when every column is usable)
        auto body = [&](auto all_usable) {
            constexpr bool kAll = decltype(all_usable)::value;
            const int ln = lane_here(), cl = ln & 15, rq = ln >> 4;
            const int wm = wv / C::kWN, wn = wv % C::kWN;   // scalar
            uint32_t colok[C::kNBK];
#pragma unroll
            for (int nb = 0; nb < C::kNBK; ++nb) colok[nb] = kAll ? 1u : col_l[(wn * C::kNBK + nb) * 16 + cl];
#pragma unroll
            for (int mb = 0; mb < C::kMB; ++mb) {
                // the four thresholds of this lane's rows in the block (INT_MIN past the needles)
                const v4i t4 = *reinterpret_cast<const v4i*>(thr_l + (wm * C::kMB + mb) * 16 + 4 * rq);
                uint32_t packed = 0;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    uint32_t cnt = 0;
#pragma unroll
                    for (int nb = 0; nb < C::kNBK; ++nb)
                        cnt += kAll ? below(acc[mb][nb][v], t4[v]) : below(acc[mb][nb][v], t4[v]) & colok[nb];
                    packed |= cnt << (8 * v);
                }
                packed = row16_prefix_sum(packed);
                if (cl == 15) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const uint32_t cnt = (packed >> (8 * v)) & 0xFFu;
                        const int lrow = (wm * C::kMB + mb) * 16 + 4 * rq + v;   // row within the tile
                        // (every row of a tile pair is a slot of the set;
                        // no wait for the ring's loads in flight)
                        if constexpr (MODE == kModePair) {
                            lds_add_u32(rowcnt + lrow, cnt);   // (no branch per count)
                        } else {
                            if (cnt && ga0 * 16 + (uint32_t)lrow < nrows) atomicAdd(rowcnt + lrow, cnt);
                        }
                    }
                }
            }
        };
        if (!(tile_flags_lds() & 8)) body(std::true_type{});   // every column usable
        else body(std::false_type{});
    };

    auto step = [&](int k, int s, const Frags& cur, Frags& nxt) {   // k = s % NS, a literal
        // outstanding loads beyond stage s+1: stages s+2 .. s+NS-2
        wait_vmcnt<(C::kNS - 3) * C::kLPW>();
        stage_barrier();
        issue((k + C::kNS - 1) % C::kNS, s + C::kNS - 1);
        read_frags((k + 1) % C::kNS, nxt);
#pragma unroll
        for (int mb = 0; mb < C::kMB; ++mb)
#pragma unroll
            for (int nb = 0; nb < C::kNBK; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(cur.a[mb], cur.b[nb], acc[mb][nb], 0, 0, 0);
        // schedule: 1 MFMA, the stage loads, then the fragment reads spread
        // over the MFMAs: 3 reads after every 6 MFMAs when the counts allow
        // (measured best for the 256 x 256 tile), else 1 read after every 2
        // (the first pair has one MFMA when there are only twice as many
        // MFMAs as reads); then the rest of the MFMAs
        constexpr int kReads = C::kMB + C::kNBK, kMfma = C::kMB * C::kNBK;
        static_assert(2 * kReads <= kMfma, "interleave pattern");
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);          // MFMA
        __builtin_amdgcn_sched_group_barrier(0x020, C::kLPW, 0);    // global -> LDS loads
        if constexpr (kReads % 3 == 0 && 1 + 2 * kReads <= kMfma) {
#pragma unroll
            for (int i = 0; i < kReads / 3; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 6, 0);   // MFMA
                __builtin_amdgcn_sched_group_barrier(0x100, 3, 0);   // LDS read
            }
            constexpr int kRest = kMfma - 1 - 2 * kReads;
            if constexpr (kRest > 0) __builtin_amdgcn_sched_group_barrier(0x008, kRest, 0);
        } else {
            constexpr bool kTight = 1 + 2 * kReads > kMfma;
            if constexpr (kTight) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            }
#pragma unroll
            for (int i = kTight ? 1 : 0; i < kReads; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);   // MFMA
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
            }
            constexpr int kRest = kMfma - 1 - 2 * kReads + (kTight ? 1 : 0);
            if constexpr (kRest > 0) __builtin_amdgcn_sched_group_barrier(0x008, kRest, 0);
        }
        if constexpr (MODE != kModePair) {
            if (k == C::kNS - 1 && (s + 1) % NB == 0 && s + 1 < nstage) {
                // end of a phase: scale the partial sum (x -128 after q, x -2
                // after D.D)
                const int sh = (hq && s + 1 == NB) ? 7 : 1;
#pragma unroll
                for (int mb = 0; mb < C::kMB; ++mb)
#pragma unroll
                    for (int nb = 0; nb < C::kNBK; ++nb) acc[mb][nb] = -(acc[mb][nb] << sh);
            }
        }
    };

    // Pair mode, end of the cross phase: -2 <D_I, D_J> kept for the third
    // phase, as int16 when every value of the wave fits (blocks nb and nb + 1
    // share block nb's 16 bytes: half the bytes), else as int32.
    auto keep_cross = [&]() {
#pragma unroll
        for (int mb = 0; mb < C::kMB; ++mb)
#pragma unroll
            for (int nb = 0; nb < C::kNBK; ++nb) acc[mb][nb] = -(acc[mb][nb] << 1);
        int32_t lo = 0, hi = 0;
#pragma unroll
        for (int mb = 0; mb < C::kMB; ++mb)
#pragma unroll
            for (int nb = 0; nb < C::kNBK; ++nb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    lo = min(lo, acc[mb][nb][v]);
                    hi = max(hi, acc[mb][nb][v]);
                }
        c16 = __ballot(lo < -32768 || hi > 32767) == 0;
        const uint32_t cvo = cslot_voff();
        // Loads and stores share the vector memory counter and need not
        // retire in order with respect to each other: the stores (and the
        // ring's stages in flight) retire before the next ring wait, so that
        // every ring wait counts loads only.
        if (c16) {
#pragma unroll
            for (int mb = 0; mb < C::kMB; ++mb)
#pragma unroll
                for (int nb = 0; nb < C::kNBK; nb += 2) {
                    v4i w;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        w[v] = (int32_t)(((uint32_t)acc[mb][nb][v] & 0xFFFFu) |
                                         ((uint32_t)acc[mb][nb + 1][v] << 16));
                    __builtin_amdgcn_raw_buffer_store_b128(w, crsrc, cvo, cslot_soff(mb, nb), 0);
                    // a store of more than 8 bytes reads its data registers
                    // after it issues: two wait states before the next pack
                    // may rewrite them
                    __builtin_amdgcn_sched_barrier(0);
                    asm volatile("s_nop 1");
                    __builtin_amdgcn_sched_barrier(0);
                }
        } else {
#pragma unroll
            for (int mb = 0; mb < C::kMB; ++mb)
#pragma unroll
                for (int nb = 0; nb < C::kNBK; ++nb)
                    __builtin_amdgcn_raw_buffer_store_b128(acc[mb][nb], crsrc, cvo, cslot_soff(mb, nb), 0);
        }
        wait_vmcnt<0>();
    };

    static_assert(C::kNS == 4 && NB % 4 == 0, "the loop below is unrolled for a 4-deep ring");
    issue(0, 0);
    issue(1, 1);
    issue(2, 2);
    wait_vmcnt<(C::kNS - 2) * C::kLPW>();
    stage_barrier();
    Frags fr0, fr1;
    read_frags(0, fr0);
    // stages [s0, s1), s0 and s1 multiples of 4
    auto run = [&](int s0, int s1) {
        for (int s = s0; s < s1; s += 4) {
            step(0, s, fr0, fr1);
            step(1, s + 1, fr1, fr0);
            step(2, s + 2, fr0, fr1);
            step(3, s + 3, fr1, fr0);
            // after 16, 32 and 48 rows of the last phase: vote, publish, decide
            if (exit_ok && s + 4 > last_phase && (s + 4 - last_phase) % 16 == 0 && s + 4 < nstage) {
                vote(128 * 63 * (NB - (s + 4 - last_phase)));
                __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): the votes are written
                stage_barrier();
                if (all_done()) {
                    wait_vmcnt<0>();   // no load may land in LDS after the tile is left
                    return true;
                }
            }
        }
        return false;
    };
    if constexpr (MODE == kModePair) {
        // one loop per phase, so that what happens between phases holds no
        // registers inside the loops; the ring keeps prefetching across
        run(0, NB);
        keep_cross();
        run(NB, 2 * NB);
        // end of the (I -> J) direction: its rows are counted (LDS only: the
        // stages in flight keep landing), and the (J -> I) r phase starts
        // from zero
        count_rows();
        zero_acc();
        run(2 * NB, 3 * NB);
    } else {
        if (run(0, nstage)) return;   // nstage is a multiple of 64
    }
    wait_vmcnt<0>();   // the repeated loads of the last steps have landed

    if constexpr (MODE == kModePair) {
        const int ln = lane_here(), cl = ln & 15, rq = ln >> 4;
        const int wm = wv / C::kWN, wn = wv % C::kWN;   // scalar
        // The kept cross term: this wave's own stores, retired in the cross
        // phase.  The loads are device-scope (cache policy sc1): they miss in
        // the CU's vector L1 and read the L2, so no line of the slot cached
        // by an earlier pair of this workgroup can be read instead.
        const uint32_t cvo = cslot_voff();
        if (c16) {
#pragma unroll
            for (int mb = 0; mb < C::kMB; ++mb) {
                v4i w[C::kNBK / 2];
#pragma unroll
                for (int nb = 0; nb < C::kNBK; nb += 2)
                    w[nb / 2] = __builtin_amdgcn_raw_buffer_load_b128(crsrc, cvo, cslot_soff(mb, nb), kDeviceScope);
#pragma unroll
                for (int nb = 0; nb < C::kNBK; nb += 2)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        acc[mb][nb][v] += (int32_t)((uint32_t)w[nb / 2][v] << 16) >> 16;   // low half, sign-extended
                        acc[mb][nb + 1][v] += w[nb / 2][v] >> 16;                         // high half (arithmetic)
                    }
            }
        } else {
#pragma unroll
            for (int mb = 0; mb < C::kMB; ++mb) {
                v4i w[C::kNBK];
#pragma unroll
                for (int nb = 0; nb < C::kNBK; ++nb)
                    w[nb] = __builtin_amdgcn_raw_buffer_load_b128(crsrc, cvo, cslot_soff(mb, nb), kDeviceScope);
#pragma unroll
                for (int nb = 0; nb < C::kNBK; ++nb) acc[mb][nb] += w[nb];
            }
        }
        // counts per column (needle of tile J): over the lane's 4 rows of
        // each block, the wave's row blocks, the 4 lanes of the column (l,
        // l ^ 16, l ^ 32, l ^ 48: lane-half swaps) and the kWM waves sharing
        // the column (LDS)
        static_assert(C::kNBK <= 4 && C::kMB * 16 < 256, "column counts must fit a byte each");
        auto body = [&](auto all_usable) {
            constexpr bool kAll = decltype(all_usable)::value;
            uint32_t packed = 0;
#pragma unroll
            for (int nb = 0; nb < C::kNBK; ++nb) {
                const int32_t t = thrc_l[(wn * C::kNBK + nb) * 16 + cl];
                uint32_t cnt = 0;
#pragma unroll
                for (int mb = 0; mb < C::kMB; ++mb) {
                    const uint32_t rowok =
                        kAll ? 0x01010101u
                             : *reinterpret_cast<const uint32_t*>(rowok_l + (wm * C::kMB + mb) * 16 + 4 * rq);
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        cnt += kAll ? below(acc[mb][nb][v], t) : below(acc[mb][nb][v], t) & (rowok >> (8 * v));
                }
                packed |= cnt << (8 * nb);
            }
            return packed;
        };
        // (every row usable: no per-row test)
        uint32_t packed = !(tile_flags_lds() & 16) ? body(std::true_type{}) : body(std::false_type{});
        {
            const auto h = __builtin_amdgcn_permlane32_swap(packed, packed, false, false);
            packed = h[0] + h[1];
            const auto q = __builtin_amdgcn_permlane16_swap(packed, packed, false, false);
            packed = q[0] + q[1];
        }
        if (rq == 0) {
#pragma unroll
            for (int nb = 0; nb < C::kNBK; ++nb) {
                const uint32_t cnt = (packed >> (8 * nb)) & 0xFFu;
                if (cnt) atomicAdd(colcnt + (wn * C::kNBK + nb) * 16 + cl, cnt);
            }
        }
        __syncthreads();
        // every slot of a paired set is a row (nrows covers the tiles)
        for (int j = tid; j < C::BM; j += C::kThreads) {
            const uint32_t r = rowcnt[j], c = colcnt[j];
            if (r) red_add(A.rank + permr_l[j], r);
            if (c) red_add(A.rank + permc_l[j], c);
        }
        return;
    }
    const int cl = lane & 15, rq = lane >> 4;
    if (ranks) {
        count_rows();
    } else {
        // original haystack index of each of the lane's columns (matrix mode)
        bool colok[C::kNBK];
        uint32_t col[C::kNBK];
#pragma unroll
        for (int nb = 0; nb < C::kNBK; ++nb) {
            const uint32_t slot = (gb0 + wn * C::kNBK + nb) * 16 + cl;
            colok[nb] = col_l[(wn * C::kNBK + nb) * 16 + cl] != 0;
            col[nb] = colok[nb] ? A.hperm[slot] : 0u;
        }
#pragma unroll
        for (int mb = 0; mb < C::kMB; ++mb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t row = ga0 * 16 + (uint32_t)((wm * C::kMB + mb) * 16 + 4 * rq + v);
                if (row < A.nn && A.nmax[row] <= kSlow) {
                    const int64_t base = A.sumsq[row];
#pragma unroll
                    for (int nb = 0; nb < C::kNBK; ++nb)
                        if (colok[nb]) A.matrix[(size_t)row * A.nh + col[nb]] = base + (int64_t)acc[mb][nb][v];
                }
            }
        }
    }
    if (ranks) {
        __syncthreads();
        for (int j = tid; j < C::BM; j += C::kThreads) {
            const uint32_t c = rowcnt[j], row = ga0 * 16 + (uint32_t)j;
            if (c && row < nrows) red_add(A.rank + (A.nperm ? ldg(A.nperm + row) : row), c);
        }
    }
}


// Both directions of tile pair (I, J) of a paired set.  A pair whose images
// all have |D| <= 15 computes the cross term once (one pass of three
// phases); a pair with a q phase on either side runs (I, J) and (J, I) as
// plain tiles.  cslot: this workgroup's BM x BN int32 slot.
template <class C>
__device__ void search_pair(const SearchArgs& A, uint32_t I, uint32_t J, int8_t* lds, int32_t* cslot)
{
    if (I != J) {
        const uint32_t fi = ldc(A.tile_flags + I), fj = ldc(A.tile_flags + J);
        if (!(fi & 1u) || !(fj & 1u)) return;   // one side has no usable image: neither direction counts
        if (!((fi | fj) & 2u)) {
            search_tile<C, false, kModePair>(A, I, J, lds, cslot);
            return;
        }
    }
    // plain tiles: the diagonal one, or both directions of a pair with a q
    // phase (one copy of the tile code, hence the loop)
    const uint32_t n = I == J ? 1u : 2u;
#pragma nounroll
    for (uint32_t d = 0; d < n; ++d) {
        if (d) __syncthreads();
        search_tile<C, false, kModeRank>(A, d ? J : I, d ? I : J, lds);
    }
}

// Next work item of a persistent search kernel: items [0, total) are split
// into 8 contiguous ranges, one per XCD (workgroup ids are dealt to the XCDs
// round robin, so the items that run at the same time on one XCD are
// neighbours and share fragments in its L2); a workgroup takes items from its
// own XCD's counter, then from the others' once its range is used up.  The
// item is broadcast through the first LDS word; returns total when done.
// (Claiming one item ahead, to hide the atomic's latency, was measured
// slower: a workgroup then holds a second item while others run dry at the
// end of the queue.)
__device__ __forceinline__ uint32_t next_item(uint32_t* __restrict__ counters, uint32_t total, uint32_t& visited,
                                              int8_t* lds)
{
    volatile __attribute__((address_space(3))) uint32_t* s_item =
        (volatile __attribute__((address_space(3))) uint32_t*)lds;
    const uint32_t xcd = blockIdx.x & 7u, per = (total + 7) / 8;
    if (threadIdx.x == 0) {
        uint32_t item = total;
        while (visited < 8) {
            const uint32_t x = (xcd + visited) & 7u;
            const uint32_t k = atomicAdd(counters + x, 1u);
            if (k < per && x * per + k < total) {
                item = x * per + k;
                break;
            }
            ++visited;
        }
        *s_item = item;
    }
    __syncthreads();
    // the item is the same in every lane: keep it in a scalar register.
    // (No second barrier: the word is next written by the ring's first stage
    // or by the next call, both behind a later workgroup barrier that every
    // wave reaches only after this read.)
    return __builtin_amdgcn_readfirstlane(*s_item);
}

// Persistent search over the tile pairs of one paired set (one workgroup per
// CU; each owns a BM x BN int32 slot of A.cross).
template <class C>
__global__ void __launch_bounds__(C::kThreads)
k_search_paired(SearchArgs A, uint32_t* __restrict__ counters)
{
    extern __shared__ __align__(16) int8_t lds[];
    const uint32_t total = pair_items(A.tiles_m);
    int32_t* cslot = A.cross + (size_t)blockIdx.x * C::BM * C::BN;
    uint32_t visited = 0;   // ranges used up (thread 0 only)
    for (;;) {
        const uint32_t item = next_item(counters, total, visited, lds);
        if (item >= total) break;
        uint32_t I, J;
        pair_coords(item, A.tiles_m, I, J);
        search_pair<C>(A, I, J, lds, cslot);
        __syncthreads();   // every wave is done with the ring before its first word is reused
    }
}

template <class C, bool EXIT>
__global__ void __launch_bounds__(C::kThreads)
k_search(SearchArgs A)
{
    extern __shared__ __align__(16) int8_t lds[];
    // consecutive workgroup ids land on different XCDs (round robin): gather
    // each XCD's ids into one contiguous range of the tile order so the tiles
    // resident on one XCD share fragments in its L2
    const uint32_t b = blockIdx.x;
    const uint32_t logical = (b & 7u) * A.per_xcd + (b >> 3);
    if (logical >= A.tiles_m * A.tiles_n) return;
    uint32_t tm, tn;
    tile_coords(logical, A.tiles_m, A.tiles_n, tm, tn);
    search_tile<C, EXIT>(A, tm, tn, lds);
}

// Persistent form for many searches.  The (job, tile) items (jobs stored
// largest first) are split into 8 contiguous ranges, one per XCD: workgroup
// ids are dealt to the XCDs round robin, so the tiles that run at the same
// time on one XCD are neighbours in the tile order and share fragments in its
// L2.  A workgroup takes items from its own XCD's counter, then from the
// others' once its range is used up.
template <class C, bool EXIT>
__global__ void __launch_bounds__(C::kThreads)
k_search_batched(const SearchJob* __restrict__ jobs, uint32_t njobs, uint32_t total, uint32_t* __restrict__ counters)
{
    extern __shared__ __align__(16) int8_t lds[];
    // the ring takes all of the LDS: the item is broadcast through its first
    // word, which no wave reads or fills between two items
    uint32_t visited = 0;   // ranges used up (thread 0 only)
    // the job of the last item and its item range: consecutive items mostly
    // belong to one job, which saves the dependent loads of the search
    uint32_t lo = 0, j_begin = 0, j_end = 0;
    for (;;) {
        const uint32_t item = next_item(counters, total, visited, lds);
        if (item >= total) break;
        // the job's arguments, loaded through the uniform item, stay scalar
        if (item < j_begin || item >= j_end) {
            uint32_t hi = njobs - 1;
            lo = 0;
            while (lo < hi) {
                const uint32_t mid = (lo + hi + 1) / 2;
                if (jobs[mid].tile_start <= item) lo = mid; else hi = mid - 1;
            }
            j_begin = jobs[lo].tile_start;
            j_end = lo + 1 < njobs ? jobs[lo + 1].tile_start : total;
        }
        const SearchArgs A = jobs[lo].A;
        bool done = false;
        if constexpr (!EXIT && C::BM == C::BN) {
            if (A.paired) {
                uint32_t I, J;
                pair_coords(item - jobs[lo].tile_start, A.tiles_m, I, J);
                search_pair<C>(A, I, J, lds, A.cross + (size_t)blockIdx.x * C::BM * C::BN);
                done = true;
            }
        }
        if (!done) {
            uint32_t tm, tn;
            tile_coords(item - jobs[lo].tile_start, A.tiles_m, A.tiles_n, tm, tn);
            search_tile<C, EXIT, kModeRank>(A, tm, tn, lds);   // batched jobs rank
        }
        __syncthreads();   // every wave is done with the ring before its first word is reused
    }
}

// One slice of a database scan (serving): item = (haystack tile of the slice,
// query, needle tile), haystack-tile major so that the workgroups running at
// the same time share the slice's haystack fragments in L2.
template <class C, bool EXIT>
__global__ void __launch_bounds__(C::kThreads)
k_search_scan(ScanTable T)
{
    extern __shared__ __align__(16) int8_t lds[];
    const uint32_t M = T.m_start[T.njobs];
    const uint32_t item = blockIdx.x;
    const uint32_t tnl = item / M, r = item % M;
    uint32_t k = 0;
    while (k + 1 < T.njobs && T.m_start[k + 1] <= r) ++k;
    const uint32_t tm = r - T.m_start[k];
    const uint32_t tn = (T.tile_begin + tnl) % T.db_tiles;
    search_tile<C, EXIT, kModeRank>(T.A[k], tm, tn, lds);   // a query ranks
}

// ------------------------------------------------------- out-of-range images

// lists[0] = #needles with |D| > 127, lists[1] = #haystack images with
// |D| > 127, then the needle ids (nn slots) and the haystack ids (nh slots).
// Order within a list is free (each entry is one independent unit of work).
// k_slow_reset clears the two counts; k_slow_lists takes one entry per thread
// (needles first, then the haystack) and appends by one atomic per wave.
__global__ void __launch_bounds__(64)
k_slow_reset(uint32_t* __restrict__ lists)
{
    if (threadIdx.x < 2) lists[threadIdx.x] = 0u;
}

__device__ __forceinline__ void slow_lists_entry(const uint32_t* __restrict__ nmax, uint32_t nn,
                                                 const uint32_t* __restrict__ hmax, uint32_t nh,
                                                 uint32_t* __restrict__ lists, uint64_t x)
{
    // x < nn: needle x; nn <= x < nn + nh: haystack image x - nn.  A wave may
    // straddle the two lists: each side gets its own ballot.
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    const bool is_n = x < nn, is_h = !is_n && x < (uint64_t)nn + nh;
    const bool slow_n = is_n && nmax[x] > kSlow;
    const bool slow_h = is_h && hmax[x - nn] > kSlow;
    const uint64_t bn = __ballot(slow_n), bh = __ballot(slow_h);
    uint32_t base_n = 0, base_h = 0;
    if (lane == 0) {
        if (bn) base_n = atomicAdd(lists + 0, (uint32_t)__popcll(bn));
        if (bh) base_h = atomicAdd(lists + 1, (uint32_t)__popcll(bh));
    }
    base_n = __shfl(base_n, 0, 64);
    base_h = __shfl(base_h, 0, 64);
    if (slow_n) lists[2 + base_n + __popcll(bn & below)] = (uint32_t)x;
    if (slow_h) lists[2 + (size_t)nn + base_h + __popcll(bh & below)] = (uint32_t)(x - nn);
}

__global__ void __launch_bounds__(256)
k_slow_lists(const uint32_t* __restrict__ nmax, uint32_t nn, const uint32_t* __restrict__ hmax, uint32_t nh,
             uint32_t* __restrict__ lists)
{
    slow_lists_entry(nmax, nn, hmax, nh, lists, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Every (needle, haystack) pair with an out-of-range image, by Eq. 7 in int64.
// A fixed grid of wavefronts walks the pair list; the list length is bounded
// by nn * nh, so every wave reaches the end.
__device__ void fallback_pairs(const uint32_t* __restrict__ needles, uint32_t nn, const uint32_t* __restrict__ hay,
                               uint32_t nh, const uint32_t* __restrict__ nmax, const uint32_t* __restrict__ lists,
                               const int64_t* __restrict__ dstar, uint32_t* __restrict__ rank,
                               int64_t* __restrict__ matrix, uint64_t wave_id, uint64_t nwaves)
{
    const int lane = threadIdx.x & 63;
    const uint64_t ns = lists[0], nhs = lists[1];
    const uint64_t part_a = ns * nh, total = part_a + nhs * nn;
    for (uint64_t w = wave_id; w < total; w += nwaves) {
        uint32_t i, j;
        if (w < part_a) {
            i = lists[2 + w / nh];
            j = (uint32_t)(w % nh);
        } else {
            const uint64_t w2 = w - part_a;
            j = lists[2 + (size_t)nn + w2 / nn];
            i = (uint32_t)(w2 % nn);
            if (nmax[i] > kSlow) continue;   // already done in part A
        }
        const int64_t d = crd_wave(needles + (size_t)i * NPIX, hay + (size_t)j * NPIX, lane);
        if (lane == 0) {
            if (matrix) matrix[(size_t)i * nh + j] = d;
            else if (dstar[i] >= 0 && d < dstar[i]) atomicAdd(rank + i, 1u);
        }
    }
}

__global__ void __launch_bounds__(256)
k_fallback(const uint32_t* __restrict__ needles, uint32_t nn, const uint32_t* __restrict__ hay, uint32_t nh,
           const uint32_t* __restrict__ nmax, const uint32_t* __restrict__ lists,
           const int64_t* __restrict__ dstar, uint32_t* __restrict__ rank, int64_t* __restrict__ matrix)
{
    fallback_pairs(needles, nn, hay, nh, nmax, lists, dstar, rank, matrix,
                   (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6),
                   (uint64_t)gridDim.x * (blockDim.x >> 6));
}

// ------------------------------------------------------------ batched prep

// job owning flat index x, given a per-job start offset selected by `which`
template <int which>
__device__ __forceinline__ uint32_t job_of(const SearchJob* __restrict__ jobs, uint32_t njobs, uint64_t x)
{
    uint32_t lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) / 2;
        const uint64_t st = which == 0 ? jobs[mid].ngrp_start : which == 1 ? jobs[mid].hslot_start
                          : which == 2 ? jobs[mid].himg_start : which == 3 ? jobs[mid].hgrp_start
                          : jobs[mid].needle_start;
        if (st <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// needle planes in image order; for a paired set (after the slot assignment)
// both plane sets in the haystack's slot order
__global__ void __launch_bounds__(kDeltaWaves * 64)
k_needle_prep_batched(const SearchJob* __restrict__ jobs, uint32_t njobs)
{
    const SearchJob& J = jobs[job_of<0>(jobs, njobs, blockIdx.x)];
    delta_group(J.needles, J.A.nn, J.A.paired ? 2 : 1, J.np.planes, J.np.ngroups,
                J.A.paired ? nullptr : J.np.sumsq, J.np.maxabs,
                J.A.paired ? J.hp.perm : nullptr, (uint32_t)(blockIdx.x - J.ngrp_start), J.hp.planes,
                J.A.paired ? J.A.tile_flags : nullptr);
}

__global__ void __launch_bounds__(256)
k_hay_init_batched(const SearchJob* __restrict__ jobs, uint32_t njobs, uint64_t total)
{
    const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= total) return;
    const SearchJob& J = jobs[job_of<1>(jobs, njobs, x)];
    const uint64_t s = x - J.hslot_start;
    J.hp.perm[s] = kPad;
    J.hp.maxabs[s] = kPad;
    if (J.A.paired) const_cast<int32_t*>(J.A.thr)[s] = INT_MIN;   // thresholds per slot
}

// paired sets: flags of every 256-slot tile (flattened over the jobs)
__global__ void __launch_bounds__(256)
k_tile_flags_batched(const SearchJob* __restrict__ jobs, uint32_t njobs, uint64_t total)
{
    const uint64_t t = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= total) return;
    const SearchJob& J = jobs[job_of<3>(jobs, njobs, t * (kFlagTile / kGroup))];
    tile_flags_one(J.hp.maxabs, const_cast<uint32_t*>(J.A.tile_flags),
                   (uint32_t)(t - J.hgrp_start / (kFlagTile / kGroup)), threadIdx.x & 63);
}

__global__ void __launch_bounds__(256)
k_hay_stats_batched(const SearchJob* __restrict__ jobs, uint32_t njobs, uint64_t total)
{
    const uint64_t x = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (x >= total) return;
    const SearchJob& J = jobs[job_of<2>(jobs, njobs, x)];
    const uint32_t img = (uint32_t)(x - J.himg_start);
    if (J.hay == J.needles && !J.A.paired) {
        // ranking a set against itself: the needle pass already found max |D|
        if ((threadIdx.x & 63) == 0) J.hp.maxabs_img[img] = J.np.maxabs[img];
    } else {
        hay_stats_one(J.hay, J.hp.maxabs_img, img, threadIdx.x & 63);
    }
}

__global__ void __launch_bounds__(1024)
k_hay_assign_batched(const SearchJob* __restrict__ jobs)
{
    const SearchJob& J = jobs[blockIdx.x];
    if (J.A.paired)
        hay_assign_block(J.hp.maxabs_img, J.A.nh, J.hp.ngroups * kGroup, J.hp.perm, J.hp.maxabs, J.hp.inv,
                         J.true_idx, J.dstar, J.np.sumsq, const_cast<int32_t*>(J.A.thr), J.A.rank);
    else
        hay_assign_block(J.hp.maxabs_img, J.A.nh, J.hp.ngroups * kGroup, J.hp.perm, J.hp.maxabs, J.hp.inv);
}

__global__ void __launch_bounds__(kDeltaWaves * 64)
k_hay_prep_batched(const SearchJob* __restrict__ jobs, uint32_t njobs)
{
    const SearchJob& J = jobs[job_of<3>(jobs, njobs, blockIdx.x)];
    delta_group(J.hay, J.A.nh, 0, J.hp.planes, J.hp.ngroups, nullptr, J.hp.maxabs, J.hp.perm,
                (uint32_t)(blockIdx.x - J.hgrp_start));
}

__global__ void __launch_bounds__(256)
k_true_distance_batched(const SearchJob* __restrict__ jobs, uint32_t njobs, uint64_t total)
{
    const uint64_t x = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (x >= total) return;
    const SearchJob& J = jobs[job_of<4>(jobs, njobs, x)];
    true_distance_one(J.needles, J.hay, J.A.nh, J.true_idx, J.np.sumsq, J.np.maxabs, J.dstar,
                      const_cast<int32_t*>(J.A.thr), J.A.rank, J.A.paired ? J.hp.inv : nullptr,
                      (uint32_t)(x - J.needle_start), threadIdx.x & 63);
}

// paired sets: statistics and true-match distances in one pass over the
// images (flattened over the jobs; needles and haystack are the same set)
__global__ void __launch_bounds__(256)
k_stats_true_batched(const SearchJob* __restrict__ jobs, uint32_t njobs, uint64_t total)
{
    const uint64_t x = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (x >= total) return;
    const SearchJob& J = jobs[job_of<4>(jobs, njobs, x)];
    stats_true_one(J.hay, J.A.nh, J.true_idx, J.hp.maxabs_img, J.np.sumsq, J.dstar, (uint32_t)(x - J.needle_start),
                   threadIdx.x & 63);
}

__global__ void __launch_bounds__(1024)
k_slow_lists_batched(const SearchJob* __restrict__ jobs)
{
    const SearchJob& J = jobs[blockIdx.x];
    if (threadIdx.x < 2) {
        atomicExch(J.lists + threadIdx.x, 0u);
        __threadfence();   // the counts are zero before any wave of the block adds to them
    }
    __syncthreads();
    const uint64_t total = (uint64_t)J.A.nn + J.A.nh;
    for (uint64_t x0 = 0; x0 < total; x0 += blockDim.x)   // uniform bound: every lane takes part in the ballots
        slow_lists_entry(J.np.maxabs, J.A.nn, J.hp.maxabs_img, J.A.nh, J.lists, x0 + threadIdx.x);
}

__global__ void __launch_bounds__(256)
k_fallback_batched(const SearchJob* __restrict__ jobs, uint32_t njobs)
{
    const uint64_t wave_id = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint32_t j = 0; j < njobs; ++j) {
        const SearchJob& J = jobs[j];
        fallback_pairs(J.needles, J.A.nn, J.hay, J.A.nh, J.np.maxabs, J.lists, J.dstar, J.A.rank, nullptr,
                       wave_id, nwaves);
    }
}

__global__ void k_zero_counters8(uint32_t* __restrict__ c) { if (threadIdx.x < 8) c[threadIdx.x] = 0u; }

}  // namespace

size_t search_groups(uint32_t n)
{
    const size_t g = (n + kGroup - 1) / kGroup;
    const size_t t = Cfg::GA > Cfg::GB ? Cfg::GA : Cfg::GB;
    return ((g + t - 1) / t) * t;
}

size_t haystack_slots(uint32_t nh)
{
    const size_t t = Cfg::BN;
    return ((size_t)nh + t - 1) / t * t + t;   // + one tile: a tile boundary inside the gap
}

hipError_t launch_delta_prep(const uint32_t* images, uint32_t n, int needle_side, const SearchPrep& p,
                             hipStream_t s, const uint32_t* known_maxabs)
{
    if (p.ngroups == 0) return hipSuccess;
    if (p.perm) {
        const uint32_t nslots = p.ngroups * kGroup;
        hipLaunchKernelGGL(k_hay_init, dim3((nslots + 255) / 256), dim3(256), 0, s, p.perm, p.maxabs,
                           (int32_t*)nullptr, nslots);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (n > 0) {
            if (known_maxabs)
                hipLaunchKernelGGL(k_copy_u32, dim3((n + 255) / 256), dim3(256), 0, s, known_maxabs, p.maxabs_img, n);
            else
                hipLaunchKernelGGL(k_hay_stats, dim3((n + 3) / 4), dim3(256), 0, s, images, n, p.maxabs_img);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_hay_assign, dim3(1), dim3(1024), 0, s, p.maxabs_img, n, nslots, p.perm, p.maxabs,
                               (uint32_t*)nullptr, (const uint32_t*)nullptr, (const int64_t*)nullptr,
                               (const int64_t*)nullptr, (int32_t*)nullptr, (uint32_t*)nullptr);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL(k_delta_prep, dim3(p.ngroups), dim3(kDeltaWaves * 64), 0, s, images, n, needle_side, p.planes,
                       p.ngroups, p.sumsq, p.maxabs, p.perm, (int8_t*)nullptr, (const uint32_t*)nullptr);
    return hipGetLastError();
}

hipError_t launch_true_distance(const uint32_t* needles, uint32_t nn, const uint32_t* hay, uint32_t nh,
                                const uint32_t* true_idx, const int64_t* sumsq, const uint32_t* nmax,
                                int64_t* dstar, int32_t* thr, uint32_t* rank, hipStream_t s, const uint32_t* inv)
{
    if (nn == 0) return hipSuccess;
    hipLaunchKernelGGL(k_true_distance, dim3((nn + 3) / 4), dim3(256), 0, s, needles, nn, hay, nh, true_idx, sumsq,
                       nmax, dstar, thr, rank, inv);
    return hipGetLastError();
}

hipError_t launch_paired_prep(const uint32_t* images, uint32_t n, const uint32_t* true_idx, const SearchPrep& np,
                              const SearchPrep& hp, int32_t* thr_slots, uint32_t* tile_flags, int64_t* dstar,
                              uint32_t* rank, hipStream_t s)
{
    const uint32_t nslots = hp.ngroups * kGroup;
    if (n == 0 || nslots == 0 || np.ngroups != hp.ngroups) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_hay_init, dim3((nslots + 255) / 256), dim3(256), 0, s, hp.perm, hp.maxabs, thr_slots, nslots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stats_true, dim3((n + 3) / 4), dim3(256), 0, s, images, n, true_idx, hp.maxabs_img,
                       np.sumsq, dstar);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hay_assign, dim3(1), dim3(1024), 0, s, hp.maxabs_img, n, nslots, hp.perm, hp.maxabs, hp.inv,
                       true_idx, (const int64_t*)dstar, (const int64_t*)np.sumsq, thr_slots, rank);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint32_t tiles = nslots / kFlagTile;
    hipLaunchKernelGGL(k_tile_flags, dim3((tiles + 3) / 4), dim3(256), 0, s, hp.maxabs, tiles, tile_flags);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the needles' mask plane and the haystack planes (D, r, q), both in slot
    // order, from one read of each image; q only where the tile flags ask
    hipLaunchKernelGGL(k_delta_prep, dim3(np.ngroups), dim3(kDeltaWaves * 64), 0, s, images, n, 2, np.planes,
                       np.ngroups, (int64_t*)nullptr, np.maxabs, (const uint32_t*)hp.perm, hp.planes,
                       (const uint32_t*)tile_flags);
    return hipGetLastError();
}

hipError_t launch_search_paired(const SearchArgs& A, uint32_t grid, uint32_t* counters, hipStream_t s)
{
    if (!A.paired || A.tiles_m == 0) return hipSuccess;
    hipError_t e = prepare_search_kernels();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_counters8, dim3(1), dim3(64), 0, s, counters);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_search_paired<Cfg>), dim3(grid), dim3(Cfg::kThreads), (size_t)Cfg::kLds, s, A, counters);
    return hipGetLastError();
}

uint32_t paired_items(uint32_t tiles) { return pair_items(tiles); }
size_t paired_slot_bytes() { return (size_t)Cfg::BM * Cfg::BN * sizeof(int32_t); }

template <class C>
static hipError_t launch_search_t(const SearchPrep& np, uint32_t nn, const SearchPrep& hp, uint32_t nh,
                                  const int32_t* thr, const int64_t* sumsq, uint32_t* rank, int64_t* matrix,
                                  int early_exit, hipStream_t s)
{
    SearchArgs A = {};
    A.early_exit = early_exit ? 1u : 0u;
    A.a_planes = np.planes; A.a_groups = np.ngroups; A.nn = nn;
    A.b_planes = hp.planes; A.b_groups = hp.ngroups; A.nh = nh;
    A.nmax = np.maxabs; A.hmax = hp.maxabs; A.hperm = hp.perm;
    A.thr = thr; A.sumsq = sumsq; A.rank = rank; A.matrix = matrix;
    A.tiles_m = (nn + C::BM - 1) / C::BM;
    A.tiles_n = hp.ngroups * kGroup / C::BN;   // every haystack slot, padding included
    const uint32_t total = A.tiles_m * A.tiles_n;
    A.per_xcd = (total + 7) / 8;
    if (A.early_exit && thr && !matrix)
        hipLaunchKernelGGL((k_search<C, true>), dim3(8 * A.per_xcd), dim3(C::kThreads), (size_t)C::kLds, s, A);
    else
        hipLaunchKernelGGL((k_search<C, false>), dim3(8 * A.per_xcd), dim3(C::kThreads), (size_t)C::kLds, s, A);
    return hipGetLastError();
}

hipError_t launch_search(const SearchPrep& np, uint32_t nn, const SearchPrep& hp, uint32_t nh,
                         const int32_t* thr, const int64_t* sumsq, uint32_t* rank, int64_t* matrix, int variant,
                         int early_exit, hipStream_t s)
{
    if (nn == 0 || nh == 0) return hipSuccess;
    hipError_t e = prepare_search_kernels();
    if (e != hipSuccess) return e;
    return variant == 1 ? launch_search_t<CfgS>(np, nn, hp, nh, thr, sumsq, rank, matrix, early_exit, s)
                        : launch_search_t<Cfg>(np, nn, hp, nh, thr, sumsq, rank, matrix, early_exit, s);
}

hipError_t launch_fallback(const uint32_t* needles, uint32_t nn, const uint32_t* hay, uint32_t nh,
                           const uint32_t* nmax, const uint32_t* hmax, const int64_t* dstar,
                           uint32_t* rank, int64_t* matrix, uint32_t* lists, hipStream_t s)
{
    if (nn == 0 || nh == 0) return hipSuccess;
    hipLaunchKernelGGL(k_slow_reset, dim3(1), dim3(64), 0, s, lists);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint64_t entries = (uint64_t)nn + nh;   // < 2^32
    hipLaunchKernelGGL(k_slow_lists, dim3((uint32_t)((entries + 255) / 256)), dim3(256), 0, s, nmax, nn, hmax, nh,
                       lists);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fallback, dim3(512), dim3(256), 0, s, needles, nn, hay, nh, nmax, lists, dstar, rank,
                       matrix);
    return hipGetLastError();
}

hipError_t launch_search_batched(const SearchJob* jobs, uint32_t njobs, const SearchTotals& T, uint32_t* counter,
                                 uint32_t grid, int variant, int early_exit, hipStream_t s, int part, int paired)
{
    if (njobs == 0) return hipSuccess;
#define RICI_LAUNCH(...)                                   \
    do {                                                   \
        hipLaunchKernelGGL(__VA_ARGS__);                   \
        hipError_t e_ = hipGetLastError();                 \
        if (e_ != hipSuccess) return e_;                   \
    } while (0)
    if ((part == 0 || part == 1) && paired) {
        // paired sets: statistics with the true-match distances (one read of
        // each image), slot assignment with the thresholds, tile flags, then
        // both plane sets in slot order (q only where the flags ask)
        if (T.hay_slots)
            RICI_LAUNCH(k_hay_init_batched, dim3((uint32_t)((T.hay_slots + 255) / 256)), dim3(256), 0, s, jobs, njobs,
                        T.hay_slots);
        if (T.needles)   // == T.hay_images
            RICI_LAUNCH(k_stats_true_batched, dim3((uint32_t)((T.needles + 3) / 4)), dim3(256), 0, s, jobs, njobs,
                        T.needles);
        RICI_LAUNCH(k_hay_assign_batched, dim3(njobs), dim3(1024), 0, s, jobs);
        if (T.hay_groups) {
            const uint64_t tiles = T.hay_groups / (kFlagTile / kGroup);
            RICI_LAUNCH(k_tile_flags_batched, dim3((uint32_t)((tiles + 3) / 4)), dim3(256), 0, s, jobs, njobs, tiles);
        }
        if (T.needle_groups)   // == T.hay_groups: both plane sets in one pass
            RICI_LAUNCH(k_needle_prep_batched, dim3((uint32_t)T.needle_groups), dim3(kDeltaWaves * 64), 0, s, jobs, njobs);
        RICI_LAUNCH(k_zero_counters8, dim3(1), dim3(64), 0, s, counter);
    } else if (part == 0 || part == 1) {
        if (T.needle_groups)
            RICI_LAUNCH(k_needle_prep_batched, dim3((uint32_t)T.needle_groups), dim3(kDeltaWaves * 64), 0, s, jobs, njobs);
        if (T.hay_slots)
            RICI_LAUNCH(k_hay_init_batched, dim3((uint32_t)((T.hay_slots + 255) / 256)), dim3(256), 0, s, jobs, njobs,
                        T.hay_slots);
        if (T.hay_images)
            RICI_LAUNCH(k_hay_stats_batched, dim3((uint32_t)((T.hay_images + 3) / 4)), dim3(256), 0, s, jobs, njobs,
                        T.hay_images);
        RICI_LAUNCH(k_hay_assign_batched, dim3(njobs), dim3(1024), 0, s, jobs);
        if (T.hay_groups)
            RICI_LAUNCH(k_hay_prep_batched, dim3((uint32_t)T.hay_groups), dim3(kDeltaWaves * 64), 0, s, jobs, njobs);
        if (T.needles)
            RICI_LAUNCH(k_true_distance_batched, dim3((uint32_t)((T.needles + 3) / 4)), dim3(256), 0, s, jobs, njobs,
                        T.needles);
        RICI_LAUNCH(k_zero_counters8, dim3(1), dim3(64), 0, s, counter);
    }
    if (part == 0 || part == 2) {
        if (T.tiles && variant == 1 && early_exit)
            RICI_LAUNCH((k_search_batched<CfgS, true>), dim3(grid), dim3(CfgS::kThreads), (size_t)CfgS::kLds, s, jobs,
                        njobs, (uint32_t)T.tiles, counter);
        else if (T.tiles && variant == 1)
            RICI_LAUNCH((k_search_batched<CfgS, false>), dim3(grid), dim3(CfgS::kThreads), (size_t)CfgS::kLds, s, jobs,
                        njobs, (uint32_t)T.tiles, counter);
        else if (T.tiles && early_exit)
            RICI_LAUNCH((k_search_batched<Cfg, true>), dim3(grid), dim3(Cfg::kThreads), (size_t)Cfg::kLds, s, jobs,
                        njobs, (uint32_t)T.tiles, counter);
        else if (T.tiles)
            RICI_LAUNCH((k_search_batched<Cfg, false>), dim3(grid), dim3(Cfg::kThreads), (size_t)Cfg::kLds, s, jobs,
                        njobs, (uint32_t)T.tiles, counter);
    }
    if (part == 0 || part == 3) {
        RICI_LAUNCH(k_slow_lists_batched, dim3(njobs), dim3(1024), 0, s, jobs);
        RICI_LAUNCH(k_fallback_batched, dim3(512), dim3(256), 0, s, jobs, njobs);
    }
#undef RICI_LAUNCH
    return hipSuccess;
}

hipError_t launch_search_scan(const ScanTable& T, int variant, hipStream_t s)
{
    if (T.njobs == 0 || T.tile_count == 0) return hipSuccess;
    const uint32_t items = T.m_start[T.njobs] * T.tile_count;
    if (items == 0) return hipSuccess;
    bool early_exit = false;
    for (uint32_t k = 0; k < T.njobs; ++k) early_exit |= T.A[k].early_exit != 0;
    if (variant == 1 && early_exit)
        hipLaunchKernelGGL((k_search_scan<CfgS, true>), dim3(items), dim3(CfgS::kThreads), (size_t)CfgS::kLds, s, T);
    else if (variant == 1)
        hipLaunchKernelGGL((k_search_scan<CfgS, false>), dim3(items), dim3(CfgS::kThreads), (size_t)CfgS::kLds, s, T);
    else if (early_exit)
        hipLaunchKernelGGL((k_search_scan<Cfg, true>), dim3(items), dim3(Cfg::kThreads), (size_t)Cfg::kLds, s, T);
    else
        hipLaunchKernelGGL((k_search_scan<Cfg, false>), dim3(items), dim3(Cfg::kThreads), (size_t)Cfg::kLds, s, T);
    return hipGetLastError();
}

template <class C, bool EXIT>
static hipError_t raise_lds()
{
    const int lds = (int)C::kLds;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_search<C, EXIT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_search_batched<C, EXIT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_search_scan<C, EXIT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if constexpr (!EXIT && C::BM == C::BN) {
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_search_paired<C>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    }
    return e;
}

hipError_t prepare_search_kernels()
{
    static hipError_t once = [] {
        hipError_t e = raise_lds<Cfg, false>();
        if (e == hipSuccess) e = raise_lds<Cfg, true>();
        if (e == hipSuccess) e = raise_lds<CfgS, false>();
        return e != hipSuccess ? e : raise_lds<CfgS, true>();
    }();
    return once;
}

uint32_t search_tile_m(int variant) { return variant == 1 ? CfgS::BM : Cfg::BM; }
uint32_t search_tile_n() { return Cfg::BN; }

}  // namespace rici
