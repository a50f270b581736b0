// RICI generation for gfx950 (Sec. 3.1 of van Blokland & Theoharis 2020).
//
// For every oriented point, every scene triangle is projected into cylindrical
// (alpha, beta) coordinates (Sec. 3.1.1), sliced by the row planes in its beta
// extent, and the radii with single and double circle intersections are
// counted into the image (Sec. 3.1.2).
//
// Mapping onto CDNA4
//   * A workgroup of 8 waves owns G images (G = 4 or 2, a tuning knob).  Their
//     FP64 frames (Eq. 1 coefficients) and per-row difference arrays live in
//     LDS (G x 16.6 KiB of uint32); with the per-wave rings and slice maps this
//     is small enough for 2 (G = 4) or 3 (G = 2) workgroups per CU.
//   * Lanes stream triangles (one per lane, coalesced float4 bounding spheres)
//     and test each against the G images with a conservative FP32 cull: the
//     bounding sphere must reach the support slab |beta| <= R/2 and the support
//     cylinder alpha <= R, with margins far above FP32 rounding.  Whole runs of
//     64 triangles are tested first through their common bounding sphere.  The
//     cull only discards triangles that provably touch no bin, so counts are
//     unchanged.
//   * Survivors (image, triangle) are appended to a per-wave LDS ring with a
//     ballot prefix; once 64 are queued every lane takes one and does the exact
//     work in FP64: projection (Eq. 2-5) and edge slopes, kept in registers.
//     The pairs' row slices are then spread evenly over the lanes, each lane
//     reading its slice's pair record from the owning lane (ds_bpermute): the
//     slice E0E1, single range (min|E|, max|E|), double range (|C|, min|E|),
//     all as comparisons of squared radii (no sqrt in any decision).
//   * Each slice adds +1 / -1 (single) and +2 / -2 (double) at its first and
//     end columns of a row's difference array (3 LDS atomics per slice, O(1)
//     per slice instead of O(64)); the final row prefix sum is a wavefront
//     scan and each row leaves as one coalesced 256 B store.
#include "rici_internal.h"

namespace rici {
namespace {

constexpr int kWaves = 8;      // wavefronts per workgroup
constexpr int kRing = 128;     // per-wave survivor ring (entries)

__device__ __forceinline__ bool finite3(float a, float b, float c)
{
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// ------------------------------------------------------------- triangle prep

// Triangle `src` of the mesh, stored at slot `t` of the cull and vertex arrays.
__device__ __forceinline__ void prep_triangle(const float* __restrict__ pos, uint32_t nv,
                                              const uint32_t* __restrict__ tri, uint32_t src, uint32_t t,
                                              float4* __restrict__ cull, float4* __restrict__ verts,
                                              uint32_t* __restrict__ err)
{
    const uint32_t i0 = tri[3 * (size_t)src], i1 = tri[3 * (size_t)src + 1], i2 = tri[3 * (size_t)src + 2];
    float4 dead = make_float4(0.f, 0.f, 0.f, -INFINITY);   // never passes the cull
    if (i0 >= nv || i1 >= nv || i2 >= nv) {
        atomicOr(err, 1u);
        cull[t] = dead;
        verts[3 * (size_t)t] = verts[3 * (size_t)t + 1] = verts[3 * (size_t)t + 2] = make_float4(0, 0, 0, 0);
        return;
    }
    const float* a = pos + 3 * (size_t)i0;
    const float* b = pos + 3 * (size_t)i1;
    const float* c = pos + 3 * (size_t)i2;
    float ax = a[0], ay = a[1], az = a[2], bx = b[0], by = b[1], bz = b[2], cx = c[0], cy = c[1], cz = c[2];
    verts[3 * (size_t)t + 0] = make_float4(ax, ay, az, 0.f);
    verts[3 * (size_t)t + 1] = make_float4(bx, by, bz, 0.f);
    verts[3 * (size_t)t + 2] = make_float4(cx, cy, cz, 0.f);
    if (!finite3(ax, ay, az) || !finite3(bx, by, bz) || !finite3(cx, cy, cz)) {
        atomicOr(err, 2u);
        cull[t] = dead;
        return;
    }
    // centre of the bounding box and the largest vertex distance from it,
    // inflated well beyond FP32 rounding of this and of the cull test
    float mx = 0.5f * (fminf(ax, fminf(bx, cx)) + fmaxf(ax, fmaxf(bx, cx)));
    float my = 0.5f * (fminf(ay, fminf(by, cy)) + fmaxf(ay, fmaxf(by, cy)));
    float mz = 0.5f * (fminf(az, fminf(bz, cz)) + fmaxf(az, fmaxf(bz, cz)));
    float ra = (ax - mx) * (ax - mx) + (ay - my) * (ay - my) + (az - mz) * (az - mz);
    float rb = (bx - mx) * (bx - mx) + (by - my) * (by - my) + (bz - mz) * (bz - mz);
    float rc = (cx - mx) * (cx - mx) + (cy - my) * (cy - my) + (cz - mz) * (cz - mz);
    float r = sqrtf(fmaxf(ra, fmaxf(rb, rc)));
    float mag = fmaxf(fabsf(mx), fmaxf(fabsf(my), fabsf(mz)));
    r = r * 1.0001f + 1e-5f * (mag + r) + 1e-30f;
    // a sphere whose centre or radius is beyond 1e18 would overflow the FP32
    // squares of the cull: it is stored with an infinite radius, which every
    // cull passes (the exact FP64 stage handles any finite coordinates)
    if (!(mag < 1e18f) || !(r < 1e18f)) { mx = my = mz = 0.f; r = INFINITY; }
    cull[t] = make_float4(mx, my, mz, r);
}

// 30-bit Morton code of a point quantised to 10 bits per axis
__device__ __forceinline__ uint32_t spread10(uint32_t v)
{
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// One workgroup (1024 threads) stores triangles b * 4096 .. b * 4096 + 4095 of
// the mesh in Morton order of their bounding-box centres within the block's
// box, so that the runs of 64 consecutive triangles tested together by k_gen
// are compact patches with small bounding spheres (the order of the triangles
// never changes a count: every triangle adds its crossings to the same
// integer image).  Keys: Morton code, then 2^30 for triangles with a bad index
// or a non-finite vertex (stored as never-passing spheres), then padding past
// the end of the mesh; the block index in the low word makes them unique.
// With sort false the block is stored in mesh order.
__device__ __forceinline__ void prep_sorted_block(const float* __restrict__ pos, uint32_t nv, const uint32_t* __restrict__ tri,
                                  uint32_t nt, uint32_t b, bool sort, float4* __restrict__ cull,
                                  float4* __restrict__ verts, uint32_t* __restrict__ err)
{
    constexpr int kT = 1024, kPer = kGenSortBlock / kT;
    __shared__ uint64_t key[kGenSortBlock];
    __shared__ float box[2][16][3];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t base = b * kGenSortBlock;
    const uint32_t n_in = min(nt - base, kGenSortBlock);
    if (!sort) {
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const uint32_t j = (uint32_t)(q * kT + tid);
            if (j < n_in) prep_triangle(pos, nv, tri, base + j, base + j, cull, verts, err);
        }
        return;
    }

    float cx[kPer], cy[kPer], cz[kPer];
    int state[kPer];                        // 0 live, 1 bad or non-finite, 2 past the end
    float lo[3] = { INFINITY, INFINITY, INFINITY }, hi[3] = { -INFINITY, -INFINITY, -INFINITY };
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const uint32_t j = (uint32_t)(q * kT + tid);
        cx[q] = cy[q] = cz[q] = 0.f;
        state[q] = 2;
        if (j < n_in) {
            const uint32_t t = base + j;
            const uint32_t i0 = tri[3 * (size_t)t], i1 = tri[3 * (size_t)t + 1], i2 = tri[3 * (size_t)t + 2];
            state[q] = 1;
            if (i0 < nv && i1 < nv && i2 < nv) {
                const float* a = pos + 3 * (size_t)i0;
                const float* bb = pos + 3 * (size_t)i1;
                const float* c = pos + 3 * (size_t)i2;
                const float x = (fminf(a[0], fminf(bb[0], c[0])) + fmaxf(a[0], fmaxf(bb[0], c[0]))) * 0.5f;
                const float y = (fminf(a[1], fminf(bb[1], c[1])) + fmaxf(a[1], fmaxf(bb[1], c[1]))) * 0.5f;
                const float z = (fminf(a[2], fminf(bb[2], c[2])) + fmaxf(a[2], fmaxf(bb[2], c[2]))) * 0.5f;
                if (finite3(x, y, z)) {
                    cx[q] = x; cy[q] = y; cz[q] = z;
                    state[q] = 0;
                    lo[0] = fminf(lo[0], x); lo[1] = fminf(lo[1], y); lo[2] = fminf(lo[2], z);
                    hi[0] = fmaxf(hi[0], x); hi[1] = fmaxf(hi[1], y); hi[2] = fmaxf(hi[2], z);
                }
            }
        }
    }
    // the block's box of live centres
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], __shfl_xor(lo[k], o, 64));
            hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], o, 64));
        }
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 3; ++k) { box[0][wave][k] = lo[k]; box[1][wave][k] = hi[k]; }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        lo[k] = box[0][0][k]; hi[k] = box[1][0][k];
        for (int w = 1; w < kT / 64; ++w) { lo[k] = fminf(lo[k], box[0][w][k]); hi[k] = fmaxf(hi[k], box[1][w][k]); }
    }
    float sc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) sc[k] = 1023.0f / fmaxf(hi[k] - lo[k], 1e-30f);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const uint32_t j = (uint32_t)(q * kT + tid);
        uint32_t code;
        if (state[q] == 0) {
            const uint32_t qx = (uint32_t)fminf(fmaxf((cx[q] - lo[0]) * sc[0], 0.f), 1023.f);
            const uint32_t qy = (uint32_t)fminf(fmaxf((cy[q] - lo[1]) * sc[1], 0.f), 1023.f);
            const uint32_t qz = (uint32_t)fminf(fmaxf((cz[q] - lo[2]) * sc[2], 0.f), 1023.f);
            code = spread10(qx) | (spread10(qy) << 1) | (spread10(qz) << 2);
        } else {
            code = state[q] == 1 ? (1u << 30) : 0xFFFFFFFFu;
        }
        key[j] = ((uint64_t)code << 32) | j;
    }
    __syncthreads();
    // bitonic sort of the 4096 keys, two compare-exchanges per thread and pass
    for (uint32_t k = 2; k <= kGenSortBlock; k <<= 1) {
        for (uint32_t h = k >> 1; h > 0; h >>= 1) {
#pragma unroll
            for (int q = 0; q < kPer / 2; ++q) {
                const uint32_t i = (uint32_t)(q * kT + tid);           // pair index, < 2048
                const uint32_t a = ((i & ~(h - 1)) << 1) | (i & (h - 1));
                const uint32_t c = a | h;
                const uint64_t ka = key[a], kc = key[c];
                const bool up = (a & k) == 0;
                if ((ka > kc) == up) { key[a] = kc; key[c] = ka; }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const uint32_t p = (uint32_t)(q * kT + tid);
        if (p < n_in)
            prep_triangle(pos, nv, tri, base + (uint32_t)(key[p] & 0xFFFFFFFFu), base + p, cull, verts, err);
    }
}

__global__ void __launch_bounds__(1024)
k_gen_prep_sorted(const float* __restrict__ pos, uint32_t nv, const uint32_t* __restrict__ tri, uint32_t nt,
                  float4* __restrict__ cull, float4* __restrict__ verts, uint32_t* __restrict__ err)
{
    prep_sorted_block(pos, nv, tri, nt, blockIdx.x, true, cull, verts, err);
}

// mesh order: one thread per triangle
__global__ void __launch_bounds__(256)
k_gen_prep(const float* __restrict__ pos, uint32_t nv, const uint32_t* __restrict__ tri, uint32_t nt,
           float4* __restrict__ cull, float4* __restrict__ verts, uint32_t* __restrict__ err)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nt) prep_triangle(pos, nv, tri, t, t, cull, verts, err);
}

// Bounding sphere of each run of 64 consecutive triangles (one wavefront's
// chunk in k_gen): it contains every triangle sphere of the run, so a run whose
// sphere misses an image's support volume can be skipped as a whole.
__device__ __forceinline__ void cluster_sphere(const float4* __restrict__ cull, uint32_t nt, uint32_t c,
                                               float4* __restrict__ clusters, int lane)
{
    const uint32_t t = c * 64 + lane;
    const float4 s = t < nt ? cull[t] : make_float4(0.f, 0.f, 0.f, -INFINITY);
    const bool giant = __ballot(s.w == INFINITY) != 0;   // then the run always passes
    const bool live = s.w >= 0.f && s.w != INFINITY;
    float lo[3] = { live ? s.x - s.w : INFINITY, live ? s.y - s.w : INFINITY, live ? s.z - s.w : INFINITY };
    float hi[3] = { live ? s.x + s.w : -INFINITY, live ? s.y + s.w : -INFINITY, live ? s.z + s.w : -INFINITY };
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], __shfl_xor(lo[k], o, 64));
            hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], o, 64));
        }
    const float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]), cz = 0.5f * (lo[2] + hi[2]);
    float r = live ? sqrtf((s.x - cx) * (s.x - cx) + (s.y - cy) * (s.y - cy) + (s.z - cz) * (s.z - cz)) + s.w : -INFINITY;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) r = fmaxf(r, __shfl_xor(r, o, 64));
    if (lane == 0) {
        const float mag = fmaxf(fabsf(cx), fmaxf(fabsf(cy), fabsf(cz)));
        const bool any = r >= 0.f;   // at least one live triangle
        clusters[c] = giant ? make_float4(0.f, 0.f, 0.f, INFINITY)
                    : any   ? make_float4(cx, cy, cz, r * 1.0001f + 1e-5f * (mag + r) + 1e-30f)
                            : make_float4(0.f, 0.f, 0.f, -INFINITY);
    }
}

__global__ void __launch_bounds__(256)
k_gen_clusters(const float4* __restrict__ cull, uint32_t nt, float4* __restrict__ clusters, uint32_t nc)
{
    const uint32_t c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c < nc) cluster_sphere(cull, nt, c, clusters, threadIdx.x & 63);
}

// ------------------------------------------------------------ exact pieces

// Per-image frame in FP64 (Eq. 1), with the second rotation and the in-plane
// y row pre-multiplied by 128/R so that projected coordinates come out in
// half-bin units: bin radii are 2c + 1 and row heights 2r - 63, all small odd
// integers.  (Scaling by a power of two changes no rounding, so every
// decision is the one made in bin units.)
struct Frame {
    double sx, sy, sz;        // Spin Vertex
    double nax, nay;          // first rotation (about z)
    double nax_d, nay_d;      // first rotation x 128/R (y coordinate)
    double nbx_d, nbz_d;      // second rotation (about y) x 128/R
    double pad;
};

// Column guesses.  In half-bin units the bin radii are the odd integers
// 2c + 1, so the first column whose radius exceeds sqrt(s) is the first c
// with (2c + 1)^2 > s.  Odd squares are 1 mod 8 and at least 8 apart, so each
// run of 8 consecutive integers 8i .. 8i + 7 holds at most one of them: a
// table entry per run (the answer at 8i) is the answer or one below it for
// every s in the run, and one exact comparison settles it.  s is clamped to
// 16640 = 129^2 - 1, the last value whose answer is 64.
constexpr int kColTab = 16640 / 8 + 1;

// entry i: the first c with (2c + 1)^2 > 8i, i.e. (isqrt(8i) + 1) / 2
__device__ void fill_col_table(uint8_t* __restrict__ tab, int tid, int nthreads)
{
    for (int i = tid; i < kColTab; i += nthreads) {
        const uint32_t x = 8u * (uint32_t)i;
        uint32_t k = (uint32_t)sqrtf((float)x);
        while (k * k > x) --k;
        while ((k + 1) * (k + 1) <= x) ++k;
        tab[i] = (uint8_t)((k + 1) / 2);
    }
}

// First column c in [0, 64] whose bin radius exceeds sqrt(s), s >= 0 the
// squared distance in half-bin units (c = 64 for s >= 16640 and for NaN).
// (2c + 1)^2 is an integer, so comparing it with floor(s) is exact.
__device__ __forceinline__ int first_col(const uint8_t* __restrict__ tab, double s)
{
    const uint32_t t = (uint32_t)fmin(s, 16640.0);
    const uint32_t c = tab[t >> 3];
    const uint32_t u = 2 * c + 1;
    return (int)(c + (u * u <= t ? 1u : 0u));
}

// Same for the ratio cr2 / dd (dd > 0): the first c with (2c + 1)^2 dd > cr2,
// decided by an FP64 comparison of the product.  The table is read at an
// estimate of the ratio from the hardware reciprocal; an estimate within 1 of
// the ratio still lands in a run whose entry is the answer or one below it.
// Results above 64 are not exact, and callers clamp them with a column that
// is at most 64.
__device__ __forceinline__ int first_col_ratio(const uint8_t* __restrict__ tab, double cr2, double dd)
{
    const double approx = cr2 * __builtin_amdgcn_rcp(dd);
    const uint32_t c = tab[(uint32_t)fmin(approx, 16640.0) >> 3];
    const uint32_t u = 2 * c + 1;
    return (int)(c + ((double)(u * u) * dd <= cr2 ? 1u : 0u));
}

__device__ __forceinline__ void csort(double& x0, double& y0, double& z0, double& x1, double& y1, double& z1)
{
    const bool sw = z1 < z0;
    const double tx = sw ? x1 : x0, ty = sw ? y1 : y0, tz = fmin(z0, z1);   // heights: one min, one max
    x1 = sw ? x0 : x1; y1 = sw ? y0 : y1; z1 = fmax(z0, z1);
    x0 = tx; y0 = ty; z0 = tz;
}

__device__ __forceinline__ double recip(double d)
{
    // 1/d: the hardware estimate (relative error up to ~6e-8 on gfx950) refined
    // by one Newton step, which leaves at most ~11 ulp (measured over 4M values
    // with exponents -100 .. 99); every decision that uses it is an FP64
    // comparison far coarser than that
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    return r;
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kDiffStride = 65;   // column 64 of each row is a sink for "past the image"
constexpr int kMapCap = 1024;     // slices mapped per round
constexpr uint32_t kOwn = 3;       // slices of a pair done by the lane that projected it

// LDS of a workgroup owning G images: the difference arrays, the per-wave
// survivor rings and slice maps, and the frames.  The per-pair records of the
// exact stage stay in registers (see process_batch), which keeps this small
// enough for two (G = 4) or three (G = 2) resident workgroups per CU.
template <int G>
struct GenLds {
    uint32_t diff[G][NB * kDiffStride];
    uint32_t ring[kWaves][kRing];
    uint8_t map[kWaves][kMapCap]; // slice -> survivor lane
    uint8_t coltab[(kColTab + 15) & ~15];   // column guesses (first_col)
    Frame frames[G];
    float cp[G][8];               // FP32 cull parameters
};

// v from lane src_x4 / 4 (every lane of the wave must be active)
__device__ __forceinline__ double lane_fetch(double v, int src_x4)
{
    const int lo = __builtin_amdgcn_ds_bpermute(src_x4, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src_x4, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ uint32_t lane_fetch(uint32_t v, int src_x4)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src_x4, (int)v);
}

// Exact work for up to 64 queued (image, triangle) pairs of one wavefront.
//
// Stage A: lane i projects pair i (Eq. 2-4 in FP64, half-bin units), sorts its
// vertices by height and keeps, in registers, the edge slopes and the first
// row of its beta extent.  Stage B: the slices of all pairs (one per row in
// the extent) are spread evenly over the lanes; a lane reads the record of
// its slice's pair from the owning lane with cross-lane permutes and adds the
// slice's single / double ranges to the row's difference array.
template <int G>
__device__ __forceinline__ void process_batch(GenLds<G>& L, int wave, int lane, uint32_t head, uint32_t cnt,
                              const float4* __restrict__ verts)
{
    wave_sync_lds();
    uint32_t nrows = 0, key = 0;
    double xa = 0.0, ya = 0.0, za = 0.0, zb = 0.0, xb = 0.0, yb = 0.0;
    double sxl = 0.0, syl = 0.0, sx1 = 0.0, sy1 = 0.0, sx2 = 0.0, sy2 = 0.0;
    int r0 = 0;
    uint32_t g = 0;
    if ((uint32_t)lane < cnt) {
        const uint32_t e = L.ring[wave][(head + lane) & (kRing - 1)];
        g = e & (G - 1);
        const uint32_t t = e / G;
        const Frame& F = L.frames[g];
        const float4 v0 = verts[3 * (size_t)t], v1 = verts[3 * (size_t)t + 1], v2 = verts[3 * (size_t)t + 2];
        double X[3], Y[3], Z[3];
        const float4 v[3] = { v0, v1, v2 };
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double px = (double)v[k].x - F.sx;          // Eq. 2
            const double py = (double)v[k].y - F.sy;
            const double pz = (double)v[k].z - F.sz;
            const double qx = F.nax * px + F.nay * py;        // Eq. 3 (x)
            Y[k] = -F.nay_d * px + F.nax_d * py;              // Eq. 3 (y), half-bin units
            X[k] = F.nbz_d * qx - F.nbx_d * pz;               // Eq. 4, half-bin units
            Z[k] = F.nbx_d * qx + F.nbz_d * pz;
        }
        double xc = X[2], yc = Y[2], zc = Z[2];
        xa = X[0]; ya = Y[0]; za = Z[0]; xb = X[1]; yb = Y[1]; zb = Z[1];
        csort(xa, ya, za, xb, yb, zb);
        csort(xb, yb, zb, xc, yc, zc);
        csort(xa, ya, za, xb, yb, zb);
        // rows r with 2r - 63 in (z_a, z_c]: a vertex is above iff z >= beta
        // (z / 2 + 31.5 rounds as z + 31.5 does in bin units)
        const double f0 = floor(fmin(fmax(fma(za, 0.5, 31.5), -2.0), 70.0)) + 1.0;
        const double f1 = floor(fmin(fmax(fma(zc, 0.5, 31.5), -2.0), 70.0));
        r0 = max((int)f0, 0);
        const int r1 = min((int)f1, 63);
        const double il = recip(zc - za);
        const double i1 = recip(zb - za);
        const double i2 = recip(zc - zb);
        nrows = (r1 >= r0 && zc > za) ? (uint32_t)(r1 - r0 + 1) : 0u;
        sxl = (xc - xa) * il; syl = (yc - ya) * il;
        sx1 = (xb - xa) * i1; sy1 = (yb - ya) * i1;
        sx2 = (xc - xb) * i2; sy2 = (yc - yb) * i2;
    }
    // One slice (pair record, row r, image gi): Sec. 3.1.2 steps 1-6 and the
    // difference-row updates.
    auto slice = [&](double Ra, double Rb, double Rxa, double Rya, double Rsxl, double Rsyl, double Rxb, double Ryb,
                     double Rsx1, double Rsy1, double Rsx2, double Rsy2, int r, uint32_t gi) {
        const double beta = (double)(2 * r - 63);
        // step 1: crossings on the long edge and on the short edge whose
        // z-range holds beta
        const double hl = beta - Ra;
        const double e0x = Rxa + hl * Rsxl, e0y = Rya + hl * Rsyl;
        const bool low = beta <= Rb;
        const double h1 = low ? hl : beta - Rb;
        const double e1x = (low ? Rxa : Rxb) + h1 * (low ? Rsx1 : Rsx2);
        const double e1y = (low ? Rya : Ryb) + h1 * (low ? Rsy1 : Rsy2);
        // steps 3-4: squared distances from the axis; single range (lo, hi)
        // (first_col is monotone, so the columns of the two ends order as
        // their distances do)
        const double d0 = e0x * e0x + e0y * e0y, d1 = e1x * e1x + e1y * e1y;
        const int k0 = first_col(L.coltab, d0), k1 = first_col(L.coltab, d1);
        // steps 5-6: double range (|C|, lo) iff the foot C of the axis on
        // line E0E1 lies strictly inside the segment
        const double dx = e1x - e0x, dy = e1y - e0y;
        const double dd = dx * dx + dy * dy;
        const bool between = (e0x * dx + e0y * dy) < 0.0 && (e1x * dx + e1y * dy) > 0.0;
        const double cr = e0x * e1y - e0y * e1x;
        const bool ok = d0 <= 1.0e300 && d1 <= 1.0e300;
        int c_lo = min(k0, k1), c_hi = max(k0, k1);
        int c_c = between ? min(first_col_ratio(L.coltab, cr * cr, dd), c_lo) : c_lo;
        if (!ok) { c_lo = c_hi = c_c = 64; }
        // +2 on [c_c, c_lo), +1 on [c_lo, c_hi) as a difference row: +2 at
        // c_c, -1 at c_lo, -1 at c_hi, with coinciding columns merged and
        // zero or past-the-image (column 64) updates dropped (LDS atomics
        // are the slice stage's most expensive instructions)
        uint32_t v0 = 2u, v1 = (uint32_t)-1, v2 = (uint32_t)-1;
        if (c_c == c_lo) { v0 = 0u; v1 = 1u; }
        if (c_lo == c_hi) { v1 -= 1u; v2 = 0u; }
        uint32_t* row = L.diff[gi] + __umul24((uint32_t)r, (uint32_t)kDiffStride);
        if (v0 != 0u && c_c < 64) atomicAdd(row + c_c, v0);
        if (v1 != 0u && c_lo < 64) atomicAdd(row + c_lo, v1);
        if (v2 != 0u && c_hi < 64) atomicAdd(row + c_hi, v2);
    };

    // The first kOwn slices of every pair stay on the lane that projected it
    // (no cross-lane reads; most pairs span only a few rows) ...
#pragma unroll
    for (uint32_t k = 0; k < kOwn; ++k)
        if (k < nrows) slice(za, zb, xa, ya, sxl, syl, xb, yb, sx1, sy1, sx2, sy2, r0 + (int)k, g);
    // ... and the rest are spread evenly over the lanes, each reading its
    // slice's pair record from the owning lane.
    const uint32_t nrest = nrows > kOwn ? nrows - kOwn : 0u;
    const uint32_t incl = wave_inclusive_scan(nrest, lane);
    const uint32_t pre = incl - nrest;
    const uint32_t total = __shfl(incl, 63, 64);
    // row of slice k of this pair = r0 + kOwn + (k - pre); stored with its image
    key = ((uint32_t)(r0 + (int)kOwn - (int)pre + 8192) << 2) | g;

    for (uint32_t base = 0; base < total; base += kMapCap) {
        const uint32_t lo = max(pre, base), hi = min(pre + nrest, base + kMapCap);
        for (uint32_t k = lo; k < hi; ++k) L.map[wave][k - base] = (uint8_t)lane;
        wave_sync_lds();
        const uint32_t n_round = min(total - base, (uint32_t)kMapCap);
        for (uint32_t k0 = 0; k0 < n_round; k0 += 64) {   // uniform trip count: permutes see every lane
            const uint32_t k = k0 + (uint32_t)lane;
            const bool valid = k < n_round;
            const int src = valid ? (int)L.map[wave][k] * 4 : 0;
            const uint32_t m = lane_fetch(key, src);
            const double Ra = lane_fetch(za, src), Rb = lane_fetch(zb, src);
            const double Rxa = lane_fetch(xa, src), Rya = lane_fetch(ya, src);
            const double Rsxl = lane_fetch(sxl, src), Rsyl = lane_fetch(syl, src);
            const double Rxb = lane_fetch(xb, src), Ryb = lane_fetch(yb, src);
            const double Rsx1 = lane_fetch(sx1, src), Rsy1 = lane_fetch(sy1, src);
            const double Rsx2 = lane_fetch(sx2, src), Rsy2 = lane_fetch(sy2, src);
            if (!valid) continue;
            const int r = (int)(m >> 2) - 8192 + (int)(base + k);
            slice(Ra, Rb, Rxa, Rya, Rsxl, Rsyl, Rxb, Ryb, Rsx1, Rsy1, Rsx2, Rsy2, r, m & (G - 1));
        }
        wave_sync_lds();
    }
}

// G images (img0 .. img0 + G - 1) of one job, by the whole workgroup.
template <int G>
__device__ void gen_images(GenLds<G>& L, const GenJob& J, uint32_t img0, float Rf, uint32_t* __restrict__ err)
{
    const float4* __restrict__ cull = J.cull;
    const float4* __restrict__ clusters = J.clusters;
    const float4* __restrict__ verts = J.verts;
    const uint32_t nt = J.nt, n = J.n;
    const float* __restrict__ op_pos = J.op_pos;
    const float* __restrict__ op_nrm = J.op_nrm;
    uint32_t* __restrict__ out = J.out;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    for (int i = tid; i < G * NB * kDiffStride; i += kWaves * 64) (&L.diff[0][0])[i] = 0u;
    if (tid < G) {
        Frame f = {};
        float* c = L.cp[tid];
        const uint32_t img = img0 + tid;
        bool live = img < n;
        if (live) {
            const float* sp = op_pos + 3 * (size_t)img;
            const float* sn = op_nrm + 3 * (size_t)img;
            if (!finite3(sp[0], sp[1], sp[2]) || !finite3(sn[0], sn[1], sn[2])) {
                atomicOr(err, 2u);
                live = false;
            } else {
                const double inv_d = (double)(2 * NB) / (double)Rf;
                f.sx = sp[0]; f.sy = sp[1]; f.sz = sp[2];
                // Eq. 1 (identity for a vanishing pair)
                const Rotation q = frame_rotation(sn[0], sn[1], sn[2]);
                const double nax = q.nax, nay = q.nay, nbx = q.nbx, nbz = q.nbz;
                f.nax = nax; f.nay = nay;
                f.nax_d = nax * inv_d; f.nay_d = nay * inv_d;
                f.nbx_d = nbx * inv_d; f.nbz_d = nbz * inv_d;
                // Central Axis direction for the cull: the pre-image of +z
                c[0] = sp[0]; c[1] = sp[1]; c[2] = sp[2];
                c[3] = (float)(nbx * nax);
                c[4] = (float)(nbx * nay);
                c[5] = (float)nbz;
                const float mag = fmaxf(fabsf(sp[0]), fmaxf(fabsf(sp[1]), fabsf(sp[2])));
                const float margin = 1e-5f * (mag + Rf) + 1e-30f;
                c[6] = 0.5f * Rf + margin;    // slab half height
                c[7] = Rf + margin;           // cylinder radius
                // a Spin Vertex or radius beyond 1e18 would overflow the FP32
                // squares of the cull: every triangle then reaches the image
                // (the exact FP64 stage handles any finite coordinates)
                if (!(mag < 1e18f) || !(Rf < 1e18f)) c[6] = c[7] = INFINITY;
            }
        }
        if (!live) {
            c[0] = c[1] = c[2] = 0.f; c[3] = c[4] = 0.f; c[5] = 1.f;
            c[6] = -INFINITY; c[7] = 0.f;
        }
        L.frames[tid] = f;
    }
    __syncthreads();

    // cull parameters of the G images, wave-uniform (scalar registers)
    float P[G][8];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < 8; ++k)
            P[g][k] = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(L.cp[g][k])));

    uint32_t head = 0, tail = 0;   // wave-uniform ring counters
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // Conservative FP32 sphere test against image g's support volume: the slab
    // |beta| <= R/2 and the cylinder alpha <= R, both with margins.  An infinite
    // radius (a sphere too large for FP32 squares) reaches every live image,
    // and an image whose own cull would overflow (infinite slab) is reached by
    // every sphere.
    auto reaches = [&](const float4& sp, int g) -> bool {
        const float dx = sp.x - P[g][0], dy = sp.y - P[g][1], dz = sp.z - P[g][2];
        const float h = P[g][3] * dx + P[g][4] * dy + P[g][5] * dz;
        const float d2 = dx * dx + dy * dy + dz * dz;
        const float a2 = d2 - h * h;
        const float la = P[g][7] + sp.w;
        return ((fabsf(h) <= P[g][6] + sp.w) & (a2 <= la * la)) | ((sp.w == INFINITY) & (P[g][6] > 0.f)) |
               (P[g][6] == INFINITY);
    };

    // Test one run of 64 triangles (spheres s, triangle t = run * 64 + lane)
    // against the images in cmask and append the survivors to the ring.
    auto test_run = [&](const float4& s, uint32_t t, uint32_t cmask) {
        uint32_t mask = 0;
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (cmask & (1u << g)) mask |= (reaches(s, g) ? 1u : 0u) << g;
        // append the pairs to the ring, one image bit per round
        while (__ballot(mask != 0)) {
            const bool has = mask != 0;
            const uint32_t g = (uint32_t)__builtin_ctz(mask | (1u << G));
            mask &= mask - 1;
            const uint64_t bal = __ballot(has);
            if (has) {
                const uint32_t slot = tail + (uint32_t)__popcll(bal & lt_mask);
                L.ring[wave][slot & (kRing - 1)] = t * G + g;
            }
            tail += (uint32_t)__popcll(bal);
            if (tail - head >= 64) {
                process_batch<G>(L, wave, lane, head, 64, verts);
                head += 64;
            }
        }
    };

    // Runs of this wave: wv, wv + 8, wv + 16, ...  Their bounding spheres are
    // tested 64 at a time (one run per lane), then the passing runs are
    // tested triangle by triangle.  (A sphere that never passes is built in
    // place: a named local would turn the guarded loads into flat loads
    // through a pointer select.)
    const uint32_t wv = __builtin_amdgcn_readfirstlane(wave);
    const uint32_t nc = (nt + 63) / 64;
    for (uint32_t c0 = wv; c0 < nc; c0 += kWaves * 64) {
        const uint32_t cl = c0 + kWaves * (uint32_t)lane;
        const float4 cs = cl < nc ? clusters[cl] : make_float4(0.f, 0.f, 0.f, -INFINITY);
        uint32_t cm = 0;
#pragma unroll
        for (int g = 0; g < G; ++g) cm |= (reaches(cs, g) ? 1u : 0u) << g;
        for (uint64_t pend = __ballot(cm != 0); pend != 0; pend &= pend - 1) {
            const int l = (int)__builtin_ctzll(pend);
            const uint32_t run = c0 + kWaves * (uint32_t)l;
            const uint32_t rmask = (uint32_t)__builtin_amdgcn_readlane((int)cm, l);
            const uint32_t t = run * 64 + (uint32_t)lane;
            const float4 s = t < nt ? cull[t] : make_float4(0.f, 0.f, 0.f, -INFINITY);
            test_run(s, t, rmask);
        }
    }
    if (tail > head) process_batch<G>(L, wave, lane, head, tail - head, verts);
    __syncthreads();

    // row prefix sums of the difference arrays -> counts; one row per wave step
    for (int row = wave; row < G * NB; row += kWaves) {
        const int g = row / NB, r = row % NB;
        const uint32_t img = img0 + g;
        if (img >= n) continue;
        const uint32_t v = wave_inclusive_scan(L.diff[g][r * kDiffStride + lane], lane);
        out[(size_t)img * NPIX + r * NB + lane] = v;
    }
    __syncthreads();   // the LDS is reused by the workgroup's next group
}

// waves per SIMD to leave room for: 3 workgroups per CU (G = 2), 2 (G = 4)
template <int G> constexpr int kGenWavesPerEU = G == 2 ? 6 : 4;

template <int G>
__global__ void __launch_bounds__(kWaves * 64, kGenWavesPerEU<G>)
k_gen(GenJob J, float Rf, uint32_t* __restrict__ err)
{
    __shared__ GenLds<G> L;
    fill_col_table(L.coltab, threadIdx.x, kWaves * 64);   // published by gen_images' first barrier
    gen_images<G>(L, J, blockIdx.x * G, Rf, err);
}

// Persistent form for many meshes: every workgroup takes (job, image group)
// items from a device counter until none are left.  Jobs are stored largest
// first, so the long items start early and the short ones fill the tail.
// (G = 2 spills a few registers of the per-item loop here, none in the
// triangle or slice loops)
template <int G>
__global__ void __launch_bounds__(kWaves * 64, kGenWavesPerEU<G>)
k_gen_batched(const GenJob* __restrict__ jobs, uint32_t njobs, uint32_t total_items, float Rf,
              uint32_t* __restrict__ counter, uint32_t* __restrict__ err)
{
    __shared__ GenLds<G> L;
    __shared__ uint32_t s_item;
    fill_col_table(L.coltab, threadIdx.x, kWaves * 64);   // published by the first barrier below
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= total_items) break;
        uint32_t lo = 0, hi = njobs - 1;          // last job with item_start <= item
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) / 2;
            if (jobs[mid].item_start <= item) lo = mid; else hi = mid - 1;
        }
        const GenJob J = jobs[lo];
        gen_images<G>(L, J, (item - J.item_start) * G, Rf, err);
    }
}

__device__ __forceinline__ uint32_t find_job(const GenJob* __restrict__ jobs, uint32_t njobs, uint64_t x, bool chunks)
{
    uint32_t lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) / 2;
        const uint64_t st = chunks ? jobs[mid].chunk_start : jobs[mid].block_start;
        if (st <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(1024)
k_gen_prep_batched(const GenJob* __restrict__ jobs, uint32_t njobs, uint32_t* __restrict__ err)
{
    // one workgroup per sort block of every mesh (block_start: the mesh's first)
    const uint64_t x = blockIdx.x;
    const GenJob& J = jobs[find_job(jobs, njobs, x, false)];
    prep_sorted_block(J.pos, J.nv, J.tri, J.nt, (uint32_t)(x - J.block_start), J.sort != 0, J.cull, J.verts, err);
}

__global__ void __launch_bounds__(256)
k_gen_clusters_batched(const GenJob* __restrict__ jobs, uint32_t njobs, uint64_t total)
{
    const uint64_t x = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (x >= total) return;
    const GenJob& J = jobs[find_job(jobs, njobs, x, true)];
    cluster_sphere(J.cull, J.nt, (uint32_t)(x - J.chunk_start), J.clusters, threadIdx.x & 63);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t n, uint32_t v)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

bool gen_sort_wanted(int mode, uint32_t nt)
{
    return mode == 1 || (mode == 2 && nt >= kGenSortAuto);
}

hipError_t launch_gen_prep(const float* pos, uint32_t nv, const uint32_t* tri, uint32_t nt, int sort_mode,
                           float4* cull, float4* verts, uint32_t* err, hipStream_t s)
{
    if (nt == 0) return hipSuccess;
    if (gen_sort_wanted(sort_mode, nt))
        hipLaunchKernelGGL(k_gen_prep_sorted, dim3((nt + kGenSortBlock - 1) / kGenSortBlock), dim3(1024), 0, s, pos,
                           nv, tri, nt, cull, verts, err);
    else
        hipLaunchKernelGGL(k_gen_prep, dim3((nt + 255) / 256), dim3(256), 0, s, pos, nv, tri, nt, cull, verts, err);
    return hipGetLastError();
}

hipError_t launch_gen_clusters(const float4* cull, uint32_t nt, float4* clusters, hipStream_t s)
{
    const uint32_t nc = (nt + 63) / 64;
    if (nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gen_clusters, dim3((nc + 3) / 4), dim3(256), 0, s, cull, nt, clusters, nc);
    return hipGetLastError();
}

hipError_t launch_gen(const float4* cull, const float4* clusters, const float4* verts, uint32_t nt,
                      const float* op_pos, const float* op_nrm, uint32_t n, float R,
                      uint32_t* out, uint32_t* err, int group, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    GenJob J = {};
    J.nt = nt; J.op_pos = op_pos; J.op_nrm = op_nrm; J.n = n; J.out = out;
    J.cull = const_cast<float4*>(cull); J.clusters = const_cast<float4*>(clusters); J.verts = const_cast<float4*>(verts);
    if (group == 2)
        hipLaunchKernelGGL(k_gen<2>, dim3((n + 1) / 2), dim3(kWaves * 64), 0, s, J, R, err);
    else
        hipLaunchKernelGGL(k_gen<4>, dim3((n + 3) / 4), dim3(kWaves * 64), 0, s, J, R, err);
    return hipGetLastError();
}

uint32_t gen_group_images(int group) { return group == 2 ? 2u : 4u; }

hipError_t gen_batched_grid(int group, int cus, uint32_t* grid)
{
    int per_cu = 0;
    hipError_t e = group == 2
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gen_batched<2>, kWaves * 64, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gen_batched<4>, kWaves * 64, 0);
    if (e != hipSuccess) return e;
    *grid = (uint32_t)(max(per_cu, 1) * cus);
    return hipSuccess;
}

hipError_t launch_gen_batched(const GenJob* jobs, uint32_t njobs, uint64_t total_blocks, uint64_t total_chunks,
                              uint32_t total_items, float R, uint32_t* counter, uint32_t* err, uint32_t grid,
                              int group, hipStream_t s, int part)
{
    if (njobs == 0) return hipSuccess;
    hipError_t e = hipSuccess;
    if (part == 0 || part == 1) {
        if (total_blocks > 0) {
            hipLaunchKernelGGL(k_gen_prep_batched, dim3((uint32_t)total_blocks), dim3(1024), 0, s, jobs, njobs, err);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_gen_clusters_batched, dim3((uint32_t)((total_chunks + 3) / 4)), dim3(256), 0, s,
                               jobs, njobs, total_chunks);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, counter, 1u, 0u);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (part == 1 || total_items == 0) return hipSuccess;
    if (group == 2)
        hipLaunchKernelGGL(k_gen_batched<2>, dim3(grid), dim3(kWaves * 64), 0, s, jobs, njobs, total_items, R, counter,
                           err);
    else
        hipLaunchKernelGGL(k_gen_batched<4>, dim3(grid), dim3(kWaves * 64), 0, s, jobs, njobs, total_items, R, counter,
                           err);
    return hipGetLastError();
}

}  // namespace rici
