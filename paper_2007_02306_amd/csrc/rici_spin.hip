// Spin Images (Sec. 2.1) for gfx950, built with the same FP64 projection as
// the RICI generator (Sec. 3.1.1 states the projection serves SI construction
// too), and the search by Pearson correlation with the rank of the true match
// (Sec. 4.1 step 6c, ties to the best rank).
//
// Generation: a workgroup owns G images in LDS (fp32, 16 KiB each); its lanes
// stream the point samples (coalesced), project each into the G frames in
// FP64 (bin units), keep the samples inside the support volume
// (0 <= alpha < R, -R/2 <= beta < R/2) and add their bilinear weights between
// bin centres to the four nearest bins with LDS float atomics; the images
// leave as coalesced rows.  Sums are fp32, so pixel values carry the rounding
// of an fp32 sum of their contributions in arbitrary order.
//
// Search: rho(a, b) = <z_a, z_b> with z = (x - mean) / |x - mean| (0 for a
// constant image).  A prep kernel writes z in fp32, fragment-major for
// v_mfma_f32_16x16x4_f32 (per group of 16 images and 16 pixels: lane
// 16 q + i holds pixels 16 kc + 4 s + q of image i, s = 0..3), with the mean
// and norm in FP64.  The contraction runs on MFMA over 128 x 128 tiles.  Its
// error is below kBand (4100 fp32 roundings of a sum of |z_a z_b| <= 1), so
// a pair whose fp32 correlation is more than kBand above the true match's is
// counted, one within kBand of it is queued, and the queue is settled by the
// exact FP64 correlation -- the same routine that gives the true match's
// correlation, so the true match never outranks itself and ranks are exact
// up to FP64 rounding of the correlations.
#include "rici_internal.h"

namespace rici {
namespace {

constexpr int kSpinG = 4;              // images per generation workgroup
constexpr int kSpinThreads = 256;
constexpr int kZTile = 128;            // images per correlation tile side
constexpr double kBand = 2.5e-4;       // > 4100 * 2^-24: fp32 contraction error bound

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bool finite3f(float a, float b, float c)
{
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// ------------------------------------------------------------ generation

struct SpinFrame {
    double sx, sy, sz;
    double nax, nay;              // first rotation
    double nax_d, nay_d;          // first rotation x 64 / R (y coordinate in bins)
    double nbx_d, nbz_d;          // second rotation x 64 / R
    int live;
};

__global__ void __launch_bounds__(kSpinThreads)
k_spin_gen(const float* __restrict__ samples, uint32_t ns, const float* __restrict__ op_pos,
           const float* __restrict__ op_nrm, uint32_t n, float R, float* __restrict__ out,
           uint32_t* __restrict__ err)
{
    extern __shared__ __align__(16) float simg[];   // [kSpinG][4096]
    __shared__ SpinFrame fr[kSpinG];
    const int tid = threadIdx.x;
    const uint32_t img0 = blockIdx.x * kSpinG;
    for (int i = tid; i < kSpinG * NPIX; i += kSpinThreads) simg[i] = 0.f;
    if (tid < kSpinG) {
        SpinFrame f = {};
        const uint32_t img = img0 + tid;
        if (img < n) {
            const float* sp = op_pos + 3 * (size_t)img;
            const float* sn = op_nrm + 3 * (size_t)img;
            if (!finite3f(sp[0], sp[1], sp[2]) || !finite3f(sn[0], sn[1], sn[2])) {
                atomicOr(err, 2u);
            } else {
                const double inv_d = (double)NB / (double)R;     // bin units
                const Rotation q = frame_rotation(sn[0], sn[1], sn[2]);
                f.sx = sp[0]; f.sy = sp[1]; f.sz = sp[2];
                f.nax = q.nax; f.nay = q.nay;
                f.nax_d = q.nax * inv_d; f.nay_d = q.nay * inv_d;
                f.nbx_d = q.nbx * inv_d; f.nbz_d = q.nbz * inv_d;
                f.live = 1;
            }
        }
        fr[tid] = f;
    }
    __syncthreads();
    for (uint32_t s = tid; s < ns; s += kSpinThreads) {
        const float x = samples[3 * (size_t)s], y = samples[3 * (size_t)s + 1], z = samples[3 * (size_t)s + 2];
        if (!finite3f(x, y, z)) {
            atomicOr(err, 2u);
            continue;
        }
#pragma unroll
        for (int g = 0; g < kSpinG; ++g) {
            const SpinFrame& F = fr[g];
            if (!F.live) continue;
            const double px = (double)x - F.sx, py = (double)y - F.sy, pz = (double)z - F.sz;   // Eq. 2
            const double qx = F.nax * px + F.nay * py;                                       // Eq. 3
            const double Y = -F.nay_d * px + F.nax_d * py;
            const double X = F.nbz_d * qx - F.nbx_d * pz;                                    // Eq. 4
            const double Z = F.nbx_d * qx + F.nbz_d * pz;
            const double a2 = X * X + Y * Y;
            // support volume in bins: alpha < 64, -32 <= beta < 32
            if (!(a2 < (double)(NB * NB)) || !(Z >= -0.5 * NB) || !(Z < 0.5 * NB)) continue;
            const double u = sqrt(a2) - 0.5, v = Z + (0.5 * NB - 0.5);                        // Eq. 5, bin centres
            const double cu = floor(u), rv = floor(v);
            const double fu = u - cu, fv = v - rv;
            const int c0 = (int)cu, r0 = (int)rv;
            float* im = simg + g * NPIX;
            // weights in FP64, each rounded once to fp32
            const float w00 = (float)((1.0 - fu) * (1.0 - fv)), w01 = (float)(fu * (1.0 - fv));
            const float w10 = (float)((1.0 - fu) * fv), w11 = (float)(fu * fv);
            // c0 >= -1 and r0 >= -1 always; c0, r0 <= 63
            if (r0 >= 0) {
                if (c0 >= 0) atomicAdd(im + r0 * NB + c0, w00);
                if (c0 + 1 < NB) atomicAdd(im + r0 * NB + c0 + 1, w01);
            }
            if (r0 + 1 < NB) {
                if (c0 >= 0) atomicAdd(im + (r0 + 1) * NB + c0, w10);
                if (c0 + 1 < NB) atomicAdd(im + (r0 + 1) * NB + c0 + 1, w11);
            }
        }
    }
    __syncthreads();
    for (int g = 0; g < kSpinG; ++g) {
        const uint32_t img = img0 + g;
        if (img >= n) break;
        float4* dst = reinterpret_cast<float4*>(out + (size_t)img * NPIX);
        const float4* src = reinterpret_cast<const float4*>(simg + g * NPIX);
        for (int i = tid; i < NPIX / 4; i += kSpinThreads) dst[i] = src[i];
    }
}

// -------------------------------------------------------- correlation prep

__device__ __forceinline__ double wave_sum_f64(double x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// One wave per image: FP64 mean and centred norm, then z = (x - mean) / norm
// in fp32, fragment-major.  Images past n (padding up to the tile) get z = 0.
__global__ void __launch_bounds__(256)
k_spin_zprep(const float* __restrict__ images, uint32_t n, uint32_t nslots, float* __restrict__ z,
             double* __restrict__ mean, double* __restrict__ norm)
{
    const int lane = threadIdx.x & 63;
    const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nslots) return;
    const uint32_t grp = i / 16, slot = i % 16;
    float* zg = z + (size_t)grp * NPIX * 16;
    if (i >= n) {
        for (int j = 0; j < 64; ++j) {
            const int k = lane + 64 * j;
            zg[((size_t)(k >> 4) * 64 + 16 * (k & 3) + slot) * 4 + ((k >> 2) & 3)] = 0.f;
        }
        return;
    }
    const float* x = images + (size_t)i * NPIX;
    float v[64];
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        v[j] = x[lane + 64 * j];
        s += (double)v[j];
    }
    const double m = wave_sum_f64(s) / (double)NPIX;
    double q = 0.0;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        const double d = (double)v[j] - m;
        q += d * d;
    }
    const double nrm = sqrt(wave_sum_f64(q));
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        const int k = lane + 64 * j;
        zg[((size_t)(k >> 4) * 64 + 16 * (k & 3) + slot) * 4 + ((k >> 2) & 3)] = (float)(((double)v[j] - m) * inv);
    }
    if (lane == 0) {
        mean[i] = m;
        norm[i] = nrm;
    }
}

// Exact correlation of one pair by one wave: FP64 centred cross sum over the
// 4096 pixels (fixed lane order and butterfly), divided by the two norms.
// Not inlined, so every caller gets bit-identical values for the same pair.
__device__ __noinline__ double rho_exact(const float* __restrict__ a, const float* __restrict__ b, double ma,
                                         double na, double mb, double nb)
{
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int j = 0; j < 64; ++j) {
        const int k = lane + 64 * j;
        s += ((double)a[k] - ma) * ((double)b[k] - mb);
    }
    s = wave_sum_f64(s);
    if (!(na > 0.0) || !(nb > 0.0)) return 0.0;
    return s / (na * nb);
}

// rho_t[i] = rho(needle i, haystack t[i]), one wave per needle
__global__ void __launch_bounds__(256)
k_spin_true(const float* __restrict__ needles, uint32_t nn, const float* __restrict__ hay, uint32_t nh,
            const uint32_t* __restrict__ true_idx, const double* __restrict__ nmean, const double* __restrict__ nnorm,
            const double* __restrict__ hmean, const double* __restrict__ hnorm, double* __restrict__ rho_t,
            uint32_t* __restrict__ rank)
{
    const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nn) return;
    const uint32_t t = true_idx[i];
    double r = INFINITY;    // an out-of-range true index: rank nh, nothing counted
    if (t < nh)
        r = rho_exact(needles + (size_t)i * NPIX, hay + (size_t)t * NPIX, nmean[i], nnorm[i], hmean[t], hnorm[t]);
    if ((threadIdx.x & 63) == 0) {
        rho_t[i] = r;
        rank[i] = t < nh ? 0u : nh;
    }
}

// ----------------------------------------------------------- contraction

// Inclusive prefix sum over the lane's row of 16 lanes (DPP row shifts).
__device__ __forceinline__ uint32_t row16_sum(uint32_t x)
{
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);   // row_shr:8
    return x;
}

struct SpinSearch {
    const float* za; const float* zb;      // fragment-major z planes
    uint32_t nn, nh, tiles_n;
    const uint32_t* true_idx;              // rank mode
    const double* rho_t;
    uint32_t* rank;
    uint2* queue; uint32_t* queue_count; uint32_t queue_cap;
    float* matrix;                         // matrix mode [nn][nh]
    uint32_t* err;
};

// 128 x 128 (needle x haystack) tile per workgroup of 4 waves, each wave a
// 64 x 64 block: 4 x 4 accumulators of 16 x 16.  Per 16 pixels a wave loads 8
// fragments (16 B per lane) and issues 64 MFMAs; the next 16 pixels' fragments
// are loaded before this step's MFMAs.
template <bool RANK>
__global__ void __launch_bounds__(256)
k_spin_search(SpinSearch S)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const uint32_t tm = blockIdx.x / S.tiles_n, tn = blockIdx.x % S.tiles_n;
    const uint32_t ga0 = tm * (kZTile / 16) + wm * 4, gb0 = tn * (kZTile / 16) + wn * 4;
    const v4f* A = reinterpret_cast<const v4f*>(S.za) + (size_t)ga0 * 256 * 64 + lane;
    const v4f* B = reinterpret_cast<const v4f*>(S.zb) + (size_t)gb0 * 256 * 64 + lane;
    constexpr size_t kGrp = 256 * 64;      // v4f per group of 16 images
    v4f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    v4f a[4], b[4], na[4], nb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        a[i] = A[i * kGrp];
        b[i] = B[i * kGrp];
    }
    for (int kc = 0; kc < 256; ++kc) {
        const int kn = kc + 1 < 256 ? kc + 1 : kc;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            na[i] = A[i * kGrp + (size_t)kn * 64];
            nb[i] = B[i * kGrp + (size_t)kn * 64];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a[i] = na[i];
            b[i] = nb[i];
        }
    }
    // accumulator layout: lane l holds column l % 16 and rows 4 (l / 16) + v
    const int cl = lane & 15, rq = lane >> 4;
    uint32_t col[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) col[j] = (gb0 + j) * 16 + cl;
    if (!RANK) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t row = (ga0 + i) * 16 + 4 * rq + v;
                if (row >= S.nn) continue;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (col[j] < S.nh) S.matrix[(size_t)row * S.nh + col[j]] = acc[i][j][v];
            }
        return;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint32_t packed = 0;
        uint32_t rows[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const uint32_t row = (ga0 + i) * 16 + 4 * rq + v;
            rows[v] = row;
            if (row >= S.nn) continue;
            const double rt = S.rho_t[row];
            const uint32_t t = S.true_idx[row];
            uint32_t cnt = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (col[j] >= S.nh || col[j] == t) continue;
                const double r = (double)acc[i][j][v];
                if (r > rt + kBand) {
                    ++cnt;
                } else if (r >= rt - kBand) {
                    const uint32_t slot = atomicAdd(S.queue_count, 1u);
                    if (slot < S.queue_cap) S.queue[slot] = make_uint2(row, col[j]);
                    else atomicOr(S.err, 4u);
                }
            }
            packed |= cnt << (8 * v);
        }
        packed = row16_sum(packed);
        if (cl == 15) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t c = (packed >> (8 * v)) & 0xFFu;
                if (c && rows[v] < S.nn) atomicAdd(S.rank + rows[v], c);
            }
        }
    }
}

// The queued pairs, settled by the exact correlation: one wave per pair.
__global__ void __launch_bounds__(256)
k_spin_settle(const float* __restrict__ needles, const float* __restrict__ hay, const uint2* __restrict__ queue,
              const uint32_t* __restrict__ queue_count, uint32_t queue_cap, const double* __restrict__ nmean,
              const double* __restrict__ nnorm, const double* __restrict__ hmean, const double* __restrict__ hnorm,
              const double* __restrict__ rho_t, uint32_t* __restrict__ rank)
{
    const uint32_t total = min(*queue_count, queue_cap);
    const uint32_t waves = gridDim.x * 4;
    for (uint32_t e = blockIdx.x * 4 + (threadIdx.x >> 6); e < total; e += waves) {
        const uint2 p = queue[e];
        const double r = rho_exact(needles + (size_t)p.x * NPIX, hay + (size_t)p.y * NPIX, nmean[p.x], nnorm[p.x],
                                   hmean[p.y], hnorm[p.y]);
        if ((threadIdx.x & 63) == 0 && r > rho_t[p.x]) atomicAdd(rank + p.x, 1u);
    }
}

__global__ void k_spin_zero(uint32_t* __restrict__ p) { if (threadIdx.x == 0) *p = 0u; }

}  // namespace

size_t spin_slots(uint32_t n) { return ((size_t)n + kZTile - 1) / kZTile * kZTile; }
double spin_band() { return kBand; }

hipError_t launch_spin_gen(const float* samples, uint32_t ns, const float* op_pos, const float* op_nrm, uint32_t n,
                           float R, float* out, uint32_t* err, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    static hipError_t once = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spin_gen),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)(kSpinG * NPIX * sizeof(float)));
    if (once != hipSuccess) return once;
    hipLaunchKernelGGL(k_spin_gen, dim3((n + kSpinG - 1) / kSpinG), dim3(kSpinThreads),
                       kSpinG * NPIX * sizeof(float), s, samples, ns, op_pos, op_nrm, n, R, out, err);
    return hipGetLastError();
}

hipError_t launch_spin_zprep(const float* images, uint32_t n, float* z, double* mean, double* norm, hipStream_t s)
{
    const size_t slots = spin_slots(n);
    if (slots == 0) return hipSuccess;
    hipLaunchKernelGGL(k_spin_zprep, dim3((uint32_t)((slots + 3) / 4)), dim3(256), 0, s, images, n, (uint32_t)slots,
                       z, mean, norm);
    return hipGetLastError();
}

hipError_t launch_spin_rank(const SpinPrep& np, const float* needles, uint32_t nn, const SpinPrep& hp,
                            const float* hay, uint32_t nh, const uint32_t* true_idx, double* rho_t, uint32_t* rank,
                            uint2* queue, uint32_t* queue_count, uint32_t queue_cap, uint32_t* err, hipStream_t s,
                            int part)
{
    if (nn == 0) return hipSuccess;
    hipError_t e = hipSuccess;
    if (part == 0 || part == 1) {
        hipLaunchKernelGGL(k_spin_zero, dim3(1), dim3(64), 0, s, queue_count);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_spin_true, dim3((nn + 3) / 4), dim3(256), 0, s, needles, nn, hay, nh, true_idx, np.mean,
                           np.norm, hp.mean, hp.norm, rho_t, rank);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (part == 0 || part == 2) {
        SpinSearch S = {};
        S.za = np.z; S.zb = hp.z; S.nn = nn; S.nh = nh;
        const uint32_t tiles_m = (uint32_t)(spin_slots(nn) / kZTile);
        S.tiles_n = (uint32_t)(spin_slots(nh) / kZTile);
        S.true_idx = true_idx; S.rho_t = rho_t; S.rank = rank;
        S.queue = queue; S.queue_count = queue_count; S.queue_cap = queue_cap; S.err = err;
        hipLaunchKernelGGL(k_spin_search<true>, dim3(tiles_m * S.tiles_n), dim3(256), 0, s, S);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (part == 0 || part == 3) {
        hipLaunchKernelGGL(k_spin_settle, dim3(1024), dim3(256), 0, s, needles, hay, queue, queue_count, queue_cap,
                           np.mean, np.norm, hp.mean, hp.norm, rho_t, rank);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_spin_matrix(const SpinPrep& np, uint32_t nn, const SpinPrep& hp, uint32_t nh, float* out,
                              hipStream_t s)
{
    if (nn == 0) return hipSuccess;
    SpinSearch S = {};
    S.za = np.z; S.zb = hp.z; S.nn = nn; S.nh = nh; S.matrix = out;
    const uint32_t tiles_m = (uint32_t)(spin_slots(nn) / kZTile);
    S.tiles_n = (uint32_t)(spin_slots(nh) / kZTile);
    hipLaunchKernelGGL(k_spin_search<false>, dim3(tiles_m * S.tiles_n), dim3(256), 0, s, S);
    return hipGetLastError();
}

}  // namespace rici
