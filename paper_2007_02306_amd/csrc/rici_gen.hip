// RICI generation for gfx950 (Sec. 3.1 of van Blokland & Theoharis 2020).
//
// For every oriented point, every scene triangle is projected into cylindrical
// (alpha, beta) coordinates (Sec. 3.1.1), sliced by the row planes in its beta
// extent, and the radii with single and double circle intersections are
// counted into the image (Sec. 3.1.2).
//
// Mapping onto CDNA4
//   * A workgroup owns G images.  Their FP64 frames (Eq. 1 coefficients) and
//     per-row difference arrays live in LDS (G x 16 KiB of uint32).
//   * Lanes stream triangles (one per lane, coalesced float4 bounding spheres)
//     and test each against the G images with a conservative FP32 cull: the
//     bounding sphere must reach the support slab |beta| <= R/2 and the support
//     cylinder alpha <= R, with margins far above FP32 rounding.  The cull only
//     discards triangles that provably touch no bin, so counts are unchanged.
//   * Survivors (image, triangle) are appended to a per-wave LDS ring with a
//     ballot prefix; once 64 are queued every lane takes one and does the exact
//     work in FP64: projection (Eq. 2-5), rows in the triangle's beta extent,
//     the slice E0E1, single range (min|E|, max|E|), double range (|C|, min|E|),
//     all as comparisons of squared radii (no sqrt in any decision).
//   * Each slice adds +1 / -1 (single) and +2 / -2 (double) at its first and
//     end columns of a row's difference array (3 LDS atomics per slice, O(1)
//     per slice instead of O(64)); the final row prefix sum is a wavefront
//     scan and each row leaves as one coalesced 256 B store.
#include "rici_internal.h"

namespace rici {
namespace {

constexpr int kG = 8;          // images per workgroup
constexpr int kWaves = 8;      // wavefronts per workgroup
constexpr int kRing = 128;     // per-wave survivor ring (entries)

__device__ __forceinline__ bool finite3(float a, float b, float c)
{
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// ------------------------------------------------------------- triangle prep

__global__ void __launch_bounds__(256)
k_gen_prep(const float* __restrict__ pos, uint32_t nv, const uint32_t* __restrict__ tri, uint32_t nt,
           float4* __restrict__ cull, float4* __restrict__ verts, uint32_t* __restrict__ err)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const uint32_t i0 = tri[3 * (size_t)t], i1 = tri[3 * (size_t)t + 1], i2 = tri[3 * (size_t)t + 2];
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
    cull[t] = make_float4(mx, my, mz, r);
}

// ------------------------------------------------------------ exact pieces

struct Frame {
    double sx, sy, sz;       // Spin Vertex
    double nax, nay;         // Eq. 1, first rotation (about z)
    double nbx, nbz;         // Eq. 1, second rotation (about y), normalising the rotated normal
    double pad;
};

// column index helpers: rho_c = (c + 1/2) * delta, exact in FP64
__device__ __forceinline__ double rho_sq(int c, double delta)
{
    double rho = ((double)c + 0.5) * delta;
    return rho * rho;
}

// first column c in [0, 64] with rho_c^2 > s (64 if none); s >= 0 or NaN-free
__device__ __forceinline__ int first_col_above(double s, double delta, float inv_delta)
{
    float f = sqrtf(fminf((float)s, 3.0e38f)) * inv_delta - 0.5f;
    f = fminf(fmaxf(f, -1.0f), 64.0f);
    int c = (int)floorf(f) + 1;
    c = min(max(c, 0), 64);
    if (c > 0 && rho_sq(c - 1, delta) > s) --c;
    if (c < 64 && rho_sq(c, delta) <= s) ++c;
    return c;
}

__device__ __forceinline__ double beta_of(int r, double R, double delta)
{
    return -0.5 * R + ((double)r + 0.5) * delta;   // exact for fp32 R
}

__device__ __forceinline__ void lds_add(uint32_t* row, int c, uint32_t v)
{
    if (c < NB) atomicAdd(row + c, v);
}

// One (image, triangle) survivor: the three steps of Sec. 3.1 in FP64.
__device__ void slice_triangle(const Frame& F, const float4 va, const float4 vb, const float4 vc,
                               double R, double delta, float inv_delta, uint32_t* diff_img)
{
    double x[3], y[3], z[3];
    const float4 v[3] = { va, vb, vc };
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double px = (double)v[k].x - F.sx;                 // Eq. 2
        double py = (double)v[k].y - F.sy;
        double pz = (double)v[k].z - F.sz;
        double qx = F.nax * px + F.nay * py;               // Eq. 3
        double qy = -F.nay * px + F.nax * py;
        x[k] = F.nbz * qx - F.nbx * pz;                    // Eq. 4
        y[k] = qy;
        z[k] = F.nbx * qx + F.nbz * pz;
    }
    const double zmin = fmin(z[0], fmin(z[1], z[2]));
    const double zmax = fmax(z[0], fmax(z[1], z[2]));
    const double inv_d = 1.0 / delta;

    // rows whose plane has vertices on both sides under "above iff z >= beta":
    // beta_r in (zmin, zmax]
    double fr0 = floor(fmin(fmax(zmin * inv_d + 31.5, -2.0), 70.0)) + 1.0;
    int r0 = min(max((int)fr0, 0), 64);
    if (r0 > 0 && beta_of(r0 - 1, R, delta) > zmin) --r0;
    if (r0 < 64 && beta_of(r0, R, delta) <= zmin) ++r0;
    double fr1 = floor(fmin(fmax(zmax * inv_d + 31.5, -2.0), 70.0));
    int r1 = min(max((int)fr1, -1), 63);
    if (r1 < 63 && beta_of(r1 + 1, R, delta) <= zmax) ++r1;
    if (r1 >= 0 && beta_of(r1, R, delta) > zmax) --r1;
    if (r0 > r1) return;

    // reciprocal vertical extent of the edges 0->1, 1->2, 2->0
    const double i01 = 1.0 / (z[1] - z[0]);
    const double i12 = 1.0 / (z[2] - z[1]);
    const double i20 = 1.0 / (z[0] - z[2]);

    for (int r = r0; r <= r1; ++r) {
        const double beta = beta_of(r, R, delta);
        const bool a0 = z[0] >= beta, a1 = z[1] >= beta, a2 = z[2] >= beta;
        // the vertex alone on its side of the plane (l) and the two edges
        // leaving it, towards a = l + 1 and b = l + 2 (mod 3)
        const bool l0 = (a0 != a1) && (a0 != a2);
        const bool l1 = !l0 && (a1 != a0) && (a1 != a2);
        const double xl = l0 ? x[0] : (l1 ? x[1] : x[2]);
        const double yl = l0 ? y[0] : (l1 ? y[1] : y[2]);
        const double zl = l0 ? z[0] : (l1 ? z[1] : z[2]);
        const double xa = l0 ? x[1] : (l1 ? x[2] : x[0]);
        const double ya = l0 ? y[1] : (l1 ? y[2] : y[0]);
        const double xb = l0 ? x[2] : (l1 ? x[0] : x[1]);
        const double yb = l0 ? y[2] : (l1 ? y[0] : y[1]);
        const double inv_a = l0 ? i01 : (l1 ? i12 : i20);      // 1 / (z_a - z_l)
        const double inv_b = l0 ? -i20 : (l1 ? -i01 : -i12);   // 1 / (z_b - z_l)
        const double hl = beta - zl;
        const double ta = hl * inv_a, tb = hl * inv_b;
        const double e0x = xl + ta * (xa - xl);
        const double e0y = yl + ta * (ya - yl);
        const double e1x = xl + tb * (xb - xl);
        const double e1y = yl + tb * (yb - yl);

        const double d0 = e0x * e0x + e0y * e0y;
        const double d1 = e1x * e1x + e1y * e1y;
        const double lo2 = fmin(d0, d1), hi2 = fmax(d0, d1);
        const double dx = e1x - e0x, dy = e1y - e0y;
        const double dd = dx * dx + dy * dy;
        const bool between = (e0x * dx + e0y * dy) < 0.0 && (e1x * dx + e1y * dy) > 0.0;

        uint32_t* row = diff_img + r * NB;
        const int c_lo = first_col_above(lo2, delta, inv_delta);
        const int c_hi = first_col_above(hi2, delta, inv_delta);
        if (between) {
            // |C|^2 = (E0 x E1)^2 / |E1 - E0|^2: distance of the axis from the line E0E1
            const double cr = e0x * e1y - e0y * e1x;
            const int c_c = first_col_above(cr * cr / dd, delta, inv_delta);
            if (c_c < c_lo) {
                lds_add(row, c_c, 2u);
                lds_add(row, c_lo, (uint32_t)-2);
            }
        }
        if (c_lo < c_hi) {
            lds_add(row, c_lo, 1u);
            lds_add(row, c_hi, (uint32_t)-1);
        }
    }
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

__global__ void __launch_bounds__(kWaves * 64)
k_gen(const float4* __restrict__ cull, const float4* __restrict__ verts, uint32_t nt,
      const float* __restrict__ op_pos, const float* __restrict__ op_nrm, uint32_t n, float Rf,
      uint32_t* __restrict__ out, uint32_t* __restrict__ err)
{
    __shared__ uint32_t diff[kG][NPIX];
    __shared__ uint32_t ring[kWaves][kRing];
    __shared__ Frame frames[kG];
    __shared__ __align__(16) float cp[kG][8];     // FP32 cull parameters per image

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t img0 = blockIdx.x * kG;
    const double R = (double)Rf;
    const double delta = R / NB;
    const float inv_delta = (float)(NB / R);

    for (int i = tid; i < kG * NPIX; i += kWaves * 64) (&diff[0][0])[i] = 0u;
    if (tid < kG) {
        Frame f = {};
        float* c = cp[tid];
        const uint32_t img = img0 + tid;
        bool live = img < n;
        if (live) {
            const float* sp = op_pos + 3 * (size_t)img;
            const float* sn = op_nrm + 3 * (size_t)img;
            if (!finite3(sp[0], sp[1], sp[2]) || !finite3(sn[0], sn[1], sn[2])) {
                atomicOr(err, 2u);
                live = false;
            } else {
                f.sx = sp[0]; f.sy = sp[1]; f.sz = sp[2];
                const double nx = sn[0], ny = sn[1], nz = sn[2];
                // Eq. 1: [N_ax, N_ay] = Normalize[S_nx, S_ny]; identity if both vanish
                const double la = sqrt(nx * nx + ny * ny);
                if (la > 0.0) { f.nax = nx / la; f.nay = ny / la; } else { f.nax = 1.0; f.nay = 0.0; }
                // second rotation normalises the normal's x after the first rotation
                const double rx = f.nax * nx + f.nay * ny;
                const double lb = sqrt(rx * rx + nz * nz);
                if (lb > 0.0) { f.nbx = rx / lb; f.nbz = nz / lb; } else { f.nbx = 0.0; f.nbz = 1.0; }
                // Central Axis direction for the cull: the pre-image of +z
                c[0] = sp[0]; c[1] = sp[1]; c[2] = sp[2];
                c[3] = (float)(f.nbx * f.nax);
                c[4] = (float)(f.nbx * f.nay);
                c[5] = (float)f.nbz;
                const float mag = fmaxf(fabsf(sp[0]), fmaxf(fabsf(sp[1]), fabsf(sp[2])));
                const float margin = 1e-5f * (mag + Rf) + 1e-30f;
                c[6] = 0.5f * Rf + margin;    // slab half height
                c[7] = Rf + margin;           // cylinder radius
            }
        }
        if (!live) {
            c[0] = c[1] = c[2] = 0.f; c[3] = c[4] = 0.f; c[5] = 1.f;
            c[6] = -INFINITY; c[7] = -INFINITY;
        }
        frames[tid] = f;
    }
    __syncthreads();

    uint32_t* my_ring = ring[wave];
    uint32_t head = 0, tail = 0;   // wave-uniform ring counters
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    for (uint32_t base = (uint32_t)wave * 64; base < nt; base += kWaves * 64) {
        const uint32_t t = base + lane;
        const float4 s = t < nt ? cull[t] : make_float4(0.f, 0.f, 0.f, -INFINITY);
#pragma unroll 1
        for (int g = 0; g < kG; ++g) {
            // uniform LDS reads (broadcast) of this image's cull parameters
            const float4 p0 = *reinterpret_cast<const float4*>(&cp[g][0]);
            const float4 p1 = *reinterpret_cast<const float4*>(&cp[g][4]);
            const float dx = s.x - p0.x, dy = s.y - p0.y, dz = s.z - p0.z;
            const float h = p0.w * dx + p1.x * dy + p1.y * dz;
            const float d2 = dx * dx + dy * dy + dz * dz;
            const float a2 = d2 - h * h;
            const float la = p1.w + s.w;
            const bool pass = fabsf(h) <= p1.z + s.w && a2 <= la * la && la > 0.f;
            const uint64_t m = __ballot(pass);
            if (pass) {
                const uint32_t slot = tail + (uint32_t)__popcll(m & lt_mask);
                my_ring[slot & (kRing - 1)] = (t << 3) | (uint32_t)g;
            }
            tail += (uint32_t)__popcll(m);
            if (tail - head >= 64) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const uint32_t e = my_ring[(head + lane) & (kRing - 1)];
                head += 64;
                const uint32_t gi = e & 7u, ti = e >> 3;
                slice_triangle(frames[gi], verts[3 * (size_t)ti], verts[3 * (size_t)ti + 1],
                               verts[3 * (size_t)ti + 2], R, delta, inv_delta, diff[gi]);
            }
        }
    }
    {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t left = tail - head;
        if ((uint32_t)lane < left) {
            const uint32_t e = my_ring[(head + lane) & (kRing - 1)];
            const uint32_t gi = e & 7u, ti = e >> 3;
            slice_triangle(frames[gi], verts[3 * (size_t)ti], verts[3 * (size_t)ti + 1],
                           verts[3 * (size_t)ti + 2], R, delta, inv_delta, diff[gi]);
        }
    }
    __syncthreads();

    // row prefix sums of the difference arrays -> counts; one row per wave step
    for (int row = wave; row < kG * NB; row += kWaves) {
        const int g = row / NB, r = row % NB;
        const uint32_t img = img0 + g;
        if (img >= n) continue;
        uint32_t v = wave_inclusive_scan(diff[g][r * NB + lane], lane);
        out[(size_t)img * NPIX + r * NB + lane] = v;
    }
}

}  // namespace

hipError_t launch_gen_prep(const float* pos, uint32_t nv, const uint32_t* tri, uint32_t nt,
                           float4* cull, float4* verts, uint32_t* err, hipStream_t s)
{
    if (nt == 0) return hipSuccess;
    const uint32_t blocks = (nt + 255) / 256;
    hipLaunchKernelGGL(k_gen_prep, dim3(blocks), dim3(256), 0, s, pos, nv, tri, nt, cull, verts, err);
    return hipGetLastError();
}

hipError_t launch_gen(const float4* cull, const float4* verts, uint32_t nt,
                      const float* op_pos, const float* op_nrm, uint32_t n, float R,
                      uint32_t* out, uint32_t* err, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint32_t blocks = (n + kG - 1) / kG;
    hipLaunchKernelGGL(k_gen, dim3(blocks), dim3(kWaves * 64), 0, s, cull, verts, nt, op_pos, op_nrm, n, R,
                       out, err);
    return hipGetLastError();
}

}  // namespace rici
