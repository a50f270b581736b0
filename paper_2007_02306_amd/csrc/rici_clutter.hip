// Clutter around oriented points (Eq. 8): the areas of the whole scene's and
// of one object's surface inside each point's support volume -- the cylinder
// alpha <= R, |beta| <= R/2 about the Central Axis (Sec. 2.1) -- from which
// clutter = (A_all - A_object) / A_all.
//
// A workgroup owns kCG oriented points; its lanes stream the triangles, move
// their vertices into each point's frame (Eq. 1-4, FP64), drop triangles that
// provably miss the volume (height range outside the slab, or a bounding
// circle of the projected vertices outside the disc of radius R) and
// integrate the area of the others exactly.  Per-lane FP64 sums are reduced
// over the workgroup at the end.
//
// Exact area of a triangle in the volume: in its plane take orthonormal
// coordinates (s, t) with e1 horizontal and e2 = m x e1.  The distance of a
// plane point from the axis depends on s and on a2 + k t only (k = the
// horizontal part of e2 along z x e1), and its height is linear in t, so at
// in-plane height t the volume covers |s| <= sqrt(R^2 - (a2 + k t)^2) inside a
// t-range set by the slab.  The triangle covers [lo(t), hi(t)], linear
// between its vertices.  Integrating the overlap length over t piece by piece
// (pieces split where an end switches: vertices, slab ends, tangency, and
// edges crossing the boundary) needs only linear integrals and that of the
// root, done in closed form arranged so that nearly vertical planes (k -> 0)
// do not cancel.
#include "rici_internal.h"

namespace rici {
namespace {

constexpr int kCG = 8;            // oriented points per workgroup
constexpr int kCThreads = 256;

struct CFrame {
    double sx, sy, sz, nax, nay, nbx, nbz;
    int live;
};

__device__ __forceinline__ double root_pos(double x) { return x > 0.0 ? sqrt(x) : 0.0; }

// integral of sqrt(R^2 - (a2 + k t)^2) over [t1, t2] (|a2 + k t| <= R there).
// In x = (a2 + k t) / R, c = sqrt(1 - x^2), the antiderivative is
// R^2 (x c + asin x) / 2 per unit of x, and dx = (k / R) dt.  Well-conditioned
// forms: nearly equal ends (a plane close to parallel with the axis) by 5-point
// Gauss-Legendre on t; ends away from tangency by the difference written as
// (x2 - x1) times bounded factors, so (x2 - x1) / (k / R) = dt exactly; near
// tangency directly, with asin x as atan2(x, c) so that the errors of c and
// of the angle cancel to first order.
__device__ double strip_integral(double R, double a2, double k, double t1, double t2)
{
    const double dt = t2 - t1;
    if (!(dt > 0.0)) return 0.0;
    if (k == 0.0) return root_pos(R * R - a2 * a2) * dt;
    const double x1 = fmin(1.0, fmax(-1.0, (a2 + k * t1) / R));
    const double x2 = fmin(1.0, fmax(-1.0, (a2 + k * t2) / R));
    const double c1 = root_pos(1.0 - x1 * x1), c2 = root_pos(1.0 - x2 * x2);
    if (fabs(x2 - x1) < 1e-6) {
        const double gx[5] = {-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831,
                              0.9061798459386640};
        const double gw[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889, 0.4786286704993665,
                              0.2369268850561891};
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const double x = fmin(1.0, fmax(-1.0, (a2 + k * (0.5 * (t1 + t2) + 0.5 * dt * gx[q])) / R));
            acc += gw[q] * root_pos(1.0 - x * x);
        }
        return 0.5 * R * dt * acc;
    }
    if (fmin(c1, c2) >= 0.1 && x1 * x2 >= 0.0 && fabs(x2 - x1) < 0.5) {
        const double h = x1 * (x1 + x2) / (c1 + c2);
        const double g = c1 + h;
        const double y = (x2 - x1) * g;
        const double r = fabs(y) < 1e-8 ? 1.0 + y * y / 6.0 : asin(y) / y;
        return 0.5 * R * dt * ((c2 - h) + r * g);
    }
    const double g1 = x1 * c1 + atan2(x1, c1), g2 = x2 * c2 + atan2(x2, c2);
    return 0.5 * R * R * (g2 - g1) / k;
}

__device__ __forceinline__ void cross(const double* a, const double* b, double* o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// area of the triangle (vertices in the point's frame) inside the volume
__device__ double area_in_volume(const double (&P)[3][3], double R)
{
    const double u[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
    const double v[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
    double n[3];
    cross(u, v, n);
    const double nl = sqrt(dot(n, n));
    if (!(nl > 0.0)) return 0.0;
    const double m[3] = {n[0] / nl, n[1] / nl, n[2] / nl};
    const double hl = sqrt(m[0] * m[0] + m[1] * m[1]);
    double e1[3] = {1.0, 0.0, 0.0};
    if (hl > 1e-300) { e1[0] = m[1] / hl; e1[1] = -m[0] / hl; }
    double e2[3];
    cross(m, e1, e2);
    const double w2[3] = {-e1[1], e1[0], 0.0};
    const double h0 = dot(P[0], m);
    const double a2 = h0 * dot(m, w2), k = dot(e2, w2);
    const double zc = h0 * m[2], ez = e2[2];
    double tlo = -INFINITY, thi = INFINITY;
    if (ez != 0.0) {
        const double ta = (-0.5 * R - zc) / ez, tb = (0.5 * R - zc) / ez;
        tlo = fmin(ta, tb);
        thi = fmax(ta, tb);
    } else if (fabs(zc) > 0.5 * R) {
        return 0.0;
    }
    if (k != 0.0) {
        const double ta = (-R - a2) / k, tb = (R - a2) / k;
        tlo = fmax(tlo, fmin(ta, tb));
        thi = fmin(thi, fmax(ta, tb));
    } else if (fabs(a2) > R) {
        return 0.0;
    }
    double s[3], t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        s[i] = dot(P[i], e1);
        t[i] = dot(P[i], e2);
    }
    // order the vertices by t: a (lowest), b, c (highest)
    int ia = 0, ib = 1, ic = 2;
    if (t[ib] < t[ia]) { const int x = ia; ia = ib; ib = x; }
    if (t[ic] < t[ib]) { const int x = ib; ib = ic; ic = x; }
    if (t[ib] < t[ia]) { const int x = ia; ia = ib; ib = x; }
    tlo = fmax(tlo, t[ia]);
    thi = fmin(thi, t[ic]);
    if (!(thi > tlo) || !(t[ic] > t[ia])) return 0.0;
    // the long edge a-c and the two short ones, as s = p + q t
    const double qac = (s[ic] - s[ia]) / (t[ic] - t[ia]), pac = s[ia] - qac * t[ia];
    const bool ab_ok = t[ib] > t[ia], bc_ok = t[ic] > t[ib];
    const double qab = ab_ok ? (s[ib] - s[ia]) / (t[ib] - t[ia]) : 0.0, pab = s[ia] - qab * t[ia];
    const double qbc = bc_ok ? (s[ic] - s[ib]) / (t[ic] - t[ib]) : 0.0, pbc = s[ib] - qbc * t[ib];
    // breakpoints (at most 2 + 1 + 2 per edge), kept sorted by insertion
    double bp[9];
    int nb = 0;
    auto add = [&](double x) {
        if (!(x > tlo && x < thi)) return;
        int j = nb++;
        while (j > 0 && bp[j - 1] > x) { bp[j] = bp[j - 1]; --j; }
        bp[j] = x;
    };
    add(t[ib]);
    auto crossings = [&](double p, double q, double t0, double t1) {
        // (p + q t)^2 + (a2 + k t)^2 = R^2 on (t0, t1)
        const double A = q * q + k * k, B = 2.0 * (p * q + a2 * k), C = p * p + a2 * a2 - R * R;
        if (!(A > 0.0)) return;
        const double disc = B * B - 4.0 * A * C;
        if (disc < 0.0) return;
        const double sq = sqrt(disc);
        const double r1 = (-B - sq) / (2.0 * A), r2 = (-B + sq) / (2.0 * A);
        if (r1 > t0 && r1 < t1) add(r1);
        if (r2 > t0 && r2 < t1) add(r2);
    };
    crossings(pac, qac, t[ia], t[ic]);
    if (ab_ok) crossings(pab, qab, t[ia], t[ib]);
    if (bc_ok) crossings(pbc, qbc, t[ib], t[ic]);
    double area = 0.0;
    double lo_t = tlo;
    for (int i = 0; i <= nb; ++i) {
        const double hi_t = i < nb ? bp[i] : thi;
        const double len = hi_t - lo_t;
        if (len > 0.0) {
            const double tm = 0.5 * (lo_t + hi_t);
            const bool first = tm <= t[ib];
            if (first ? ab_ok : bc_ok) {
                const double qo = first ? qab : qbc, po = first ? pab : pbc;
                // ends of the triangle's cross-section at the piece's mid-height
                const double sl = pac + qac * tm, so = po + qo * tm;
                const double low = fmin(sl, so), high = fmax(sl, so);
                const double dm = a2 + k * tm;
                const double wm = root_pos(R * R - dm * dm);
                if (fmin(high, wm) > fmax(low, -wm)) {
                    // linear ends integrate to their value at mid-height times the length
                    const bool top_w = high >= wm, bot_w = low <= -wm;
                    const double iw = (top_w || bot_w) ? strip_integral(R, a2, k, lo_t, hi_t) : 0.0;
                    area += (top_w ? iw : high * len) - (bot_w ? -iw : low * len);
                }
            }
        }
        lo_t = hi_t;
    }
    return area;
}

__device__ __forceinline__ double block_sum(double x, double* red)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = x;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kCThreads / 64; ++w) s += red[w];
    return s;
}

__global__ void __launch_bounds__(kCThreads)
k_clutter(const float* __restrict__ pos, uint32_t nv, const uint32_t* __restrict__ tri, uint32_t nt,
          uint32_t obj_first, uint32_t obj_count, const float* __restrict__ op_pos, const float* __restrict__ op_nrm,
          uint32_t n, float Rf, double* __restrict__ a_all, double* __restrict__ a_obj, uint32_t* __restrict__ err)
{
    __shared__ CFrame fr[kCG];
    __shared__ double red[kCThreads / 64];
    const int tid = threadIdx.x;
    const uint32_t p0 = blockIdx.x * kCG;
    if (tid < kCG) {
        CFrame f = {};
        const uint32_t p = p0 + tid;
        if (p < n) {
            const float* sp = op_pos + 3 * (size_t)p;
            const float* sn = op_nrm + 3 * (size_t)p;
            if (isfinite(sp[0]) && isfinite(sp[1]) && isfinite(sp[2]) && isfinite(sn[0]) && isfinite(sn[1]) &&
                isfinite(sn[2])) {
                const Rotation q = frame_rotation(sn[0], sn[1], sn[2]);
                f.sx = sp[0]; f.sy = sp[1]; f.sz = sp[2];
                f.nax = q.nax; f.nay = q.nay; f.nbx = q.nbx; f.nbz = q.nbz;
                f.live = 1;
            } else {
                atomicOr(err, 2u);
            }
        }
        fr[tid] = f;
    }
    __syncthreads();
    const double R = Rf;
    double sum_all[kCG], sum_obj[kCG];
#pragma unroll
    for (int g = 0; g < kCG; ++g) sum_all[g] = sum_obj[g] = 0.0;
    for (uint32_t i = tid; i < nt; i += kCThreads) {
        const uint32_t i0 = tri[3 * (size_t)i], i1 = tri[3 * (size_t)i + 1], i2 = tri[3 * (size_t)i + 2];
        if (i0 >= nv || i1 >= nv || i2 >= nv) {
            atomicOr(err, 1u);
            continue;
        }
        const uint32_t vi[3] = {i0, i1, i2};
        double V[3][3];
        bool fin = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float x = pos[3 * (size_t)vi[k] + c];
                fin = fin && isfinite(x);
                V[k][c] = x;
            }
        }
        if (!fin) {
            atomicOr(err, 2u);
            continue;
        }
        const bool in_obj = i - obj_first < obj_count && i >= obj_first;
#pragma unroll
        for (int g = 0; g < kCG; ++g) {
            const CFrame& F = fr[g];
            if (!F.live) continue;
            double P[3][3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double px = V[k][0] - F.sx, py = V[k][1] - F.sy, pz = V[k][2] - F.sz;   // Eq. 2
                const double qx = F.nax * px + F.nay * py;                                  // Eq. 3
                P[k][1] = -F.nay * px + F.nax * py;
                P[k][0] = F.nbz * qx - F.nbx * pz;                                          // Eq. 4
                P[k][2] = F.nbx * qx + F.nbz * pz;
            }
            // provable misses (margins far above FP64 rounding)
            const double zmin = fmin(P[0][2], fmin(P[1][2], P[2][2])), zmax = fmax(P[0][2], fmax(P[1][2], P[2][2]));
            const double margin = 1e-9 * (R + fabs(zmin) + fabs(zmax));
            if (zmin > 0.5 * R + margin || zmax < -0.5 * R - margin) continue;
            const double cx = (P[0][0] + P[1][0] + P[2][0]) / 3.0, cy = (P[0][1] + P[1][1] + P[2][1]) / 3.0;
            double r2 = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                r2 = fmax(r2, (P[k][0] - cx) * (P[k][0] - cx) + (P[k][1] - cy) * (P[k][1] - cy));
            const double cd = sqrt(cx * cx + cy * cy), rr = sqrt(r2);
            if (cd - rr > R * (1.0 + 1e-9) + 1e-12) continue;
            const double a = area_in_volume(P, R);
            sum_all[g] += a;
            if (in_obj) sum_obj[g] += a;
        }
    }
#pragma unroll
    for (int g = 0; g < kCG; ++g) {
        const double sa = block_sum(sum_all[g], red);
        const double so = block_sum(sum_obj[g], red);
        if (tid == 0 && p0 + g < n) {
            a_all[p0 + g] = sa;
            a_obj[p0 + g] = so;
        }
    }
}

}  // namespace

hipError_t launch_clutter(const float* pos, uint32_t nv, const uint32_t* tri, uint32_t nt, uint32_t obj_first,
                          uint32_t obj_count, const float* op_pos, const float* op_nrm, uint32_t n, float R,
                          double* a_all, double* a_obj, uint32_t* err, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_clutter, dim3((n + kCG - 1) / kCG), dim3(kCThreads), 0, s, pos, nv, tri, nt, obj_first,
                       obj_count, op_pos, op_nrm, n, R, a_all, a_obj, err);
    return hipGetLastError();
}

}  // namespace rici
