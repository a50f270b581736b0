/*
 * rici_oracle.c -- plain, slow, FP64 CPU oracle for the Radial Intersection
 * Count Image (RICI) method (van Blokland & Theoharis, "Radial intersection
 * count image: a clutter resistant 3D shape descriptor", 2020).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header or table with the HIP implementation.
 *
 * Contents
 *   rowrange : the paper's generation algorithm (Sec. 3.1: project the
 *              triangle, slice it with each row plane, single/double radius
 *              ranges, increment bins), with degeneracy flags and work counters.
 *   brute    : the plain definition of a RICI bin (number of points where the
 *              bin's circle meets the scene's triangles), solved per circle and
 *              triangle with trigonometry and barycentric coordinates.
 *   crd      : the clutter-resistant distance, Sec. 3.2 (Eq. 6-7), summed
 *              literally in int64.
 *   rank     : 0-based rank of the true match, ties taking the best rank
 *              (Sec. 4.1, clutterbox step 6c, and the tie rule of Sec. 4.2).
 *
 * Readings of the paper used here (each one is also listed in the design notes):
 *   R1  Eq. 1, second line: the second rotation normalises the *rotated*
 *       normal, N_b = Normalize(|(S_nx, S_ny)|, S_nz); the printed
 *       Normalize(S_nx, S_nz) does not align S_n with z when S_ny != 0.
 *       A pair that normalises from (0, 0) is the identity rotation (Sec. 3.1.1).
 *   R2  Pixel grid (Sec. 2.1 square plane, Sec. 3.1): the support square spans
 *       alpha in [0, R] and beta in [-R/2, R/2]; bins are sampled at their
 *       centres: rho_c = (c + 1/2) R/64, beta_r = -R/2 + (r + 1/2) R/64.
 *       Column c grows with radius, row r with beta.
 *   R3  A vertex lies "above" a row plane iff z >= beta (half-open).
 *   R4  Counts use open intervals; any pixel whose decision lies within
 *       EPS of its threshold is flagged as degenerate instead (C-D rules).
 *   R5  CRD sums r in [0, 64) and c in [1, 64) (64 x 63 terms); the printed
 *       ranges [0..N_bins] / [1..N_bins] are read half-open.
 *   R6  rank = #{h : CRD(n, h) < CRD(n, h_true)} (strict: ties -> best rank).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -pthread (no fast-math).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define NBINS 64
#define EPS 1e-9          /* decision band in scene units (R4)                  */
#define VBAND 1e-6        /* radial band around a vertex that sits on a row plane */
#define FLAT_DZ 1e-6      /* a crossing edge flatter than this is ill-conditioned */
#define SHORT_SLICE 1e-6  /* a slice shorter than this has an ill-conditioned |C| */

/* ------------------------------------------------------------------ pixel grid */

/* R2: bin-centre radius of column c and height of row r.  Both are exact in
 * FP64 for fp32 R: (c + 1/2) * R / 64 has at most 7 + 24 significant bits. */
static double bin_radius(double R, int c) { return ((double)c + 0.5) * (R / NBINS); }
static double bin_height(double R, int r) { return -0.5 * R + ((double)r + 0.5) * (R / NBINS); }

/* ----------------------------------------------------- projection, Eq. 1 - 5 */

typedef struct {
    double nax, nay;   /* first rotation (about z), Eq. 1 line 1 */
    double nbx, nbz;   /* second rotation (about y), Eq. 1 line 2 (R1) */
    double sv[3];      /* spin vertex */
    int zero_normal;   /* |S_n| == 0: identity frame, image flagged */
} frame_t;

/* Normalize[a, b], with (0, 0) giving the identity pair (1, 0) when `x_first`
 * (rotation about z: cos = 1) or (0, 1) otherwise (rotation about y: N_bz = 1). */
static void normalize2(double a, double b, double* oa, double* ob, int identity_first)
{
    double len = sqrt(a * a + b * b);
    if (len > 0.0) {
        *oa = a / len;
        *ob = b / len;
    } else if (identity_first) {
        *oa = 1.0; *ob = 0.0;
    } else {
        *oa = 0.0; *ob = 1.0;
    }
}

static void make_frame(const float* sv, const float* sn, frame_t* f)
{
    double nx = sn[0], ny = sn[1], nz = sn[2];
    f->sv[0] = sv[0]; f->sv[1] = sv[1]; f->sv[2] = sv[2];
    f->zero_normal = (nx == 0.0 && ny == 0.0 && nz == 0.0);
    /* Eq. 1, first line: [N_ax, N_ay] = Normalize[S_nx, S_ny] */
    normalize2(nx, ny, &f->nax, &f->nay, 1);
    /* R1: the x component of the normal after the first rotation */
    double rx = f->nax * nx + f->nay * ny;
    /* Eq. 1, second line as read in R1: [N_bx, N_bz] = Normalize[S''_nx, S_nz] */
    normalize2(rx, nz, &f->nbx, &f->nbz, 0);
}

/* Eq. 2 (translation), Eq. 3 (rotation about z), Eq. 4 (rotation about y). */
static void project(const frame_t* f, double px, double py, double pz,
                    double* tx, double* ty, double* tz)
{
    double p1x = px - f->sv[0];                 /* Eq. 2 */
    double p1y = py - f->sv[1];
    double p1z = pz - f->sv[2];
    double p2x = f->nax * p1x + f->nay * p1y;   /* Eq. 3 */
    double p2y = -f->nay * p1x + f->nax * p1y;
    *tx = f->nbz * p2x - f->nbx * p1z;          /* Eq. 4 */
    *ty = p2y;
    *tz = f->nbx * p2x + f->nbz * p1z;
}

/* Eq. 1 - 5 for a list of points (used by the projection tests).  `printed`
 * selects Eq. 1 exactly as printed (second line Normalize[S_nx, S_nz]). */
void oracle_project(const float* sv, const float* sn, const double* pts, int64_t n,
                    int printed, double* alpha, double* beta, double* txy)
{
    frame_t f;
    make_frame(sv, sn, &f);
    if (printed) normalize2((double)sn[0], (double)sn[2], &f.nbx, &f.nbz, 0);
    for (int64_t i = 0; i < n; ++i) {
        double tx, ty, tz;
        project(&f, pts[3 * i], pts[3 * i + 1], pts[3 * i + 2], &tx, &ty, &tz);
        alpha[i] = sqrt(tx * tx + ty * ty);   /* Eq. 5 */
        beta[i] = tz;
        if (txy) { txy[2 * i] = tx; txy[2 * i + 1] = ty; }
    }
}

/* ------------------------------------------------------ row-range generation */

typedef struct {
    const float* pos; uint32_t nv;
    const uint32_t* tri; uint32_t nt;
    const float* op_pos; const float* op_nrm; uint32_t n;
    double R;
    uint32_t* images;   /* [n][64][64] */
    uint8_t* flags;     /* [n][64][64] or NULL */
    uint64_t* work;     /* [n][3]: triangles visited, slices, pixel updates */
    int64_t first, last;
    int status;
} gen_job_t;

static void flag_band(uint8_t* fl, int r, double R, double lo, double hi)
{
    if (!fl) return;
    for (int c = 0; c < NBINS; ++c) {
        double rho = bin_radius(R, c);
        if (rho >= lo && rho <= hi) fl[r * NBINS + c] = 1;
    }
}

/* distance from the origin to the 2-D triangle (0 when it contains the origin) */
static double origin_triangle_dist2d(const double* x, const double* y)
{
    double s0 = x[0] * y[1] - y[0] * x[1];
    double s1 = x[1] * y[2] - y[1] * x[2];
    double s2 = x[2] * y[0] - y[2] * x[0];
    if ((s0 >= 0 && s1 >= 0 && s2 >= 0) || (s0 <= 0 && s1 <= 0 && s2 <= 0)) return 0.0;
    double best = INFINITY;
    for (int k = 0; k < 3; ++k) {
        int j = (k + 1) % 3;
        double dx = x[j] - x[k], dy = y[j] - y[k];
        double l2 = dx * dx + dy * dy;
        double t = l2 > 0 ? -(x[k] * dx + y[k] * dy) / l2 : 0.0;
        if (t < 0) t = 0;
        if (t > 1) t = 1;
        double qx = x[k] + t * dx, qy = y[k] + t * dy;
        double d = sqrt(qx * qx + qy * qy);
        if (d < best) best = d;
    }
    return best;
}

static void rici_one_image(const gen_job_t* J, int64_t img)
{
    const double R = J->R;
    uint32_t* out = J->images + (size_t)img * NBINS * NBINS;
    uint8_t* fl = J->flags ? J->flags + (size_t)img * NBINS * NBINS : NULL;
    uint64_t slices = 0, updates = 0;
    memset(out, 0, sizeof(uint32_t) * NBINS * NBINS);
    if (fl) memset(fl, 0, NBINS * NBINS);

    frame_t f;
    make_frame(J->op_pos + 3 * img, J->op_nrm + 3 * img, &f);
    if (f.zero_normal && fl) memset(fl, 1, NBINS * NBINS);

    const double beta_lo = bin_height(R, 0), beta_hi = bin_height(R, NBINS - 1);

    for (uint32_t t = 0; t < J->nt; ++t) {
        /* Step 1: project the triangle's vertices (Eq. 2 - 5). */
        double x[3], y[3], z[3], a[3];
        for (int k = 0; k < 3; ++k) {
            const float* p = J->pos + 3 * (size_t)J->tri[3 * (size_t)t + k];
            project(&f, p[0], p[1], p[2], &x[k], &y[k], &z[k]);
            a[k] = sqrt(x[k] * x[k] + y[k] * y[k]);
        }
        double zmin = fmin(z[0], fmin(z[1], z[2])), zmax = fmax(z[0], fmax(z[1], z[2]));
        if (zmax < beta_lo - VBAND || zmin > beta_hi + VBAND) continue;

        /* Step 2: for each row plane in the triangle's beta extent, the radius
         * ranges of single and double intersections. */
        for (int r = 0; r < NBINS; ++r) {
            const double beta = bin_height(R, r);
            uint8_t* flr = fl ? fl + r * NBINS : NULL;

            /* C-D (iii): a vertex (almost) on the row plane */
            int on_plane = 0;
            for (int k = 0; k < 3; ++k) {
                if (fabs(z[k] - beta) < EPS) {
                    ++on_plane;
                    flag_band(flr, r, R, a[k] - VBAND, a[k] + VBAND);
                }
            }
            /* C-D (iv): the whole triangle lies in the row plane (Sec. 3.1.2:
             * infinitely many intersections are not handled) */
            if (on_plane == 3) {
                double amax = fmax(a[0], fmax(a[1], a[2]));
                flag_band(flr, r, R, origin_triangle_dist2d(x, y) - VBAND, amax + VBAND);
            }

            int above[3], na = 0;
            for (int k = 0; k < 3; ++k) { above[k] = (z[k] >= beta); na += above[k]; }  /* R3 */
            if (na == 0 || na == 3) continue;

            /* the vertex alone on its side; the slice joins its two edges */
            int lone = 0;
            for (int k = 0; k < 3; ++k)
                if ((na == 1 && above[k]) || (na == 2 && !above[k])) lone = k;
            int ia = (lone + 1) % 3, ib = (lone + 2) % 3;

            /* Sec. 3.1.2 step 1: intersection points E0, E1 of the plane with
             * the two crossing edges */
            double t0 = (beta - z[lone]) / (z[ia] - z[lone]);
            double t1 = (beta - z[lone]) / (z[ib] - z[lone]);
            double e0x = x[lone] + t0 * (x[ia] - x[lone]);
            double e0y = y[lone] + t0 * (y[ia] - y[lone]);
            double e1x = x[lone] + t1 * (x[ib] - x[lone]);
            double e1y = y[lone] + t1 * (y[ib] - y[lone]);

            /* step 2: rotate about z so that E0 -> E1 points along +x; the
             * normalised E0E1 vector supplies cosine and sine directly */
            double dx = e1x - e0x, dy = e1y - e0y;
            double len = sqrt(dx * dx + dy * dy);
            double x0r = 0, x1r = 0, yr = 0;
            if (len > 0.0) {
                double cs = dx / len, sn = dy / len;
                x0r = e0x * cs + e0y * sn;
                x1r = e1x * cs + e1y * sn;
                yr = -e0x * sn + e0y * cs;
            }
            /* step 3: distances of E0 and E1 from the z axis */
            double d0 = sqrt(e0x * e0x + e0y * e0y);
            double d1 = sqrt(e1x * e1x + e1y * e1y);
            /* step 4: single intersections for radii in (min, max) */
            double lo = fmin(d0, d1), hi = fmax(d0, d1);
            /* step 5: a double intersection exists iff the rotated x
             * coordinates of E0 and E1 have different signs */
            int dbl = (len > 0.0) && ((x0r < 0.0 && x1r > 0.0) || (x0r > 0.0 && x1r < 0.0));
            /* step 6: double intersections for radii in (|y|, min(|E0|, |E1|)) */
            double cdist = fabs(yr);

            /* Step 3 of the triangle loop: increment the bins */
            ++slices;
            for (int c = 0; c < NBINS; ++c) {
                double rho = bin_radius(R, c);
                uint32_t add = 0;
                if (lo < rho && rho < hi) add += 1;
                if (dbl && cdist < rho && rho < lo) add += 2;
                if (add) { out[r * NBINS + c] += add; ++updates; }
                if (flr) {
                    if (fabs(rho - d0) < EPS || fabs(rho - d1) < EPS) flr[c] = 1;   /* C-D (i)  */
                    if (dbl && fabs(rho - cdist) < EPS) flr[c] = 1;                 /* C-D (ii) */
                }
            }
            /* C-D (v): a crossing edge almost parallel to the row plane puts
             * the intersection point out of reach of FP64 rounding bounds */
            if (fabs(z[ia] - z[lone]) < FLAT_DZ || fabs(z[ib] - z[lone]) < FLAT_DZ)
                flag_band(flr, r, R, (dbl ? cdist : lo) - VBAND, hi + VBAND);
            /* C-D (vi): for a very short slice the direction E0 -> E1, hence
             * |C| and the double/single decision, is ill-conditioned; every
             * radius it can affect lies within SHORT_SLICE of lo */
            if (len < SHORT_SLICE)
                flag_band(flr, r, R, lo - SHORT_SLICE - VBAND, hi + VBAND);
        }
    }
    if (J->work) {
        J->work[3 * img + 0] = J->nt;
        J->work[3 * img + 1] = slices;
        J->work[3 * img + 2] = updates;
    }
}

/* ------------------------------------------------ brute force (plain definition) */

/* Orthonormal basis (u, w) perpendicular to the unit vector n; the branchless
 * construction of Duff et al., "Building an Orthonormal Basis, Revisited"
 * (JCGT 2017). */
static void basis(const double* n, double* u, double* w)
{
    double s = n[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (s + n[2]);
    double b = n[0] * n[1] * a;
    u[0] = 1.0 + s * n[0] * n[0] * a; u[1] = s * b; u[2] = -s * n[0];
    w[0] = b; w[1] = s + n[1] * n[1] * a; w[2] = -n[1];
}

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(const double* a, const double* b, double* o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static void cross3(const double* a, const double* b, double* o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static double point_segment_dist(const double* x, const double* p, const double* q)
{
    double d[3], v[3];
    sub3(q, p, d);
    sub3(x, p, v);
    double l2 = dot3(d, d);
    double t = l2 > 0 ? dot3(v, d) / l2 : 0.0;
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    double c[3] = { p[0] + t * d[0] - x[0], p[1] + t * d[1] - x[1], p[2] + t * d[2] - x[2] };
    return sqrt(dot3(c, c));
}

/* barycentric coordinates of x (assumed in the plane of p0 p1 p2) */
static void barycentric(const double* x, const double* p0, const double* p1, const double* p2, double* l)
{
    double e1[3], e2[3], v[3];
    sub3(p1, p0, e1); sub3(p2, p0, e2); sub3(x, p0, v);
    double d11 = dot3(e1, e1), d12 = dot3(e1, e2), d22 = dot3(e2, e2);
    double v1 = dot3(v, e1), v2 = dot3(v, e2);
    double den = d11 * d22 - d12 * d12;
    l[1] = (d22 * v1 - d12 * v2) / den;
    l[2] = (d11 * v2 - d12 * v1) / den;
    l[0] = 1.0 - l[1] - l[2];
}

static double point_triangle_boundary_dist(const double* x, const double* p0, const double* p1, const double* p2)
{
    double d0 = point_segment_dist(x, p0, p1);
    double d1 = point_segment_dist(x, p1, p2);
    double d2 = point_segment_dist(x, p2, p0);
    return fmin(d0, fmin(d1, d2));
}

static void brute_one_image(const gen_job_t* J, int64_t img)
{
    const double R = J->R;
    uint32_t* out = J->images + (size_t)img * NBINS * NBINS;
    uint8_t* fl = J->flags ? J->flags + (size_t)img * NBINS * NBINS : NULL;
    memset(out, 0, sizeof(uint32_t) * NBINS * NBINS);
    if (fl) memset(fl, 0, NBINS * NBINS);

    const float* svf = J->op_pos + 3 * img;
    const float* snf = J->op_nrm + 3 * img;
    double sv[3] = { svf[0], svf[1], svf[2] };
    double n[3] = { snf[0], snf[1], snf[2] };
    double nl = sqrt(dot3(n, n));
    if (nl > 0) { n[0] /= nl; n[1] /= nl; n[2] /= nl; }
    else { n[0] = 0; n[1] = 0; n[2] = 1; if (fl) memset(fl, 1, NBINS * NBINS); }
    double u[3], w[3];
    basis(n, u, w);

    for (uint32_t t = 0; t < J->nt; ++t) {
        double p[3][3];
        for (int k = 0; k < 3; ++k) {
            const float* q = J->pos + 3 * (size_t)J->tri[3 * (size_t)t + k];
            p[k][0] = q[0]; p[k][1] = q[1]; p[k][2] = q[2];
        }
        double e1[3], e2[3], m[3];
        sub3(p[1], p[0], e1); sub3(p[2], p[0], e2);
        cross3(e1, e2, m);
        double mn = sqrt(dot3(m, m));
        if (mn == 0.0) continue;   /* zero-area triangle: no surface */
        double mu = dot3(m, u), mw = dot3(m, w);

        for (int r = 0; r < NBINS; ++r) {
            double beta = bin_height(R, r);
            double Q[3] = { sv[0] + beta * n[0], sv[1] + beta * n[1], sv[2] + beta * n[2] };
            double qp[3];
            sub3(Q, p[0], qp);
            /* f(theta) = m.(Gamma(theta) - p0) = K + A cos(theta) + B sin(theta) */
            double K = dot3(m, qp);
            for (int c = 0; c < NBINS; ++c) {
                double rho = bin_radius(R, c);
                double A = rho * mu, B = rho * mw;
                double M = sqrt(A * A + B * B);
                int idx = r * NBINS + c;
                if (fabs(K) + M < EPS * mn) {      /* circle within EPS of the triangle's plane */
                    if (fl) fl[idx] = 1;
                    continue;
                }
                double phi = atan2(B, A);
                /* tangency: |rho - dist(axis point, line)| < EPS, and the
                 * touching point near the triangle */
                if (M > 0 && fabs(M - fabs(K)) < EPS * M / rho) {
                    double th = K > 0 ? phi + M_PI : phi;
                    double X[3];
                    for (int k = 0; k < 3; ++k) X[k] = Q[k] + rho * (cos(th) * u[k] + sin(th) * w[k]);
                    double l[3];
                    barycentric(X, p[0], p[1], p[2], l);
                    int inside = l[0] > 0 && l[1] > 0 && l[2] > 0;
                    if (inside || point_triangle_boundary_dist(X, p[0], p[1], p[2]) < VBAND) {
                        if (fl) fl[idx] = 1;
                    }
                }
                if (!(M > fabs(K))) continue;        /* the circle misses the plane */
                double dphi = acos(-K / M);
                for (int s = 0; s < 2; ++s) {
                    double th = s ? phi - dphi : phi + dphi;
                    double X[3];
                    for (int k = 0; k < 3; ++k) X[k] = Q[k] + rho * (cos(th) * u[k] + sin(th) * w[k]);
                    double l[3];
                    barycentric(X, p[0], p[1], p[2], l);
                    if (l[0] > 0 && l[1] > 0 && l[2] > 0) out[idx] += 1;
                    if (fl && point_triangle_boundary_dist(X, p[0], p[1], p[2]) < EPS) fl[idx] = 1;
                }
            }
        }
    }
}

/* ------------------------------------------------------------- thread helpers */

typedef void (*img_fn)(const gen_job_t*, int64_t);
typedef struct { gen_job_t* job; img_fn fn; } gen_thread_t;

static void* gen_worker(void* arg)
{
    gen_thread_t* T = (gen_thread_t*)arg;
    for (int64_t i = T->job->first; i < T->job->last; ++i) T->fn(T->job, i);
    return NULL;
}

static int resolve_threads(int nthreads)
{
    if (nthreads > 0) return nthreads;
    long n = sysconf(_SC_NPROCESSORS_ONLN);
    return n > 0 ? (int)n : 1;
}

static int run_images(gen_job_t* base, img_fn fn, int nthreads)
{
    int nt = resolve_threads(nthreads);
    if ((int64_t)nt > (int64_t)base->n) nt = base->n > 0 ? (int)base->n : 1;
    pthread_t th[512];
    gen_job_t jobs[512];
    gen_thread_t args[512];
    if (nt > 512) nt = 512;
    int started = 0;
    for (int k = 0; k < nt; ++k) {
        jobs[k] = *base;
        jobs[k].first = (int64_t)base->n * k / nt;
        jobs[k].last = (int64_t)base->n * (k + 1) / nt;
        args[k].job = &jobs[k];
        args[k].fn = fn;
        if (pthread_create(&th[k], NULL, gen_worker, &args[k]) != 0) {
            gen_worker(&args[k]);
            th[k] = 0;
        } else {
            ++started;
        }
    }
    for (int k = 0; k < nt; ++k) if (th[k]) pthread_join(th[k], NULL);
    (void)started;
    return 0;
}

static int check_mesh(const uint32_t* tri, uint32_t nt, uint32_t nv)
{
    for (size_t i = 0; i < (size_t)nt * 3; ++i)
        if (tri[i] >= nv) return -1;
    return 0;
}

/* RICI images by the paper's row-range algorithm.  flags / work may be NULL.
 * Returns 0, or -1 when a triangle index is out of range. */
int oracle_rici_rowrange(const float* pos, uint32_t nv, const uint32_t* tri, uint32_t nt,
                         const float* op_pos, const float* op_nrm, uint32_t n, float R,
                         uint32_t* images, uint8_t* flags, uint64_t* work, int nthreads)
{
    if (check_mesh(tri, nt, nv)) return -1;
    gen_job_t J = { pos, nv, tri, nt, op_pos, op_nrm, n, (double)R, images, flags, work, 0, n, 0 };
    return run_images(&J, rici_one_image, nthreads);
}

/* RICI images by the plain definition (brute force per circle and triangle). */
int oracle_rici_brute(const float* pos, uint32_t nv, const uint32_t* tri, uint32_t nt,
                      const float* op_pos, const float* op_nrm, uint32_t n, float R,
                      uint32_t* images, uint8_t* flags, int nthreads)
{
    if (check_mesh(tri, nt, nv)) return -1;
    gen_job_t J = { pos, nv, tri, nt, op_pos, op_nrm, n, (double)R, images, flags, NULL, 0, n, 0 };
    return run_images(&J, brute_one_image, nthreads);
}

/* ------------------------------------------------------ distance and rank */

/* Eq. 6: D(rici, r, c) = rici(r, c) - rici(r, c - 1), in signed 64-bit. */
static int64_t delta(const uint32_t* img, int r, int c)
{
    return (int64_t)img[r * NBINS + c] - (int64_t)img[r * NBINS + c - 1];
}

/* Eq. 7: squared differences of column deltas where the needle's delta is
 * non-zero (R5 index ranges). */
int64_t oracle_crd(const uint32_t* needle, const uint32_t* haystack)
{
    int64_t score = 0;
    for (int r = 0; r < NBINS; ++r) {
        for (int c = 1; c < NBINS; ++c) {
            int64_t nd = delta(needle, r, c);
            int64_t hd = delta(haystack, r, c);
            if (nd != 0) score += (nd - hd) * (nd - hd);
        }
    }
    return score;
}

typedef struct {
    const uint32_t* needles; uint32_t nn;
    const uint32_t* hay; uint32_t nh;
    const uint32_t* true_idx;
    uint32_t* rank; int64_t* dstar; int64_t* matrix;
    int64_t first, last;
} search_job_t;

static void* rank_worker(void* arg)
{
    search_job_t* J = (search_job_t*)arg;
    for (int64_t i = J->first; i < J->last; ++i) {
        const uint32_t* nd = J->needles + (size_t)i * NBINS * NBINS;
        int64_t d = oracle_crd(nd, J->hay + (size_t)J->true_idx[i] * NBINS * NBINS);
        uint32_t k = 0;
        for (uint32_t h = 0; h < J->nh; ++h)
            if (oracle_crd(nd, J->hay + (size_t)h * NBINS * NBINS) < d) ++k;   /* R6 */
        J->rank[i] = k;
        if (J->dstar) J->dstar[i] = d;
    }
    return NULL;
}

static void* matrix_worker(void* arg)
{
    search_job_t* J = (search_job_t*)arg;
    for (int64_t i = J->first; i < J->last; ++i) {
        const uint32_t* nd = J->needles + (size_t)i * NBINS * NBINS;
        for (uint32_t h = 0; h < J->nh; ++h)
            J->matrix[(size_t)i * J->nh + h] = oracle_crd(nd, J->hay + (size_t)h * NBINS * NBINS);
    }
    return NULL;
}

static int run_search(search_job_t* base, void* (*fn)(void*), int nthreads)
{
    int nt = resolve_threads(nthreads);
    if (nt > 512) nt = 512;
    if ((int64_t)nt > (int64_t)base->nn) nt = base->nn > 0 ? (int)base->nn : 1;
    pthread_t th[512];
    search_job_t jobs[512];
    for (int k = 0; k < nt; ++k) {
        jobs[k] = *base;
        jobs[k].first = (int64_t)base->nn * k / nt;
        jobs[k].last = (int64_t)base->nn * (k + 1) / nt;
        if (pthread_create(&th[k], NULL, fn, &jobs[k]) != 0) { fn(&jobs[k]); th[k] = 0; }
    }
    for (int k = 0; k < nt; ++k) if (th[k]) pthread_join(th[k], NULL);
    return 0;
}

/* rank[i] = #{h : CRD(needle_i, h) < CRD(needle_i, haystack[true_idx[i]])};
 * dstar (may be NULL) receives the true-match distances.  -1 on a bad index. */
int oracle_rank(const uint32_t* needles, uint32_t nn, const uint32_t* hay, uint32_t nh,
                const uint32_t* true_idx, uint32_t* rank, int64_t* dstar, int nthreads)
{
    for (uint32_t i = 0; i < nn; ++i) if (true_idx[i] >= nh) return -1;
    search_job_t J = { needles, nn, hay, nh, true_idx, rank, dstar, NULL, 0, nn };
    return run_search(&J, rank_worker, nthreads);
}

/* full CRD matrix [nn][nh] */
int oracle_distance_matrix(const uint32_t* needles, uint32_t nn, const uint32_t* hay, uint32_t nh,
                           int64_t* out, int nthreads)
{
    search_job_t J = { needles, nn, hay, nh, NULL, NULL, NULL, out, 0, nn };
    return run_search(&J, matrix_worker, nthreads);
}

int oracle_threads(int nthreads) { return resolve_threads(nthreads); }
