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
 *              Inputs are fp32 (converted exactly) or FP64.
 *   brute    : the plain definition of a RICI bin (number of points where the
 *              bin's circle meets the scene's triangles), solved per circle and
 *              triangle with trigonometry and barycentric coordinates.
 *   crd      : the clutter-resistant distance, Sec. 3.2: the Eq. 6 delta
 *              planes of both images, then the Eq. 7 sum of squared
 *              differences over the needle's non-zero deltas, in int64.
 *   rank     : 0-based rank of the true match, ties taking the best rank
 *              (Sec. 4.1, clutterbox step 6c, and the tie rule of Sec. 4.2).
 *   spin     : Spin Images from point samples (Sec. 2.1, with the projection
 *              of Sec. 3.1.1), their Pearson correlation and the rank of the
 *              true match under it (readings S1 - S4 below).
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
 *   R4  Counts use open intervals.  A pixel is flagged as degenerate (and
 *       excluded from parity) when a decision that sets its count lies within
 *       EPS of its threshold, widened by a forward bound on the FP64 rounding
 *       error of the compared quantity (so that the count of every unflagged
 *       pixel is certain, whatever the FP64 evaluation order):
 *         (i)   the bin radius vs a slice end |E0|, |E1|;
 *         (ii)  the bin radius vs the foot point |C| of a double range, and
 *               the whole double range when "C inside E0E1" is uncertain;
 *         (iii) a vertex within that band of the row plane: the slice is also
 *               taken with the vertex on the other side, and the pixels where
 *               the two slices disagree, or near the second one's decisions,
 *               are flagged;
 *         (iv)  an edge or the whole triangle within the band of the row
 *               plane (Sec. 3.1.2 leaves infinite intersections out): every
 *               radius the edge or triangle covers.
 *       A zero normal flags the whole image.
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
#define EPS 1e-9          /* decision band in scene units (R4)                       */
#define U64 0x1p-53       /* unit roundoff of FP64                                     */
#define CULL_MARGIN 1e-6  /* rows further than this from a triangle are not examined  */
#define VBAND 1e-6        /* brute force: touching points this close to an edge count */

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

static void make_frame(const double* sv, const double* sn, frame_t* f)
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
    double svd[3] = { sv[0], sv[1], sv[2] }, snd[3] = { sn[0], sn[1], sn[2] };
    make_frame(svd, snd, &f);
    if (printed) normalize2(snd[0], snd[2], &f.nbx, &f.nbz, 0);
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
    const double* pos; uint32_t nv;
    const uint32_t* tri; uint32_t nt;
    const double* op_pos; const double* op_nrm; uint32_t n;
    double R;
    uint32_t* images;   /* [n][64][64] */
    uint8_t* flags;     /* [n][64][64] or NULL */
    uint64_t* work;     /* [n][5]: triangles visited, slices, pixel updates,
                         * triangles and slices that reach inside the support
                         * radius (the work left after exact culling) */
    int64_t first, last;
} gen_job_t;

/* One projected triangle: Eq. 2-4 coordinates of its vertices, their
 * distances from the axis (Eq. 5), and a bound `ep` on the absolute rounding
 * error of any projected coordinate.  The bound covers this file's FP64
 * evaluation and any other FP64 evaluation of Eq. 1-4 from the same fp32
 * inputs (a handful of roundings, each at most U64 times the magnitude of
 * P - S_v), with a factor of 4 to spare. */
typedef struct {
    double x[3], y[3], z[3], a[3];
    double ep;
} ptri_t;

/* Flag every column whose bin radius lies in [lo, hi] (row-relative: `fr` is
 * the row's own 64 flags). */
static void flag_band(uint8_t* fr, double R, double lo, double hi)
{
    if (!fr || !(lo <= hi)) return;
    for (int c = 0; c < NBINS; ++c) {
        double rho = bin_radius(R, c);
        if (rho >= lo && rho <= hi) fr[c] = 1;
    }
}

/* distance from the origin to the 2-D segment p q */
static double origin_segment_dist2d(double px, double py, double qx, double qy)
{
    double dx = qx - px, dy = qy - py;
    double l2 = dx * dx + dy * dy;
    double t = l2 > 0 ? -(px * dx + py * dy) / l2 : 0.0;
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    return hypot(px + t * dx, py + t * dy);
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
        double d = origin_segment_dist2d(x[k], y[k], x[j], y[j]);
        if (d < best) best = d;
    }
    return best;
}

/* The slice of a triangle by one row plane (Sec. 3.1.2 steps 1-6) under a
 * given classification of its vertices (bit k of `above` set: vertex k lies
 * above the plane), with error bounds for every quantity a decision compares.
 * The crossing parameters are clamped to [0, 1], so a classification that
 * disagrees with the computed heights (used for the alternatives of rule
 * (iii)) still yields points on the triangle's edges. */
typedef struct {
    double d0, d1;        /* |E0|, |E1| */
    double err0, err1;    /* bounds on their rounding errors */
    double lo, hi;        /* single-intersection radii (lo, hi) */
    int dbl;              /* double range (|C|, lo) present */
    int dbl_unsure;       /* that decision lies within its error bound */
    double cdist, errc;   /* |C| and its error bound */
} slice_t;

/* error bound of a crossing point on edge l -> o: the crossing parameter
 * (beta - z_l) / (z_o - z_l) moves by about ep / |z_o - z_l| per unit error of
 * a height, which the edge's length in the plane carries over to the point;
 * clamping keeps the point on the edge, so the error never exceeds that
 * length (plus the projection's own error) */
static double crossing_err(const ptri_t* T, int l, int o)
{
    double dz = fabs(T->z[o] - T->z[l]);
    double len = hypot(T->x[o] - T->x[l], T->y[o] - T->y[l]);
    double e = dz > 0.0 ? 4.0 * T->ep * (1.0 + len / dz) : INFINITY;
    return fmin(e, len + 4.0 * T->ep);
}

static double clamp01(double t) { return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t); }

static int slice_row(const ptri_t* T, double beta, int above, slice_t* s)
{
    int na = ((above >> 0) & 1) + ((above >> 1) & 1) + ((above >> 2) & 1);
    if (na == 0 || na == 3) return 0;
    /* the vertex alone on its side; the slice joins its two edges */
    int lone = 0;
    for (int k = 0; k < 3; ++k) {
        int up = (above >> k) & 1;
        if ((na == 1 && up) || (na == 2 && !up)) lone = k;
    }
    int ia = (lone + 1) % 3, ib = (lone + 2) % 3;
    const double* x = T->x; const double* y = T->y; const double* z = T->z;

    /* step 1: the points E0, E1 where the plane crosses the two edges */
    double t0 = clamp01((beta - z[lone]) / (z[ia] - z[lone]));
    double t1 = clamp01((beta - z[lone]) / (z[ib] - z[lone]));
    if (t0 != t0) t0 = 0.5;   /* 0/0: an edge lying in the plane (rule (iv) flags it) */
    if (t1 != t1) t1 = 0.5;
    double e0x = x[lone] + t0 * (x[ia] - x[lone]);
    double e0y = y[lone] + t0 * (y[ia] - y[lone]);
    double e1x = x[lone] + t1 * (x[ib] - x[lone]);
    double e1y = y[lone] + t1 * (y[ib] - y[lone]);
    double eE0 = crossing_err(T, lone, ia), eE1 = crossing_err(T, lone, ib);

    /* step 2: rotate about z so that E0 -> E1 points along +x; the normalised
     * E0E1 vector supplies cosine and sine directly */
    double dx = e1x - e0x, dy = e1y - e0y;
    double len = sqrt(dx * dx + dy * dy);
    double x0r = 0, x1r = 0, yr = 0;
    if (len > 0.0) {
        double cs = dx / len, sn = dy / len;
        x0r = e0x * cs + e0y * sn;
        x1r = e1x * cs + e1y * sn;
        yr = -e0x * sn + e0y * cs;
    }
    /* step 3: distances of E0 and E1 from the axis */
    s->d0 = sqrt(e0x * e0x + e0y * e0y);
    s->d1 = sqrt(e1x * e1x + e1y * e1y);
    s->err0 = eE0 + 4.0 * U64 * s->d0;
    s->err1 = eE1 + 4.0 * U64 * s->d1;
    /* step 4: single intersections for radii in (min, max) */
    s->lo = fmin(s->d0, s->d1);
    s->hi = fmax(s->d0, s->d1);
    /* step 5: a double intersection iff the rotated x coordinates of E0 and
     * E1 have different signs (the foot C of the axis lies inside E0E1) */
    s->dbl = (len > 0.0) && ((x0r < 0.0 && x1r > 0.0) || (x0r > 0.0 && x1r < 0.0));
    /* step 6: double intersections for radii in (|C|, min(|E0|, |E1|)) */
    s->cdist = len > 0.0 ? fabs(yr) : s->lo;

    /* Error bounds of the step 5-6 quantities.  |C| = |E0 x E1| / |E1 - E0|:
     * the cross product carries the points' errors times the other point's
     * length, and the division amplifies both by 1 / |E1 - E0|.  When C lies
     * inside the segment, |C| is at least lo - |E1 - E0|, so no bound needs
     * to exceed the segment's length plus the points' errors. */
    double eE = eE0 + eE1;
    double dsum = s->d0 + s->d1;
    double bound_c = len > 0.0 ? (eE * dsum + 4.0 * U64 * s->d0 * s->d1) / len
                                 + s->cdist * (eE + 4.0 * U64 * len) / len + 4.0 * U64 * dsum
                               : INFINITY;
    s->errc = fmin(bound_c, len + 2.0 * eE);
    /* the rotated x coordinates are E_k . (E1 - E0) / |E1 - E0|; their error
     * is the points' errors times the lengths involved */
    double err_x = eE * (dsum + len) / (len > 0.0 ? len : 1.0) + eE + 8.0 * U64 * dsum;
    s->dbl_unsure = (len == 0.0) || fabs(x0r) <= err_x || fabs(x1r) <= err_x;
    return 1;
}

/* Add one slice's counts to a row (Sec. 3.1 step 3) and return the number of
 * pixels it changes. */
static uint64_t slice_counts(const slice_t* s, double R, uint32_t* add)
{
    uint64_t updates = 0;
    for (int c = 0; c < NBINS; ++c) {
        double rho = bin_radius(R, c);
        uint32_t v = 0;
        if (s->lo < rho && rho < s->hi) v += 1;
        if (s->dbl && s->cdist < rho && rho < s->lo) v += 2;
        add[c] += v;
        updates += v != 0;
    }
    return updates;
}

/* Rules (i) and (ii): pixels whose radius lies within EPS (plus the rounding
 * bound of the computed quantity) of a slice end or of the foot point. */
static void slice_flags(const slice_t* s, double R, uint8_t* fr)
{
    if (!fr) return;
    flag_band(fr, R, s->d0 - EPS - s->err0, s->d0 + EPS + s->err0);                  /* (i)  */
    flag_band(fr, R, s->d1 - EPS - s->err1, s->d1 + EPS + s->err1);
    if (s->dbl_unsure) {                                                              /* (ii) */
        /* were C inside the exact slice, its double range would lie between
         * the exact slice's distance from the axis and its nearer end; the
         * exact slice lies within the end points' errors of the computed one,
         * whose distance from the axis is |C| (C inside) or lo (C outside) */
        double elo = s->d0 <= s->d1 ? s->err0 : s->err1;
        double emax = fmax(s->err0, s->err1);
        double from = s->dbl ? s->cdist - fmax(s->errc, emax) : s->lo - emax;
        flag_band(fr, R, from - EPS, s->lo + EPS + elo);
    } else if (s->dbl) {
        flag_band(fr, R, s->cdist - EPS - s->errc, s->cdist + EPS + s->errc);
    }
}

static void rici_one_image(const gen_job_t* J, int64_t img)
{
    const double R = J->R;
    uint32_t* out = J->images + (size_t)img * NBINS * NBINS;
    uint8_t* fl = J->flags ? J->flags + (size_t)img * NBINS * NBINS : NULL;
    uint64_t slices = 0, updates = 0, tris_in = 0, slices_in = 0;
    memset(out, 0, sizeof(uint32_t) * NBINS * NBINS);
    if (fl) memset(fl, 0, NBINS * NBINS);

    frame_t f;
    make_frame(J->op_pos + 3 * img, J->op_nrm + 3 * img, &f);
    if (f.zero_normal && fl) memset(fl, 1, NBINS * NBINS);

    const double beta_lo = bin_height(R, 0), beta_hi = bin_height(R, NBINS - 1);

    for (uint32_t t = 0; t < J->nt; ++t) {
        /* Step 1: project the triangle's vertices (Eq. 2 - 5). */
        ptri_t T;
        double mag = 0.5 * R;
        for (int k = 0; k < 3; ++k) {
            const double* p = J->pos + 3 * (size_t)J->tri[3 * (size_t)t + k];
            project(&f, p[0], p[1], p[2], &T.x[k], &T.y[k], &T.z[k]);
            T.a[k] = sqrt(T.x[k] * T.x[k] + T.y[k] * T.y[k]);
            mag = fmax(mag, fabs(p[0] - f.sv[0]) + fabs(p[1] - f.sv[1]) + fabs(p[2] - f.sv[2]));
        }
        T.ep = 64.0 * U64 * mag;
        const double band = EPS + T.ep;   /* a height this close to a row plane is ambiguous */
        double zmin = fmin(T.z[0], fmin(T.z[1], T.z[2])), zmax = fmax(T.z[0], fmax(T.z[1], T.z[2]));
        if (zmax < beta_lo - CULL_MARGIN || zmin > beta_hi + CULL_MARGIN) continue;

        /* Step 2: for each row plane in the triangle's beta extent, the radius
         * ranges of single and double intersections. */
        int reaches = 0;
        for (int r = 0; r < NBINS; ++r) {
            const double beta = bin_height(R, r);
            uint8_t* fr = fl ? fl + (size_t)r * NBINS : NULL;
            int above = 0, amb = 0, namb = 0;
            for (int k = 0; k < 3; ++k) {
                if (T.z[k] >= beta) above |= 1 << k;                      /* R3 */
                if (fabs(T.z[k] - beta) <= band) { amb |= 1 << k; ++namb; }
            }

            slice_t s;
            if (slice_row(&T, beta, above, &s)) {
                /* Step 3 of the triangle loop: increment the bins */
                ++slices;
                /* the slice comes closer to the axis than R: it meets the
                 * support cylinder */
                if ((s.dbl ? s.cdist : s.lo) < R) {
                    ++slices_in;
                    reaches = 1;
                }
                updates += slice_counts(&s, R, out + (size_t)r * NBINS);
                slice_flags(&s, R, fr);
            }
            if (!fr || namb == 0) continue;

            if (namb == 3) {
                /* (iv) the whole triangle lies in the row plane (Sec. 3.1.2:
                 * infinitely many intersections are not handled): every radius
                 * the triangle covers is flagged */
                double amax = fmax(T.a[0], fmax(T.a[1], T.a[2]));
                flag_band(fr, R, origin_triangle_dist2d(T.x, T.y) - band, amax + band);
            } else if (namb == 2) {
                /* (iv) an edge lies in the row plane: the crossing can be
                 * anywhere on it, so every radius the edge covers is flagged,
                 * widened by the error of the crossings near its ends on the
                 * third vertex's edges */
                int m = (amb & 1) == 0 ? 0 : ((amb & 2) == 0 ? 1 : 2);
                int k = (m + 1) % 3, j = (m + 2) % 3;
                double w = band + fmax(crossing_err(&T, m, k), crossing_err(&T, m, j));
                flag_band(fr, R, origin_segment_dist2d(T.x[k], T.y[k], T.x[j], T.y[j]) - w,
                          fmax(T.a[k], T.a[j]) + w);
            } else {
                /* (iii) one vertex within `band` of the row plane: its side is
                 * ambiguous, so the slice is also taken with that vertex on the
                 * other side, and every pixel where the two disagree, or near a
                 * decision of the other slice, is flagged */
                uint32_t base[NBINS] = { 0 }, alt[NBINS] = { 0 };
                slice_t s2;
                if (slice_row(&T, beta, above, &s)) slice_counts(&s, R, base);
                if (slice_row(&T, beta, above ^ amb, &s2)) {
                    slice_counts(&s2, R, alt);
                    slice_flags(&s2, R, fr);
                }
                for (int c = 0; c < NBINS; ++c)
                    if (base[c] != alt[c]) fr[c] = 1;
            }
        }
        tris_in += reaches;
    }
    if (J->work) {
        J->work[5 * img + 0] = J->nt;
        J->work[5 * img + 1] = slices;
        J->work[5 * img + 2] = updates;
        J->work[5 * img + 3] = tris_in;
        J->work[5 * img + 4] = slices_in;
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

    const double* svf = J->op_pos + 3 * img;
    const double* snf = J->op_nrm + 3 * img;
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
            const double* q = J->pos + 3 * (size_t)J->tri[3 * (size_t)t + k];
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

static double* widen(const float* a, size_t n)
{
    double* d = (double*)malloc((n ? n : 1) * sizeof(double));
    if (d) for (size_t i = 0; i < n; ++i) d[i] = a[i];
    return d;
}

static int run_widened(const float* pos, uint32_t nv, const uint32_t* tri, uint32_t nt,
                       const float* op_pos, const float* op_nrm, uint32_t n, float R,
                       uint32_t* images, uint8_t* flags, uint64_t* work, img_fn fn, int nthreads)
{
    if (check_mesh(tri, nt, nv)) return -1;
    double* p = widen(pos, (size_t)nv * 3);
    double* o = widen(op_pos, (size_t)n * 3);
    double* m = widen(op_nrm, (size_t)n * 3);
    int rc = -2;
    if (p && o && m) {
        gen_job_t J = { p, nv, tri, nt, o, m, n, (double)R, images, flags, work, 0, n };
        rc = run_images(&J, fn, nthreads);
    }
    free(p); free(o); free(m);
    return rc;
}

/* RICI images by the paper's row-range algorithm, from fp32 inputs (converted
 * exactly to FP64).  flags / work may be NULL.  Returns 0, -1 when a triangle
 * index is out of range, -2 when host memory runs out. */
int oracle_rici_rowrange(const float* pos, uint32_t nv, const uint32_t* tri, uint32_t nt,
                         const float* op_pos, const float* op_nrm, uint32_t n, float R,
                         uint32_t* images, uint8_t* flags, uint64_t* work, int nthreads)
{
    return run_widened(pos, nv, tri, nt, op_pos, op_nrm, n, R, images, flags, work, rici_one_image, nthreads);
}

/* The same from FP64 inputs (for pins that need positions fp32 cannot hold). */
int oracle_rici_rowrange_f64(const double* pos, uint32_t nv, const uint32_t* tri, uint32_t nt,
                             const double* op_pos, const double* op_nrm, uint32_t n, double R,
                             uint32_t* images, uint8_t* flags, uint64_t* work, int nthreads)
{
    if (check_mesh(tri, nt, nv)) return -1;
    gen_job_t J = { pos, nv, tri, nt, op_pos, op_nrm, n, R, images, flags, work, 0, n };
    return run_images(&J, rici_one_image, nthreads);
}

/* RICI images by the plain definition (brute force per circle and triangle). */
int oracle_rici_brute(const float* pos, uint32_t nv, const uint32_t* tri, uint32_t nt,
                      const float* op_pos, const float* op_nrm, uint32_t n, float R,
                      uint32_t* images, uint8_t* flags, int nthreads)
{
    return run_widened(pos, nv, tri, nt, op_pos, op_nrm, n, R, images, flags, NULL, brute_one_image, nthreads);
}

int oracle_rici_brute_f64(const double* pos, uint32_t nv, const uint32_t* tri, uint32_t nt,
                          const double* op_pos, const double* op_nrm, uint32_t n, double R,
                          uint32_t* images, uint8_t* flags, int nthreads)
{
    if (check_mesh(tri, nt, nv)) return -1;
    gen_job_t J = { pos, nv, tri, nt, op_pos, op_nrm, n, R, images, flags, NULL, 0, n };
    return run_images(&J, brute_one_image, nthreads);
}

/* ------------------------------------------------------ distance and rank */

#define NDELTA (NBINS * (NBINS - 1))   /* R5: rows 0..63, columns 1..63 */

/* Eq. 6 for every pixel the distance uses: D(r, c) = I(r, c) - I(r, c - 1),
 * signed, stored at r * 63 + (c - 1). */
static void delta_plane(const uint32_t* img, int64_t* D)
{
    for (int r = 0; r < NBINS; ++r)
        for (int c = 1; c < NBINS; ++c)
            D[r * (NBINS - 1) + c - 1] = (int64_t)img[r * NBINS + c] - (int64_t)img[r * NBINS + c - 1];
}

/* Eq. 7 over two delta planes: the squared difference of the deltas, summed
 * over the pixels where the needle's delta is non-zero. */
static int64_t masked_sq_sum(const int64_t* Dn, const int64_t* Dh)
{
    int64_t sum = 0;
    for (int i = 0; i < NDELTA; ++i) {
        int64_t diff = Dn[i] - Dh[i];
        int64_t mask = Dn[i] != 0;
        sum += mask * diff * diff;
    }
    return sum;
}

/* CRD(needle, haystack) of Eq. 7 (Sec. 3.2). */
int64_t oracle_crd(const uint32_t* needle, const uint32_t* haystack)
{
    int64_t Dn[NDELTA], Dh[NDELTA];
    delta_plane(needle, Dn);
    delta_plane(haystack, Dh);
    return masked_sq_sum(Dn, Dh);
}

/* Needles are handled in blocks: their delta planes are built once, then the
 * threads split the haystack, each counting (or writing distances) for every
 * needle of the block over its own range of haystack images. */
#define NEEDLE_BLOCK 64

typedef struct {
    const int64_t* planes; uint32_t nb;     /* this block's needle planes */
    const uint32_t* hay; uint32_t nh;
    const int64_t* dstar;                   /* rank: thresholds of the block, else NULL */
    uint32_t* counts;                       /* rank: this thread's [nb] counts */
    int64_t* matrix; size_t row_stride;     /* matrix: rows of the block */
    int64_t first, last;                    /* haystack range */
} search_job_t;

static void* search_worker(void* arg)
{
    search_job_t* J = (search_job_t*)arg;
    int64_t Dh[NDELTA];
    for (int64_t h = J->first; h < J->last; ++h) {
        delta_plane(J->hay + (size_t)h * NBINS * NBINS, Dh);
        for (uint32_t i = 0; i < J->nb; ++i) {
            int64_t d = masked_sq_sum(J->planes + (size_t)i * NDELTA, Dh);
            if (J->matrix) J->matrix[(size_t)i * J->row_stride + (size_t)h] = d;
            else if (d < J->dstar[i]) ++J->counts[i];                         /* R6 */
        }
    }
    return NULL;
}

/* rank (counts != NULL) or matrix (matrix != NULL) of one needle block */
static int search_block(const int64_t* planes, uint32_t nb, const uint32_t* hay, uint32_t nh,
                        const int64_t* dstar, uint32_t* rank, int64_t* matrix, size_t row_stride, int nthreads)
{
    int nt = resolve_threads(nthreads);
    if (nt > 512) nt = 512;
    if ((int64_t)nt > (int64_t)nh) nt = nh > 0 ? (int)nh : 1;
    pthread_t th[512];
    search_job_t jobs[512];
    uint32_t* counts = rank ? (uint32_t*)calloc((size_t)nt * nb, sizeof(uint32_t)) : NULL;
    if (rank && !counts) return -2;
    for (int k = 0; k < nt; ++k) {
        search_job_t j = { planes, nb, hay, nh, dstar, counts ? counts + (size_t)k * nb : NULL, matrix, row_stride,
                           (int64_t)nh * k / nt, (int64_t)nh * (k + 1) / nt };
        jobs[k] = j;
        if (pthread_create(&th[k], NULL, search_worker, &jobs[k]) != 0) { search_worker(&jobs[k]); th[k] = 0; }
    }
    for (int k = 0; k < nt; ++k) if (th[k]) pthread_join(th[k], NULL);
    if (rank) {
        for (uint32_t i = 0; i < nb; ++i) {
            uint32_t s = 0;
            for (int k = 0; k < nt; ++k) s += counts[(size_t)k * nb + i];
            rank[i] = s;
        }
        free(counts);
    }
    return 0;
}

/* rank[i] = #{h : CRD(needle_i, h) < CRD(needle_i, haystack[true_idx[i]])};
 * dstar (may be NULL) receives the true-match distances.  -1 on a bad index,
 * -2 when host memory runs out. */
int oracle_rank(const uint32_t* needles, uint32_t nn, const uint32_t* hay, uint32_t nh,
                const uint32_t* true_idx, uint32_t* rank, int64_t* dstar, int nthreads)
{
    for (uint32_t i = 0; i < nn; ++i) if (true_idx[i] >= nh) return -1;
    int64_t* planes = (int64_t*)malloc((size_t)NEEDLE_BLOCK * NDELTA * sizeof(int64_t));
    int64_t thr[NEEDLE_BLOCK];
    int64_t Dh[NDELTA];
    if (!planes) return -2;
    int rc = 0;
    for (uint32_t b = 0; b < nn && rc == 0; b += NEEDLE_BLOCK) {
        uint32_t nb = nn - b < NEEDLE_BLOCK ? nn - b : NEEDLE_BLOCK;
        for (uint32_t i = 0; i < nb; ++i) {
            int64_t* Dn = planes + (size_t)i * NDELTA;
            delta_plane(needles + (size_t)(b + i) * NBINS * NBINS, Dn);
            delta_plane(hay + (size_t)true_idx[b + i] * NBINS * NBINS, Dh);
            thr[i] = masked_sq_sum(Dn, Dh);
            if (dstar) dstar[b + i] = thr[i];
        }
        rc = search_block(planes, nb, hay, nh, thr, rank + b, NULL, 0, nthreads);
    }
    free(planes);
    return rc;
}

/* full CRD matrix [nn][nh] */
int oracle_distance_matrix(const uint32_t* needles, uint32_t nn, const uint32_t* hay, uint32_t nh,
                           int64_t* out, int nthreads)
{
    int64_t* planes = (int64_t*)malloc((size_t)NEEDLE_BLOCK * NDELTA * sizeof(int64_t));
    if (!planes) return -2;
    int rc = 0;
    for (uint32_t b = 0; b < nn && rc == 0; b += NEEDLE_BLOCK) {
        uint32_t nb = nn - b < NEEDLE_BLOCK ? nn - b : NEEDLE_BLOCK;
        for (uint32_t i = 0; i < nb; ++i)
            delta_plane(needles + (size_t)(b + i) * NBINS * NBINS, planes + (size_t)i * NDELTA);
        rc = search_block(planes, nb, hay, nh, NULL, NULL, out + (size_t)b * nh, nh, nthreads);
    }
    free(planes);
    return rc;
}

int oracle_threads(int nthreads) { return resolve_threads(nthreads); }

/* ================================================================ spin images
 *
 * Spin Image (Sec. 2.1), built from point samples of the scene with the
 * projection of Sec. 3.1.1 (which the paper states applies to SI construction
 * as well), and compared by the Pearson correlation coefficient.
 *
 * Readings (also in the design notes):
 *   S1  Support volume: a sample counts when 0 <= alpha < R and
 *       -R/2 <= beta < R/2 (the square plane of Sec. 2.1, width and height R,
 *       half-open like the bins).  No support-angle filter (Sec. 4.2: the
 *       paper's SI results apply none).
 *   S2  Bilinear interpolation between bin centres: with u = alpha / d - 1/2
 *       and v = (beta + R/2) / d - 1/2 (d = R/64), a sample adds
 *       (1 - fu)(1 - fv), fu (1 - fv), (1 - fu) fv, fu fv to the bins
 *       (floor v, floor u), (floor v, floor u + 1), (floor v + 1, floor u),
 *       (floor v + 1, floor u + 1), fu and fv being the fractional parts;
 *       bins outside the 64 x 64 grid receive nothing.  Row = beta, column =
 *       alpha, as for the RICI.
 *   S3  The Pearson coefficient of two images over their 4096 pixels; it is
 *       undefined for a constant image, which is given correlation 0.
 *   S4  Rank of the true match under correlation (higher is closer):
 *       #{h : rho(n, h) > rho(n, h_true)}, ties taking the best rank.
 *
 * Flags: a sample within EPS (plus the projection's rounding bound) of the
 * support boundary (alpha = R, beta = +-R/2) might be counted or not by an
 * implementation with other rounding; the pixels it would reach are flagged.
 * counts[] receives how many non-zero weights each pixel summed (it sets the
 * accumulation error bound of an fp32 implementation).
 */

typedef void (*item_fn)(const void* ctx, int64_t i);
typedef struct { const void* ctx; item_fn fn; int64_t first, last; } par_range_t;

static void* par_worker(void* arg)
{
    par_range_t* P = (par_range_t*)arg;
    for (int64_t i = P->first; i < P->last; ++i) P->fn(P->ctx, i);
    return NULL;
}

/* fn(ctx, i) for i in [0, n) over `nthreads` threads (0: all cores) */
static void parallel_for(const void* ctx, item_fn fn, int64_t n, int nthreads)
{
    int nt = resolve_threads(nthreads);
    if (nt > 512) nt = 512;
    if ((int64_t)nt > n) nt = n > 0 ? (int)n : 1;
    pthread_t th[512];
    par_range_t rg[512];
    for (int k = 0; k < nt; ++k) {
        rg[k].ctx = ctx;
        rg[k].fn = fn;
        rg[k].first = n * k / nt;
        rg[k].last = n * (k + 1) / nt;
        if (pthread_create(&th[k], NULL, par_worker, &rg[k]) != 0) {
            par_worker(&rg[k]);
            th[k] = 0;
        }
    }
    for (int k = 0; k < nt; ++k) if (th[k]) pthread_join(th[k], NULL);
}

typedef struct {
    const double* samples; int64_t ns;
    const double* op_pos; const double* op_nrm;
    double R;
    double* images; uint32_t* counts; uint8_t* flags;
} si_job_t;

static void si_one_image(const void* ctx, int64_t img)
{
    const si_job_t* J = (const si_job_t*)ctx;
    const double R = J->R, d = R / NBINS;
    double* out = J->images + (size_t)img * NBINS * NBINS;
    uint32_t* cnt = J->counts ? J->counts + (size_t)img * NBINS * NBINS : NULL;
    uint8_t* fl = J->flags ? J->flags + (size_t)img * NBINS * NBINS : NULL;
    memset(out, 0, sizeof(double) * NBINS * NBINS);
    if (cnt) memset(cnt, 0, sizeof(uint32_t) * NBINS * NBINS);
    if (fl) memset(fl, 0, NBINS * NBINS);
    frame_t f;
    make_frame(J->op_pos + 3 * img, J->op_nrm + 3 * img, &f);
    if (f.zero_normal && fl) memset(fl, 1, NBINS * NBINS);
    for (int64_t s = 0; s < J->ns; ++s) {
        const double* p = J->samples + 3 * s;
        double x, y, z;
        project(&f, p[0], p[1], p[2], &x, &y, &z);                 /* Eq. 2 - 4 */
        const double alpha = sqrt(x * x + y * y), beta = z;        /* Eq. 5 */
        const double mag = fabs(p[0] - f.sv[0]) + fabs(p[1] - f.sv[1]) + fabs(p[2] - f.sv[2]);
        const double band = EPS + 64.0 * U64 * (mag + R);
        const int inside = alpha < R && beta >= -0.5 * R && beta < 0.5 * R;          /* S1 */
        const int near = fabs(alpha - R) <= band || fabs(beta + 0.5 * R) <= band || fabs(beta - 0.5 * R) <= band;
        if (!inside && !near) continue;
        const double u = alpha / d - 0.5, v = (beta + 0.5 * R) / d - 0.5;             /* S2 */
        const double cu = floor(u), rv = floor(v);
        const double fu = u - cu, fv = v - rv;
        const int c0 = (int)cu, r0 = (int)rv;
        const double w[4] = { (1.0 - fu) * (1.0 - fv), fu * (1.0 - fv), (1.0 - fu) * fv, fu * fv };
        const int rr[4] = { r0, r0, r0 + 1, r0 + 1 }, cc[4] = { c0, c0 + 1, c0, c0 + 1 };
        for (int k = 0; k < 4; ++k) {
            if (rr[k] < 0 || rr[k] >= NBINS || cc[k] < 0 || cc[k] >= NBINS) continue;
            const size_t px = (size_t)rr[k] * NBINS + (size_t)cc[k];
            if (inside) {
                out[px] += w[k];
                if (cnt && w[k] != 0.0) ++cnt[px];
            }
            if (near && fl) fl[px] = 1;
        }
    }
}

/* Spin Images of n oriented points over ns fp32 point samples [ns][3];
 * images [n][64][64] FP64; counts / flags may be NULL. */
int oracle_spin_images(const float* samples, int64_t ns, const float* op_pos, const float* op_nrm, uint32_t n,
                       float R, double* images, uint32_t* counts, uint8_t* flags, int nthreads)
{
    double* p = widen(samples, (size_t)ns * 3);
    double* o = widen(op_pos, (size_t)n * 3);
    double* m = widen(op_nrm, (size_t)n * 3);
    int rc = -2;
    if (p && o && m) {
        si_job_t J = { p, ns, o, m, (double)R, images, counts, flags };
        parallel_for(&J, si_one_image, n, nthreads);
        rc = 0;
    }
    free(p); free(o); free(m);
    return rc;
}

/* S3: Pearson correlation of two fp32 images, FP64, two passes (means, then
 * the centred sums). */
double oracle_pearson(const float* a, const float* b)
{
    const int N = NBINS * NBINS;
    double ma = 0.0, mb = 0.0;
    for (int i = 0; i < N; ++i) { ma += a[i]; mb += b[i]; }
    ma /= N;
    mb /= N;
    double sab = 0.0, saa = 0.0, sbb = 0.0;
    for (int i = 0; i < N; ++i) {
        const double x = a[i] - ma, y = b[i] - mb;
        sab += x * y;
        saa += x * x;
        sbb += y * y;
    }
    if (saa == 0.0 || sbb == 0.0) return 0.0;
    return sab / sqrt(saa * sbb);
}

typedef struct {
    const float* needles; const float* hay; uint32_t nh;
    const uint32_t* true_idx; double band;
    uint32_t* rank; uint32_t* lo; uint32_t* hi; double* rho_true;
    double* matrix;
} pearson_job_t;

static void pearson_rank_one(const void* ctx, int64_t i)
{
    const pearson_job_t* J = (const pearson_job_t*)ctx;
    const float* a = J->needles + (size_t)i * NBINS * NBINS;
    const uint32_t t = J->true_idx[i];
    const double rt = oracle_pearson(a, J->hay + (size_t)t * NBINS * NBINS);
    uint32_t r = 0, lo = 0, hi = 0;
    for (uint32_t h = 0; h < J->nh; ++h) {
        const double rho = oracle_pearson(a, J->hay + (size_t)h * NBINS * NBINS);
        r += rho > rt;                                                  /* S4 */
        if (h != t) {
            lo += rho > rt + J->band;
            hi += rho > rt - J->band;
        }
    }
    J->rank[i] = r;
    if (J->lo) J->lo[i] = lo;
    if (J->hi) J->hi[i] = hi;
    if (J->rho_true) J->rho_true[i] = rt;
}

/* rank[i] = #{h : rho(n_i, h) > rho(n_i, h_true)}; lo / hi (may be NULL): the
 * same count over h != h_true with the threshold raised / lowered by `band`
 * (the range of ranks an implementation whose correlations are within band/2
 * of these may return).  -1 on a bad index. */
int oracle_pearson_rank(const float* needles, uint32_t nn, const float* hay, uint32_t nh, const uint32_t* true_idx,
                        double band, uint32_t* rank, uint32_t* lo, uint32_t* hi, double* rho_true, int nthreads)
{
    for (uint32_t i = 0; i < nn; ++i) if (true_idx[i] >= nh) return -1;
    pearson_job_t J = { needles, hay, nh, true_idx, band, rank, lo, hi, rho_true, NULL };
    parallel_for(&J, pearson_rank_one, nn, nthreads);
    return 0;
}

static void pearson_row(const void* ctx, int64_t i)
{
    const pearson_job_t* J = (const pearson_job_t*)ctx;
    for (uint32_t h = 0; h < J->nh; ++h)
        J->matrix[(size_t)i * J->nh + h] = oracle_pearson(J->needles + (size_t)i * NBINS * NBINS,
                                                          J->hay + (size_t)h * NBINS * NBINS);
}

/* out[i][j] = rho(needle_i, haystack_j), FP64 */
int oracle_pearson_matrix(const float* needles, uint32_t nn, const float* hay, uint32_t nh, double* out,
                          int nthreads)
{
    pearson_job_t J = { needles, hay, nh, NULL, 0.0, NULL, NULL, NULL, NULL, out };
    parallel_for(&J, pearson_row, nn, nthreads);
    return 0;
}

/* =================================================================== clutter
 *
 * Clutter around an oriented point (Eq. 8): (A_all - A_object) / A_all, the
 * areas of the whole scene's surface and of the object's surface inside the
 * support volume.  Reading C1: the support volume is the descriptor's, the
 * cylinder alpha <= R, |beta| <= R/2 about the Central Axis (Sec. 2.1); a
 * point whose volume holds no surface has clutter 0.
 *
 * Area of a triangle inside the volume, in the frame of Eq. 1-4 (axis = z,
 * Spin Vertex at the origin).  The triangle's plane gets orthonormal
 * coordinates (s, t): e1 horizontal, e2 = m x e1 (m its unit normal).  Since
 * e1 and the horizontal part of e2 are orthogonal, a point's squared distance
 * from the axis is s^2 + (a2 + k t)^2 (k = e2 . w2, a2 the plane's own offset
 * along w2 = z x e1) and its height is h0 m_z + t e2_z.  At each t the volume
 * therefore cuts the line of constant t in |s| <= w(t) = sqrt(R^2 - (a2 +
 * k t)^2), inside the slab's t-range; the triangle cuts it in [lo(t), hi(t)],
 * linear between its vertices.  The area is the integral over t of the
 * overlap, split where the choice of ends can change: the vertices' t, the
 * slab's ends, tangency (a2 + k t = +-R) and edge-boundary crossings (roots of
 * s(t)^2 + (a2 + k t)^2 = R^2 along each edge).  On each piece the integrand
 * is a difference of linear functions and +-w, integrated exactly; the
 * integral of w is written so that it does not cancel when k is small.
 */

static double chord_w(double R, double d)
{
    double q = R * R - d * d;
    return q > 0.0 ? sqrt(q) : 0.0;
}

/* integral over [t1, t2] of sqrt(R^2 - (a2 + k t)^2), with |a2 + k t| <= R there.
 * With x = (a2 + k t) / R and c = sqrt(1 - x^2) the antiderivative in x is
 * R^2 (x c + asin x) / 2, so the integral is R (G(x2) - G(x1)) / (2 x') with
 * x' = k / R.  Three forms keep it well conditioned:
 *   - the ends within 1e-6 of each other in x (a plane near parallel to the
 *     axis, or a tiny piece): 5-point Gauss-Legendre of the smooth root;
 *   - both ends away from tangency (c >= 0.1): the difference of G written
 *     without cancellation (x2 c2 - x1 c1 and asin x2 - asin x1 each as
 *     (x2 - x1) times a bounded factor), so that the division by x' is exact;
 *   - otherwise G directly, with asin x taken as atan2(x, c): near tangency
 *     the errors of c and of the angle then cancel to first order. */
static double int_w(double R, double a2, double k, double t1, double t2)
{
    const double dt = t2 - t1;
    if (!(dt > 0.0)) return 0.0;
    if (k == 0.0) return chord_w(R, a2) * dt;
    const double x1 = fmax(-1.0, fmin(1.0, (a2 + k * t1) / R));
    const double x2 = fmax(-1.0, fmin(1.0, (a2 + k * t2) / R));
    const double c1 = chord_w(1.0, x1), c2 = chord_w(1.0, x2);
    if (fabs(x2 - x1) < 1e-6) {
        static const double node[5] = { -0.9061798459386640, -0.5384693101056831, 0.0,
                                        0.5384693101056831, 0.9061798459386640 };
        static const double weight[5] = { 0.2369268850561891, 0.4786286704993665, 0.5688888888888889,
                                          0.4786286704993665, 0.2369268850561891 };
        double sum = 0.0;
        for (int q = 0; q < 5; ++q) {
            const double t = 0.5 * (t1 + t2) + 0.5 * dt * node[q];
            sum += weight[q] * chord_w(R, fmax(-R, fmin(R, a2 + k * t)));
        }
        return 0.5 * dt * sum;
    }
    if (fmin(c1, c2) >= 0.1 && x1 * x2 >= 0.0 && fabs(x2 - x1) < 0.5) {
        /* x2 c2 - x1 c1 = (x2 - x1) [c2 - x1 (x1 + x2) / (c1 + c2)];
         * asin x2 - asin x1 = asin((x2 - x1) g), g = c1 + x1 (x1 + x2) / (c1 + c2);
         * and (x2 - x1) / x' = dt */
        const double f = c2 - x1 * (x1 + x2) / (c1 + c2);
        const double g = c1 + x1 * (x1 + x2) / (c1 + c2);
        const double y = (x2 - x1) * g;
        const double ratio = fabs(y) < 1e-8 ? 1.0 + y * y / 6.0 : asin(y) / y;
        return 0.5 * R * dt * (f + ratio * g);
    }
    const double G1 = x1 * c1 + atan2(x1, c1), G2 = x2 * c2 + atan2(x2, c2);
    return 0.5 * R * R * (G2 - G1) / k;
}

typedef struct { double s0, t0, s1, t1; } edge_st_t;

/* s on an edge at t (t within the edge's t-range, edge not horizontal in t) */
static double edge_s(const edge_st_t* e, double t)
{
    return e->s0 + (e->s1 - e->s0) * ((t - e->t0) / (e->t1 - e->t0));
}

static int cmp_double(const void* a, const void* b)
{
    const double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* area of triangle (P0, P1, P2), frame coordinates, inside the support volume */
static double tri_area_in_volume(double R, const double* P0, const double* P1, const double* P2)
{
    double u[3], v[3], n[3];
    sub3(P1, P0, u);
    sub3(P2, P0, v);
    cross3(u, v, n);
    const double nl = sqrt(dot3(n, n));
    if (!(nl > 0.0)) return 0.0;
    const double m[3] = { n[0] / nl, n[1] / nl, n[2] / nl };
    double e1[3];
    const double hl = sqrt(m[0] * m[0] + m[1] * m[1]);
    if (hl > 1e-300) { e1[0] = m[1] / hl; e1[1] = -m[0] / hl; e1[2] = 0.0; }
    else { e1[0] = 1.0; e1[1] = 0.0; e1[2] = 0.0; }
    double e2[3];
    cross3(m, e1, e2);
    const double w2v[3] = { -e1[1], e1[0], 0.0 };          /* z x e1 */
    const double h0 = dot3(P0, m);
    const double a2 = h0 * dot3(m, w2v), k = dot3(e2, w2v);
    const double zc = h0 * m[2], ez = e2[2];
    /* slab: -R/2 <= zc + t ez <= R/2 */
    double tlo = -INFINITY, thi = INFINITY;
    if (ez != 0.0) {
        double ta = (-0.5 * R - zc) / ez, tb = (0.5 * R - zc) / ez;
        tlo = fmin(ta, tb);
        thi = fmax(ta, tb);
    } else if (fabs(zc) > 0.5 * R) {
        return 0.0;
    }
    /* the distance condition: |a2 + k t| <= R */
    if (k != 0.0) {
        double ta = (-R - a2) / k, tb = (R - a2) / k;
        tlo = fmax(tlo, fmin(ta, tb));
        thi = fmin(thi, fmax(ta, tb));
    } else if (fabs(a2) > R) {
        return 0.0;
    }
    const double* P[3] = { P0, P1, P2 };
    double s[3], t[3];
    for (int i = 0; i < 3; ++i) { s[i] = dot3(P[i], e1); t[i] = dot3(P[i], e2); }
    /* vertices sorted by t */
    int ia = 0, ib = 1, ic = 2, tmp;
    if (t[ib] < t[ia]) { tmp = ia; ia = ib; ib = tmp; }
    if (t[ic] < t[ib]) { tmp = ib; ib = ic; ic = tmp; }
    if (t[ib] < t[ia]) { tmp = ia; ia = ib; ib = tmp; }
    tlo = fmax(tlo, t[ia]);
    thi = fmin(thi, t[ic]);
    if (!(thi > tlo)) return 0.0;
    const edge_st_t eac = { s[ia], t[ia], s[ic], t[ic] };
    const edge_st_t eab = { s[ia], t[ia], s[ib], t[ib] };
    const edge_st_t ebc = { s[ib], t[ib], s[ic], t[ic] };
    double bp[16];
    int nb = 0;
    bp[nb++] = tlo;
    bp[nb++] = thi;
    bp[nb++] = t[ib];
    const edge_st_t* edges[3] = { &eac, &eab, &ebc };
    for (int j = 0; j < 3; ++j) {
        const edge_st_t* e = edges[j];
        if (!(e->t1 > e->t0)) continue;
        /* s(t) = p + q t; (p + q t)^2 + (a2 + k t)^2 = R^2 */
        const double q = (e->s1 - e->s0) / (e->t1 - e->t0), p = e->s0 - q * e->t0;
        const double A = q * q + k * k, B = 2.0 * (p * q + a2 * k), C = p * p + a2 * a2 - R * R;
        if (A == 0.0) continue;
        const double disc = B * B - 4.0 * A * C;
        if (disc < 0.0) continue;
        const double sq = sqrt(disc);
        const double r1 = (-B - sq) / (2.0 * A), r2 = (-B + sq) / (2.0 * A);
        if (r1 > e->t0 && r1 < e->t1) bp[nb++] = r1;
        if (r2 > e->t0 && r2 < e->t1) bp[nb++] = r2;
    }
    qsort(bp, (size_t)nb, sizeof(double), cmp_double);
    double area = 0.0;
    for (int i = 0; i + 1 < nb; ++i) {
        const double ua = fmax(bp[i], tlo), ub = fmin(bp[i + 1], thi);
        if (!(ub > ua)) continue;
        const double tm = 0.5 * (ua + ub);
        const edge_st_t* other = tm <= t[ib] ? &eab : &ebc;
        if (!(other->t1 > other->t0) || !(eac.t1 > eac.t0)) continue;
        double sa_u = edge_s(&eac, ua), sa_v = edge_s(&eac, ub), sa_m = edge_s(&eac, tm);
        double so_u = edge_s(other, ua), so_v = edge_s(other, ub), so_m = edge_s(other, tm);
        const int ac_low = sa_m <= so_m;
        const double lo_u = ac_low ? sa_u : so_u, lo_v = ac_low ? sa_v : so_v, lo_m = fmin(sa_m, so_m);
        const double hi_u = ac_low ? so_u : sa_u, hi_v = ac_low ? so_v : sa_v, hi_m = fmax(sa_m, so_m);
        const double wm = chord_w(R, a2 + k * tm);
        const double top = fmin(hi_m, wm), bot = fmax(lo_m, -wm);
        if (!(top > bot)) continue;
        const double len = ub - ua;
        const double iw = (hi_m > wm || lo_m < -wm) ? int_w(R, a2, k, ua, ub) : 0.0;
        const double upper = hi_m < wm ? 0.5 * (hi_u + hi_v) * len : iw;
        const double lower = lo_m > -wm ? 0.5 * (lo_u + lo_v) * len : -iw;
        area += upper - lower;
    }
    return area;
}

typedef struct {
    const double* pos; const uint32_t* tri; uint32_t nt;
    uint32_t obj_first, obj_count;
    const double* op_pos; const double* op_nrm;
    double R;
    double* a_all; double* a_obj;
} clutter_job_t;

static void clutter_one(const void* ctx, int64_t img)
{
    const clutter_job_t* J = (const clutter_job_t*)ctx;
    frame_t f;
    make_frame(J->op_pos + 3 * img, J->op_nrm + 3 * img, &f);
    double all = 0.0, obj = 0.0;
    for (uint32_t i = 0; i < J->nt; ++i) {
        double Q[3][3];
        for (int k = 0; k < 3; ++k) {
            const double* p = J->pos + 3 * (size_t)J->tri[3 * (size_t)i + k];
            project(&f, p[0], p[1], p[2], &Q[k][0], &Q[k][1], &Q[k][2]);
        }
        const double a = tri_area_in_volume(J->R, Q[0], Q[1], Q[2]);
        all += a;
        if (i >= J->obj_first && i - J->obj_first < J->obj_count) obj += a;
    }
    J->a_all[img] = all;
    J->a_obj[img] = obj;
}

/* Areas of the scene's and of the object's surface inside each oriented
 * point's support volume; triangles obj_first .. obj_first + obj_count - 1 are
 * the object.  fp32 inputs converted exactly.  -1 on a bad index. */
int oracle_clutter_areas(const float* pos, uint32_t nv, const uint32_t* tri, uint32_t nt, uint32_t obj_first,
                         uint32_t obj_count, const float* op_pos, const float* op_nrm, uint32_t n, float R,
                         double* a_all, double* a_obj, int nthreads)
{
    if (check_mesh(tri, nt, nv)) return -1;
    double* p = widen(pos, (size_t)nv * 3);
    double* o = widen(op_pos, (size_t)n * 3);
    double* m = widen(op_nrm, (size_t)n * 3);
    int rc = -2;
    if (p && o && m) {
        clutter_job_t J = { p, tri, nt, obj_first, obj_count, o, m, (double)R, a_all, a_obj };
        parallel_for(&J, clutter_one, n, nthreads);
        rc = 0;
    }
    free(p); free(o); free(m);
    return rc;
}

/* area of one triangle given in frame coordinates (FP64), for the pins */
double oracle_triangle_area_in_volume(const double* p0, const double* p1, const double* p2, double R)
{
    return tri_area_in_volume(R, p0, p1, p2);
}
