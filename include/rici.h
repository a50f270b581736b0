/*
 * rici.h -- C ABI of the MI355X (gfx950) implementation of the Radial
 * Intersection Count Image (RICI) pipeline of van Blokland & Theoharis,
 * "Radial intersection count image: a clutter resistant 3D shape descriptor"
 * (2020): descriptor generation (Sec. 3.1) and clutter-resistant-distance rank
 * search (Sec. 3.2, Sec. 4.1).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers on the handle's device, allocated and
 *     owned by the caller.  The library never frees or retains them beyond the
 *     work it enqueues.  Outputs must not overlap inputs.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     work is enqueued on it and the call returns without waiting.
 *   - Every call returns a rici_status.  Argument errors are detected on the
 *     host before anything is enqueued; rici_last_error() then describes them.
 *     Errors found by the kernels (a triangle index >= num_vertices, a
 *     non-finite coordinate) set a sticky per-handle device word that the next
 *     rici_sync() reports (and clears); the images of such a call are
 *     unspecified.
 *   - A handle owns its scratch memory and is NOT safe for concurrent calls:
 *     use one handle per stream that issues work concurrently.  Scratch grows
 *     on demand; growing it synchronises the device.
 *   - Zero-sized work (num_points == 0, num_needles == 0) is a valid no-op.
 *
 * Image layout: uint32 [N][64][64], row-major; every image array (generation
 * output, needles, haystack, database) must start on a 16-byte boundary
 * (RICI_ERR_INVALID otherwise).  Row r is the circle plane at
 * height beta_r = -R/2 + (r + 1/2) R/64 along the Central Axis, column c the
 * circle of radius rho_c = (c + 1/2) R/64, so pixel (r, c) counts the points
 * where that circle meets the scene's triangles (Sec. 3.1; the square support
 * plane of width and height R of Sec. 2.1, sampled at bin centres).
 */
#ifndef RICI_H
#define RICI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RICI_BINS 64

typedef struct rici_ctx* rici_handle;

typedef enum {
    RICI_OK = 0,
    RICI_ERR_INVALID = -1,      /* bad argument (null pointer, size, radius, overlap) */
    RICI_ERR_OOM = -2,          /* scratch allocation failed                          */
    RICI_ERR_HIP = -3,          /* a HIP runtime call failed                          */
    RICI_ERR_DEVICE = -4,       /* a kernel flagged bad input (reported by rici_sync) */
    RICI_ERR_UNSUPPORTED = -5   /* no gfx950 device / size beyond the documented cap  */
} rici_status;

/* Device-side error bits reported through rici_sync / rici_device_errors. */
#define RICI_DEVERR_INDEX 1u       /* a triangle index >= num_vertices */
#define RICI_DEVERR_NONFINITE 2u   /* a non-finite position, normal or sample  */
#define RICI_DEVERR_QUEUE 4u       /* rici_spin_rank: more pairs near a true match's
                                      correlation than its settle queue holds; ranks
                                      of that call may be too low                   */

/* Create a handle bound to HIP device `device` (must be gfx950).  */
int rici_create(rici_handle* out, int device);
/* Release the handle and its scratch (waits for the handle's device). */
void rici_destroy(rici_handle h);
/* Message describing the last failing call made by this thread ("" if none). */
const char* rici_last_error(void);
/* Wait for `stream`, then report and clear the handle's sticky device errors:
 * RICI_OK, RICI_ERR_DEVICE (bits readable via rici_device_errors) or RICI_ERR_HIP. */
int rici_sync(rici_handle h, void* stream);
/* Device error bits seen by the last rici_sync on this handle. */
uint32_t rici_device_errors(rici_handle h);

/*
 * rici_generate -- one RICI per oriented point (Sec. 3.1; one descriptor per
 * unique vertex, Sec. 4.1 step 5).
 *   positions     [num_vertices][3] fp32 scene vertices.
 *   triangles     [num_triangles][3] uint32 vertex indices (every triangle of
 *                 the scene contributes, Sec. 3.1: O(T) per image).
 *   op_positions  [num_points][3] fp32 Spin Vertices S_v.
 *   op_normals    [num_points][3] fp32 Spin Normals S_n (any length; a zero
 *                 normal selects the +z axis, the identity rotation of Sec. 3.1.1).
 *   support_radius  R, finite and > 0.
 *   out_images    [num_points][64][64] uint32, overwritten.
 * Projection: Eq. 1-5 with the second rotation normalising the first
 * rotation's output; intersection counting: Sec. 3.1.2 (single range
 * (min|E|, max|E|), double range (|C|, min|E|)); all decisions in FP64.
 * num_triangles == 0 gives all-zero images.  Limits: num_triangles < 2^29,
 * num_points < 2^31.
 */
int rici_generate(rici_handle h,
                  const float* positions, uint32_t num_vertices,
                  const uint32_t* triangles, uint32_t num_triangles,
                  const float* op_positions, const float* op_normals, uint32_t num_points,
                  float support_radius, uint32_t* out_images, void* stream);

/*
 * rici_generate_noalloc -- rici_generate for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, checks, kernels and results as
 * rici_generate; the difference is where the triangle preparation records
 * live: in a static workspace of the library (one per GPU, about 64 MiB, held
 * until the process ends, its address looked up by rici_create) instead of the
 * handle's growable scratch.  The call allocates nothing and never
 * synchronises.
 *   num_triangles  at most RICI_NOALLOC_MAX_TRIANGLES; a larger mesh returns
 *                  RICI_ERR_UNSUPPORTED (checked right after the handle,
 *                  before the other arguments) and nothing is enqueued.
 * Every call on one GPU shares that GPU's workspace, whatever the handle:
 * calls whose work overlaps on one GPU (on different streams, or from
 * different threads) race and give unspecified images.  Serialise them, for
 * instance on one stream.  Nothing in the workspace needs to start at zero
 * (each call rewrites the records it reads).  Kernel timing does not cover
 * this call.  RICI_ERR_HIP if the workspace's address could not be found.
 */
#define RICI_NOALLOC_MAX_TRIANGLES (1u << 20)

int rici_generate_noalloc(rici_handle h,
                          const float* positions, uint32_t num_vertices,
                          const uint32_t* triangles, uint32_t num_triangles,
                          const float* op_positions, const float* op_normals, uint32_t num_points,
                          float support_radius, uint32_t* out_images, void* stream);

/*
 * rici_distance_rank -- rank of the true match (Sec. 4.1 step 6c) under the
 * clutter-resistant distance CRD (Sec. 3.2, Eq. 6-7):
 *   CRD(n, h) = sum over rows r in [0, 64), columns c in [1, 64) with
 *               D(n,r,c) != 0 of (D(n,r,c) - D(h,r,c))^2,
 *   D(x,r,c)  = x(r,c) - x(r,c-1) (signed).
 *   rank[i]   = #{ j : CRD(n_i, h_j) < CRD(n_i, h_true[i]) }   (ties take the
 *               best rank, Sec. 4.2), so 0 <= rank[i] <= num_haystack - 1.
 *   needles       [num_needles][64][64] uint32.
 *   haystack      [num_haystack][64][64] uint32 (may be the same memory).
 *   true_index    [num_needles] uint32, each < num_haystack (checked on device;
 *                 an out-of-range entry yields rank = num_haystack).
 *   out_rank      [num_needles] uint32.
 *   out_true_distance  [num_needles] int64 CRD(n_i, h_true[i]), or NULL.
 * Exact integer arithmetic: int8 x int8 -> int32 MFMA contractions when the
 * column deltas fit (|D| <= 127 for every image; two contraction phases when
 * every haystack image of a tile has |D| <= 15, three otherwise), exact int64
 * VALU arithmetic for any image outside that range.  When needles and
 * haystack are the same array with the same count, the search runs over
 * pairs of tiles that share the cross term (tuning key "search_pairs").
 */
int rici_distance_rank(rici_handle h,
                       const uint32_t* needles, uint32_t num_needles,
                       const uint32_t* haystack, uint32_t num_haystack,
                       const uint32_t* true_index,
                       uint32_t* out_rank, int64_t* out_true_distance, void* stream);

/*
 * rici_distance_matrix -- out[i][j] = CRD(needle_i, haystack_j), int64,
 * row-major [num_needles][num_haystack] (same arithmetic as rici_distance_rank).
 */
int rici_distance_matrix(rici_handle h,
                         const uint32_t* needles, uint32_t num_needles,
                         const uint32_t* haystack, uint32_t num_haystack,
                         int64_t* out, void* stream);

/*
 * Spin Images and their Pearson search (Sec. 2.1; the paper's comparison
 * descriptor, built with the same projection, Sec. 3.1.1).
 *
 * rici_spin_generate -- one Spin Image per oriented point from a point cloud.
 *   samples       [num_samples][3] fp32 point samples of the scene surface.
 *   op_positions, op_normals  [num_points][3] fp32 oriented points (a zero
 *                 normal selects +z).
 *   support_radius  R, finite and > 0.
 *   out_images    [num_points][64][64] fp32, overwritten (16-byte aligned).
 * A sample counts when 0 <= alpha < R and -R/2 <= beta < R/2 (Eq. 1-5 in
 * FP64, no support-angle filter); it adds bilinear weights between bin centres
 * (alpha = (c + 1/2) R/64, beta = -R/2 + (r + 1/2) R/64) to its four nearest
 * bins, dropping bins outside the grid.  Pixel sums are fp32 in arbitrary
 * order: each pixel is within n 2^-24 of its exact sum times that sum, n being
 * the number of contributions it received.
 *
 * rici_spin_rank -- rank of the true match under the Pearson correlation
 * coefficient rho over the 4096 pixels (0 for a constant image, where it is
 * undefined); higher is closer:
 *   rank[i] = #{ j : rho(n_i, h_j) > rho(n_i, h_true[i]) }  (ties: best rank).
 *   needles [num_needles][64][64], haystack [num_haystack][64][64] fp32 (may be
 *   the same memory); true_index [num_needles] uint32 (an entry >= num_haystack
 *   gives rank num_haystack and correlation +inf); out_rank [num_needles];
 *   out_true_correlation [num_needles] double or NULL.
 * The contraction runs in fp32 on the matrix cores; pairs within its error
 * bound of the true match's correlation are settled by the FP64 correlation,
 * which also gives out_true_correlation, so ranks are those of the FP64
 * correlations.  If more pairs need settling than the call's queue holds
 * (at least 2^20 or 1024 per needle), rici_sync reports RICI_DEVERR_QUEUE.
 *
 * rici_spin_correlation_matrix -- out[i][j] = rho(n_i, h_j) as fp32 from the
 * same contraction (row-major [num_needles][num_haystack]); within 2.5e-4 of
 * the FP64 value.
 */
int rici_spin_generate(rici_handle h, const float* samples, uint32_t num_samples,
                       const float* op_positions, const float* op_normals, uint32_t num_points,
                       float support_radius, float* out_images, void* stream);
int rici_spin_rank(rici_handle h, const float* needles, uint32_t num_needles,
                   const float* haystack, uint32_t num_haystack, const uint32_t* true_index,
                   uint32_t* out_rank, double* out_true_correlation, void* stream);
int rici_spin_correlation_matrix(rici_handle h, const float* needles, uint32_t num_needles,
                                 const float* haystack, uint32_t num_haystack, float* out,
                                 void* stream);

/*
 * rici_clutter_areas -- the areas behind Eq. 8's clutter measure,
 *   clutter = (A_all - A_object) / A_all,
 * for each oriented point: A_all = surface area of all triangles, A_object =
 * of the object's triangles object_first .. object_first + object_count - 1,
 * inside the point's support volume (the descriptor's cylinder: distance from
 * the Central Axis <= R and |beta| <= R/2, Sec. 2.1).
 *   positions [num_vertices][3], triangles [num_triangles][3] as for
 *   rici_generate; op_positions, op_normals [num_points][3] fp32;
 *   out_area_all, out_area_object [num_points] double.
 * Each triangle's area inside the volume is integrated exactly over its
 * in-plane height in FP64 (closed forms for the circular boundary), so the
 * results are the exact areas up to FP64 rounding.
 */
int rici_clutter_areas(rici_handle h, const float* positions, uint32_t num_vertices,
                       const uint32_t* triangles, uint32_t num_triangles,
                       uint32_t object_first, uint32_t object_count,
                       const float* op_positions, const float* op_normals, uint32_t num_points,
                       float support_radius, double* out_area_all, double* out_area_object,
                       void* stream);

/*
 * Batched describe-and-rank over many meshes (one plan, replayed as a HIP graph).
 *
 * Each job is one mesh with its own oriented points; its RICIs are written to
 * out_images and, when true_index is given, every one of them is ranked as a
 * needle against the job's own RICIs as the haystack (rank of the true match,
 * Sec. 4.1 step 6c, same arithmetic as rici_distance_rank).
 * rici_batch_create validates the jobs, allocates the plan's scratch (freed by
 * rici_batch_destroy), uploads the job tables and records the launch sequence
 * -- triangle preparation, one persistent generation kernel over (mesh, image
 * group) items, delta planes, one persistent search kernel over (mesh, tile)
 * items, exact fallback -- into a HIP graph.  Work items are taken from device
 * counters, largest meshes first.  rici_batch_run replays the graph on
 * `stream`; the device pointers of the jobs must stay valid for the life of the
 * plan.  A plan must not run concurrently with itself.
 */
typedef struct {
    const float* positions; uint32_t num_vertices;    /* [V][3] fp32                     */
    const uint32_t* triangles; uint32_t num_triangles;/* [T][3] uint32                   */
    const float* op_positions;                        /* [N][3] fp32                     */
    const float* op_normals; uint32_t num_points;     /* [N][3] fp32                     */
    uint32_t* out_images;                             /* [N][64][64] uint32              */
    const uint32_t* true_index;                       /* [N] or NULL (describe only)     */
    uint32_t* out_rank;                               /* [N], required with true_index   */
    int64_t* out_true_distance;                       /* [N] or NULL                     */
} rici_mesh_job;

typedef struct rici_batch_ctx* rici_batch;

int rici_batch_create(rici_handle h, const rici_mesh_job* jobs /* host array */, uint32_t num_jobs,
                      float support_radius, rici_batch* out);
int rici_batch_run(rici_batch b, void* stream);
void rici_batch_destroy(rici_batch b);
/* Bytes of device scratch the plan holds. */
uint64_t rici_batch_scratch_bytes(rici_batch b);
/* Measurement support: duration in ms of the persistent generation ("gen") or
 * search ("search") kernel in the plan's most recent replay, from HIP events
 * recorded inside the graph right around that kernel.  Waits for that replay to
 * pass the kernel; 0 if the plan has no such work; RICI_ERR_UNSUPPORTED if the
 * runtime refused event nodes in the graph (the plan runs without them).
 * Undefined before the first rici_batch_run. */
int rici_batch_kernel_ms(rici_batch b, const char* kernel, float* ms);

/*
 * Device-resident descriptor database and incremental queries (serving).
 *
 * rici_db_create prepares a haystack once: delta planes (partitioned by delta
 * range), per-image statistics and the list of images outside the int8 range.
 * The caller's images must stay valid while the database exists (true-match
 * distances and exact out-of-range counts read them).  The database's tiles
 * (rici_db_tiles, 256 haystack slots each) can then be scanned in any order and
 * in any number of slices.
 *
 * rici_query_create prepares a set of needles against a database: delta planes,
 * true-match distances d*_i = CRD(n_i, h_true[i]) (Eq. 7), out_rank zeroed, and
 * the exact counts of every pair that involves an image outside the int8 range
 * added to out_rank.  rici_db_scan adds, for each query, the counts
 * #{h in tiles : CRD(n_i, h) < d*_i} of `tile_count` database tiles starting at
 * `tile_begin` (wrapping around).  After every tile has been scanned exactly
 * once for a query, its out_rank holds the rank of Sec. 4.1 step 6c -- whatever
 * the order of the slices and whichever other queries shared them (integer
 * counts, no rounding).  out_rank / out_true_distance are caller device buffers
 * of num_needles entries.  A query's scratch is its own; queries and databases
 * may be used from several handles on several streams, but a query must not be
 * scanned by two calls at once.  At most RICI_SCAN_MAX_QUERIES queries per scan.
 */
#define RICI_SCAN_MAX_QUERIES 24

typedef struct rici_db_ctx* rici_db;
typedef struct rici_query_ctx* rici_query;

int rici_db_create(rici_handle h, const uint32_t* images, uint32_t num_images, void* stream, rici_db* out);
uint32_t rici_db_tiles(rici_db db);
uint64_t rici_db_scratch_bytes(rici_db db);
void rici_db_destroy(rici_db db);

/* workspace: NULL (the query allocates and rici_query_destroy frees, after
 * waiting for the device) or caller device memory of at least
 * rici_query_footprint bytes that outlives the query (then rici_query_destroy
 * neither frees nor waits: the caller must know the query's work is done). */
int rici_query_create(rici_handle h, rici_db db, const uint32_t* needles, uint32_t num_needles,
                      const uint32_t* true_index, uint32_t* out_rank, int64_t* out_true_distance,
                      void* workspace, uint64_t workspace_bytes, void* stream, rici_query* out);
/* Device bytes a query of num_needles needles against db holds (its admission footprint). */
uint64_t rici_query_footprint(rici_db db, uint32_t num_needles);
void rici_query_destroy(rici_query q);

int rici_db_scan(rici_handle h, rici_db db, const rici_query* queries, uint32_t num_queries,
                 uint32_t tile_begin, uint32_t tile_count, void* stream);

/*
 * Kernel timing (measurement support).  When enabled, every kernel the handle
 * launches is bracketed by HIP events on its stream; rici_timing_get sums the
 * elapsed times of the completed launches of the named kernel ("gen",
 * "gen_prep", "delta_needle", "delta_haystack", "true_distance", "search",
 * "fallback", "matrix", "spin_gen", "spin_zprep", "spin_true", "spin_search",
 * "spin_settle", "spin_matrix", "clutter").  Reading synchronises the handle's device.
 */
int rici_timing_enable(rici_handle h, int on);
int rici_timing_reset(rici_handle h);
int rici_timing_get(rici_handle h, const char* kernel, double* total_ms, uint64_t* launches);

/*
 * Tuning knobs of a handle (launch shapes only: results never depend on them).
 *
 *   "gen_images_per_group"  images sharing one generation workgroup (and its
 *                    triangle stream): 2 (default) or 4.  Read by
 *                    rici_generate and rici_batch_create (fixed into the plan).
 *   "gen_sort_triangles"  order in which the triangle preparation stores a
 *                    mesh's triangles for the generation kernel's culls: 0 mesh
 *                    order, 1 Morton order of their bounding-box centres within
 *                    blocks of 4096 (compact runs of 64 whose bounding spheres
 *                    miss more images), 2 (default) Morton order for meshes of
 *                    at least 131072 triangles.  Read by rici_generate and
 *                    rici_batch_create (per mesh, fixed into the plan).
 *   "search_early_exit"  0 (default) or 1: in rank mode a search tile stops
 *                    once every partial distance of its last contraction phase
 *                    exceeds its needle's threshold by more than it can still
 *                    fall (at most 128 x 63 per remaining image row), so the
 *                    tile can add to no rank.  Ranks are unchanged; it saves
 *                    work when true matches are close (clutter, serving).
 *                    Read by rici_distance_rank, rici_batch_create and
 *                    rici_query_create.
 *   "search_pairs"   1 (default) or 0: a set ranked against itself (the same
 *                    array and count as needles and haystack, and every mesh
 *                    of a batched plan) is searched by pairs of tiles that
 *                    serve both directions and compute the cross term
 *                    <D_a, D_b> of Eq. 7 once for both (about a quarter fewer
 *                    contraction operations).  Taken only with 256-needle
 *                    tiles and without the early exit.  Read by
 *                    rici_distance_rank and rici_batch_create (fixed into the
 *                    plan).
 *   "search_tile_m"  needles per search workgroup tile: 256 (default) or 128.
 *                    The smaller tile wastes less work on padding when a
 *                    needle set is small or just above a multiple of 256.
 *                    Read by rici_distance_rank, rici_distance_matrix,
 *                    rici_batch_create (fixed into the plan) and
 *                    rici_query_create (fixed into the query: queries scanned
 *                    together by rici_db_scan must share it).
 *
 * rici_set_tuning returns RICI_ERR_INVALID for an unknown key or a value the
 * key does not allow; rici_get_tuning writes the current value to *value.
 */
int rici_set_tuning(rici_handle h, const char* key, int value);
int rici_get_tuning(rici_handle h, const char* key, int* value);

#ifdef __cplusplus
}
#endif

#endif /* RICI_H */
