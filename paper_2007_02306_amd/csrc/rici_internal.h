// Internal declarations shared by the HIP translation units of librici.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rici {

constexpr int NB = 64;              // bins per image side (64 x 64 images)
constexpr int NPIX = NB * NB;       // pixels per image

// ------------------------------------------------------------ projection
// Eq. 1 in FP64 for one oriented point: the first rotation (about z) takes
// the normal's (x, y) onto +x, the second (about y) normalises the normal's x
// after the first rotation against its z, so that the normal ends on +z.  A
// pair that normalises from (0, 0) gives the identity rotation.  Shared by the
// RICI and the Spin Image generators.
struct Rotation { double nax, nay, nbx, nbz; };

__device__ __forceinline__ Rotation frame_rotation(double nx, double ny, double nz)
{
    Rotation q = {1.0, 0.0, 0.0, 1.0};
    const double la = sqrt(nx * nx + ny * ny);
    if (la > 0.0) { q.nax = nx / la; q.nay = ny / la; }
    const double rx = q.nax * nx + q.nay * ny;
    const double lb = sqrt(rx * rx + nz * nz);
    if (lb > 0.0) { q.nbx = rx / lb; q.nbz = nz / lb; }
    return q;
}

// ---------------------------------------------------------------- generation
// Scratch per triangle: a conservative bounding sphere (cx, cy, cz, radius) and
// the three vertices as float4 (w unused).
constexpr size_t kTriCullBytes = 16;
constexpr size_t kTriVertBytes = 48;

// One mesh of a batched call (device copy).  cull / clusters / verts point at
// this job's part of the scratch; block_start / chunk_start / item_start are
// the job's first triangle sort block (kGenSortBlock triangles), 64-triangle
// chunk and image-group work item in the flattened index spaces of the batched
// kernels.
// triangles per Morton-sorted block of the triangle preparation (one
// workgroup), and the mesh size from which the automatic mode sorts (measured:
// the sort pays on the 691k-triangle clutter scene, not on the 47k-triangle
// union of 12 shapes)
constexpr uint32_t kGenSortBlock = 4096;
constexpr uint32_t kGenSortAuto = 1u << 17;

struct GenJob {
    const float* pos; uint32_t nv;
    const uint32_t* tri; uint32_t nt;
    const float* op_pos; const float* op_nrm; uint32_t n;
    uint32_t* out;
    float4* cull; float4* clusters; float4* verts;
    uint64_t block_start, chunk_start;
    uint32_t item_start;
    int sort;                     // triangles stored in Morton order within blocks
};

// sort mode: 0 mesh order, 1 Morton order within blocks, 2 Morton order for
// meshes of at least kGenSortAuto triangles
bool gen_sort_wanted(int mode, uint32_t nt);
hipError_t launch_gen_prep(const float* pos, uint32_t nv, const uint32_t* tri, uint32_t nt, int sort_mode,
                           float4* cull, float4* verts, uint32_t* err, hipStream_t s);
hipError_t launch_gen_clusters(const float4* cull, uint32_t nt, float4* clusters, hipStream_t s);
hipError_t launch_gen(const float4* cull, const float4* clusters, const float4* verts, uint32_t nt,
                      const float* op_pos, const float* op_nrm, uint32_t n, float R,
                      uint32_t* out, uint32_t* err, int group, hipStream_t s);
// images per workgroup (and per work item of the batched kernel): 2 or 4
uint32_t gen_group_images(int group);
// workgroups of the persistent generation kernel that fit the device at once
hipError_t gen_batched_grid(int group, int cus, uint32_t* grid);
// prep + clusters + persistent generation over `njobs` jobs stored largest first
// part: 0 everything; 1 the launches before the persistent kernel (triangle
// preparation, cluster spheres, work counter); 2 the persistent kernel alone
hipError_t launch_gen_batched(const GenJob* jobs, uint32_t njobs, uint64_t total_blocks, uint64_t total_chunks,
                              uint32_t total_items, float R, uint32_t* counter, uint32_t* err, uint32_t grid,
                              int group, hipStream_t s, int part = 0);

// -------------------------------------------------------------------- search
// Column-delta planes in "fragment-major" order: for every group of 16 images
// and every image row (64 deltas = one 64-wide K chunk), the 16 x 64 int8 values
// sit in 1 KiB exactly as the 64 lanes of one v_mfma_i32_16x16x64_i8 operand
// read them: lane l = 16 * (c / 16) + (image % 16) holds columns c .. c + 15.
constexpr int kGroup = 16;                       // images per fragment group
constexpr size_t kFragBytes = 1024;              // 16 images x 64 columns
constexpr size_t kPlaneGroupBytes = NB * kFragBytes;   // one group, all 64 rows

// needle planes: 0 = D (int8), 1 = mask [D != 0] (0/1)
// haystack planes: 0 = D, 1 = r = (D^2 mod 256) - 128, 2 = q = D^2 div 256
// (a set ranked against itself writes needle plane 1 only: its needles read
// the haystack's D plane, in the same slot order)
// Needles keep their order (slot = image).  The haystack is permuted: images
// whose deltas all satisfy |D| <= 15 (so q = 0) take slots from the front, the others
// from the back, with at least one whole tile of padding in between, so that a
// search tile holds only one kind and only tiles of the second kind pay the
// third contraction phase.  Ranks are counts, so the order is free; the
// distance matrix maps slots back through `perm`.
struct SearchPrep {
    int8_t* planes;        // [nplanes][ngroups][64][1024]
    int64_t* sumsq;        // needles: |D|^2 + 128 * #(D != 0) per slot (the contraction's constant)
    uint32_t* maxabs;      // max |D| per slot (saturating; padding = 0xFFFFFFFF)
    uint32_t* maxabs_img;  // max |D| per original image (== maxabs for needles)
    uint32_t* perm;        // haystack: slot -> image (0xFFFFFFFF = padding); needles: nullptr
    uint32_t* inv;         // paired sets (haystack side): image -> slot; else nullptr
    uint32_t ngroups;      // slots / 16
};

// Arguments of the MFMA search over one (needles, haystack) pair of sets.
struct SearchArgs {
    const int8_t* a_planes; uint32_t a_groups; uint32_t nn;
    const int8_t* b_planes; uint32_t b_groups; uint32_t nh;
    const uint32_t* nmax;
    const uint32_t* hmax;      // per haystack slot
    const uint32_t* hperm;     // haystack slot -> image
    const int32_t* thr;
    const int64_t* sumsq;
    uint32_t* rank;
    int64_t* matrix;
    uint32_t tiles_m, tiles_n, per_xcd;
    // rank mode only: leave a tile once no pair can still end below its
    // needle's threshold: in the last phase a partial sum can fall by at most
    // 128 * 63 per remaining row (r >= -128), so a tile stops when every
    // partial sum exceeds its threshold by that slack
    uint32_t early_exit;
    // Paired mode (rank mode, a set ranked against itself): needles and
    // haystack share the haystack's slot order, so tile (I, J) holds the pairs
    // of both directions.  Work items are the tile pairs I <= J; a pair of
    // tiles whose images all have |D| <= 15 computes the cross term once and
    // reuses it for the mirrored direction through a per-workgroup slot of
    // `cross` (BM x BN int32 per resident workgroup).  nperm maps a needle
    // slot to its image (rank index); tile_flags[t]: bit 0 = some image of
    // tile t is usable (|D| <= 127), bit 1 = some usable image has |D| > 15.
    uint32_t paired;
    const uint32_t* nperm;
    const uint32_t* tile_flags;
    int32_t* cross;
};

// One ranking job of a batched call (device copy): its arguments, its scratch
// and its first index in each flattened index space of the batched kernels.
struct SearchJob {
    SearchArgs A;
    const uint32_t* needles; const uint32_t* hay; const uint32_t* true_idx;
    int64_t* dstar;
    uint32_t* lists;
    SearchPrep np, hp;
    uint64_t ngrp_start, hslot_start, himg_start, hgrp_start, needle_start;
    uint32_t tile_start;
};

// One slice of a database scan: every listed query against database tiles
// tile_begin .. tile_begin + tile_count - 1 (mod db_tiles).  Passed by value.
constexpr int kMaxScanJobs = 24;
struct ScanTable {
    SearchArgs A[kMaxScanJobs];
    uint32_t m_start[kMaxScanJobs + 1];   // prefix of the queries' needle tiles
    uint32_t njobs, tile_begin, tile_count, db_tiles;
};
// variant: search tile shape (0: 256 x 256, 1: 128 x 256; see search_tile_m)
hipError_t launch_search_scan(const ScanTable& T, int variant, hipStream_t s);

struct SearchTotals {
    uint64_t needle_groups, hay_slots, hay_images, hay_groups, needles, tiles;
};

// known_maxabs (haystack side, optional): per-image max |D| already computed
// for the same images (by the needle pass when a set is ranked against itself)
hipError_t launch_delta_prep(const uint32_t* images, uint32_t n, int needle_side,
                             const SearchPrep& p, hipStream_t s, const uint32_t* known_maxabs = nullptr);
// every prep, rank and fallback step of `njobs` jobs (stored largest first),
// with a persistent search kernel of `grid` workgroups
// part: 0 everything; 1 the launches before the persistent kernel (delta
// planes, statistics, true-match distances, work counters); 2 the persistent
// search kernel alone; 3 the launches after it (exact fallback)
// paired: every job is a paired set (variant 0, no early exit); its needle
// planes are then written after the slot assignment
hipError_t launch_search_batched(const SearchJob* jobs, uint32_t njobs, const SearchTotals& T, uint32_t* counter,
                                 uint32_t grid, int variant, int early_exit, hipStream_t s, int part = 0,
                                 int paired = 0);
size_t haystack_slots(uint32_t nh);   // slots allocated for a haystack of nh images
// inv (paired sets): thresholds are written per slot, thr[inv[i]]
hipError_t launch_true_distance(const uint32_t* needles, uint32_t nn, const uint32_t* hay, uint32_t nh,
                                const uint32_t* true_idx, const int64_t* sumsq, const uint32_t* nmax,
                                int64_t* dstar, int32_t* thr, uint32_t* rank, hipStream_t s,
                                const uint32_t* inv = nullptr);
// A set of n images ranked against itself ("paired"): statistics per image
// (hp.maxabs_img, np.sumsq) and the true-match distances (dstar, -1 for
// true_idx[i] >= n) in one pass, slot assignment (hp.perm, hp.inv,
// hp.maxabs) with the thresholds per slot (INT_MIN where no count) and the
// ranks' start values, the flags of each 256-slot tile, then the needle mask
// plane and the haystack planes in the same slot order.  np.ngroups ==
// hp.ngroups == haystack_slots(n) / 16.
hipError_t launch_paired_prep(const uint32_t* images, uint32_t n, const uint32_t* true_idx, const SearchPrep& np,
                              const SearchPrep& hp, int32_t* thr_slots, uint32_t* tile_flags, int64_t* dstar,
                              uint32_t* rank, hipStream_t s);
// persistent search over the tile pairs of a paired set (A.paired, square
// tiles); grid <= resident workgroups, each with a paired_slot_bytes() slot
// of A.cross; counters: 8 words of scratch
hipError_t launch_search_paired(const SearchArgs& A, uint32_t grid, uint32_t* counters, hipStream_t s);
uint32_t paired_items(uint32_t tiles);   // work items of a paired set of `tiles` tiles
size_t paired_slot_bytes();              // cross-term slot per persistent workgroup
hipError_t launch_search(const SearchPrep& np, uint32_t nn, const SearchPrep& hp, uint32_t nh,
                         const int32_t* thr, const int64_t* sumsq, uint32_t* rank, int64_t* matrix, int variant,
                         int early_exit, hipStream_t s);
// `lists` scratch: 2 + nn + nh uint32
hipError_t launch_fallback(const uint32_t* needles, uint32_t nn, const uint32_t* hay, uint32_t nh,
                           const uint32_t* nmax, const uint32_t* hmax, const int64_t* dstar,
                           uint32_t* rank, int64_t* matrix, uint32_t* lists, hipStream_t s);

// ---------------------------------------------------------- spin images
// Correlation planes of one image set: z = (x - mean) / norm in fp32,
// fragment-major for v_mfma_f32_16x16x4_f32, spin_slots(n) images; FP64 mean
// and centred norm per image.
struct SpinPrep { float* z; double* mean; double* norm; };
size_t spin_slots(uint32_t n);          // images per plane set (n rounded up to the tile)
double spin_band();                     // fp32 contraction error bound used by the rank
hipError_t launch_spin_gen(const float* samples, uint32_t ns, const float* op_pos, const float* op_nrm, uint32_t n,
                           float R, float* out, uint32_t* err, hipStream_t s);
hipError_t launch_spin_zprep(const float* images, uint32_t n, float* z, double* mean, double* norm, hipStream_t s);
// rank[i] = #{h : rho(n_i, h) > rho(n_i, h_true)}; queue: scratch for pairs
// near the threshold (queue_cap entries; overflow sets bit 4 of *err)
hipError_t launch_spin_rank(const SpinPrep& np, const float* needles, uint32_t nn, const SpinPrep& hp,
                            const float* hay, uint32_t nh, const uint32_t* true_idx, double* rho_t, uint32_t* rank,
                            uint2* queue, uint32_t* queue_count, uint32_t queue_cap, uint32_t* err, hipStream_t s,
                            int part = 0);   // 0 all; 1 true correlations; 2 contraction; 3 settle the queue
hipError_t launch_spin_matrix(const SpinPrep& np, uint32_t nn, const SpinPrep& hp, uint32_t nh, float* out,
                              hipStream_t s);

// ------------------------------------------------------------- clutter
// a_all / a_obj: surface area of all triangles / of triangles obj_first ..
// obj_first + obj_count - 1 inside each oriented point's support volume
hipError_t launch_clutter(const float* pos, uint32_t nv, const uint32_t* tri, uint32_t nt, uint32_t obj_first,
                          uint32_t obj_count, const float* op_pos, const float* op_nrm, uint32_t n, float R,
                          double* a_all, double* a_obj, uint32_t* err, hipStream_t s);

size_t search_groups(uint32_t n);   // fragment groups allocated for n images
size_t search_lds_bytes();          // dynamic LDS of the search kernel
hipError_t prepare_search_kernels(); // raise the search kernels' LDS limit (before any graph capture)
uint32_t search_tile_m(int variant);  // needles per search tile
uint32_t search_tile_n();             // haystack slots per search tile (same for every variant)

}  // namespace rici
