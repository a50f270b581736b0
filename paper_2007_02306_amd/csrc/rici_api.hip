// Host side of librici: handles, scratch, argument checks, kernel timing and
// the extern "C" entry points declared in include/rici.h.
#include "rici.h"
#include "rici_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

struct TimedLaunch {
    const char* name;
    hipEvent_t start, stop;
};

struct rici_ctx {
    int device = 0;
    uint32_t* d_err = nullptr;      // sticky device error word
    uint32_t last_dev_err = 0;
    void* ws = nullptr;             // scratch
    size_t ws_size = 0;
    void* noalloc = nullptr;        // this device's address of the static generation workspace
    bool timing = false;
    int search_variant = 0;         // search tile: 0 = 256 x 256, 1 = 128 x 256
    int gen_group = 2;              // images per generation workgroup: 2 or 4
    int gen_sort = 2;               // triangle order: 0 mesh, 1 Morton, 2 Morton for large meshes
    int early_exit = 0;             // search tiles may stop once no pair can count (rank mode)
    int search_pairs = 1;           // a set ranked against itself: tile pairs share the cross term
    int cus = 0;                    // compute units of the device
    std::vector<TimedLaunch> launches;
    std::vector<hipEvent_t> free_events;
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(RICI_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Makes the handle's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

hipEvent_t get_event(rici_ctx* h)
{
    if (!h->free_events.empty()) {
        hipEvent_t e = h->free_events.back();
        h->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs one launch, bracketed by events when timing is on.
template <class F>
hipError_t timed(rici_ctx* h, const char* name, hipStream_t s, F&& launch)
{
    if (!h->timing) return launch();
    TimedLaunch t{name, get_event(h), get_event(h)};
    if (t.start) (void)hipEventRecord(t.start, s);
    hipError_t e = launch();
    if (t.stop) (void)hipEventRecord(t.stop, s);
    if (t.start && t.stop) h->launches.push_back(t);
    return e;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ------------------------------------------------ static generation workspace
// rici_generate_noalloc keeps the triangle preparation records of at most
// RICI_NOALLOC_MAX_TRIANGLES triangles (bounding spheres, 64-triangle cluster
// spheres, vertices) in this array instead of the handle's growable scratch.
// Every GPU the library runs on holds one copy until the process ends.  In
// host code `scratch` only names the variable: its device address is looked up
// once per device (noalloc_address) and only that address is used.
constexpr size_t kNoallocCullBytes = ((size_t)RICI_NOALLOC_MAX_TRIANGLES * rici::kTriCullBytes + 255) & ~(size_t)255;
constexpr size_t kNoallocClusBytes =
    (((size_t)RICI_NOALLOC_MAX_TRIANGLES + 63) / 64 * rici::kTriCullBytes + 255) & ~(size_t)255;
constexpr size_t kNoallocVertBytes = ((size_t)RICI_NOALLOC_MAX_TRIANGLES * rici::kTriVertBytes + 255) & ~(size_t)255;
constexpr size_t kNoallocBytes = kNoallocCullBytes + kNoallocClusBytes + kNoallocVertBytes;

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices];
hipError_t g_noalloc_err[kMaxDevices];
bool g_noalloc_done[kMaxDevices];

// Device address of `scratch` on `device` (which must be current), looked up on
// the first call for that device and kept.  Returns the lookup's error code.
hipError_t noalloc_address(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_done[device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        g_noalloc_ptr[device] = p;
        g_noalloc_err[device] = e;
        g_noalloc_done[device] = true;
    }
    *out = g_noalloc_ptr[device];
    return g_noalloc_err[device];
}

// Grows the handle's scratch to at least `bytes` (synchronises the device).
int ensure_ws(rici_ctx* h, size_t bytes)
{
    if (bytes <= h->ws_size) return RICI_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    if (h->ws) {
        (void)hipFree(h->ws);
        h->ws = nullptr;
        h->ws_size = 0;
    }
    size_t want = bytes + bytes / 4;
    e = hipMalloc(&h->ws, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        h->ws = nullptr;
        e = hipMalloc(&h->ws, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            h->ws = nullptr;
            return fail(RICI_ERR_OOM, "cannot allocate %zu bytes of scratch", bytes);
        }
        want = bytes;
    }
    h->ws_size = want;
    return RICI_OK;
}

// image arrays are read and written with 16-byte vector accesses
bool misaligned(const void* p) { return ((uintptr_t)p & 15u) != 0; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb)
{
    if (!a || !b || na == 0 || nb == 0) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

}  // namespace

extern "C" {

const char* rici_last_error(void) { return g_last_error.c_str(); }

int rici_create(rici_handle* out, int device)
{
    if (!out) return fail(RICI_ERR_INVALID, "rici_create: out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(RICI_ERR_UNSUPPORTED, "rici_create: no HIP device");
    if (device < 0 || device >= count) return fail(RICI_ERR_INVALID, "rici_create: device %d of %d", device, count);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(RICI_ERR_UNSUPPORTED, "rici_create: device %d is %s, this library is built for gfx950",
                    device, prop.gcnArchName);
    DeviceGuard g(device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    rici_ctx* h = new rici_ctx();
    h->device = device;
    h->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    e = hipMalloc(&h->d_err, sizeof(uint32_t));
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipMalloc(error word)");
    }
    e = hipMemset(h->d_err, 0, sizeof(uint32_t));
    if (e != hipSuccess) {
        (void)hipFree(h->d_err);
        delete h;
        return hip_fail(e, "hipMemset(error word)");
    }
    // a failed lookup only disables rici_generate_noalloc (which reports it)
    (void)noalloc_address(device, &h->noalloc);
    *out = h;
    return RICI_OK;
}

void rici_destroy(rici_handle h)
{
    if (!h) return;
    DeviceGuard g(h->device);
    (void)hipDeviceSynchronize();
    for (auto& t : h->launches) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    for (auto e : h->free_events) (void)hipEventDestroy(e);
    if (h->ws) (void)hipFree(h->ws);
    if (h->d_err) (void)hipFree(h->d_err);
    delete h;
}

int rici_sync(rici_handle h, void* stream)
{
    if (!h) return fail(RICI_ERR_INVALID, "rici_sync: NULL handle");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    uint32_t word = 0;
    e = hipMemcpy(&word, h->d_err, sizeof word, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(error word)");
    h->last_dev_err = word;
    if (word) {
        e = hipMemset(h->d_err, 0, sizeof(uint32_t));
        if (e != hipSuccess) return hip_fail(e, "hipMemset(error word)");
        return fail(RICI_ERR_DEVICE, "device reported:%s%s%s",
                    (word & RICI_DEVERR_INDEX) ? " triangle index out of range" : "",
                    (word & RICI_DEVERR_NONFINITE) ? " non-finite coordinate" : "",
                    (word & RICI_DEVERR_QUEUE) ? " correlation settle queue full (ranks too low)" : "");
    }
    return RICI_OK;
}

uint32_t rici_device_errors(rici_handle h) { return h ? h->last_dev_err : 0u; }

}  // extern "C"

namespace {

// Argument checks shared by rici_generate and rici_generate_noalloc.
int check_generate_args(const char* fn, rici_handle h, const float* positions, uint32_t num_vertices,
                        const uint32_t* triangles, uint32_t num_triangles, const float* op_positions,
                        const float* op_normals, uint32_t num_points, float support_radius, const uint32_t* out_images)
{
    if (!h) return fail(RICI_ERR_INVALID, "%s: NULL handle", fn);
    if (!(isfinite(support_radius) && support_radius > 0.0f))
        return fail(RICI_ERR_INVALID, "%s: support_radius must be finite and > 0", fn);
    if (num_triangles >= (1u << 29)) return fail(RICI_ERR_UNSUPPORTED, "%s: num_triangles >= 2^29", fn);
    if (num_points >= (1u << 31)) return fail(RICI_ERR_UNSUPPORTED, "%s: num_points >= 2^31", fn);
    if (num_points == 0) return RICI_OK;
    if (!op_positions || !op_normals || !out_images)
        return fail(RICI_ERR_INVALID, "%s: NULL oriented-point or output pointer", fn);
    if (num_triangles > 0 && (!triangles || !positions || num_vertices == 0))
        return fail(RICI_ERR_INVALID, "%s: NULL mesh pointer or no vertices", fn);
    if (misaligned(out_images)) return fail(RICI_ERR_INVALID, "%s: out_images is not 16-byte aligned", fn);
    const size_t out_bytes = (size_t)num_points * rici::NPIX * sizeof(uint32_t);
    if (overlaps(out_images, out_bytes, positions, (size_t)num_vertices * 12) ||
        overlaps(out_images, out_bytes, triangles, (size_t)num_triangles * 12) ||
        overlaps(out_images, out_bytes, op_positions, (size_t)num_points * 12) ||
        overlaps(out_images, out_bytes, op_normals, (size_t)num_points * 12))
        return fail(RICI_ERR_INVALID, "%s: output overlaps an input", fn);
    return RICI_OK;
}

// Triangle preparation, cluster spheres and the generation kernel, with the
// preparation records at cull / clusters / verts.
int enqueue_generate(rici_ctx* h, const float* positions, uint32_t num_vertices, const uint32_t* triangles,
                     uint32_t num_triangles, const float* op_positions, const float* op_normals, uint32_t num_points,
                     float support_radius, uint32_t* out_images, float4* cull, float4* clusters, float4* verts,
                     hipStream_t s)
{
    hipError_t e = timed(h, "gen_prep", s, [&] {
        hipError_t e1 = rici::launch_gen_prep(positions, num_vertices, triangles, num_triangles, h->gen_sort, cull, verts,
                                              h->d_err, s);
        return e1 != hipSuccess ? e1 : rici::launch_gen_clusters(cull, num_triangles, clusters, s);
    });
    if (e != hipSuccess) return hip_fail(e, "gen_prep launch");
    e = timed(h, "gen", s, [&] {
        return rici::launch_gen(cull, clusters, verts, num_triangles, op_positions, op_normals, num_points,
                                support_radius, out_images, h->d_err, h->gen_group, s);
    });
    if (e != hipSuccess) return hip_fail(e, "gen launch");
    return RICI_OK;
}

}  // namespace

extern "C" {

int rici_generate(rici_handle h, const float* positions, uint32_t num_vertices, const uint32_t* triangles,
                  uint32_t num_triangles, const float* op_positions, const float* op_normals, uint32_t num_points,
                  float support_radius, uint32_t* out_images, void* stream)
{
    int rc = check_generate_args("rici_generate", h, positions, num_vertices, triangles, num_triangles, op_positions,
                                 op_normals, num_points, support_radius, out_images);
    if (rc || num_points == 0) return rc;
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    const size_t cull_bytes = align256((size_t)num_triangles * rici::kTriCullBytes);
    const size_t clus_bytes = align256(((size_t)num_triangles + 63) / 64 * rici::kTriCullBytes);
    const size_t vert_bytes = align256((size_t)num_triangles * rici::kTriVertBytes);
    rc = ensure_ws(h, cull_bytes + clus_bytes + vert_bytes + 256);
    if (rc) return rc;
    float4* cull = (float4*)h->ws;
    float4* clusters = (float4*)((char*)h->ws + cull_bytes);
    float4* verts = (float4*)((char*)h->ws + cull_bytes + clus_bytes);
    return enqueue_generate(h, positions, num_vertices, triangles, num_triangles, op_positions, op_normals, num_points,
                            support_radius, out_images, cull, clusters, verts, (hipStream_t)stream);
}

int rici_generate_noalloc(rici_handle h, const float* positions, uint32_t num_vertices, const uint32_t* triangles,
                          uint32_t num_triangles, const float* op_positions, const float* op_normals,
                          uint32_t num_points, float support_radius, uint32_t* out_images, void* stream)
{
    if (!h) return fail(RICI_ERR_INVALID, "rici_generate_noalloc: NULL handle");
    if (num_triangles > RICI_NOALLOC_MAX_TRIANGLES)
        return fail(RICI_ERR_UNSUPPORTED,
                    "rici_generate_noalloc: %u triangles exceed the static workspace of %u triangles "
                    "(use rici_generate)", num_triangles, (unsigned)RICI_NOALLOC_MAX_TRIANGLES);
    int rc = check_generate_args("rici_generate_noalloc", h, positions, num_vertices, triangles, num_triangles,
                                 op_positions, op_normals, num_points, support_radius, out_images);
    if (rc) return rc;
    if (!h->noalloc) {
        void* p = nullptr;
        hipError_t e = noalloc_address(h->device, &p);
        return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                        "rici_generate_noalloc: hipGetSymbolAddress(static workspace)");
    }
    if (num_points == 0) return RICI_OK;
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    char* base = (char*)h->noalloc;
    float4* cull = (float4*)base;
    float4* clusters = (float4*)(base + kNoallocCullBytes);
    float4* verts = (float4*)(base + kNoallocCullBytes + kNoallocClusBytes);
    // no event bracketing: timing would create events
    const bool timing = h->timing;
    h->timing = false;
    rc = enqueue_generate(h, positions, num_vertices, triangles, num_triangles, op_positions, op_normals, num_points,
                          support_radius, out_images, cull, clusters, verts, (hipStream_t)stream);
    h->timing = timing;
    return rc;
}

namespace {

struct SearchScratch {
    rici::SearchPrep np, hp;
    int32_t* thr = nullptr;
    int64_t* dstar = nullptr;
    uint32_t* lists = nullptr;
};

int search_scratch(rici_ctx* h, uint32_t nn, uint32_t nh, bool want_dstar, SearchScratch& S)
{
    const size_t ga = rici::search_groups(nn);
    const size_t hslots = rici::haystack_slots(nh), gb = hslots / rici::kGroup;
    const size_t a_planes = align256(2 * ga * rici::kPlaneGroupBytes);
    const size_t b_planes = align256(3 * gb * rici::kPlaneGroupBytes);
    const size_t sumsq = align256(ga * rici::kGroup * sizeof(int64_t));
    const size_t nmax = align256(ga * rici::kGroup * sizeof(uint32_t));
    const size_t hmax = align256(hslots * sizeof(uint32_t));
    const size_t hmax_img = align256((size_t)nh * sizeof(uint32_t));
    const size_t hperm = align256(hslots * sizeof(uint32_t));
    const size_t thr = align256((size_t)nn * sizeof(int32_t));
    const size_t dstar = want_dstar ? align256((size_t)nn * sizeof(int64_t)) : 0;
    const size_t lists = align256((2 + (size_t)nn + nh) * sizeof(uint32_t));
    const size_t total = a_planes + b_planes + sumsq + nmax + hmax + hmax_img + hperm + thr + dstar + lists;
    int rc = ensure_ws(h, total);
    if (rc) return rc;
    char* p = (char*)h->ws;
    S.np.planes = (int8_t*)p; p += a_planes;
    S.hp.planes = (int8_t*)p; p += b_planes;
    S.np.sumsq = (int64_t*)p; p += sumsq;
    S.hp.sumsq = nullptr;
    S.np.maxabs = (uint32_t*)p; p += nmax;
    S.np.maxabs_img = S.np.maxabs;
    S.np.perm = nullptr;
    S.hp.maxabs = (uint32_t*)p; p += hmax;
    S.hp.maxabs_img = (uint32_t*)p; p += hmax_img;
    S.hp.perm = (uint32_t*)p; p += hperm;
    S.thr = (int32_t*)p; p += thr;
    S.dstar = want_dstar ? (int64_t*)p : nullptr; p += dstar;
    S.lists = (uint32_t*)p;
    S.np.ngroups = (uint32_t)ga;
    S.hp.ngroups = (uint32_t)gb;
    S.np.inv = S.hp.inv = nullptr;
    return RICI_OK;
}

// Whether a rank call takes the paired path: one set ranked against itself,
// square tiles, no early exit.
bool use_pairs(const rici_ctx* h, const uint32_t* needles, uint32_t nn, const uint32_t* hay, uint32_t nh)
{
    return h->search_pairs && h->search_variant == 0 && !h->early_exit && needles == hay && nn == nh;
}

// The paired path of rici_distance_rank: needles and haystack in one slot
// order, the tile pairs (I <= J) searched by a persistent kernel, each
// workgroup holding one cross-term slot.
int rank_paired(rici_ctx* h, const uint32_t* images, uint32_t n, const uint32_t* true_index, uint32_t* out_rank,
                int64_t* out_true_distance, hipStream_t s)
{
    const size_t hslots = rici::haystack_slots(n), gb = hslots / rici::kGroup;
    const uint32_t tiles = (uint32_t)(hslots / rici::search_tile_n());
    const uint32_t items = rici::paired_items(tiles);
    const uint32_t grid = std::min<uint32_t>((uint32_t)h->cus, items);
    const size_t a_planes = align256(2 * gb * rici::kPlaneGroupBytes);
    const size_t b_planes = align256(3 * gb * rici::kPlaneGroupBytes);
    const size_t sumsq = align256((size_t)n * sizeof(int64_t));
    const size_t slot_u32 = align256(hslots * sizeof(uint32_t));
    const size_t img_u32 = align256((size_t)n * sizeof(uint32_t));
    const size_t flags = align256((size_t)tiles * sizeof(uint32_t));
    const size_t dstar = out_true_distance ? 0 : align256((size_t)n * sizeof(int64_t));
    const size_t lists = align256((2 + 2 * (size_t)n) * sizeof(uint32_t));
    const size_t counters = 256;
    const size_t cross = (size_t)grid * rici::paired_slot_bytes();
    // planes, sumsq, maxabs/perm/thr per slot, maxabs/inv per image, flags, ...
    const size_t total = a_planes + b_planes + sumsq + 3 * slot_u32 + 2 * img_u32 + flags + dstar + lists + counters +
                         cross;
    int rc = ensure_ws(h, total);
    if (rc) return rc;
    char* p = (char*)h->ws;
    rici::SearchPrep np = {}, hp = {};
    np.planes = (int8_t*)p; p += a_planes;
    hp.planes = (int8_t*)p; p += b_planes;
    np.sumsq = (int64_t*)p; p += sumsq;
    hp.maxabs = (uint32_t*)p; p += slot_u32;
    hp.perm = (uint32_t*)p; p += slot_u32;
    int32_t* thr = (int32_t*)p; p += slot_u32;
    hp.maxabs_img = (uint32_t*)p; p += img_u32;
    hp.inv = (uint32_t*)p; p += img_u32;
    uint32_t* tile_flags = (uint32_t*)p; p += flags;
    int64_t* ds = out_true_distance ? out_true_distance : (int64_t*)p; p += dstar;
    uint32_t* lst = (uint32_t*)p; p += lists;
    uint32_t* cnt = (uint32_t*)p; p += counters;
    int32_t* cslots = (int32_t*)p;
    np.maxabs = np.maxabs_img = hp.maxabs_img;   // per image (the needle pass writes no statistics)
    np.ngroups = hp.ngroups = (uint32_t)gb;

    // statistics, true-match distances, thresholds and planes
    hipError_t e = timed(h, "paired_prep", s, [&] {
        return rici::launch_paired_prep(images, n, true_index, np, hp, thr, tile_flags, ds, out_rank, s);
    });
    if (e != hipSuccess) return hip_fail(e, "paired_prep launch");
    rici::SearchArgs A = {};
    A.a_planes = np.planes; A.a_groups = (uint32_t)gb; A.nn = n;
    A.b_planes = hp.planes; A.b_groups = (uint32_t)gb; A.nh = n;
    A.nmax = hp.maxabs; A.hmax = hp.maxabs; A.hperm = hp.perm;
    A.thr = thr; A.sumsq = np.sumsq; A.rank = out_rank; A.matrix = nullptr;
    A.tiles_m = A.tiles_n = tiles;
    A.paired = 1; A.nperm = hp.perm; A.tile_flags = tile_flags; A.cross = cslots;
    e = timed(h, "search", s, [&] { return rici::launch_search_paired(A, grid, cnt, s); });
    if (e != hipSuccess) return hip_fail(e, "search launch");
    e = timed(h, "fallback", s, [&] {
        return rici::launch_fallback(images, n, images, n, hp.maxabs_img, hp.maxabs_img, ds, out_rank, nullptr, lst,
                                     s);
    });
    if (e != hipSuccess) return hip_fail(e, "fallback launch");
    return RICI_OK;
}

int check_search_args(const char* fn, const uint32_t* needles, uint32_t nn, const uint32_t* hay, uint32_t nh)
{
    if (nn > 0 && !needles) return fail(RICI_ERR_INVALID, "%s: NULL needles", fn);
    if (nh == 0 && nn > 0) return fail(RICI_ERR_INVALID, "%s: empty haystack", fn);
    if (nh > 0 && !hay) return fail(RICI_ERR_INVALID, "%s: NULL haystack", fn);
    if (nn >= (1u << 31) || nh >= (1u << 31)) return fail(RICI_ERR_UNSUPPORTED, "%s: more than 2^31 images", fn);
    if ((nn > 0 && misaligned(needles)) || (nh > 0 && misaligned(hay)))
        return fail(RICI_ERR_INVALID, "%s: image arrays must be 16-byte aligned", fn);
    return RICI_OK;
}

int prep_both(rici_ctx* h, SearchScratch& S, const uint32_t* needles, uint32_t nn, const uint32_t* hay, uint32_t nh,
              hipStream_t s)
{
    hipError_t e = timed(h, "delta_needle", s, [&] { return rici::launch_delta_prep(needles, nn, 1, S.np, s); });
    if (e != hipSuccess) return hip_fail(e, "delta_needle launch");
    // a set ranked against itself: the haystack's max |D| comes from the needle pass
    const uint32_t* known = (hay == needles && nh == nn) ? S.np.maxabs : nullptr;
    e = timed(h, "delta_haystack", s, [&] { return rici::launch_delta_prep(hay, nh, 0, S.hp, s, known); });
    if (e != hipSuccess) return hip_fail(e, "delta_haystack launch");
    return RICI_OK;
}

}  // namespace

int rici_distance_rank(rici_handle h, const uint32_t* needles, uint32_t num_needles, const uint32_t* haystack,
                       uint32_t num_haystack, const uint32_t* true_index, uint32_t* out_rank,
                       int64_t* out_true_distance, void* stream)
{
    if (!h) return fail(RICI_ERR_INVALID, "rici_distance_rank: NULL handle");
    int rc = check_search_args("rici_distance_rank", needles, num_needles, haystack, num_haystack);
    if (rc) return rc;
    if (num_needles == 0) return RICI_OK;
    if (!true_index || !out_rank) return fail(RICI_ERR_INVALID, "rici_distance_rank: NULL true_index or out_rank");
    const size_t nb = (size_t)num_needles;
    const size_t img_n = nb * rici::NPIX * 4, img_h = (size_t)num_haystack * rici::NPIX * 4;
    if (overlaps(out_rank, nb * 4, needles, img_n) || overlaps(out_rank, nb * 4, haystack, img_h) ||
        overlaps(out_rank, nb * 4, true_index, nb * 4) ||
        (out_true_distance && (overlaps(out_true_distance, nb * 8, needles, img_n) ||
                               overlaps(out_true_distance, nb * 8, haystack, img_h) ||
                               overlaps(out_true_distance, nb * 8, out_rank, nb * 4) ||
                               overlaps(out_true_distance, nb * 8, true_index, nb * 4))))
        return fail(RICI_ERR_INVALID, "rici_distance_rank: an output overlaps another array");

    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (use_pairs(h, needles, num_needles, haystack, num_haystack))
        return rank_paired(h, needles, num_needles, true_index, out_rank, out_true_distance, s);
    SearchScratch S;
    rc = search_scratch(h, num_needles, num_haystack, out_true_distance == nullptr, S);
    if (rc) return rc;
    int64_t* dstar = out_true_distance ? out_true_distance : S.dstar;
    rc = prep_both(h, S, needles, num_needles, haystack, num_haystack, s);
    if (rc) return rc;
    hipError_t e = timed(h, "true_distance", s, [&] {
        return rici::launch_true_distance(needles, num_needles, haystack, num_haystack, true_index, S.np.sumsq,
                                          S.np.maxabs, dstar, S.thr, out_rank, s);
    });
    if (e != hipSuccess) return hip_fail(e, "true_distance launch");
    e = timed(h, "search", s, [&] {
        return rici::launch_search(S.np, num_needles, S.hp, num_haystack, S.thr, S.np.sumsq, out_rank, nullptr,
                                   h->search_variant, h->early_exit, s);
    });
    if (e != hipSuccess) return hip_fail(e, "search launch");
    e = timed(h, "fallback", s, [&] {
        return rici::launch_fallback(needles, num_needles, haystack, num_haystack, S.np.maxabs, S.hp.maxabs_img, dstar,
                                     out_rank, nullptr, S.lists, s);
    });
    if (e != hipSuccess) return hip_fail(e, "fallback launch");
    return RICI_OK;
}

int rici_distance_matrix(rici_handle h, const uint32_t* needles, uint32_t num_needles, const uint32_t* haystack,
                         uint32_t num_haystack, int64_t* out, void* stream)
{
    if (!h) return fail(RICI_ERR_INVALID, "rici_distance_matrix: NULL handle");
    int rc = check_search_args("rici_distance_matrix", needles, num_needles, haystack, num_haystack);
    if (rc) return rc;
    if (num_needles == 0) return RICI_OK;
    if (!out) return fail(RICI_ERR_INVALID, "rici_distance_matrix: NULL out");
    const size_t ob = (size_t)num_needles * num_haystack * 8;
    if (overlaps(out, ob, needles, (size_t)num_needles * rici::NPIX * 4) ||
        overlaps(out, ob, haystack, (size_t)num_haystack * rici::NPIX * 4))
        return fail(RICI_ERR_INVALID, "rici_distance_matrix: output overlaps an input");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    SearchScratch S;
    rc = search_scratch(h, num_needles, num_haystack, false, S);
    if (rc) return rc;
    rc = prep_both(h, S, needles, num_needles, haystack, num_haystack, s);
    if (rc) return rc;
    hipError_t e = timed(h, "matrix", s, [&] {
        return rici::launch_search(S.np, num_needles, S.hp, num_haystack, nullptr, S.np.sumsq, nullptr, out,
                                   h->search_variant, 0, s);
    });
    if (e != hipSuccess) return hip_fail(e, "matrix launch");
    e = timed(h, "fallback", s, [&] {
        return rici::launch_fallback(needles, num_needles, haystack, num_haystack, S.np.maxabs, S.hp.maxabs_img, nullptr,
                                     nullptr, out, S.lists, s);
    });
    if (e != hipSuccess) return hip_fail(e, "fallback launch");
    return RICI_OK;
}

// ---------------------------------------------------------------- clutter

int rici_clutter_areas(rici_handle h, const float* positions, uint32_t num_vertices, const uint32_t* triangles,
                       uint32_t num_triangles, uint32_t object_first, uint32_t object_count,
                       const float* op_positions, const float* op_normals, uint32_t num_points,
                       float support_radius, double* out_area_all, double* out_area_object, void* stream)
{
    if (!h) return fail(RICI_ERR_INVALID, "rici_clutter_areas: NULL handle");
    if (!(isfinite(support_radius) && support_radius > 0.0f))
        return fail(RICI_ERR_INVALID, "rici_clutter_areas: support_radius must be finite and > 0");
    if (num_points >= (1u << 31)) return fail(RICI_ERR_UNSUPPORTED, "rici_clutter_areas: num_points >= 2^31");
    if (num_points == 0) return RICI_OK;
    if (!op_positions || !op_normals || !out_area_all || !out_area_object)
        return fail(RICI_ERR_INVALID, "rici_clutter_areas: NULL oriented-point or output pointer");
    if (num_triangles > 0 && (!triangles || !positions || num_vertices == 0))
        return fail(RICI_ERR_INVALID, "rici_clutter_areas: NULL mesh pointer or no vertices");
    const size_t ob = (size_t)num_points * 8;
    if (overlaps(out_area_all, ob, out_area_object, ob) ||
        overlaps(out_area_all, ob, positions, (size_t)num_vertices * 12) ||
        overlaps(out_area_object, ob, positions, (size_t)num_vertices * 12) ||
        overlaps(out_area_all, ob, triangles, (size_t)num_triangles * 12) ||
        overlaps(out_area_object, ob, triangles, (size_t)num_triangles * 12))
        return fail(RICI_ERR_INVALID, "rici_clutter_areas: an output overlaps another array");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = timed(h, "clutter", s, [&] {
        return rici::launch_clutter(positions, num_vertices, triangles, num_triangles, object_first, object_count,
                                    op_positions, op_normals, num_points, support_radius, out_area_all,
                                    out_area_object, h->d_err, s);
    });
    if (e != hipSuccess) return hip_fail(e, "clutter launch");
    return RICI_OK;
}

// ------------------------------------------------------------ spin images

int rici_spin_generate(rici_handle h, const float* samples, uint32_t num_samples, const float* op_positions,
                       const float* op_normals, uint32_t num_points, float support_radius, float* out_images,
                       void* stream)
{
    if (!h) return fail(RICI_ERR_INVALID, "rici_spin_generate: NULL handle");
    if (!(isfinite(support_radius) && support_radius > 0.0f))
        return fail(RICI_ERR_INVALID, "rici_spin_generate: support_radius must be finite and > 0");
    if (num_points >= (1u << 31) || num_samples >= (1u << 31))
        return fail(RICI_ERR_UNSUPPORTED, "rici_spin_generate: more than 2^31 points or samples");
    if (num_points == 0) return RICI_OK;
    if (!op_positions || !op_normals || !out_images)
        return fail(RICI_ERR_INVALID, "rici_spin_generate: NULL oriented-point or output pointer");
    if (num_samples > 0 && !samples) return fail(RICI_ERR_INVALID, "rici_spin_generate: NULL samples");
    if (misaligned(out_images)) return fail(RICI_ERR_INVALID, "rici_spin_generate: out_images is not 16-byte aligned");
    const size_t ob = (size_t)num_points * rici::NPIX * sizeof(float);
    if (overlaps(out_images, ob, samples, (size_t)num_samples * 12) ||
        overlaps(out_images, ob, op_positions, (size_t)num_points * 12) ||
        overlaps(out_images, ob, op_normals, (size_t)num_points * 12))
        return fail(RICI_ERR_INVALID, "rici_spin_generate: output overlaps an input");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = timed(h, "spin_gen", s, [&] {
        return rici::launch_spin_gen(samples, num_samples, op_positions, op_normals, num_points, support_radius,
                                     out_images, h->d_err, s);
    });
    if (e != hipSuccess) return hip_fail(e, "spin_gen launch");
    return RICI_OK;
}

}  // extern "C"

namespace {

struct SpinScratch {
    rici::SpinPrep np, hp;
    double* rho_t = nullptr;
    uint2* queue = nullptr;
    uint32_t* queue_count = nullptr;
    uint32_t queue_cap = 0;
};

int check_spin_args(const char* fn, const float* needles, uint32_t nn, const float* hay, uint32_t nh)
{
    if (nn > 0 && !needles) return fail(RICI_ERR_INVALID, "%s: NULL needles", fn);
    if (nh == 0 && nn > 0) return fail(RICI_ERR_INVALID, "%s: empty haystack", fn);
    if (nh > 0 && !hay) return fail(RICI_ERR_INVALID, "%s: NULL haystack", fn);
    if (nn >= (1u << 31) || nh >= (1u << 31)) return fail(RICI_ERR_UNSUPPORTED, "%s: more than 2^31 images", fn);
    return RICI_OK;
}

// z planes and statistics of both sets (one set when the needles are the
// haystack), true correlations and the queue of pairs near the threshold
int spin_prep(rici_ctx* h, const float* needles, uint32_t nn, const float* hay, uint32_t nh, bool ranks,
              SpinScratch& S, hipStream_t s)
{
    const bool same = needles == hay && nn == nh;
    const size_t sa = rici::spin_slots(nn), sb = same ? 0 : rici::spin_slots(nh);
    const uint64_t pairs = (uint64_t)nn * nh;
    const uint64_t want = std::max<uint64_t>((uint64_t)1 << 20, (uint64_t)1024 * nn);
    S.queue_cap = ranks ? (uint32_t)std::min<uint64_t>(std::min<uint64_t>(pairs, want), (uint64_t)1 << 30) : 0u;
    const size_t za = align256(sa * rici::NPIX * sizeof(float)), zb = align256(sb * rici::NPIX * sizeof(float));
    const size_t st_a = align256(sa * 2 * sizeof(double)), st_b = align256(sb * 2 * sizeof(double));
    const size_t rt = ranks ? align256((size_t)nn * sizeof(double)) : 0;
    const size_t qb = align256((size_t)S.queue_cap * sizeof(uint2)), qc = ranks ? 256 : 0;
    int rc = ensure_ws(h, za + zb + st_a + st_b + rt + qb + qc);
    if (rc) return rc;
    char* p = (char*)h->ws;
    S.np.z = (float*)p; p += za;
    S.np.mean = (double*)p; S.np.norm = S.np.mean + sa; p += st_a;
    if (same) {
        S.hp = S.np;
    } else {
        S.hp.z = (float*)p; p += zb;
        S.hp.mean = (double*)p; S.hp.norm = S.hp.mean + sb; p += st_b;
    }
    S.rho_t = ranks ? (double*)p : nullptr; p += rt;
    S.queue = ranks ? (uint2*)p : nullptr; p += qb;
    S.queue_count = ranks ? (uint32_t*)p : nullptr;
    hipError_t e = timed(h, "spin_zprep", s, [&] {
        hipError_t e1 = rici::launch_spin_zprep(needles, nn, S.np.z, S.np.mean, S.np.norm, s);
        if (e1 == hipSuccess && !same) e1 = rici::launch_spin_zprep(hay, nh, S.hp.z, S.hp.mean, S.hp.norm, s);
        return e1;
    });
    if (e != hipSuccess) return hip_fail(e, "spin_zprep launch");
    return RICI_OK;
}

}  // namespace

extern "C" {

int rici_spin_rank(rici_handle h, const float* needles, uint32_t num_needles, const float* haystack,
                   uint32_t num_haystack, const uint32_t* true_index, uint32_t* out_rank,
                   double* out_true_correlation, void* stream)
{
    if (!h) return fail(RICI_ERR_INVALID, "rici_spin_rank: NULL handle");
    int rc = check_spin_args("rici_spin_rank", needles, num_needles, haystack, num_haystack);
    if (rc) return rc;
    if (num_needles == 0) return RICI_OK;
    if (!true_index || !out_rank) return fail(RICI_ERR_INVALID, "rici_spin_rank: NULL true_index or out_rank");
    const size_t nb = num_needles;
    const size_t img_n = nb * rici::NPIX * 4, img_h = (size_t)num_haystack * rici::NPIX * 4;
    if (overlaps(out_rank, nb * 4, needles, img_n) || overlaps(out_rank, nb * 4, haystack, img_h) ||
        overlaps(out_rank, nb * 4, true_index, nb * 4) ||
        (out_true_correlation && (overlaps(out_true_correlation, nb * 8, needles, img_n) ||
                                  overlaps(out_true_correlation, nb * 8, haystack, img_h) ||
                                  overlaps(out_true_correlation, nb * 8, out_rank, nb * 4) ||
                                  overlaps(out_true_correlation, nb * 8, true_index, nb * 4))))
        return fail(RICI_ERR_INVALID, "rici_spin_rank: an output overlaps another array");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    SpinScratch S;
    rc = spin_prep(h, needles, num_needles, haystack, num_haystack, true, S, s);
    if (rc) return rc;
    double* rho_t = out_true_correlation ? out_true_correlation : S.rho_t;
    const char* names[3] = {"spin_true", "spin_search", "spin_settle"};
    for (int part = 1; part <= 3; ++part) {
        hipError_t e = timed(h, names[part - 1], s, [&] {
            return rici::launch_spin_rank(S.np, needles, num_needles, S.hp, haystack, num_haystack, true_index,
                                          rho_t, out_rank, S.queue, S.queue_count, S.queue_cap, h->d_err, s, part);
        });
        if (e != hipSuccess) return hip_fail(e, "spin rank launch");
    }
    return RICI_OK;
}

int rici_spin_correlation_matrix(rici_handle h, const float* needles, uint32_t num_needles, const float* haystack,
                                 uint32_t num_haystack, float* out, void* stream)
{
    if (!h) return fail(RICI_ERR_INVALID, "rici_spin_correlation_matrix: NULL handle");
    int rc = check_spin_args("rici_spin_correlation_matrix", needles, num_needles, haystack, num_haystack);
    if (rc) return rc;
    if (num_needles == 0) return RICI_OK;
    if (!out) return fail(RICI_ERR_INVALID, "rici_spin_correlation_matrix: NULL out");
    const size_t ob = (size_t)num_needles * num_haystack * 4;
    if (overlaps(out, ob, needles, (size_t)num_needles * rici::NPIX * 4) ||
        overlaps(out, ob, haystack, (size_t)num_haystack * rici::NPIX * 4))
        return fail(RICI_ERR_INVALID, "rici_spin_correlation_matrix: output overlaps an input");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    SpinScratch S;
    rc = spin_prep(h, needles, num_needles, haystack, num_haystack, false, S, s);
    if (rc) return rc;
    hipError_t e = timed(h, "spin_matrix", s, [&] {
        return rici::launch_spin_matrix(S.np, num_needles, S.hp, num_haystack, out, s);
    });
    if (e != hipSuccess) return hip_fail(e, "spin_matrix launch");
    return RICI_OK;
}

int rici_set_tuning(rici_handle h, const char* key, int value)
{
    if (!h || !key) return fail(RICI_ERR_INVALID, "rici_set_tuning: NULL handle or key");
    if (strcmp(key, "search_early_exit") == 0) {
        if (value != 0 && value != 1)
            return fail(RICI_ERR_INVALID, "rici_set_tuning: search_early_exit must be 0 or 1 (got %d)", value);
        h->early_exit = value;
        return RICI_OK;
    }
    if (strcmp(key, "gen_sort_triangles") == 0) {
        if (value < 0 || value > 2)
            return fail(RICI_ERR_INVALID, "rici_set_tuning: gen_sort_triangles must be 0, 1 or 2 (got %d)", value);
        h->gen_sort = value;
        return RICI_OK;
    }
    if (strcmp(key, "gen_images_per_group") == 0) {
        if (value != 4 && value != 2)
            return fail(RICI_ERR_INVALID, "rici_set_tuning: gen_images_per_group must be 4 or 2 (got %d)", value);
        h->gen_group = value;
        return RICI_OK;
    }
    if (strcmp(key, "search_tile_m") == 0) {
        if (value != 256 && value != 128)
            return fail(RICI_ERR_INVALID, "rici_set_tuning: search_tile_m must be 256 or 128 (got %d)", value);
        h->search_variant = value == 128 ? 1 : 0;
        return RICI_OK;
    }
    if (strcmp(key, "search_pairs") == 0) {
        if (value != 0 && value != 1)
            return fail(RICI_ERR_INVALID, "rici_set_tuning: search_pairs must be 0 or 1 (got %d)", value);
        h->search_pairs = value;
        return RICI_OK;
    }
    return fail(RICI_ERR_INVALID, "rici_set_tuning: unknown key '%s'", key);
}

int rici_get_tuning(rici_handle h, const char* key, int* value)
{
    if (!h || !key || !value) return fail(RICI_ERR_INVALID, "rici_get_tuning: NULL argument");
    if (strcmp(key, "gen_images_per_group") == 0) {
        *value = h->gen_group;
        return RICI_OK;
    }
    if (strcmp(key, "search_early_exit") == 0) {
        *value = h->early_exit;
        return RICI_OK;
    }
    if (strcmp(key, "gen_sort_triangles") == 0) {
        *value = h->gen_sort;
        return RICI_OK;
    }
    if (strcmp(key, "search_tile_m") == 0) {
        *value = (int)rici::search_tile_m(h->search_variant);
        return RICI_OK;
    }
    if (strcmp(key, "search_pairs") == 0) {
        *value = h->search_pairs;
        return RICI_OK;
    }
    return fail(RICI_ERR_INVALID, "rici_get_tuning: unknown key '%s'", key);
}

int rici_timing_enable(rici_handle h, int on)
{
    if (!h) return fail(RICI_ERR_INVALID, "rici_timing_enable: NULL handle");
    h->timing = on != 0;
    return RICI_OK;
}

int rici_timing_reset(rici_handle h)
{
    if (!h) return fail(RICI_ERR_INVALID, "rici_timing_reset: NULL handle");
    DeviceGuard g(h->device);
    (void)hipDeviceSynchronize();
    for (auto& t : h->launches) {
        h->free_events.push_back(t.start);
        h->free_events.push_back(t.stop);
    }
    h->launches.clear();
    return RICI_OK;
}

int rici_timing_get(rici_handle h, const char* kernel, double* total_ms, uint64_t* launches)
{
    if (!h || !kernel || !total_ms || !launches) return fail(RICI_ERR_INVALID, "rici_timing_get: NULL argument");
    DeviceGuard g(h->device);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    double sum = 0.0;
    uint64_t n = 0;
    for (auto& t : h->launches) {
        if (strcmp(t.name, kernel) != 0) continue;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, t.start, t.stop);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        sum += ms;
        ++n;
    }
    *total_ms = sum;
    *launches = n;
    return RICI_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batched plans

struct rici_batch_ctx {
    rici_ctx* h = nullptr;
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int search_variant = 0;
    // recorded inside the graph around the two persistent kernels:
    // [0, 1] generation, [2, 3] search
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool has_gen = false, has_search = false, timing_ok = false;
};

namespace {

bool job_ok(const rici_mesh_job& j, uint32_t k)
{
    if (j.num_points == 0) return true;
    if (!j.op_positions || !j.op_normals || !j.out_images) {
        fail(RICI_ERR_INVALID, "rici_batch_create: job %u has a NULL oriented-point or image pointer", k);
        return false;
    }
    if (misaligned(j.out_images)) {
        fail(RICI_ERR_INVALID, "rici_batch_create: job %u: out_images is not 16-byte aligned", k);
        return false;
    }
    if (j.num_triangles > 0 && (!j.triangles || !j.positions || j.num_vertices == 0)) {
        fail(RICI_ERR_INVALID, "rici_batch_create: job %u has a NULL mesh pointer", k);
        return false;
    }
    if (j.num_triangles >= (1u << 29) || j.num_points >= (1u << 31)) {
        fail(RICI_ERR_UNSUPPORTED, "rici_batch_create: job %u is beyond the size limits", k);
        return false;
    }
    if (j.true_index && !j.out_rank) {
        fail(RICI_ERR_INVALID, "rici_batch_create: job %u has true_index but no out_rank", k);
        return false;
    }
    return true;
}

void destroy_plan(rici_batch_ctx* b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->scratch) (void)hipFree(b->scratch);
    for (hipEvent_t e : b->ev)
        if (e) (void)hipEventDestroy(e);
    delete b;
}

}  // namespace

extern "C" {

int rici_batch_create(rici_handle h, const rici_mesh_job* jobs, uint32_t num_jobs, float support_radius,
                      rici_batch* out)
{
    if (!out) return fail(RICI_ERR_INVALID, "rici_batch_create: out is NULL");
    *out = nullptr;
    if (!h) return fail(RICI_ERR_INVALID, "rici_batch_create: NULL handle");
    if (num_jobs > 0 && !jobs) return fail(RICI_ERR_INVALID, "rici_batch_create: NULL jobs");
    if (!(isfinite(support_radius) && support_radius > 0.0f))
        return fail(RICI_ERR_INVALID, "rici_batch_create: support_radius must be finite and > 0");
    for (uint32_t k = 0; k < num_jobs; ++k)
        if (!job_ok(jobs[k], k)) return RICI_ERR_INVALID;

    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, h->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    const int gen_group = h->gen_group;
    uint32_t gen_grid = 0;   // as many persistent generation workgroups as fit at once
    e = rici::gen_batched_grid(gen_group, prop.multiProcessorCount, &gen_grid);
    if (e != hipSuccess) return hip_fail(e, "rici_batch_create: occupancy");
    const uint32_t grid = (uint32_t)prop.multiProcessorCount;   // search: one resident workgroup per CU

    // generation jobs, largest triangle count first (longest items start first)
    std::vector<uint32_t> gorder;
    for (uint32_t k = 0; k < num_jobs; ++k)
        if (jobs[k].num_points > 0) gorder.push_back(k);
    std::stable_sort(gorder.begin(), gorder.end(),
                     [&](uint32_t a, uint32_t b2) { return jobs[a].num_triangles > jobs[b2].num_triangles; });
    // ranking jobs, most tiles first
    std::vector<uint32_t> sorder;
    for (uint32_t k = 0; k < num_jobs; ++k)
        if (jobs[k].num_points > 0 && jobs[k].true_index) sorder.push_back(k);
    std::stable_sort(sorder.begin(), sorder.end(),
                     [&](uint32_t a, uint32_t b2) { return jobs[a].num_points > jobs[b2].num_points; });

    const uint32_t G = rici::gen_group_images(gen_group);
    const int variant = h->search_variant;
    const size_t tm = rici::search_tile_m(variant), tn = rici::search_tile_n();

    // generation scratch (triangle soup); the search scratch reuses the same
    // memory because it is only written after generation has finished
    size_t gen_bytes = 0;
    std::vector<size_t> goff(gorder.size());
    for (size_t i = 0; i < gorder.size(); ++i) {
        const rici_mesh_job& j = jobs[gorder[i]];
        goff[i] = gen_bytes;
        gen_bytes += align256((size_t)j.num_triangles * rici::kTriCullBytes) +
                     align256(((size_t)j.num_triangles + 63) / 64 * rici::kTriCullBytes) +
                     align256((size_t)j.num_triangles * rici::kTriVertBytes);
    }
    // paired sets (each mesh ranked against itself): needle planes in the
    // haystack's slot order, thresholds per slot, tile flags, and one
    // cross-term slot per persistent search workgroup
    const bool paired = h->search_pairs && variant == 0 && !h->early_exit;
    auto needle_groups = [&](uint32_t n) {
        return paired ? rici::haystack_slots(n) / rici::kGroup : rici::search_groups(n);
    };
    size_t srch_bytes = 0;
    std::vector<size_t> soff(sorder.size());
    for (size_t i = 0; i < sorder.size(); ++i) {
        const uint32_t n = jobs[sorder[i]].num_points;
        const size_t ga = needle_groups(n), hs = rici::haystack_slots(n), gb = hs / rici::kGroup;
        soff[i] = srch_bytes;
        srch_bytes += align256(2 * ga * rici::kPlaneGroupBytes) + align256(3 * gb * rici::kPlaneGroupBytes) +
                      align256(ga * rici::kGroup * 8) + align256(ga * rici::kGroup * 4) + align256(hs * 4) +
                      align256((size_t)n * 4) + align256(hs * 4) + align256(std::max<size_t>(hs, n) * 4) +
                      align256((size_t)n * 8) + align256((2 + 2 * (size_t)n) * 4) +
                      (paired ? align256((size_t)n * 4) + align256(hs / tn * 4) : 0);
    }
    const size_t cross_bytes = paired && !sorder.empty() ? (size_t)grid * rici::paired_slot_bytes() : 0;
    const size_t tables = align256(gorder.size() * sizeof(rici::GenJob)) +
                          align256(sorder.size() * sizeof(rici::SearchJob)) + 256 + cross_bytes;
    const size_t total = tables + std::max(gen_bytes, srch_bytes);

    rici_batch_ctx* b = new rici_batch_ctx();
    b->h = h;
    b->search_variant = variant;
    e = hipMalloc(&b->scratch, total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b->scratch = nullptr;
        destroy_plan(b);
        return fail(RICI_ERR_OOM, "rici_batch_create: cannot allocate %zu bytes of scratch", total);
    }
    b->scratch_bytes = total;
    char* base = (char*)b->scratch;
    rici::GenJob* d_gjobs = (rici::GenJob*)base;
    rici::SearchJob* d_sjobs = (rici::SearchJob*)(base + align256(gorder.size() * sizeof(rici::GenJob)));
    uint32_t* d_counters = (uint32_t*)(base + tables - cross_bytes - 256);
    int32_t* d_cross = cross_bytes ? (int32_t*)(base + tables - cross_bytes) : nullptr;
    char* work = base + tables;

    // ---- generation table
    std::vector<rici::GenJob> gj(gorder.size());
    uint64_t blocks = 0, chunks = 0;
    uint32_t items = 0;
    for (size_t i = 0; i < gorder.size(); ++i) {
        const rici_mesh_job& j = jobs[gorder[i]];
        rici::GenJob& J = gj[i];
        J.pos = j.positions; J.nv = j.num_vertices; J.tri = j.triangles; J.nt = j.num_triangles;
        J.op_pos = j.op_positions; J.op_nrm = j.op_normals; J.n = j.num_points; J.out = j.out_images;
        char* p = work + goff[i];
        J.cull = (float4*)p; p += align256((size_t)j.num_triangles * rici::kTriCullBytes);
        J.clusters = (float4*)p; p += align256(((size_t)j.num_triangles + 63) / 64 * rici::kTriCullBytes);
        J.verts = (float4*)p;
        J.block_start = blocks; J.chunk_start = chunks; J.item_start = items;
        J.sort = rici::gen_sort_wanted(h->gen_sort, j.num_triangles) ? 1 : 0;
        blocks += (j.num_triangles + rici::kGenSortBlock - 1) / rici::kGenSortBlock;
        chunks += (j.num_triangles + 63) / 64;
        items += (j.num_points + G - 1) / G;
    }
    // ---- search table
    std::vector<rici::SearchJob> sj(sorder.size());
    rici::SearchTotals T = {};
    uint32_t tiles = 0;
    for (size_t i = 0; i < sorder.size(); ++i) {
        const rici_mesh_job& j = jobs[sorder[i]];
        const uint32_t n = j.num_points;
        const size_t ga = needle_groups(n), hs = rici::haystack_slots(n), gb = hs / rici::kGroup;
        rici::SearchJob& S = sj[i];
        char* p = work + soff[i];
        S.np.planes = (int8_t*)p; p += align256(2 * ga * rici::kPlaneGroupBytes);
        S.hp.planes = (int8_t*)p; p += align256(3 * gb * rici::kPlaneGroupBytes);
        S.np.sumsq = (int64_t*)p; p += align256(ga * rici::kGroup * 8);
        S.np.maxabs = (uint32_t*)p; p += align256(ga * rici::kGroup * 4);
        S.hp.maxabs = (uint32_t*)p; p += align256(hs * 4);
        S.hp.maxabs_img = (uint32_t*)p; p += align256((size_t)n * 4);
        S.hp.perm = (uint32_t*)p; p += align256(hs * 4);
        int32_t* thr = (int32_t*)p; p += align256(std::max<size_t>(hs, n) * 4);
        int64_t* dstar = (int64_t*)p; p += align256((size_t)n * 8);
        S.lists = (uint32_t*)p; p += align256((2 + 2 * (size_t)n) * 4);
        S.np.maxabs_img = S.np.maxabs; S.np.perm = nullptr; S.hp.sumsq = nullptr;
        S.np.inv = S.hp.inv = nullptr;
        uint32_t* tile_flags = nullptr;
        if (paired) {
            S.hp.inv = (uint32_t*)p; p += align256((size_t)n * 4);
            tile_flags = (uint32_t*)p;
            S.np.maxabs = S.np.maxabs_img = S.hp.maxabs_img;   // per image
        }
        S.np.ngroups = (uint32_t)ga; S.hp.ngroups = (uint32_t)gb;
        S.needles = j.out_images; S.hay = j.out_images; S.true_idx = j.true_index;
        S.dstar = j.out_true_distance ? j.out_true_distance : dstar;
        rici::SearchArgs& A = S.A;
        A = {};
        A.a_planes = S.np.planes; A.a_groups = S.np.ngroups; A.nn = n;
        A.b_planes = S.hp.planes; A.b_groups = S.hp.ngroups; A.nh = n;
        A.nmax = S.np.maxabs; A.hmax = S.hp.maxabs; A.hperm = S.hp.perm;
        A.thr = thr; A.sumsq = S.np.sumsq; A.rank = j.out_rank; A.matrix = nullptr;
        A.tiles_m = paired ? (uint32_t)(hs / tn) : (uint32_t)((n + tm - 1) / tm);
        A.tiles_n = (uint32_t)(hs / tn);
        A.per_xcd = 0;
        A.early_exit = (uint32_t)h->early_exit;
        if (paired) {
            A.paired = 1; A.nperm = S.hp.perm; A.tile_flags = tile_flags; A.cross = d_cross;
        }
        S.ngrp_start = T.needle_groups; S.hslot_start = T.hay_slots; S.himg_start = T.hay_images;
        S.hgrp_start = T.hay_groups; S.needle_start = T.needles; S.tile_start = tiles;
        T.needle_groups += ga; T.hay_slots += hs; T.hay_images += n; T.hay_groups += gb; T.needles += n;
        tiles += paired ? rici::paired_items(A.tiles_m) : A.tiles_m * A.tiles_n;
    }
    T.tiles = tiles;
    if (!gj.empty()) e = hipMemcpy(d_gjobs, gj.data(), gj.size() * sizeof(rici::GenJob), hipMemcpyHostToDevice);
    if (e == hipSuccess && !sj.empty())
        e = hipMemcpy(d_sjobs, sj.data(), sj.size() * sizeof(rici::SearchJob), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        destroy_plan(b);
        return hip_fail(e, "rici_batch_create: job table upload");
    }
    e = rici::prepare_search_kernels();
    if (e != hipSuccess) {
        destroy_plan(b);
        return hip_fail(e, "rici_batch_create: kernel attributes");
    }

    for (hipEvent_t& ev : b->ev) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            ev = nullptr;
            destroy_plan(b);
            return hip_fail(e, "rici_batch_create: hipEventCreate");
        }
    }
    b->has_gen = items > 0;
    b->has_search = T.tiles > 0;

    // ---- record the launch sequence as a graph: five captured segments
    // (generation preparation, persistent generation kernel, search
    // preparation, persistent search kernel, exact fallback) chained as child
    // graphs, with event records right around the two persistent kernels
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        destroy_plan(b);
        return hip_fail(e, "hipStreamCreate");
    }
    hipGraph_t seg[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hipError_t le = hipSuccess;
    for (int k = 0; k < 5 && e == hipSuccess && le == hipSuccess; ++k) {
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) break;
        if (k < 2)
            le = rici::launch_gen_batched(d_gjobs, (uint32_t)gj.size(), blocks, chunks, items, support_radius,
                                          d_counters, h->d_err, gen_grid, gen_group, cs, k + 1);
        else
            le = rici::launch_search_batched(d_sjobs, (uint32_t)sj.size(), T, d_counters + 1, grid, variant,
                                             h->early_exit, cs, k - 1, paired ? 1 : 0);
        hipError_t ee = hipStreamEndCapture(cs, &seg[k]);
        if (e == hipSuccess) e = ee;
    }
    (void)hipStreamDestroy(cs);
    if (e == hipSuccess && le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphCreate(&b->graph, 0);
    hipGraphNode_t prev = nullptr;
    bool events_ok = true;
    for (int k = 0; k < 5 && e == hipSuccess; ++k) {
        size_t nodes = 0;
        e = hipGraphGetNodes(seg[k], nullptr, &nodes);
        if (e == hipSuccess && nodes > 0) {
            hipGraphNode_t node = nullptr;
            e = hipGraphAddChildGraphNode(&node, b->graph, prev ? &prev : nullptr, prev ? 1 : 0, seg[k]);
            if (e == hipSuccess) prev = node;
        }
        // events before and after segments 1 (generation kernel) and 3 (search kernel)
        const int ev = k == 0 ? 0 : k == 1 ? 1 : k == 2 ? 2 : k == 3 ? 3 : -1;
        if (e == hipSuccess && ev >= 0 && events_ok) {
            hipGraphNode_t node = nullptr;
            hipError_t ee = hipGraphAddEventRecordNode(&node, b->graph, prev ? &prev : nullptr, prev ? 1 : 0,
                                                       b->ev[ev]);
            if (ee == hipSuccess) {
                prev = node;
            } else {
                (void)hipGetLastError();   // no in-graph timing on this runtime; the plan still runs
                events_ok = false;
            }
        }
    }
    for (hipGraph_t g2 : seg)
        if (g2) (void)hipGraphDestroy(g2);
    b->timing_ok = events_ok;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        destroy_plan(b);
        return hip_fail(e, "rici_batch_create: graph construction");
    }
    *out = b;
    return RICI_OK;
}

int rici_batch_run(rici_batch b, void* stream)
{
    if (!b || !b->exec) return fail(RICI_ERR_INVALID, "rici_batch_run: NULL plan");
    DeviceGuard g(b->h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    rici_ctx* h = b->h;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = timed(h, "batch", s, [&] { return hipGraphLaunch(b->exec, s); });
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return RICI_OK;
}

void rici_batch_destroy(rici_batch b)
{
    if (!b) return;
    DeviceGuard g(b->h->device);
    (void)hipDeviceSynchronize();
    destroy_plan(b);
}

uint64_t rici_batch_scratch_bytes(rici_batch b) { return b ? (uint64_t)b->scratch_bytes : 0u; }

int rici_batch_kernel_ms(rici_batch b, const char* kernel, float* ms)
{
    if (!b || !kernel || !ms) return fail(RICI_ERR_INVALID, "rici_batch_kernel_ms: NULL argument");
    int k;
    bool present;
    if (strcmp(kernel, "gen") == 0) {
        k = 0;
        present = b->has_gen;
    } else if (strcmp(kernel, "search") == 0) {
        k = 2;
        present = b->has_search;
    } else {
        return fail(RICI_ERR_INVALID, "rici_batch_kernel_ms: unknown kernel '%s' (gen, search)", kernel);
    }
    *ms = 0.0f;
    if (!present) return RICI_OK;
    if (!b->timing_ok) return fail(RICI_ERR_UNSUPPORTED, "rici_batch_kernel_ms: no event nodes in this plan's graph");
    DeviceGuard g(b->h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = hipEventSynchronize(b->ev[k + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, b->ev[k], b->ev[k + 1]);
    if (e != hipSuccess) return hip_fail(e, "rici_batch_kernel_ms");
    return RICI_OK;
}

}  // extern "C"

// ------------------------------------------------------- database and queries

struct rici_db_ctx {
    rici_ctx* h = nullptr;
    void* scratch = nullptr;
    size_t bytes = 0;
    rici::SearchPrep hp = {};
    const uint32_t* images = nullptr;
    uint32_t n = 0, tiles = 0;
};

struct rici_query_ctx {
    rici_db db = nullptr;
    void* scratch = nullptr;
    bool owns = false;
    size_t bytes = 0;
    rici::SearchPrep np = {};
    int32_t* thr = nullptr;
    int64_t* dstar = nullptr;
    uint32_t* rank = nullptr;
    uint32_t nn = 0, tiles_m = 0;
    int variant = 0;                // search tile shape the needle tiles were counted for
    int early_exit = 0;
};

namespace {

struct QueryLayout {
    size_t planes, sumsq, nmax, thr, dstar, lists, total;
};

QueryLayout query_layout(uint32_t nn, uint32_t nh)
{
    QueryLayout L;
    const size_t ga = rici::search_groups(nn);
    L.planes = align256(2 * ga * rici::kPlaneGroupBytes);
    L.sumsq = align256(ga * rici::kGroup * sizeof(int64_t));
    L.nmax = align256(ga * rici::kGroup * sizeof(uint32_t));
    L.thr = align256((size_t)nn * sizeof(int32_t));
    L.dstar = align256((size_t)nn * sizeof(int64_t));
    L.lists = align256((2 + (size_t)nn + nh) * sizeof(uint32_t));
    L.total = L.planes + L.sumsq + L.nmax + L.thr + L.dstar + L.lists;
    return L;
}

}  // namespace

extern "C" {

int rici_db_create(rici_handle h, const uint32_t* images, uint32_t num_images, void* stream, rici_db* out)
{
    if (!out) return fail(RICI_ERR_INVALID, "rici_db_create: out is NULL");
    *out = nullptr;
    if (!h) return fail(RICI_ERR_INVALID, "rici_db_create: NULL handle");
    if (num_images == 0 || !images) return fail(RICI_ERR_INVALID, "rici_db_create: empty database");
    if (num_images >= (1u << 31)) return fail(RICI_ERR_UNSUPPORTED, "rici_db_create: more than 2^31 images");
    if (misaligned(images)) return fail(RICI_ERR_INVALID, "rici_db_create: images are not 16-byte aligned");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipError_t e = rici::prepare_search_kernels();
    if (e != hipSuccess) return hip_fail(e, "kernel attributes");
    const size_t hs = rici::haystack_slots(num_images), gb = hs / rici::kGroup;
    const size_t planes = align256(3 * gb * rici::kPlaneGroupBytes), hmax = align256(hs * 4),
                 himg = align256((size_t)num_images * 4), perm = align256(hs * 4);
    rici_db_ctx* db = new rici_db_ctx();
    db->h = h;
    db->bytes = planes + hmax + himg + perm;
    e = hipMalloc(&db->scratch, db->bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete db;
        return fail(RICI_ERR_OOM, "rici_db_create: cannot allocate %zu bytes", planes + hmax + himg + perm);
    }
    char* p = (char*)db->scratch;
    db->hp.planes = (int8_t*)p; p += planes;
    db->hp.maxabs = (uint32_t*)p; p += hmax;
    db->hp.maxabs_img = (uint32_t*)p; p += himg;
    db->hp.perm = (uint32_t*)p;
    db->hp.sumsq = nullptr;
    db->hp.ngroups = (uint32_t)gb;
    db->images = images;
    db->n = num_images;
    db->tiles = (uint32_t)(hs / rici::search_tile_n());
    hipStream_t s = (hipStream_t)stream;
    e = timed(h, "delta_haystack", s, [&] { return rici::launch_delta_prep(images, num_images, 0, db->hp, s); });
    if (e != hipSuccess) {
        (void)hipFree(db->scratch);
        delete db;
        return hip_fail(e, "rici_db_create: delta planes");
    }
    *out = db;
    return RICI_OK;
}

uint32_t rici_db_tiles(rici_db db) { return db ? db->tiles : 0u; }
uint64_t rici_db_scratch_bytes(rici_db db) { return db ? (uint64_t)db->bytes : 0u; }

void rici_db_destroy(rici_db db)
{
    if (!db) return;
    DeviceGuard g(db->h->device);
    (void)hipDeviceSynchronize();
    if (db->scratch) (void)hipFree(db->scratch);
    delete db;
}

uint64_t rici_query_footprint(rici_db db, uint32_t num_needles)
{
    return db ? (uint64_t)query_layout(num_needles, db->n).total : 0u;
}

int rici_query_create(rici_handle h, rici_db db, const uint32_t* needles, uint32_t num_needles,
                      const uint32_t* true_index, uint32_t* out_rank, int64_t* out_true_distance, void* workspace,
                      uint64_t workspace_bytes, void* stream, rici_query* out)
{
    if (!out) return fail(RICI_ERR_INVALID, "rici_query_create: out is NULL");
    *out = nullptr;
    if (!h || !db) return fail(RICI_ERR_INVALID, "rici_query_create: NULL handle or database");
    if (num_needles == 0 || !needles || !true_index || !out_rank)
        return fail(RICI_ERR_INVALID, "rici_query_create: empty query or NULL pointer");
    if (num_needles >= (1u << 31)) return fail(RICI_ERR_UNSUPPORTED, "rici_query_create: too many needles");
    if (misaligned(needles)) return fail(RICI_ERR_INVALID, "rici_query_create: needles are not 16-byte aligned");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    const QueryLayout L = query_layout(num_needles, db->n);
    if (workspace && workspace_bytes < L.total)
        return fail(RICI_ERR_INVALID, "rici_query_create: workspace of %llu bytes, %zu needed",
                    (unsigned long long)workspace_bytes, L.total);
    rici_query_ctx* q = new rici_query_ctx();
    q->db = db;
    q->bytes = L.total;
    hipError_t e = hipSuccess;
    if (workspace) {
        q->scratch = workspace;
    } else {
        e = hipMalloc(&q->scratch, L.total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete q;
            return fail(RICI_ERR_OOM, "rici_query_create: cannot allocate %zu bytes", L.total);
        }
        q->owns = true;
    }
    char* p = (char*)q->scratch;
    q->np.planes = (int8_t*)p; p += L.planes;
    q->np.sumsq = (int64_t*)p; p += L.sumsq;
    q->np.maxabs = (uint32_t*)p; p += L.nmax;
    q->np.maxabs_img = q->np.maxabs;
    q->np.perm = nullptr;
    q->np.ngroups = (uint32_t)rici::search_groups(num_needles);
    q->thr = (int32_t*)p; p += L.thr;
    int64_t* own_dstar = (int64_t*)p; p += L.dstar;
    uint32_t* lists = (uint32_t*)p;
    q->dstar = out_true_distance ? out_true_distance : own_dstar;
    q->rank = out_rank;
    q->nn = num_needles;
    q->variant = h->search_variant;
    q->early_exit = h->early_exit;
    q->tiles_m = (num_needles + rici::search_tile_m(q->variant) - 1) / rici::search_tile_m(q->variant);
    hipStream_t s = (hipStream_t)stream;
    e = timed(h, "delta_needle", s, [&] { return rici::launch_delta_prep(needles, num_needles, 1, q->np, s); });
    if (e == hipSuccess)
        e = timed(h, "true_distance", s, [&] {
            return rici::launch_true_distance(needles, num_needles, db->images, db->n, true_index, q->np.sumsq,
                                              q->np.maxabs, q->dstar, q->thr, out_rank, s);
        });
    if (e == hipSuccess)
        e = timed(h, "fallback", s, [&] {
            return rici::launch_fallback(needles, num_needles, db->images, db->n, q->np.maxabs, db->hp.maxabs_img,
                                         q->dstar, out_rank, nullptr, lists, s);
        });
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        if (q->owns) (void)hipFree(q->scratch);
        delete q;
        return hip_fail(e, "rici_query_create: launch");
    }
    *out = q;
    return RICI_OK;
}

void rici_query_destroy(rici_query q)
{
    if (!q) return;
    if (q->owns) {
        DeviceGuard g(q->db->h->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(q->scratch);
    }
    delete q;
}

int rici_db_scan(rici_handle h, rici_db db, const rici_query* queries, uint32_t num_queries, uint32_t tile_begin,
                 uint32_t tile_count, void* stream)
{
    if (!h || !db) return fail(RICI_ERR_INVALID, "rici_db_scan: NULL handle or database");
    if (num_queries > (uint32_t)rici::kMaxScanJobs)
        return fail(RICI_ERR_INVALID, "rici_db_scan: more than %d queries", rici::kMaxScanJobs);
    if (num_queries > 0 && !queries) return fail(RICI_ERR_INVALID, "rici_db_scan: NULL queries");
    if (tile_count > db->tiles || tile_begin >= db->tiles)
        return fail(RICI_ERR_INVALID, "rici_db_scan: tile range beyond the database");
    rici::ScanTable T = {};
    uint32_t m = 0;
    const int variant = num_queries > 0 && queries[0] ? queries[0]->variant : 0;
    for (uint32_t k = 0; k < num_queries; ++k) {
        const rici_query_ctx* q = queries[k];
        if (!q || q->db != db) return fail(RICI_ERR_INVALID, "rici_db_scan: query %u is not of this database", k);
        if (q->variant != variant)
            return fail(RICI_ERR_INVALID, "rici_db_scan: queries %u and 0 were created with different search tiles", k);
        rici::SearchArgs& A = T.A[k];
        A.a_planes = q->np.planes; A.a_groups = q->np.ngroups; A.nn = q->nn;
        A.b_planes = db->hp.planes; A.b_groups = db->hp.ngroups; A.nh = db->n;
        A.nmax = q->np.maxabs; A.hmax = db->hp.maxabs; A.hperm = db->hp.perm;
        A.thr = q->thr; A.sumsq = q->np.sumsq; A.rank = q->rank; A.matrix = nullptr;
        A.tiles_m = q->tiles_m; A.tiles_n = db->tiles; A.per_xcd = 0;
        A.early_exit = (uint32_t)q->early_exit;
        T.m_start[k] = m;
        m += q->tiles_m;
    }
    T.m_start[num_queries] = m;
    T.njobs = num_queries;
    T.tile_begin = tile_begin;
    T.tile_count = tile_count;
    T.db_tiles = db->tiles;
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = timed(h, "scan", s, [&] { return rici::launch_search_scan(T, variant, s); });
    if (e != hipSuccess) return hip_fail(e, "rici_db_scan: launch");
    return RICI_OK;
}

}  // extern "C"
