// Internal declarations shared by the libdect translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dect.h"

namespace dect {

// ---------------------------------------------------------------- errors ---
void set_error(const std::string &msg);
dect_status fail(dect_status st, const std::string &msg);

#define DECT_HIP(expr)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::dect::fail(DECT_ERR_HIP, std::string(#expr " failed: ") +            \
                                                  hipGetErrorString(e_));                 \
    } while (0)

// -------------------------------------------------------------- tracing ---
// A roctx range over a scope (host side: it brackets the enqueueing of the
// scope's launches, and shows in rocprofv3 --marker-trace beside the kernels).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};
#define DECT_TRACE_CAT2(a, b) a##b
#define DECT_TRACE_CAT(a, b) DECT_TRACE_CAT2(a, b)
#define DECT_TRACE(name) ::dect::TraceRange DECT_TRACE_CAT(trace_range_, __LINE__)(name)

// ------------------------------------------------------------- geometry ---
// Joseph line coordinate in 32.32 fixed point: the crossing of ray (v,b)
// with driving line i (column for x-major rays, row for y-major rays) is at
// q(i) = (a_fx + k_fx * i) / 2^32 in units of pixels along the other axis.
// The integer form is exact, so the forward pass (incremental) and the
// adjoint (direct, in FP64, which holds these integers exactly) agree bit
// for bit on every interpolation weight.
struct RayFwd {
    int64_t a_fx;
    int64_t k_fx;
};
// Siddon model: a_fx above is the coordinate q' = q - |k|/2 + 1/2 of the
// ray's lower end within the driving line, shifted by half a pixel, so that
// h = floor(q') is the first of the (at most two) pixels the ray crosses on
// that line.  Its share of the line's path length that falls in pixel h + 1
// is (frac(q') - (1 - |k|)) / |k| when positive, else 0; with frac(q') as
// the 32-bit word lo, that is (lo - c) * inv * 2^-32 for lo > c, where
// c = 2^32 - |k_fx| and inv = 1 / |k| (c = 2^32 - 1, inv = 0 when k = 0).
struct SidW {
    uint32_t c;
    float inv;
};
// Per (view, 64-bin bundle): union of the valid driving-line ranges of the
// bundle's x-major lanes [x0, x1] and y-major lanes [y0, y1] (empty: x0 > x1).
struct Bundle {
    int32_t x0, x1, y0, y1;
};
// Per view: detector-plane projection constants and the bin ranges of the
// two ray classes (x-major bins [xb0, xb1), y-major bins [yb0, yb1)).
struct ViewInfo {
    float ct, st;
    int32_t xb0, xb1, yb0, yb1;
    int32_t pad0, pad1;
};

// A forward wavefront holds kFwdViews adjacent views x kBundle adjacent bins
// (lane = view offset * kBundle + bin offset): their rays cross each image
// line close together, so a wavefront's tap loads touch few cache lines.
#ifndef DECT_FWD_VIEWS
#define DECT_FWD_VIEWS 4
#endif
constexpr int kFwdViews = DECT_FWD_VIEWS;
constexpr int kBundle = 64 / kFwdViews;  // bins per forward wavefront and view
constexpr int kPad = 2;       // zero border of the padded image copies

// Adjoint strips.  The two ray classes are gathered separately: x-major rays
// on strips of kSW image rows x kSL columns (lane = column, taps along the
// rows), y-major rays on strips of kSW columns x kSL rows (lane = row, taps
// along the columns) -- the same walk on the transposed image.  Strips are
// numbered x-major first: strip = ts * ceil(n_lane / kSL) + ls within a class.
#ifndef DECT_ADJ_STRIP_WIDTH
#define DECT_ADJ_STRIP_WIDTH 8
#endif
#ifndef DECT_ADJ_WAVES
#define DECT_ADJ_WAVES 4
#endif
#ifndef DECT_ADJ_BLOCKS
#define DECT_ADJ_BLOCKS 4096
#endif
#ifndef DECT_FWD_WAVES
#define DECT_FWD_WAVES 8
#endif
constexpr int kFwdWaves = DECT_FWD_WAVES;  // forward: wavefronts per (view, bundle) block
constexpr int kFwdThreads = 64 * kFwdWaves;
#ifndef DECT_FWD_GROUP
#define DECT_FWD_GROUP 4
#endif
constexpr int kFwdGroup = DECT_FWD_GROUP;  // forward: samples per FP32 partial sum
constexpr int kSL = 64;                    // strip length along the lane axis (one wavefront)
constexpr int kSW = DECT_ADJ_STRIP_WIDTH;  // strip width along the tap axis
constexpr int kAdjWaves = DECT_ADJ_WAVES;  // wavefronts per block (sharing one strip)
constexpr int kAdjThreads = 64 * kAdjWaves;
constexpr int kAdjBlocks = DECT_ADJ_BLOCKS;  // launch size the view grouping aims for
__host__ __device__ inline int adj_strips_cls(int n_lane, int n_tap)
{
    return ((n_lane + kSL - 1) / kSL) * ((n_tap + kSW - 1) / kSW);
}
__host__ __device__ inline int adj_strips_x(int nx, int ny) { return adj_strips_cls(nx, ny); }
__host__ __device__ inline int adj_strips(int nx, int ny)
{
    return adj_strips_cls(nx, ny) + adj_strips_cls(ny, nx);
}
// Bins [lo, hi] of one view whose rays put a tap inside one strip (empty:
// lo > hi); exact, from the fixed-point ray table.
struct BinRange {
    int32_t lo, hi;
    int32_t steps;  // longest per-lane range (below), at most 64: bin steps per 64-bin chunk
    int32_t pad;
};
// Bins [lo + first, lo + last] of one view that put a tap inside one strip at
// one lane (its driving line); empty: first > last.  Exact, from the
// fixed-point ray table, relative to the strip's BinRange lo.  A strip range
// of more than 256 bins keeps no lane ranges: its lanes take the whole range.
struct LaneRange {
    uint8_t first, last;
};
constexpr int kLaneRangeMax = 255;

struct GeomKey {
    int32_t nx, ny, V, B, model;
    double pixel, bin, off, sod, sdd;
    std::vector<double> angles;
    int device;
    bool operator==(const GeomKey &o) const;
};

// Device-resident tables of one geometry (shared by every batch item).
struct GeomTables {
    GeomKey key;
    int nbundle = 0;
    RayFwd *fwd = nullptr;     // [V*B]
    float *len = nullptr;      // [V*B] path length per driving line (pixel/|cos|)
    Bundle *bundles = nullptr; // [ceil(V / kFwdViews) * nbundle]
    ViewInfo *views = nullptr; // [V]
    BinRange *adj_bins = nullptr;  // [adj_strips][V]
    LaneRange *adj_lanes = nullptr;  // [adj_strips][V][kSL]
    SidW *sid = nullptr;       // [V*B] Siddon weight terms (null for Joseph)
    int64_t samples = 0;       // Joseph samples with q in (-1, n)
    ~GeomTables();
};

// Validates the geometry (DECT_ERR_GEOMETRY / DECT_ERR_INVALID_ARG) and
// returns the cached tables for the current device, building them on first
// use.
dect_status get_tables(const dect_geometry *g, GeomTables **out);
dect_status validate_geometry(const dect_geometry *g);
void release_tables();

// ----------------------------------------------------------- workspaces ---
// Every device allocation of the library goes through dev_alloc / dev_free.
// Without a caller workspace they are hipMalloc / hipFree.  With one (set by
// dect_set_workspace for the current device) dev_alloc hands out consecutive
// 256-byte-aligned pieces of it and dev_free ignores them: the pieces are
// released together when the workspace is replaced.
dect_status dev_alloc(void **p, size_t n);
void dev_free(void *p);

// A dry run that only counts bytes: while one is active on a thread,
// dev_alloc returns distinct placeholder addresses that must never be
// touched (DevBuf skips its clearing and the table upload its copies) and
// adds the 256-byte-aligned size to `bytes`; dev_free does nothing.
// get_tables builds tables into the scope instead of the cache.
struct GeomTables;
struct SizingScope {
    size_t bytes = 0;
    uintptr_t next = 256;
    std::vector<std::unique_ptr<GeomTables>> tables;
    SizingScope();
    ~SizingScope();
    SizingScope(const SizingScope &) = delete;
    SizingScope &operator=(const SizingScope &) = delete;
};
bool sizing_active();

// A growable device buffer owned by the library.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    dect_status ensure(size_t n, bool zero = false);
    ~DevBuf();
};

// Frees every library-owned device buffer of the current device: geometry
// tables, work buffers and the ADM states the library made for calls
// without one (not states or batches that callers created).
void release_device_buffers();
void release_adm_states();
void release_proj_work();
void release_fbp_work();
void release_pls_work();
void release_pls3_work();
void release_cone_work();
void release_adm3_work();
void release_unrolled_work();
dect_status set_workspace(void *p, size_t bytes);
dect_status workspace_used(size_t *bytes);
dect_status workspace_size(const dect_geometry *g, int batch, size_t *bytes);
// dry runs of each part (under a SizingScope)
dect_status adm_size_run(const dect_geometry *g);
dect_status proj_size_run(const dect_geometry *g, int batch);
dect_status fbp_size_run(const dect_geometry *g, int batch);
dect_status pls_size_run(size_t n_pixels);

// ------------------------------------------------------------ projector ---
struct ProjWork {
    // interleaved padded copies of item pairs, [pair][ny+4][nx+4][2] and
    // transposed [pair][nx+4][ny+4][2]; adjoint partial images (per item, ray
    // class and view group)
    DevBuf pad, padT, partial;
};

// Pairs of items (2p, 2p + 1) that the projectors process together.
int pairs_of(int batch);
// img [batch][ny][nx] -> both interleaved padded layouts of every pair
// (borders zero; the second image of an odd batch's last pair is zero).
dect_status launch_pad(const GeomTables &t, const float *img, float *pad2, float *padT2, int batch,
                       hipStream_t s);
// sino[e] = scale * A img[e] from the interleaved padded layouts.
// norm_partial (may be NULL) receives per-block sums of squares (double),
// [item][fwd_blocks], for a later reduction.  With sub0/sub1 (items 0 and
// 1), sino[e] = scale * A img[e] - ss_e * sub_e, formed in FP64 and rounded
// once; with lo, lo[e] receives the rounding remainder of every value (same
// layout as sino).
dect_status launch_fwd(const GeomTables &t, const float *pad2, const float *padT2, float *sino,
                       int batch, float scale, double *norm_partial, hipStream_t s,
                       const float *sub0 = nullptr, const float *sub1 = nullptr,
                       double ss0 = 0.0, double ss1 = 0.0, float *lo = nullptr);
int fwd_blocks(const GeomTables &t);
// img[e] = scale * A^T sino[e], through `partial`: adj_partial_floats()
// floats of scratch (per item, both ray classes and every view group).  With
// img == NULL only the partial planes are formed ([item][class][group][N];
// img[e] = scale * their sum in that order).  nvg: view groups, <= 0 for
// adj_groups(t, batch).
int adj_groups(const GeomTables &t, int batch);
size_t adj_partial_floats(const GeomTables &t, int batch, int nvg = 0);
dect_status launch_adj(const GeomTables &t, const float *sino, float *img, float *partial,
                       int batch, float scale, hipStream_t s, int nvg = 0);

dect_status project(const dect_geometry *g, const float *img, float *sino, int batch,
                    hipStream_t s);
dect_status fbp(const dect_geometry *g, const float *sino, float *img, int batch, hipStream_t s);
dect_status cone_project(const dect_cone_geometry *g, const float *vol, float *proj,
                         hipStream_t s);
dect_status cone_backproject(const dect_cone_geometry *g, const float *proj, float *vol,
                             hipStream_t s);
dect_status backproject(const dect_geometry *g, const float *sino, float *img, int batch,
                        hipStream_t s);

}  // namespace dect

struct dect_adm_state;  // defined in adm.hip
