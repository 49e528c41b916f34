// Device-side bodies of the projector kernels, shared by the single-geometry
// launches and the batched work-list launches.
#pragma once

#include "common.h"

namespace dect {

// Adjoint tiling: a block owns a kTW x kTH output tile, each of its four
// wavefronts a kSH-row strip of it, accumulated in LDS with one spare row and
// one spare column that absorb out-of-strip contributions (branch-free).
constexpr int kTW = 64;                  // tile width (columns) = lanes
constexpr int kSH = 32;                  // rows per wavefront strip
constexpr int kTH = 4 * kSH;             // tile height (rows)
constexpr int kAccLd = kTW + 1;          // strip row stride; column kTW is spare
constexpr int kAccSize = (kSH + 1) * kAccLd;  // row kSH is spare
constexpr int kTilePix = kTW * kTH;
constexpr int kStage = 256;              // bins staged per block and view chunk

struct AdjShared {
    float acc[4][kAccSize];
    double2 ak[kStage];  // (a, k) of the staged bins
    float ly[kStage];    // |path length per line| * sinogram value
    int is_last;
};

__host__ __device__ inline int adj_tiles_x(int nx) { return (nx + kTW - 1) / kTW; }
__host__ __device__ inline int adj_tiles(int nx, int ny) { return adj_tiles_x(nx) * ((ny + kTH - 1) / kTH); }
constexpr float kTwoM32 = 2.3283064365386963e-10f;  // 2^-32

// ------------------------------------------------------------ forward ---
// One driving-line loop over `line` in [l0, l1] for the lanes of one class.
// base: padded line l0 at offset kPad (the element of index 0 of the line);
// step: floats between consecutive lines.  q: this lane's 32.32 coordinate
// at l0 (a sentinel far below -2 for lanes of the other class), dq its step.
__device__ __forceinline__ void walk(const float *__restrict__ base, int step, int l0, int l1,
                                     int64_t q, int64_t dq, int nq, double &acc0, double &acc1)
{
    const float *line = base;
#pragma unroll 4
    for (int i = l0; i <= l1; ++i) {
        int h = (int)(q >> 32);
        unsigned lo = (unsigned)q;
        h = min(max(h, -2), nq);  // outside [-1, nq-1]: both taps read zero padding
        const double v0 = line[h];
        const double v1 = line[h + 1];
        acc0 += v0;
        acc1 = fma((double)lo, v1 - v0, acc1);  // product of a 32-bit and a 25-bit value
        q += dq;
        line += step;
    }
}

// One forward wavefront: view v and 64-bin bundle j from the wave index gw
// (= v * nbundle + j) of one batch item.  pad_e/padT_e: that item's padded
// image copies, sino_e its sinogram.  The ray sum is accumulated in FP64 and
// rounded once (an FP32 running sum over ~700 samples would carry ~1e-6
// relative error, which the reconstruction iteration amplifies).  With sub_e
// the stored value is scale * (A x) - sub_scale * sub_e, also rounded once.
// Returns this lane's value (0 when the lane has no ray) after writing it.
__device__ __forceinline__ float fwd_wave(const float *__restrict__ pad_e,
                                          const float *__restrict__ padT_e,
                                          const RayFwd *__restrict__ rays,
                                          const float *__restrict__ len,
                                          const Bundle *__restrict__ bundles,
                                          float *__restrict__ sino_e, int nx, int ny, int B,
                                          int nbundle, int gw, int lane, float scale,
                                          const float *__restrict__ sub_e = nullptr,
                                          float sub_scale = 0.f)
{
    const int v = gw / nbundle, j = gw - v * nbundle;
    const int b = j * kBundle + lane;
    const bool act = b < B;
    const size_t ray = (size_t)v * B + (act ? b : 0);
    const RayFwd rf = rays[ray];
    const float L = len[ray];
    const Bundle bu = bundles[(size_t)v * nbundle + j];
    const int pnx = nx + 2 * kPad, pny = ny + 2 * kPad;
    double acc0 = 0.0, acc1 = 0.0;
    const int64_t far = -(int64_t(1000000) << 32);
    const int64_t a = rf.a_fx, k = rf.k_fx;
    // the sign of the stored path length marks the ray class (+ x-major)
    const bool is_x = act && L > 0.f;
    const bool is_y = act && L < 0.f;
    if (bu.x0 <= bu.x1) {
        int64_t q = is_x ? a + k * (int64_t)bu.x0 : far;
        int64_t dq = is_x ? k : 0;
        walk(padT_e + (size_t)(bu.x0 + kPad) * pny + kPad, pny, bu.x0, bu.x1, q, dq, ny, acc0,
             acc1);
    }
    if (bu.y0 <= bu.y1) {
        int64_t q = is_y ? a + k * (int64_t)bu.y0 : far;
        int64_t dq = is_y ? k : 0;
        walk(pad_e + (size_t)(bu.y0 + kPad) * pnx + kPad, pnx, bu.y0, bu.y1, q, dq, nx, acc0,
             acc1);
    }
    double sum = (double)fabsf(L) * fma(acc1, (double)kTwoM32, acc0) * (double)scale;
    if (sub_e && act) sum -= (double)sub_scale * (double)sub_e[(size_t)v * B + b];
    const float result = (float)sum;
    if (act) sino_e[(size_t)v * B + b] = result;
    return act ? result : 0.f;
}

// Fixed-order sum of one double per thread over a 256-thread block; the
// total is returned to thread 0.
__device__ __forceinline__ double block_sum_256(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    double out = red[0];
    __syncthreads();
    return out;
}

// ------------------------------------------------------------ adjoint ---
struct AdjGeo {
    float R, D, inv_du, beta0;  // beta(p) = D (p.e_u) / (R - p.e_s) * inv_du + beta0
    float dl, xoff, yoff;       // pixel centre x = c*dl - xoff, y = r*dl - yoff
    float margin;
};

// Detector projection constants of a geometry for the adjoint (host).
AdjGeo adj_geometry(const GeomTables &t);

__device__ __forceinline__ float beta_of(const AdjGeo &g, float ct, float st, float px, float py)
{
    float pu = -px * st + py * ct;
    float ps = px * ct + py * st;
    return g.D * pu / (g.R - ps) * g.inv_du + g.beta0;
}

// The whole adjoint block for output tile `tile` of one batch item, view
// group g of nvg: sino_e/out_e are the item's sinogram and image.  Per view
// the block stages the bins whose rays can reach its tile (their (a, k) and
// |L| y) in LDS; then, per wavefront strip, x-major rays are walked by
// column (lane = column) and y-major rays by row (lane = row within the strip
// and column half).  With nvg > 1, tiles_part holds this (item, tile)'s nvg
// parked tiles and counter its completion counter (zero between launches);
// the last group to finish sums the parked tiles in group order.
__device__ __forceinline__ void adj_block(AdjShared &sh, const float *__restrict__ sino_e,
                                          const RayAdj *__restrict__ rays,
                                          const float *__restrict__ len,
                                          const ViewInfo *__restrict__ views, const AdjGeo &geo,
                                          int nx, int ny, int V, int B, int tile, int g, int nvg,
                                          float *__restrict__ out_e,
                                          float *__restrict__ tiles_part, int *__restrict__ counter,
                                          float scale)
{
    const int ntx = adj_tiles_x(nx);
    const int tr0 = (tile / ntx) * kTH, tc0 = (tile % ntx) * kTW;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r0s = tr0 + kSH * wid;          // first row of this wave's strip
    float *my = sh.acc[wid];
    for (int i = lane; i < kAccSize; i += 64) my[i] = 0.f;

    const int c = tc0 + lane;                 // x-major walk: this lane's column
    const int yrow = lane & (kSH - 1);        // y-major walk: strip row ...
    const int half = lane >> 5;               // ... and column half
    const int yr = r0s + yrow, cl = tc0 + 32 * half;
    const bool xlane = c < nx && r0s < ny;
    const bool ylane = yr < ny && cl < nx;
    // strip / half extents in mm (one pixel beyond on the low side, clamped)
    const float px = c * geo.dl - geo.xoff;
    const float ya = (r0s - 1) * geo.dl - geo.yoff, yb = min(r0s + kSH, ny) * geo.dl - geo.yoff;
    const float py = yr * geo.dl - geo.yoff;
    const float xa = (cl - 1) * geo.dl - geo.xoff, xb = min(cl + 32, nx) * geo.dl - geo.xoff;
    // block tile corners
    const float Xa = (tc0 - 1) * geo.dl - geo.xoff, Xb = min(tc0 + kTW, nx) * geo.dl - geo.xoff;
    const float Ya = (tr0 - 1) * geo.dl - geo.yoff, Yb = min(tr0 + kTH, ny) * geo.dl - geo.yoff;
    const double cd = (double)c, rd = (double)yr;

    const int v_begin = (int)((int64_t)V * g / nvg), v_end = (int)((int64_t)V * (g + 1) / nvg);
    for (int v = v_begin; v < v_end; ++v) {
        const ViewInfo vi = views[v];
        const float *yv = sino_e + (size_t)v * B;
        const RayAdj *rv = rays + (size_t)v * B;
        const float *lv = len + (size_t)v * B;
        // bins whose rays can meet the tile: hull of the corner projections
        float b00 = beta_of(geo, vi.ct, vi.st, Xa, Ya), b01 = beta_of(geo, vi.ct, vi.st, Xa, Yb);
        float b10 = beta_of(geo, vi.ct, vi.st, Xb, Ya), b11 = beta_of(geo, vi.ct, vi.st, Xb, Yb);
        int lo = max(0, (int)ceilf(fminf(fminf(b00, b01), fminf(b10, b11)) - geo.margin));
        int hi = min(B - 1, (int)floorf(fmaxf(fmaxf(b00, b01), fmaxf(b10, b11)) + geo.margin));
        // per-lane ranges of the two walks
        int xb0 = 1, xb1 = 0, yb0 = 1, yb1 = 0;
        if (xlane && vi.xb0 < vi.xb1) {
            float ba = beta_of(geo, vi.ct, vi.st, px, ya), bb = beta_of(geo, vi.ct, vi.st, px, yb);
            xb0 = max(vi.xb0, (int)ceilf(fminf(ba, bb) - geo.margin));
            xb1 = min(vi.xb1 - 1, (int)floorf(fmaxf(ba, bb) + geo.margin));
        }
        if (ylane && vi.yb0 < vi.yb1) {
            float ba = beta_of(geo, vi.ct, vi.st, xa, py), bb = beta_of(geo, vi.ct, vi.st, xb, py);
            yb0 = max(vi.yb0, (int)ceilf(fminf(ba, bb) - geo.margin));
            yb1 = min(vi.yb1 - 1, (int)floorf(fmaxf(ba, bb) + geo.margin));
        }
        for (int cb = lo; cb <= hi; cb += kStage) {
            const int ce = min(hi, cb + kStage - 1);
            __syncthreads();  // the previous chunk is consumed
            for (int i = threadIdx.x; i <= ce - cb; i += 256) {
                const RayAdj t = rv[cb + i];
                sh.ak[i] = make_double2(t.a, t.k);
                sh.ly[i] = fabsf(lv[cb + i]) * yv[cb + i];
            }
            __syncthreads();
            // x-major rays: rows of this strip along column c
            {
                const int b0 = max(xb0, cb), b1 = min(xb1, ce);
                for (int b = b0; b <= b1; ++b) {
                    const double2 t = sh.ak[b - cb];
                    const float ly = sh.ly[b - cb];
                    const double q = fma(t.y, cd, t.x);
                    const double fl = floor(q);
                    const int i0 = (int)fl - r0s;
                    const float w = (float)(q - fl);
                    const float wl = w * ly, ol = ly - wl;
                    const int ia = (unsigned)i0 < (unsigned)kSH ? i0 : kSH;
                    const int ib = (unsigned)(i0 + 1) < (unsigned)kSH ? i0 + 1 : kSH;
                    my[ia * kAccLd + lane] += ol;
                    my[ib * kAccLd + lane] += wl;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // y-major rays: columns of this half along row yr
            {
                const int b0 = max(yb0, cb), b1 = min(yb1, ce);
                float *rowp = my + yrow * kAccLd;
                for (int b = b0; b <= b1; ++b) {
                    const double2 t = sh.ak[b - cb];
                    const float ly = sh.ly[b - cb];
                    const double q = fma(t.y, rd, t.x);
                    const double fl = floor(q);
                    const int i0 = (int)fl - cl;
                    const float w = (float)(q - fl);
                    const float wl = w * ly, ol = ly - wl;
                    const int ia = (unsigned)i0 < 32u ? i0 + 32 * half : kTW;
                    const int ib = (unsigned)(i0 + 1) < 32u ? i0 + 1 + 32 * half : kTW;
                    rowp[ia] += ol;
                    rowp[ib] += wl;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    __syncthreads();
    if (nvg == 1) {  // each wave writes its own strip
        for (int i = lane; i < kSH * kTW; i += 64) {
            const int rr = i / kTW, cc = i % kTW;
            const int r = r0s + rr, cx = tc0 + cc;
            if (r < ny && cx < nx) out_e[(size_t)r * nx + cx] = my[rr * kAccLd + cc] * scale;
        }
        return;
    }
    // several view groups: park this group's tile; the last group to finish
    // sums all of them in group order (deterministic) and writes the tile
    float *tiles = tiles_part;
    for (int i = lane; i < kSH * kTW; i += 64) {
        const int rr = i / kTW, cc = i % kTW;
        tiles[(size_t)g * kTilePix + (size_t)(kSH * wid + rr) * kTW + cc] = my[rr * kAccLd + cc];
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        int prev = atomicAdd(counter, 1);
        sh.is_last = prev == nvg - 1;
    }
    __syncthreads();
    if (!sh.is_last) return;
    __threadfence();
    for (int i = threadIdx.x; i < kTilePix; i += 256) {
        const int rr = i / kTW, cc = i % kTW;
        const int r = tr0 + rr, cx = tc0 + cc;
        if (r < ny && cx < nx) {
            float sum = 0.f;
            for (int q = 0; q < nvg; ++q) sum += tiles[(size_t)q * kTilePix + i];
            out_e[(size_t)r * nx + cx] = sum * scale;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) *counter = 0;  // ready for the next launch
}

}  // namespace dect
