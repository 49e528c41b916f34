// Device-side bodies of the projector kernels, shared by the single-geometry
// launches and the batched work-list launches.
#pragma once

#include "common.h"

namespace dect {

constexpr int kTile = 64;        // adjoint tile side
constexpr int kTileLd = 65;      // LDS row stride (avoids bank conflicts)
constexpr int kTilePix = kTile * kTile;
constexpr float kTwoM32 = 2.3283064365386963e-10f;  // 2^-32

// ------------------------------------------------------------ forward ---
// One driving-line loop over `line` in [l0, l1] for the lanes of one class.
// base: padded line l0 at offset kPad (the element of index 0 of the line);
// step: floats between consecutive lines.  q: this lane's 32.32 coordinate
// at l0 (a sentinel far below -2 for lanes of the other class), dq its step.
__device__ __forceinline__ void walk(const float *__restrict__ base, int step, int l0, int l1,
                                     int64_t q, int64_t dq, int nq, float &acc0, float &acc1)
{
    const float *line = base;
#pragma unroll 4
    for (int i = l0; i <= l1; ++i) {
        int h = (int)(q >> 32);
        unsigned lo = (unsigned)q;
        h = min(max(h, -2), nq);  // outside [-1, nq-1]: both taps read zero padding
        float v0 = line[h];
        float v1 = line[h + 1];
        acc0 += v0;
        acc1 = fmaf((float)lo, v1 - v0, acc1);
        q += dq;
        line += step;
    }
}

// One forward wavefront: view v and 64-bin bundle j from the wave index gw
// (= v * nbundle + j) of one batch item.  pad_e/padT_e: that item's padded
// image copies, sino_e its sinogram.  Returns this lane's value (0 when the
// lane has no ray) after writing it.
__device__ __forceinline__ float fwd_wave(const float *__restrict__ pad_e,
                                          const float *__restrict__ padT_e,
                                          const RayFwd *__restrict__ rays,
                                          const float *__restrict__ len,
                                          const Bundle *__restrict__ bundles,
                                          float *__restrict__ sino_e, int nx, int ny, int B,
                                          int nbundle, int gw, int lane, float scale)
{
    const int v = gw / nbundle, j = gw - v * nbundle;
    const int b = j * kBundle + lane;
    const bool act = b < B;
    const size_t ray = (size_t)v * B + (act ? b : 0);
    const RayFwd rf = rays[ray];
    const float L = len[ray];
    const Bundle bu = bundles[(size_t)v * nbundle + j];
    const int pnx = nx + 2 * kPad, pny = ny + 2 * kPad;
    float acc0 = 0.f, acc1 = 0.f;
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
    float result = fabsf(L) * (acc0 + acc1 * kTwoM32) * scale;
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

// The whole adjoint block for output tile `tile` (ntx tiles per row), view
// group g of nvg, of one batch item: sino_e/out_e are the item's sinogram
// and image.  acc: 4 x kTile*kTileLd floats of LDS; is_last: one LDS int.
// With nvg > 1, tiles_part holds this (item, tile)'s nvg parked tiles and
// counter its completion counter (zero between launches).
__device__ __forceinline__ void adj_block(float (*acc)[kTile * kTileLd], int *is_last,
                                          const float *__restrict__ sino_e,
                                          const RayAdj *__restrict__ rays,
                                          const float *__restrict__ len,
                                          const ViewInfo *__restrict__ views, const AdjGeo &geo,
                                          int nx, int ny, int V, int B, int ntx, int tile, int g,
                                          int nvg, float *__restrict__ out_e,
                                          float *__restrict__ tiles_part, int *__restrict__ counter,
                                          float scale)
{
    const int tr0 = (tile / ntx) * kTile, tc0 = (tile % ntx) * kTile;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float *my = acc[wid];
    for (int i = lane; i < kTile * kTileLd; i += 64) my[i] = 0.f;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();

    const int v_begin = (int)((int64_t)V * g / nvg), v_end = (int)((int64_t)V * (g + 1) / nvg);
    const float *y_e = sino_e;
    for (int v = v_begin + wid; v < v_end; v += 4) {
        const ViewInfo vi = views[v];
        const float *yv = y_e + (size_t)v * B;
        const RayAdj *rv = rays + (size_t)v * B;
        const float *lv = len + (size_t)v * B;
        // x-major rays: lane owns tile column lane, rows tr0 .. tr0+63
        if (vi.xb0 < vi.xb1) {
            const int c = tc0 + lane;
            if (c < nx) {
                float px = c * geo.dl - geo.xoff;
                float ya = (tr0 - 1) * geo.dl - geo.yoff;
                float yb = min(tr0 + kTile, ny) * geo.dl - geo.yoff;
                float ba = beta_of(geo, vi.ct, vi.st, px, ya);
                float bb = beta_of(geo, vi.ct, vi.st, px, yb);
                int b0 = max(vi.xb0, (int)ceilf(fminf(ba, bb) - geo.margin));
                int b1 = min(vi.xb1 - 1, (int)floorf(fmaxf(ba, bb) + geo.margin));
                const double cd = (double)c;
                for (int b = b0; b <= b1; ++b) {
                    const RayAdj t = rv[b];
                    double q = fma(t.k, cd, t.a);
                    double fl = floor(q);
                    int i0 = (int)fl - tr0;
                    float w = (float)(q - fl);
                    float ly = fabsf(lv[b]) * yv[b];
                    float wl = w * ly;
                    float ol = ly - wl;
                    if ((unsigned)i0 < (unsigned)kTile) my[i0 * kTileLd + lane] += ol;
                    if ((unsigned)(i0 + 1) < (unsigned)kTile) my[(i0 + 1) * kTileLd + lane] += wl;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        // y-major rays: lane owns tile row lane, columns tc0 .. tc0+63
        if (vi.yb0 < vi.yb1) {
            const int r = tr0 + lane;
            if (r < ny) {
                float py = r * geo.dl - geo.yoff;
                float xa = (tc0 - 1) * geo.dl - geo.xoff;
                float xb = min(tc0 + kTile, nx) * geo.dl - geo.xoff;
                float ba = beta_of(geo, vi.ct, vi.st, xa, py);
                float bb = beta_of(geo, vi.ct, vi.st, xb, py);
                int b0 = max(vi.yb0, (int)ceilf(fminf(ba, bb) - geo.margin));
                int b1 = min(vi.yb1 - 1, (int)floorf(fmaxf(ba, bb) + geo.margin));
                const double rd = (double)r;
                for (int b = b0; b <= b1; ++b) {
                    const RayAdj t = rv[b];
                    double q = fma(t.k, rd, t.a);
                    double fl = floor(q);
                    int i0 = (int)fl - tc0;
                    float w = (float)(q - fl);
                    float ly = fabsf(lv[b]) * yv[b];
                    float wl = w * ly;
                    float ol = ly - wl;
                    if ((unsigned)i0 < (unsigned)kTile) my[lane * kTileLd + i0] += ol;
                    if ((unsigned)(i0 + 1) < (unsigned)kTile) my[lane * kTileLd + i0 + 1] += wl;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    __syncthreads();
    float *dst = out_e;
    if (nvg == 1) {  // sum the four wave accumulators in order and write the tile
        for (int i = threadIdx.x; i < kTile * kTile; i += 256) {
            int rr = i / kTile, cc = i % kTile;
            int r = tr0 + rr, c = tc0 + cc;
            if (r < ny && c < nx) {
                int o = rr * kTileLd + cc;
                float sum = ((acc[0][o] + acc[1][o]) + acc[2][o]) + acc[3][o];
                dst[(size_t)r * nx + c] = sum * scale;
            }
        }
        return;
    }
    // several view groups: park this group's tile, and let the last group to
    // finish sum all of them in group order (deterministic) and write it
    float *tiles = tiles_part;
    for (int i = threadIdx.x; i < kTile * kTile; i += 256) {
        int o = (i / kTile) * kTileLd + i % kTile;
        tiles[(size_t)g * (kTile * kTile) + i] = ((acc[0][o] + acc[1][o]) + acc[2][o]) + acc[3][o];
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        int prev = atomicAdd(counter, 1);
        *is_last = prev == nvg - 1;
    }
    __syncthreads();
    if (!*is_last) return;
    __threadfence();
    for (int i = threadIdx.x; i < kTile * kTile; i += 256) {
        int rr = i / kTile, cc = i % kTile;
        int r = tr0 + rr, c = tc0 + cc;
        if (r < ny && c < nx) {
            float sum = 0.f;
            for (int q = 0; q < nvg; ++q) sum += tiles[(size_t)q * (kTile * kTile) + i];
            dst[(size_t)r * nx + c] = sum * scale;
        }
    }
    if (threadIdx.x == 0) *counter = 0;  // ready for the next launch
}


}  // namespace dect
