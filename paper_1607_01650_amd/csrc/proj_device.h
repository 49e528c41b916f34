// Device-side bodies of the projector kernels, shared by the single-geometry
// launches and the batched work-list launches.
#pragma once

#include "common.h"

namespace dect {

// Adjoint accumulation: a block's four wavefronts share one strip and split
// its view group between them; each adds into its own LDS copy of the strip,
// stored tap-line-major with row stride kSL (the 64 lanes of an access hit
// distinct banks) plus a spare line on each side for the taps that fall just
// outside the strip.
constexpr int kAccRows = kSW + 2;
constexpr int kAccSize = kAccRows * kSL;
constexpr int kAdjWaves = 4;

struct AdjShared {
    float acc[kAdjWaves][kAccSize];
};

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
        // the weight is the FP32 value (float)lo * 2^-32 that the adjoint also
        // uses, so the two passes apply the same matrix
        acc1 = fma((double)(float)lo, v1 - v0, acc1);
        q += dq;
        line += step;
    }
}

// One forward wavefront: view v and 64-bin bundle j from the wave index gw
// (= v * nbundle + j) of one batch item.  pad_e/padT_e: that item's padded
// image copies, sino_e its sinogram.  The ray sum is accumulated in FP64 (an
// FP32 running sum over ~700 samples would carry ~1e-6 relative error, which
// the reconstruction iteration amplifies).  With sub_e the value is
// scale * (A x) - sub_scale * sub_e, formed in FP64.  sino_e receives the
// value rounded to FP32 and, when lo_e is given, lo_e the rounding remainder
// (so that sino_e + lo_e carries the FP64 value to ~2^-48).  Returns this
// lane's FP64 value (0 when the lane has no ray).
__device__ __forceinline__ double fwd_wave(const float *__restrict__ pad_e,
                                          const float *__restrict__ padT_e,
                                          const RayFwd *__restrict__ rays,
                                          const float *__restrict__ len,
                                          const Bundle *__restrict__ bundles,
                                          float *__restrict__ sino_e, int nx, int ny, int B,
                                          int nbundle, int gw, int lane, float scale,
                                          const float *__restrict__ sub_e = nullptr,
                                          double sub_scale = 0.0,
                                          float *__restrict__ lo_e = nullptr)
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
    if (sub_e && act) sum -= sub_scale * (double)sub_e[(size_t)v * B + b];
    const float hi = (float)sum;
    if (act) {
        sino_e[(size_t)v * B + b] = hi;
        if (lo_e) lo_e[(size_t)v * B + b] = (float)(sum - (double)hi);
    }
    return act ? sum : 0.0;
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
// One adjoint block: strip `strip` (combined numbering) of one batch item,
// view group g of nvg.  The block's partial image of this (class, group) is
// written to `part` (a full [ny][nx] plane, normal layout; only this strip's
// pixels).  Per view, each wavefront walks the bins `bins` lists for its
// strip: up to 64 bins' ray data are loaded at once (lane j holds bin j) and
// broadcast bin by bin; every lane evaluates the ray on its own driving line
// and adds the two interpolation taps, which lie on consecutive tap lines,
// with one paired LDS read and write (no atomics: the copy is the wave's own).
__device__ __forceinline__ void adj_block(AdjShared &sh, const float *__restrict__ sino_e,
                                          const RayAdj *__restrict__ rays,
                                          const float *__restrict__ len,
                                          const BinRange *__restrict__ bins, int nx, int ny,
                                          int V, int B, int strip, int g, int nvg,
                                          float *__restrict__ part)
{
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nsx = adj_strips_x(nx, ny);
    const int cls = strip < nsx ? 0 : 1;
    const int sidx = cls ? strip - nsx : strip;
    const int nL = cls ? ny : nx;  // lane axis size
    const int nsL = (nL + kSL - 1) / kSL;
    const int t0 = (sidx / nsL) * kSW, l0 = (sidx % nsL) * kSL;
    float *my = sh.acc[wid];
    for (int i = lane; i < kAccSize; i += 64) my[i] = 0.f;
    // acc line 0 holds tap line t0 - 1 (spare), lines 1..kSW the strip, line
    // kSW + 1 tap line t0 + kSW (spare)
    float *col = my + lane;
    const double ld = (double)(l0 + lane);  // this lane's driving line
    const BinRange *sb = bins + (size_t)strip * V;

    const int v_begin = (int)((int64_t)V * g / nvg), v_end = (int)((int64_t)V * (g + 1) / nvg);
    for (int v = v_begin + wid; v < v_end; v += kAdjWaves) {
        const BinRange br = sb[v];
        const int lo = __builtin_amdgcn_readfirstlane(br.lo);
        const int hi = __builtin_amdgcn_readfirstlane(br.hi);
        const RayAdj *rv = rays + (size_t)v * B;
        const float *lv = len + (size_t)v * B;
        const float *yv = sino_e + (size_t)v * B;
        for (int cb = lo; cb <= hi; cb += 64) {
            // lane j: bin cb + j
            const int bj = cb + lane;
            double aj = 0.0, kj = 0.0;
            float lyj = 0.f;
            if (bj <= hi) {
                const RayAdj t = rv[bj];
                aj = t.a;
                kj = t.k;
                lyj = fabsf(lv[bj]) * yv[bj];
            }
            const int64_t ai = __double_as_longlong(aj), ki = __double_as_longlong(kj);
            const int alo = (int)ai, ahi = (int)(ai >> 32), klo = (int)ki, khi = (int)(ki >> 32);
            const int ly_bits = __float_as_int(lyj);
            const int nj = min(64, hi - cb + 1);
            for (int j = 0; j < nj; ++j) {
                const double a = __longlong_as_double(
                    ((int64_t)__builtin_amdgcn_readlane(ahi, j) << 32) |
                    (uint32_t)__builtin_amdgcn_readlane(alo, j));
                const double k = __longlong_as_double(
                    ((int64_t)__builtin_amdgcn_readlane(khi, j) << 32) |
                    (uint32_t)__builtin_amdgcn_readlane(klo, j));
                const float ly = __int_as_float(__builtin_amdgcn_readlane(ly_bits, j));
                const double q = fma(k, ld, a);
                const double fl = floor(q);
                const int i0 = (int)fl - t0;  // first tap line, strip-relative
                const float w = (float)(q - fl);
                float wl = w * ly, ol = ly - wl;
                // taps on lines i0 and i0 + 1 -> acc lines ic + 1, ic + 2; a ray
                // that misses the strip adds zeros
                const int ic = min(max(i0, -1), kSW - 1);
                if (ic != i0) {
                    ol = 0.f;
                    wl = 0.f;
                }
                float *pp = col + (ic + 1) * kSL;
                const float u0 = pp[0], u1 = pp[kSL];
                pp[0] = u0 + ol;
                pp[kSL] = u1 + wl;
            }
        }
    }
    __syncthreads();
    // the four copies summed in wave order; stored in normal image layout
    const float *a0 = sh.acc[0], *a1 = sh.acc[1], *a2 = sh.acc[2], *a3 = sh.acc[3];
    for (int i = threadIdx.x; i < kSW * kSL; i += 64 * kAdjWaves) {
        int r, c, k;
        if (cls == 0) {  // strip row = tap line, column = lane
            const int ti = i / kSL, li = i % kSL;
            r = t0 + ti;
            c = l0 + li;
            k = (ti + 1) * kSL + li;
        } else {         // strip row = lane, column = tap line
            const int li = i / kSW, ti = i % kSW;
            r = l0 + li;
            c = t0 + ti;
            k = (ti + 1) * kSL + li;
        }
        if (r < ny && c < nx) part[(size_t)r * nx + c] = ((a0[k] + a1[k]) + a2[k]) + a3[k];
    }
}

// out = scale * (sum over groups of the x-major partials + sum over groups of
// the y-major partials), in that fixed order.  part_e: [2][nvg] planes of
// stride `pstride` floats for this item; i: pixel index.
__device__ __forceinline__ float adj_sum_pixel(const float *__restrict__ part_e, size_t pstride,
                                               int nvg, size_t i)
{
    float s = 0.f;
    for (int q = 0; q < 2 * nvg; ++q) s += part_e[(size_t)q * pstride + i];
    return s;
}

}  // namespace dect
