// Device-side bodies of the projector kernels, shared by the single-geometry
// launches and the batched work-list launches.
#pragma once

#include "common.h"

namespace dect {

// Adjoint accumulation: a block's kAdjWaves wavefronts share one strip and split
// its view group between them; each adds into its own LDS copy of the strip,
// stored tap-line-major with row stride kSL (the 64 lanes of an access hit
// distinct banks) plus two spare lines on each side: a tap pair whose first
// line is clamped to [-2, kSW] then always lands on real lines only when it
// belongs there, and on spare lines otherwise.
constexpr int kAccRows = kSW + 4;
constexpr int kAccSize = kAccRows * kSL;

struct AdjShared {
    float acc[kAdjWaves][kAccSize];
};

constexpr float kTwoM32 = 2.3283064365386963e-10f;  // 2^-32

// ------------------------------------------------------------ forward ---
// One driving-line loop over lines [l0, l1] for the lanes of one class, on
// the padded plane `rs` (a buffer resource over the whole plane).  soff: byte
// offset of line l0's element -2 (the plane's line start) and bstep the line
// stride in bytes, both the same for every lane.  q: this lane's 32.32
// coordinate at l0 (a sentinel far below -2 for lanes of the other class),
// dq its step.  The taps h, h + 1 (h clamped to [-2, nq], so outside the grid
// both read zero padding) are addressed by a 32-bit per-lane byte offset.
// Groups of four samples are summed in FP32 and the group sums added in FP64
// (acc0: first taps, acc1: weight x tap difference, the weight being the FP32
// value (float)lo, scaled by 2^-32 at the end).
__device__ __forceinline__ void walk(__amdgpu_buffer_rsrc_t rs, unsigned soff, unsigned bstep,
                                     int l0, int l1, int64_t q, int64_t dq, int nq,
                                     double &acc0, double &acc1)
{
    auto sample = [&](float &s0, float &s1) {
        const int h = min(max((int)(q >> 32), -2), nq);
        const unsigned lo = (unsigned)q;
        const unsigned vo = (unsigned)(h + 2) * 4u;
        const float v0 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, soff, 0));
        const float v1 =
            __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo + 4u, soff, 0));
        s0 += v0;
        s1 = fmaf((float)lo, v1 - v0, s1);
        q += dq;
        soff += bstep;
    };
    int i = l0;
    for (; i + 3 <= l1; i += 4) {
        float s0 = 0.f, s1 = 0.f;
        sample(s0, s1);
        sample(s0, s1);
        sample(s0, s1);
        sample(s0, s1);
        acc0 += (double)s0;
        acc1 += (double)s1;
    }
    float s0 = 0.f, s1 = 0.f;
    for (; i <= l1; ++i) sample(s0, s1);
    acc0 += (double)s0;
    acc1 += (double)s1;
}

// Raw buffer resource over n_bytes at p (word 3 as for gfx9-family raw
// buffers).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float *p, unsigned n_bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)n_bytes, 0x00020000);
}

// One forward block: view v and 64-bin bundle j from the index vb (= v *
// nbundle + j) of one batch item; lane = bin.  Wavefront `part` (of 4) walks
// the part-th quarter of each of the bundle's line ranges, so every
// wavefront of the launch carries about the same work, and the four partial
// sums are combined in part order.  pad_e/padT_e: that item's padded image
// copies, sino_e its sinogram.  The ray sum is accumulated in FP64 (an FP32
// running sum over ~700 samples would carry ~1e-6 relative error, which the
// reconstruction iteration amplifies).  With sub_e the value is
// scale * (A x) - sub_scale * sub_e, formed in FP64.  sino_e receives the
// value rounded to FP32 and, when lo_e is given, lo_e the rounding remainder
// (so that sino_e + lo_e carries the FP64 value to ~2^-48).  Returns, in
// wavefront 0, this lane's FP64 value (0 when the lane has no ray); 0 in the
// other wavefronts.
struct FwdShared {
    double acc[4][2][64];
};

__device__ __forceinline__ double fwd_block(FwdShared &sh, const float *__restrict__ pad_e,
                                           const float *__restrict__ padT_e,
                                           const RayFwd *__restrict__ rays,
                                           const float *__restrict__ len,
                                           const Bundle *__restrict__ bundles,
                                           float *__restrict__ sino_e, int nx, int ny, int B,
                                           int nbundle, int vb, float scale,
                                           const float *__restrict__ sub_e = nullptr,
                                           double sub_scale = 0.0,
                                           float *__restrict__ lo_e = nullptr)
{
    const int lane = threadIdx.x & 63;
    const int part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int v = vb / nbundle, j = vb - v * nbundle;
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
    const unsigned plane_bytes = (unsigned)((size_t)pnx * pny * sizeof(float));
    auto quarter = [&](int l0, int l1, int &s0, int &s1) {
        const int n = l1 - l0 + 1;
        s0 = l0 + n * part / 4;
        s1 = l0 + n * (part + 1) / 4 - 1;
    };
    if (bu.x0 <= bu.x1) {  // x-major: lines are columns of the transposed copy
        int s0, s1;
        quarter(bu.x0, bu.x1, s0, s1);
        if (s0 <= s1) {
            int64_t q = is_x ? a + k * (int64_t)s0 : far;
            int64_t dq = is_x ? k : 0;
            walk(plane_rsrc(padT_e, plane_bytes), (unsigned)((s0 + kPad) * pny * 4),
                 (unsigned)(pny * 4), s0, s1, q, dq, ny, acc0, acc1);
        }
    }
    if (bu.y0 <= bu.y1) {  // y-major: lines are rows of the padded image
        int s0, s1;
        quarter(bu.y0, bu.y1, s0, s1);
        if (s0 <= s1) {
            int64_t q = is_y ? a + k * (int64_t)s0 : far;
            int64_t dq = is_y ? k : 0;
            walk(plane_rsrc(pad_e, plane_bytes), (unsigned)((s0 + kPad) * pnx * 4),
                 (unsigned)(pnx * 4), s0, s1, q, dq, nx, acc0, acc1);
        }
    }
    sh.acc[part][0][lane] = acc0;
    sh.acc[part][1][lane] = acc1;
    __syncthreads();
    double sum = 0.0;
    if (part == 0) {
        acc0 = ((sh.acc[0][0][lane] + sh.acc[1][0][lane]) + sh.acc[2][0][lane]) + sh.acc[3][0][lane];
        acc1 = ((sh.acc[0][1][lane] + sh.acc[1][1][lane]) + sh.acc[2][1][lane]) + sh.acc[3][1][lane];
        sum = (double)fabsf(L) * fma(acc1, (double)kTwoM32, acc0) * (double)scale;
        if (sub_e && act) sum -= sub_scale * (double)sub_e[(size_t)v * B + b];
        const float hi = (float)sum;
        if (act) {
            sino_e[(size_t)v * B + b] = hi;
            if (lo_e) lo_e[(size_t)v * B + b] = (float)(sum - (double)hi);
        } else {
            sum = 0.0;
        }
    }
    __syncthreads();  // the partials are consumed (persistent callers reuse them)
    return sum;
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
    // acc line j holds tap line t0 + j - 2: lines 0, 1 and kSW + 2, kSW + 3
    // are spare
    float *col = my + lane;
    const double ld = (double)lane;  // this lane's driving line, relative to l0
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
            // lane j: bin cb + j, its line coordinate moved to the strip
            // origin, q' = (a + k l0 - t0) + k lane (exact: all terms are
            // multiples of 2^-32 below 2^21)
            const int bj = cb + lane;
            double aj = 0.0, kj = 0.0;
            float lyj = 0.f;
            if (bj <= hi) {
                const RayAdj t = rv[bj];
                aj = fma(t.k, (double)l0, t.a) - (double)t0;
                kj = t.k;
                lyj = fabsf(lv[bj]) * yv[bj];
            }
            const int64_t ai = __double_as_longlong(aj), ki = __double_as_longlong(kj);
            const int alo = (int)ai, ahi = (int)(ai >> 32), klo = (int)ki, khi = (int)(ki >> 32);
            const int ly_bits = __float_as_int(lyj);
            const int nj = min(64, hi - cb + 1);
            // one bin: this lane's tap pair, added in bin order
            auto tap = [&](int j) {
                const double a = __longlong_as_double(
                    ((int64_t)__builtin_amdgcn_readlane(ahi, j) << 32) |
                    (uint32_t)__builtin_amdgcn_readlane(alo, j));
                const double k = __longlong_as_double(
                    ((int64_t)__builtin_amdgcn_readlane(khi, j) << 32) |
                    (uint32_t)__builtin_amdgcn_readlane(klo, j));
                const float ly = __int_as_float(__builtin_amdgcn_readlane(ly_bits, j));
                const double q = fma(k, ld, a);
                const double fl = floor(q);
                const int i0 = min(max((int)fl, -2), kSW);  // first tap line, strip-relative
                const float w = (float)(q - fl);
                const float wl = w * ly, ol = ly - wl;
                float *pp = col + (i0 + 2) * kSL;
                const float u0 = pp[0], u1 = pp[kSL];
                pp[0] = u0 + ol;
                pp[kSL] = u1 + wl;
            };
            int j = 0;
            for (; j + 1 < nj; j += 2) {
                tap(j);
                tap(j + 1);
            }
            if (j < nj) tap(j);
        }
    }
    __syncthreads();
    // the copies summed in wave order; stored in normal image layout
    for (int i = threadIdx.x; i < kSW * kSL; i += kAdjThreads) {
        int r, c, k;
        if (cls == 0) {  // strip row = tap line, column = lane
            const int ti = i / kSL, li = i % kSL;
            r = t0 + ti;
            c = l0 + li;
            k = (ti + 2) * kSL + li;
        } else {         // strip row = lane, column = tap line
            const int li = i / kSW, ti = i % kSW;
            r = l0 + li;
            c = t0 + ti;
            k = (ti + 2) * kSL + li;
        }
        if (r < ny && c < nx) {
            float sum = sh.acc[0][k];
#pragma unroll
            for (int w = 1; w < kAdjWaves; ++w) sum += sh.acc[w][k];
            part[(size_t)r * nx + c] = sum;
        }
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
