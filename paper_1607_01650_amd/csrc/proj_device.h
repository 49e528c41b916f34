// Device-side bodies of the projector kernels, shared by the single-geometry
// launches and the batched work-list launches.
//
// Both projectors work on PAIRS of images that share one geometry (the two
// energies of a slice, or two batch items): the position and weight of every
// interpolation tap are computed once and applied to both images.
#pragma once

#include <type_traits>

#include "common.h"

namespace dect {

typedef float f2v __attribute__((ext_vector_type(2)));
// four floats at 8-byte alignment: the taps h and h + 1 of both images of a
// pair in the interleaved padded layout
typedef float f4a8 __attribute__((ext_vector_type(4), aligned(8)));

// Adjoint accumulation: a block's kAdjWaves wavefronts share one strip and split
// its view group between them; each adds into its own LDS copy of the strip,
// stored tap-line-major with row stride kSL (the 64 lanes of an access hit
// distinct banks) plus one spare line on each side.  Every lane walks only
// the bins that hit its own driving line inside the strip (exact per-lane
// ranges from the host), so every bin it takes has its first tap on lines
// -1 .. kSW - 1; a lane with no bin left adds zero to lines -1 and 0, which
// leaves them as they are.  For a pair of images each element holds both
// images' values side by side.
constexpr int kAccOff = 1;
constexpr int kAccRows = kSW + 2 * kAccOff;
constexpr int kAccSize = kAccRows * kSL;

template <int NE> struct AdjElem;
template <> struct AdjElem<1> { typedef float T; };
template <> struct AdjElem<2> { typedef f2v T; };

template <int NE>
struct AdjShared {
    typename AdjElem<NE>::T acc[kAdjWaves][kAccSize];
};

struct alignas(16) AdjRay {
    int64_t a, k;  // strip-relative 32.32 line coordinate at lane 0, slope
};
// Stage slots: one 64-bin chunk per wavefront, then one null slot per
// wavefront (a bin that puts zero weight on the spare line -1 and adds zero)
// for the steps of a lane past its last bin.
constexpr int kStageSlots = kAdjWaves * 64 + kAdjWaves;
struct AdjStage {
    AdjRay ray[kStageSlots];
    f2v ly[kStageSlots];  // |path length| x sinogram value of each image
};

constexpr float kTwoM32 = 2.3283064365386963e-10f;  // 2^-32

// ------------------------------------------------------------ forward ---
// One driving-line loop over lines [l0, l1] for the lanes of one class, on an
// interleaved padded plane.  line: the start of line l0 (the same for every
// lane), bstep the line stride in bytes.  q: this lane's 32.32 coordinate at
// l0 (a sentinel far below -2 for lanes of the other class), dq its step.
// The taps h, h + 1 (h clamped to [-2, nq], so outside the grid both read
// zero padding) of both images are one 16-byte load at a 32-bit per-lane
// byte offset.  Groups of kFwdGroup samples are summed in FP32 and the group sums
// added in FP64; per image i, acc[2i] sums the first taps and acc[2i + 1] the
// weight times the tap difference, the weight being the FP32 value (float)lo
// (Joseph) or (float)(lo - c) * inv for lo > c, else 0 (Siddon, sw = (c,
// inv)), scaled by 2^-32 at the end.
template <bool SID>
__device__ __forceinline__ void walk(const char *line, unsigned bstep, int l0, int l1, int64_t q,
                                     int64_t dq, int nq, SidW sw, double (&acc)[4])
{
    // q as (signed whole part, fraction) stepped with an explicit carry
    int qh = (int)(q >> 32);
    unsigned ql = (unsigned)q;
    const int dh = (int)(dq >> 32);
    const unsigned dl = (unsigned)dq;
    auto sample = [&](float (&s)[4]) {
        const int h = min(max(qh, -2), nq);
        float wq;
        if constexpr (SID) wq = ql > sw.c ? (float)(ql - sw.c) * sw.inv : 0.f;
        else wq = (float)ql;
        const f4a8 v = *(const f4a8 *)(line + (unsigned)(h + 2) * 8u);
        s[0] += v.x;
        s[1] = fmaf(wq, v.z - v.x, s[1]);
        s[2] += v.y;
        s[3] = fmaf(wq, v.w - v.y, s[3]);
        const unsigned nl = ql + dl;
        qh += dh + (nl < ql ? 1 : 0);
        ql = nl;
        line += bstep;
    };
    int i = l0;
    for (; i + kFwdGroup - 1 <= l1; i += kFwdGroup) {
        float s[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < kFwdGroup; ++u) sample(s);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += (double)s[c];
    }
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    for (; i <= l1; ++i) sample(s);
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] += (double)s[c];
}

// Outputs of one forward block for the two images of a pair (image 1 absent
// when sino[1] is NULL).  With sub[i], the value is scale * (A x) -
// sub_scale[i] * sub[i], formed in FP64; sino[i] receives it rounded to FP32
// and, when lo[i] is given, lo[i] the rounding remainder (so that sino + lo
// carries the FP64 value to ~2^-48).
struct FwdOut {
    float *sino[2];
    float *lo[2];
    const float *sub[2];
    double sub_scale[2];
};

// One forward block: views [kFwdViews g, kFwdViews (g + 1)) and kBundle-bin
// bundle j from the index vb (= g * nbundle + j) of one pair; lane = (view
// offset, bin offset).  Wavefront `part` (of kFwdWaves)
// walks the part-th share of each of the bundle's line ranges, so every
// wavefront of the launch carries about the same work, and the partial sums
// are combined in part order.  pad2/padT2: the pair's interleaved padded planes.
// The ray sum is accumulated in FP64 (an FP32 running sum over ~700 samples
// would carry ~1e-6 relative error, which the reconstruction iteration
// amplifies).  On return, wavefront 0 holds this lane's FP64 values in
// res[0..1] (0 where the lane has no ray or the image is absent); the other
// wavefronts hold 0.
struct FwdShared {
    double acc[kFwdWaves][4][64];
};

template <bool SID>
__device__ __forceinline__ void fwd_block(FwdShared &sh, const float *__restrict__ pad2,
                                          const float *__restrict__ padT2,
                                          const RayFwd *__restrict__ rays,
                                          const float *__restrict__ len,
                                          const SidW *__restrict__ sid,
                                          const Bundle *__restrict__ bundles, const FwdOut &o,
                                          int nx, int ny, int V, int B, int nbundle, int vb,
                                          float scale, double (&res)[2])
{
    const int lane = threadIdx.x & 63;
    const int part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int vg = vb / nbundle, j = vb - vg * nbundle;
    const int v = vg * kFwdViews + lane / kBundle;
    const int b = j * kBundle + lane % kBundle;
    const bool act = v < V && b < B;
    const size_t ray = act ? (size_t)v * B + b : 0;
    const RayFwd rf = rays[ray];
    const float L = len[ray];
    SidW sw{0xFFFFFFFFu, 0.f};
    if constexpr (SID) sw = sid[ray];
    const Bundle bu = bundles[vb];
    const int pnx = nx + 2 * kPad, pny = ny + 2 * kPad;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t far = -(int64_t(1000000) << 32);
    const int64_t a = rf.a_fx, k = rf.k_fx;
    // the sign of the stored path length marks the ray class (+ x-major)
    const bool is_x = act && L > 0.f;
    const bool is_y = act && L < 0.f;
    auto share = [&](int l0, int l1, int &s0, int &s1) {
        const int n = l1 - l0 + 1;
        s0 = l0 + n * part / kFwdWaves;
        s1 = l0 + n * (part + 1) / kFwdWaves - 1;
    };
    if (bu.x0 <= bu.x1) {  // x-major: lines are columns of the transposed copy
        int s0, s1;
        share(bu.x0, bu.x1, s0, s1);
        if (s0 <= s1) {
            const int64_t q = is_x ? a + k * (int64_t)s0 : far;
            walk<SID>((const char *)padT2 + (size_t)(s0 + kPad) * pny * 8, (unsigned)(pny * 8), s0,
                      s1, q, is_x ? k : 0, ny, sw, acc);
        }
    }
    if (bu.y0 <= bu.y1) {  // y-major: lines are rows of the padded image
        int s0, s1;
        share(bu.y0, bu.y1, s0, s1);
        if (s0 <= s1) {
            const int64_t q = is_y ? a + k * (int64_t)s0 : far;
            walk<SID>((const char *)pad2 + (size_t)(s0 + kPad) * pnx * 8, (unsigned)(pnx * 8), s0,
                      s1, q, is_y ? k : 0, nx, sw, acc);
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) sh.acc[part][c][lane] = acc[c];
    __syncthreads();
    res[0] = res[1] = 0.0;
    if (part == 0) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            if (!o.sino[i]) continue;
            double a0 = sh.acc[0][2 * i][lane], a1 = sh.acc[0][2 * i + 1][lane];
#pragma unroll
            for (int w = 1; w < kFwdWaves; ++w) {
                a0 += sh.acc[w][2 * i][lane];
                a1 += sh.acc[w][2 * i + 1][lane];
            }
            double sum = (double)fabsf(L) * fma(a1, (double)kTwoM32, a0) * (double)scale;
            if (!act) continue;
            const size_t idx = (size_t)v * B + b;
            if (o.sub[i]) sum -= o.sub_scale[i] * (double)o.sub[i][idx];
            const float hi = (float)sum;
            o.sino[i][idx] = hi;
            if (o.lo[i]) o.lo[i][idx] = (float)(sum - (double)hi);
            res[i] = sum;
        }
    }
    __syncthreads();  // the partials are consumed (persistent callers reuse them)
}

// Fixed-order butterfly sum over the 64 lanes of a wavefront (every lane
// receives the total).
__device__ __forceinline__ double lane_sum(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------------------------ adjoint ---
// One adjoint block: strip `strip` (combined numbering) of NE images (1 or
// 2) that share the geometry, view group g of nvg.  The block's partial image
// of this (class, group) for image i is written to part[i] (a full [ny][nx]
// plane, normal layout; only this strip's pixels).  Per view, each wavefront
// stages the ray data of up to 64 of the strip's bins in LDS (lane j holds
// bin j: the strip-relative 32.32 line coordinate and slope, and |path
// length| x sinogram value per image); every lane then takes the bins of its
// own range in bin order, evaluates the ray on its own driving line (one
// 32 x 32 -> 64-bit multiply-add, so the tap line and FP32 weight are the
// forward pass's) and adds the two interpolation taps of every image, which
// lie on consecutive tap lines, with one paired LDS read and write (no
// atomics: the copy is the wave's own).
template <int NE, bool SID>
__device__ __forceinline__ void adj_block(AdjShared<NE> &sh, const float *const (&sino)[NE],
                                          const RayFwd *__restrict__ rays_fx,
                                          const float *__restrict__ len,
                                          const SidW *__restrict__ sid,
                                          const BinRange *__restrict__ bins,
                                          const LaneRange *__restrict__ lanes, int nx, int ny,
                                          int V, int B, int strip, int g, int nvg,
                                          float *const (&part)[NE],
                                          AdjStage &stage, SidW *sid_stage)
{
    typedef typename AdjElem<NE>::T E;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nsx = adj_strips_x(nx, ny);
    const int cls = strip < nsx ? 0 : 1;
    const int sidx = cls ? strip - nsx : strip;
    const int nL = cls ? ny : nx;  // lane axis size
    const int nsL = (nL + kSL - 1) / kSL;
    const int t0 = (sidx / nsL) * kSW, l0 = (sidx % nsL) * kSL;
    E *my = sh.acc[wid];
    for (int i = lane; i < kAccSize; i += 64) my[i] = E(0.f);
    // acc line j holds tap line t0 + j - kAccOff
    E *col = my + lane;
    // this wavefront's null slot: tap line -1 (strip-relative) at every
    // lane with weight zero on line 0, and zero values
    if (lane == 0) {
        stage.ray[kAdjWaves * 64 + wid] = AdjRay{-(int64_t(1) << 32), 0};
        stage.ly[kAdjWaves * 64 + wid] = f2v(0.f);
        if constexpr (SID) sid_stage[kAdjWaves * 64 + wid] = SidW{0xFFFFFFFFu, 0.f};
    }
    const BinRange *sb = bins + (size_t)strip * V;

    // Views v_begin + wid, + kAdjWaves, ... of this wavefront.  The ray data
    // of a view's first 64-bin chunk and its lane ranges are loaded while the
    // previous view is walked: right after a view's first chunk is staged,
    // the same registers receive the next view's, whose bin range was read
    // one view earlier still.  These loads are unconditional (a bin past the
    // range reads the range's first bin, or bin 0 of an empty range, and a
    // view past the end reads the wavefront's first view; none of it is
    // used), so the compiler does not wait for them at a branch, and the bin
    // range is read by every lane (a vector load: a scalar one would be
    // waited for together with the walk's LDS reads).  Further chunks of a
    // view are loaded when they are reached.
    const int v_begin = (int)((int64_t)V * g / nvg), v_end = (int)((int64_t)V * (g + 1) / nvg);
    const int vfirst = v_begin + wid;
    if (vfirst >= v_end) goto done;
    {
        int vzero;
        asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
        auto load_br = [&](int v) {
            return *(const BinRange *)((const char *)(sb + (v < v_end ? v : vfirst)) +
                                       (unsigned)vzero);
        };
        struct Pre {
            RayFwd t;
            float L, y0, y1;
            SidW sw;
            LaneRange lr;
        };
        auto load_pre = [&](int v, int lo, int hi) {
            // wavefront-uniform bases (scalar registers) plus 32-bit byte
            // offsets per lane
            Pre q;
            const int vv = v < v_end ? v : vfirst;
            const bool empty = lo > hi;
            const unsigned bc = empty ? 0u : (unsigned)min(lo + lane, hi);
            // an empty range reads the tables' first entries (lines that stay in
            // cache), not each view's own
            const size_t vb = empty ? 0 : (size_t)vv * B;
            auto at = [](const auto *base, unsigned bytes) {
                return *(const std::remove_cv_t<std::remove_reference_t<decltype(*base)>> *)(
                    (const char *)base + bytes);
            };
            q.t = at(rays_fx + vb, bc * (unsigned)sizeof(RayFwd));
            q.L = at(len + vb, bc * 4u);
            q.y0 = at(sino[0] + vb, bc * 4u);
            q.y1 = at(sino[NE - 1] + vb, bc * 4u);
            q.sw = SidW{0xFFFFFFFFu, 0.f};
            if constexpr (SID) q.sw = at(sid + vb, bc * (unsigned)sizeof(SidW));
            // (the lane-range table is the kernel's largest input)
            q.lr = at(empty ? lanes : lanes + ((size_t)strip * V + vv) * kSL,
                      empty ? 0u : (unsigned)lane * (unsigned)sizeof(LaneRange));
            return q;
        };
        const int snull = kAdjWaves * 64 + wid;
        const int sbase = wid * 64;
        BinRange bcur = load_br(vfirst);
        int lo = __builtin_amdgcn_readfirstlane(bcur.lo);
        int hi = __builtin_amdgcn_readfirstlane(bcur.hi);
        int steps = __builtin_amdgcn_readfirstlane(bcur.steps);
        Pre pre = load_pre(vfirst, lo, hi);
        BinRange bnext = load_br(vfirst + kAdjWaves);
        for (int v = vfirst; v < v_end; v += kAdjWaves) {
            const RayFwd *rfv = rays_fx + (size_t)v * B;
            const float *lv = len + (size_t)v * B;
            // a strip range too long for the table: every lane takes all of it
            // (and bins that miss a lane's line are masked)
            const bool whole = hi - lo > kLaneRangeMax;
            const int lfirst = whole ? 0 : (int)pre.lr.first, llast = whole ? hi - lo : (int)pre.lr.last;
            // stage chunk cb: lane j holds bin cb + j (strip-relative line
            // coordinate); the first chunk from the prefetched registers
            auto stage_chunk = [&](int cb) {
                const int bj = cb + lane;
                AdjRay me{0, 0};
                f2v my_ly = f2v(0.f);
                SidW my_sw{0xFFFFFFFFu, 0.f};
                if (cb == lo) {
                    if (bj <= hi) {
                        me.a = pre.t.a_fx + pre.t.k_fx * l0 - ((int64_t)t0 << 32);
                        me.k = pre.t.k_fx;
                        const float L = fabsf(pre.L);
                        my_ly.x = L * pre.y0;
                        if constexpr (NE > 1) my_ly.y = L * pre.y1;
                        if constexpr (SID) my_sw = pre.sw;
                    }
                } else if (bj <= hi) {
                    const RayFwd t = rfv[bj];
                    me.a = t.a_fx + t.k_fx * l0 - ((int64_t)t0 << 32);
                    me.k = t.k_fx;
                    const float L = fabsf(lv[bj]);
                    my_ly.x = L * sino[0][(size_t)v * B + bj];
                    if constexpr (NE > 1) my_ly.y = L * sino[NE - 1][(size_t)v * B + bj];
                    if constexpr (SID) my_sw = sid[(size_t)v * B + bj];
                }
                stage.ray[sbase + lane] = me;
                stage.ly[sbase + lane] = my_ly;
                if constexpr (SID) sid_stage[sbase + lane] = my_sw;
            };
            if (lo <= hi) stage_chunk(lo);
            // the next view's bin range (read one view ago), then its first
            // chunk into the registers just staged, and the range after it
            const int nlo = __builtin_amdgcn_readfirstlane(bnext.lo);
            const int nhi = __builtin_amdgcn_readfirstlane(bnext.hi);
            const int nsteps = __builtin_amdgcn_readfirstlane(bnext.steps);
            pre = load_pre(v + kAdjWaves, nlo, nhi);
            bnext = load_br(v + 2 * kAdjWaves);
            // the 64-bin chunks of the strip range; kExact: every bin a lane
            // takes is one of its own (its first tap line lies in -1 .. kSW - 1
            // by the host's exact per-lane ranges), so only the steps past its
            // last bin need care, and they take the null slot
            auto chunks = [&](auto exact_tag) {
                constexpr bool kExact = decltype(exact_tag)::value;
                for (int cb = lo; cb <= hi; cb += 64) {
                    if (cb != lo) stage_chunk(cb);
                    // this lane's bins in the chunk: [f, e], chunk-relative
                    const int rel = cb - lo;
                    const int f = max(lfirst, rel) - rel;
                    const int e = min(llast, rel + 63) - rel;
                    const int n = e - f + 1;
                    // one step: bin b (staged) at this lane.  Masked mode: a lane
                    // past its last bin, or taking a bin that misses its line,
                    // adds zero to lines -1 and 0
                    auto step = [&](const AdjRay &b, f2v y, SidW sw, bool ok) {
                        const uint64_t p = (uint64_t)(uint32_t)b.k * (uint32_t)lane + (uint64_t)b.a;
                        // high word + k_hi lane as a 24-bit multiply-add (k_hi is -1, 0
                    // or 1); written out, because the compiler otherwise forms it
                    // with a second 64-bit multiply-add
                    int qh;
                    asm("v_mad_i32_i24 %0, %1, %2, %3"
                        : "=v"(qh)
                        : "v"((int)(b.k >> 32)), "v"(lane), "v"((int)(uint32_t)(p >> 32)));
                        int i0 = qh;
                        if constexpr (!kExact) {
                            ok = ok && qh >= -1 && qh <= kSW - 1;
                            i0 = ok ? qh : -1;
                            if (!ok) y = f2v(0.f);
                        }
                        const uint32_t lo32 = (uint32_t)p;
                        float w;
                        if constexpr (SID)
                            w = (lo32 > sw.c ? (float)(lo32 - sw.c) * sw.inv : 0.f) * kTwoM32;
                        else
                            w = (float)lo32 * kTwoM32;
                        E *pp = col + (i0 + kAccOff) * kSL;
                        E u0 = pp[0], u1 = pp[kSL];
                        if constexpr (NE == 1) {
                            u0 += fmaf(-w, y.x, y.x);
                            u1 = fmaf(w, y.x, u1);
                        } else {
                            u0.x += fmaf(-w, y.x, y.x);
                            u0.y += fmaf(-w, y.y, y.y);
                            u1.x = fmaf(w, y.x, u1.x);
                            u1.y = fmaf(w, y.y, u1.y);
                        }
                        pp[0] = u0;
                        pp[kSL] = u1;
                    };
                    // the stage slot of step t at this lane
                    auto slot = [&](int t) {
                        if constexpr (kExact) return t < n ? sbase + f + t : snull;
                        else return sbase + (t < n ? f + t : 0);
                    };
                    // two steps at a time, both bins' stage reads issued first
                    int t = 0;
                    for (; t + 1 < steps; t += 2) {
                        const int j0 = slot(t), j1 = slot(t + 1);
                        const AdjRay b0 = stage.ray[j0], b1 = stage.ray[j1];
                        const f2v y0 = stage.ly[j0], y1 = stage.ly[j1];
                        SidW s0{0u, 0.f}, s1{0u, 0.f};
                        if constexpr (SID) {
                            s0 = sid_stage[j0];
                            s1 = sid_stage[j1];
                        }
                        step(b0, y0, s0, t < n);
                        step(b1, y1, s1, t + 1 < n);
                    }
                    if (t < steps) {
                        const int j = slot(t);
                        SidW sj{0u, 0.f};
                        if constexpr (SID) sj = sid_stage[j];
                        step(stage.ray[j], stage.ly[j], sj, t < n);
                    }
                }
            };
            if (lo <= hi) {
                if (whole) chunks(std::false_type{});
                else chunks(std::true_type{});
            }
            lo = nlo;
            hi = nhi;
            steps = nsteps;
        }
    }
done:
    __syncthreads();
    // the copies summed in wave order; stored in normal image layout
    for (int i = threadIdx.x; i < kSW * kSL; i += kAdjThreads) {
        int r, c, k;
        if (cls == 0) {  // strip row = tap line, column = lane
            const int ti = i / kSL, li = i % kSL;
            r = t0 + ti;
            c = l0 + li;
            k = (ti + kAccOff) * kSL + li;
        } else {         // strip row = lane, column = tap line
            const int li = i / kSW, ti = i % kSW;
            r = l0 + li;
            c = t0 + ti;
            k = (ti + kAccOff) * kSL + li;
        }
        if (r < ny && c < nx) {
            E sum = sh.acc[0][k];
#pragma unroll
            for (int w = 1; w < kAdjWaves; ++w) sum += sh.acc[w][k];
            if constexpr (NE == 1) {
                part[0][(size_t)r * nx + c] = sum;
            } else {
                part[0][(size_t)r * nx + c] = sum.x;
                part[1][(size_t)r * nx + c] = sum.y;
            }
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
