// Device-side bodies of the ADM-TV kernels (Eq. 10), shared by the
// single-geometry launches and the batched work-list launches.  Every body
// keeps all threads of the block on the same path through its barriers, so a
// persistent loop can run several items per block.
#pragma once

#include "common.h"

namespace dect {

// TV stencil tile: kTX columns x kTY rows, one pixel per thread of a 256-thread
// block (wide tiles read longer row segments of every plane)
#ifndef DECT_TV_TX
#define DECT_TV_TX 32
#endif
constexpr int kTX = DECT_TV_TX;
constexpr int kTY = 256 / kTX;
static_assert(kTX * kTY == 256 && kTX >= 8 && kTY >= 4, "tv tile must hold 256 pixels");
constexpr int kGW = kTX + 1, kGH = kTY + 1;  // G region (rows/cols -1 .. tile - 1)
constexpr int kWW = kTX + 2, kWH = kTY + 2;  // w region (rows/cols -1 .. tile)
constexpr int kFW = kTX + 3, kFH = kTY + 3;  // f region (rows/cols -2 .. tile)
static_assert(kGW * kGH <= 512 && kWW * kWH <= 512, "two pixels per thread at most");
// FP64 partial sums one TV tile leaves per energy: TV(f), |G|^2, |grad G|^2,
// |grad f - z|^2, |f|^2, <G_prev, h>, <G, h>
constexpr int kTvParts = 7;
// Device log row: J_high, J_low, alpha_high, alpha_low, |grad f - z|_high,
// |grad f - z|_low, |G|_high, |G|_low (the last four before the row's step;
// zero on the final row)
constexpr int kLogW = 8;

struct AdmScalars {
    double alpha;   // step used by the next update
    double c_prev;  // Cauchy step of the previous G
    double rr;      // |r^k|^2 of the current f
    double J;       // last logged objective
    double relchg;  // last relative image change
    double beta;    // Eq. 3 weight of this energy
    double ss, sy;  // non-negative variant: <s,s> and <s,y> of the last projected step
    double den_prev;  // mu |A G|^2 + rho |grad G|^2 of the previous G (BB2 numerator)
    double gg_prev, gh_prev, gradg_prev;  // |G|^2, <G, h>, |grad G|^2 of the previous G
    int32_t has_prev, stopped, nonfinite_iter, pending;
    int32_t stop_next;  // the stop rule held: stop once this iteration's update is done
    int64_t iter;      // iterations completed
    int64_t log_base;  // iteration index of log row 0 for this call
};

// v of this lane moved along the wavefront by the DPP control CTRL (rows of 16
// lanes not in ROW_MASK, and lanes whose source lies outside their row, get
// 0); an FP64 value moves as its two 32-bit halves
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, true);
    return __hiloint2double(hi, lo);
}

// Sum of v over the 64 lanes of a full wavefront, in a fixed order, returned
// to every lane: a prefix sum within each row of 16 lanes (shifts by 1, 2, 4
// and 8 lanes), then rows 1 and 3 add the total of the row before them (the
// row's last lane, broadcast), and rows 2 and 3 add lane 31; lane 63 then
// holds the total, which is read back as a wavefront-uniform value.  Every
// step is a VALU lane move, with no LDS round trip.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<0x111>(v);       // row_shr:1
    v += dpp_f64<0x112>(v);       // row_shr:2
    v += dpp_f64<0x114>(v);       // row_shr:4
    v += dpp_f64<0x118>(v);       // row_shr:8
    v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// x + y where lanes 0-31 take x of lanes l and l + 32, lanes 32-63 y of lanes
// l - 32 and l (permlane32 swap of the upper half of x with the lower half of
// y); with ROWS16, rows of 16 lanes instead: even rows take x of rows r and
// r + 1, odd rows y of rows r - 1 and r
template <bool ROWS16>
__device__ __forceinline__ double swap_add(double x, double y)
{
    const unsigned xl = (unsigned)__double2loint(x), xh = (unsigned)__double2hiint(x);
    const unsigned yl = (unsigned)__double2loint(y), yh = (unsigned)__double2hiint(y);
    if constexpr (ROWS16) {
        const auto lo = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
        return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
    } else {
        const auto lo = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
        return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
    }
}

// Fixed-order sum over a 256-thread block of NV values; every thread gets
// the totals in `out` (LDS).  Ends with a barrier.  For 3 to 8 values the
// wavefront reduces them together: each exchange step halves the values a
// lane holds and doubles the lanes each partial covers (wave halves, then
// row pairs, then the two halves of each row: 8 values, 4, 2, 1), and a
// butterfly over the last 8 lanes completes each sum, so that lane 8 j holds
// value j's wavefront total.  The four wavefronts' totals are added in
// wavefront order.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *out)
{
    __shared__ double sh[4][NV];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if constexpr (NV >= 3 && NV <= 8) {
        double a[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = j < NV ? v[j] : 0.0;
        double b[4], c[2];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = swap_add<false>(a[j], a[j + 4]);
#pragma unroll
        for (int j = 0; j < 2; ++j) c[j] = swap_add<true>(b[j], b[j + 2]);
        // lanes with bit 3 clear keep c[0] and send c[1] to lane l ^ 8
        // (row_ror:8), the others the reverse
        const bool up = (lane & 8) != 0;
        const double keep = up ? c[1] : c[0], send = up ? c[0] : c[1];
        double d = keep + dpp_f64<0x128>(send);
        d += dpp_f64<0xB1>(d);   // quad_perm [1, 0, 3, 2]
        d += dpp_f64<0x4E>(d);   // quad_perm [2, 3, 0, 1]
        d += dpp_f64<0x141>(d);  // row_half_mirror
        if ((lane & 7) == 0 && (lane >> 3) < NV) sh[wid][lane >> 3] = d;
    } else {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
        if (lane == 0)
#pragma unroll
            for (int i = 0; i < NV; ++i) sh[wid][i] = v[i];
    }
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        int t = threadIdx.x;
        out[t] = ((sh[0][t] + sh[1][t]) + sh[2][t]) + sh[3][t];
    }
    __syncthreads();
}

// Device pointers of one slice's ADM state (both energies).  Layouts: f, flo
// [2][N]; r, rlo, p, plo [2][M]; lambda, z [parity][energy][comp][N];
// gpad, gpadT [(ny+4)(nx+4)][2] / [(nx+4)(ny+4)][2] (the projector's
// interleaved padded layouts, both energies of a pixel side by side); partials per energy
// and block; adjpart the back-projector's partial planes of h = mu A^T r
// ([energy][class][view group][N]).  The image and the residual r = A f - beta m are carried as
// unevaluated sums of two FP32 values (f + flo, r + rlo, |lo| <= half an ulp
// of the first part), and A G arrives as p + plo from the projector's FP64
// sum; both updates are formed in FP64.  The iterates then take no FP32
// rounding per step, which the iteration would amplify.  The projector,
// the back-projector and the finite differences read FP32 values (f, r and
// f + flo respectively).
struct AdmPtrs {
    float *f, *flo, *r, *rlo, *p, *plo, *lam, *z, *gpad, *gpadT, *adjpart;
    double *p_tv, *p_fwd, *p_rr, *p_tvo, *log;
    double *p_ss, *p_ff, *p_gs;  // non-negative variant: [2][nbi] step partials
    int log_rows;
    AdmScalars *sc;
    int nb_tv, nb_fwd, nbi, nbs;
};

dect_status adm_init(const GeomTables &t, const AdmPtrs &P, int nvg, const float *mh,
                     const float *ml, double mu, double bh, double bl, const float *x0h,
                     const float *x0l, hipStream_t s);
dect_status adm_mark_log(const AdmPtrs &P, hipStream_t s);
dect_status adm_finish(const GeomTables &t, const AdmPtrs &P, float *xh, float *xl, double mu,
                       double bh, double bl, hipStream_t s,
                       bool coupled = false);

// Pointers of one energy image's ADM state.  h: hq partial planes whose sum
// times hmu is mu A^T r (summed here in plane order, as the back-projector's
// own summation kernel does).  gpad/gpadT point at this energy's first
// element of the interleaved padded layouts (element stride 2).
struct AdmImg {
    const float *f, *h, *lxi, *lyi, *zxi, *zyi;
    float *lxo, *lyo, *zxo, *zyo, *gpad, *gpadT;
    const float *flo;
    int hq;
    float hmu;
    // coupled TV: the other energy's f, f_lo, lambda and z (the z-step
    // shrinks both energies' gradients together), whether its deferred
    // multiplier step is pending, and whether this block records the joint
    // TV (energy 0 does, energy 1 records none)
    const float *f2, *flo2, *lxi2, *lyi2, *zxi2, *zyi2;
    int pending2, record_tv;
};

// ------------------------------------------------------------- tv_fused ---
// Tile origin (r0, c0).  Regions relative to it: f on rows/cols -2 .. tile,
// w on -1 .. tile, G on -1 .. tile - 1, grad G on the kTX x kTY tile.  part
// receives the kTvParts sums (TV(f), |G|^2, |grad G|^2, |grad f - z|^2, |f|^2,
// <G_prev, h>, <G, h>) of the tile, where G_prev is the value the padded G
// buffer holds at the tile's pixels before this tile overwrites it (the
// previous iteration's G) and h = mu A^T r the data term of this G.
//
// A tile runs in two stages.  tv_load issues every global read the tile
// needs into registers and uses none of them: the first kTvHq partial planes
// of h on the thread's (at most two) G-region pixels, lambda and z on its
// w-region pixels, f and f_lo on its f-region pixels, and the previous G at
// its own pixel.  tv_compute then does the arithmetic.  The tile's reads thus
// go out as one batch: one memory latency, not one per plane group and input
// kind.
constexpr int kTvHq = 8;
static_assert(kFW * kFH <= 512, "f region: two pixels per thread at most");

template <bool COUPLED>
struct TvIn {
    float h[2][kTvHq];
    float lx[2], ly[2], zx[2], zy[2];
    float lx2[2], ly2[2], zx2[2], zy2[2];  // coupled TV: the other energy's
    float f[2], fl[2], f2[2], fl2[2];
    float gprev;
};

// Region pixel i of a tile (rows and columns from (r0 + d, c0 + d), w wide, n
// pixels): its image offset, and whether it exists and lies in the image.
__device__ __forceinline__ bool tv_pix(int i, int w, int n, int r0, int c0, int d, int nx, int ny,
                                       size_t &o)
{
    const int r = r0 + d + i / w, c = c0 + d + i % w;
    const bool ok = i < n && r >= 0 && r < ny && c >= 0 && c < nx;
    o = ok ? (size_t)r * nx + c : 0;
    return ok;
}

// Every load is unconditional: one outside the image (or a plane beyond the
// slice's count, or z while no multiplier step is pending) reads element 0
// of its array instead, and tv_compute discards it.  No load sits under a
// branch, where the compiler would fold the first use into the branch and
// wait for the load there.
template <bool COUPLED>
__device__ __forceinline__ void tv_load(int r0, int c0, const AdmImg &m, int nx, int ny,
                                        TvIn<COUPLED> &in)
{
    const size_t N = (size_t)nx * ny;
    const int hq = m.hq < kTvHq ? m.hq : kTvHq;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        size_t o;
        tv_pix(threadIdx.x + 256 * k, kGW, kGW * kGH, r0, c0, -1, nx, ny, o);
#pragma unroll
        for (int u = 0; u < kTvHq; ++u) in.h[k][u] = m.h[u < hq ? o + (size_t)u * N : 0];
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        size_t o;
        tv_pix(threadIdx.x + 256 * k, kWW, kWW * kWH, r0, c0, -1, nx, ny, o);
        in.lx[k] = m.lxi[o];
        in.ly[k] = m.lyi[o];
        in.zx[k] = m.zxi[o];
        in.zy[k] = m.zyi[o];
        if constexpr (COUPLED) {
            in.lx2[k] = m.lxi2[o];
            in.ly2[k] = m.lyi2[o];
            in.zx2[k] = m.zxi2[o];
            in.zy2[k] = m.zyi2[o];
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        size_t o;
        tv_pix(threadIdx.x + 256 * k, kFW, kFW * kFH, r0, c0, -2, nx, ny, o);
        in.f[k] = m.f[o];
        in.fl[k] = m.flo[o];
        if constexpr (COUPLED) {
            in.f2[k] = m.f2[o];
            in.fl2[k] = m.flo2[o];
        }
    }
    {
        const int r = r0 + (int)threadIdx.x / kTX, c = c0 + (int)threadIdx.x % kTX;
        const size_t pnx = (size_t)nx + 2 * kPad;
        in.gprev = m.gpad[r < ny && c < nx ? 2 * ((size_t)(r + kPad) * pnx + c + kPad) : 0];
    }
}

template <bool COUPLED>
__device__ __forceinline__ void tv_compute(int r0, int c0, const AdmImg &m, const TvIn<COUPLED> &in,
                                           double *part, bool pending, int nx, int ny, float rho,
                                           float xi)
{
    __shared__ float sf[kFH][kFW + 1], sl[kFH][kFW + 1];
    __shared__ float sf2[COUPLED ? kFH : 1][COUPLED ? kFW + 1 : 1];
    __shared__ float sl2[COUPLED ? kFH : 1][COUPLED ? kFW + 1 : 1];
    __shared__ float swx[kWH][kWW + 1], swy[kWH][kWW + 1];
    __shared__ float sg[kGH][kGW + 1], sh[kGH][kGW + 1];
    __shared__ double outv[kTvParts];
    const float inv_rho = 1.0f / rho;

#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i < kFW * kFH) {
            size_t o;
            const bool ok = tv_pix(i, kFW, kFW * kFH, r0, c0, -2, nx, ny, o);
            const int rr = i / kFW, cc = i % kFW;
            sf[rr][cc] = ok ? in.f[k] : 0.f;
            sl[rr][cc] = ok ? in.fl[k] : 0.f;
            if constexpr (COUPLED) {
                sf2[rr][cc] = ok ? in.f2[k] : 0.f;
                sl2[rr][cc] = ok ? in.fl2[k] : 0.f;
            }
        }
    }

    // h = hmu * (sum of the partial planes, in plane order) on the G region;
    // planes beyond the first kTvHq are read here
    float hsum[2] = {0.f, 0.f};
    {
        const size_t N = (size_t)nx * ny;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int i = threadIdx.x + 256 * k;
            const int rr = i / kGW, cc = i % kGW;
            const int r = r0 - 1 + rr, c = c0 - 1 + cc;
            if (i < kGW * kGH && r >= 0 && r < ny && c >= 0 && c < nx) {
                float acc = 0.f;
#pragma unroll
                for (int u = 0; u < kTvHq; ++u)
                    if (u < m.hq) acc += in.h[k][u];
                if (m.hq > kTvHq) {
                    const float *hp = m.h + (size_t)r * nx + c;
                    for (int q = kTvHq; q < m.hq; ++q) acc += hp[(size_t)q * N];
                }
                hsum[k] = acc * m.hmu;
            }
        }
    }
    __syncthreads();

    double tv = 0.0, pres = 0.0, ff = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i >= kWW * kWH) break;
        int rr = i / kWW, cc = i % kWW;
        int r = r0 - 1 + rr, c = c0 - 1 + cc;
        float wx = 0.f, wy = 0.f;
        if (r >= 0 && r < ny && c >= 0 && c < nx) {
            size_t o = (size_t)r * nx + c;
            float fc = sf[rr + 1][cc + 1], lc = sl[rr + 1][cc + 1];
            float dx = c >= 1 ? (fc - sf[rr + 1][cc]) + (lc - sl[rr + 1][cc]) : 0.f;
            float dy = r >= 1 ? (fc - sf[rr][cc + 1]) + (lc - sl[rr][cc + 1]) : 0.f;
            float lx = in.lx[k], ly = in.ly[k];  // loaded at this pixel (it is in the image)
            if (pending) {
                lx -= xi * (dx - in.zx[k]);
                ly -= xi * (dy - in.zy[k]);
            }
            float vx = dx - lx / rho, vy = dy - ly / rho;
            float n, tvi;
            if constexpr (COUPLED) {
                // the other energy's gradient and multiplier at this pixel, as
                // its own block computes them; the joint norms are summed in
                // energy order (own pair first in energy 0's block)
                float f2c = sf2[rr + 1][cc + 1], l2c = sl2[rr + 1][cc + 1];
                float dx2 = c >= 1 ? (f2c - sf2[rr + 1][cc]) + (l2c - sl2[rr + 1][cc]) : 0.f;
                float dy2 = r >= 1 ? (f2c - sf2[rr][cc + 1]) + (l2c - sl2[rr][cc + 1]) : 0.f;
                float lx2 = in.lx2[k], ly2 = in.ly2[k];
                if (m.pending2) {
                    lx2 -= xi * (dx2 - in.zx2[k]);
                    ly2 -= xi * (dy2 - in.zy2[k]);
                }
                float vx2 = dx2 - lx2 / rho, vy2 = dy2 - ly2 / rho;
                const float a = vx * vx + vy * vy, b = vx2 * vx2 + vy2 * vy2;
                n = sqrtf(m.record_tv ? a + b : b + a);
                const float ta = dx * dx + dy * dy, tb = dx2 * dx2 + dy2 * dy2;
                tvi = m.record_tv ? sqrtf(ta + tb) : 0.f;
            } else {
                n = sqrtf(vx * vx + vy * vy);
                tvi = sqrtf(dx * dx + dy * dy);
            }
            float s = n > inv_rho ? (n - inv_rho) / n : 0.f;
            float zx = s * vx, zy = s * vy;
            wx = rho * (dx - zx) - lx;
            wy = rho * (dy - zy) - ly;
            if (rr >= 1 && rr <= kTY && cc >= 1 && cc <= kTX) {
                m.lxo[o] = lx;
                m.lyo[o] = ly;
                m.zxo[o] = zx;
                m.zyo[o] = zy;
                tv += (double)tvi;
                double ex = (double)dx - zx, ey = (double)dy - zy;
                pres += ex * ex + ey * ey;
                ff += (double)fc * fc;
            }
        }
        swx[rr][cc] = wx;
        swy[rr][cc] = wy;
    }
    __syncthreads();

    // G = h + grad^T w on the G region
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i >= kGW * kGH) break;
        int rr = i / kGW, cc = i % kGW;
        int r = r0 - 1 + rr, c = c0 - 1 + cc;
        float gv = 0.f;
        if (r >= 0 && r < ny && c >= 0 && c < nx) {
            float s = hsum[k];
            if (c >= 1) s += swx[rr][cc];
            if (c + 1 <= nx - 1) s -= swx[rr][cc + 1];
            if (r >= 1) s += swy[rr][cc];
            if (r + 1 <= ny - 1) s -= swy[rr + 1][cc];
            gv = s;
        }
        sg[rr][cc] = gv;
        sh[rr][cc] = hsum[k];
    }
    __syncthreads();

    double gg = 0.0, gradg = 0.0, gh_old = 0.0, gh = 0.0;
    const int pnx = nx + 2 * kPad, pny = ny + 2 * kPad;
    {
        int rr = threadIdx.x / kTX, cc = threadIdx.x % kTX;
        int r = r0 + rr, c = c0 + cc;
        if (r < ny && c < nx) {
            float gv = sg[rr + 1][cc + 1];
            float hv = sh[rr + 1][cc + 1];
            float gx = c >= 1 ? gv - sg[rr + 1][cc] : 0.f;
            float gy = r >= 1 ? gv - sg[rr][cc + 1] : 0.f;
            gg = (double)gv * gv;
            gradg = (double)gx * gx + (double)gy * gy;
            // the previous G at this pixel was read by this thread alone (in
            // tv_load), before it is replaced here
            gh_old = (double)in.gprev * hv;
            gh = (double)gv * hv;
            m.gpad[2 * ((size_t)(r + kPad) * pnx + c + kPad)] = gv;
        }
        // transposed write: consecutive threads take consecutive rows of one
        // column, i.e. consecutive elements of a line of the transposed copy
        const int cl = threadIdx.x / kTY, rl = threadIdx.x % kTY;
        int rt = r0 + rl, ct = c0 + cl;
        if (rt < ny && ct < nx)
            m.gpadT[2 * ((size_t)(ct + kPad) * pny + rt + kPad)] = sg[rl + 1][cl + 1];
    }
    double v[kTvParts] = {tv, gg, gradg, pres, ff, gh_old, gh};
    block_sum<kTvParts>(v, outv);
    if (threadIdx.x < kTvParts) part[threadIdx.x] = outv[threadIdx.x];
    __syncthreads();
}

template <bool COUPLED = false>
__device__ __forceinline__ void tv_tile(int r0, int c0, const AdmImg &m, double *part,
                                        bool pending, int nx, int ny, float rho, float xi)
{
    TvIn<COUPLED> in;
    tv_load<COUPLED>(r0, c0, m, nx, ny, in);
    tv_compute<COUPLED>(r0, c0, m, in, part, pending, nx, ny, rho, xi);
}

// ------------------------------------------------------------- scalar ---
// c^k = |G|^2 / (mu |A G|^2 + rho |grad G|^2) from the partials of one
// energy; alpha^k = c^{k-1} (c^0 at the first step); J^k logged in column
// `col` (and the step in column col + 2) of a [rows][4] log.
// fold: also take over the bookkeeping of the previous update (the plain
// iteration has no separate kernel for it): |r|^2 of the residual it left,
// from its per-block partials p_rr (once an update has run), then, for the
// update about to run, the iteration count, the pending multiplier step and
// the relative-change stop rule (stop_next, turned into stopped here one
// iteration later, so that this iteration's update still runs).
__device__ __forceinline__ void scalar_energy(AdmScalars &s, const double *__restrict__ pt,
                                              int nb_tv, const double *__restrict__ pf, int nb_fwd,
                                              double *__restrict__ log, int log_rows, int col,
                                              double mu, double rho, bool nonneg = false,
                                              bool fold = false,
                                              const double *__restrict__ p_rr = nullptr,
                                              int nbs = 0, double tol = 0.0, int step_rule = 0,
                                              const double *__restrict__ p_yy = nullptr,
                                              int nyy = 0)
{
    constexpr int kP = kTvParts, kFwd = kP, kRR = kP + 1, kYY = kP + 2, kNV = kP + 3;
    __shared__ double tot[kNV];
    const bool stop_now = fold && s.stop_next;
    const bool run = !s.stopped && !stop_now;
    const bool fresh_rr = fold && s.pending;
    const bool want_yy = step_rule != 0 && s.has_prev;
    double v[kNV];
#pragma unroll
    for (int j = 0; j < kNV; ++j) v[j] = 0.0;
    if (run) {
        if (want_yy)
            for (int i = threadIdx.x; i < nyy; i += 256) v[kYY] += p_yy[i];
        // thread t adds entries t, t + 256, ... of each list in that order.
        // The reads go out in rounds: one round loads the next kScRR, kScTV
        // and kScF of the thread's entries of p_rr, the tile partials and the
        // forward partials, unconditionally (an index past a list's end reads
        // its entry 0, which is not added), and only then adds them: a read
        // under a branch would be waited for where the branches join.  At
        // 512 x 512 and 360 views one round holds them all.
        constexpr int kScRR = 2, kScTV = 4, kScF = 24;
        const int nrr = fresh_rr ? nbs : 0;
        const int rounds = std::max(std::max((nrr + 256 * kScRR - 1) / (256 * kScRR),
                                             (nb_tv + 256 * kScTV - 1) / (256 * kScTV)),
                                    (nb_fwd + 256 * kScF - 1) / (256 * kScF));
        for (int q = 0; q < rounds; ++q) {
            double trr[kScRR], ttv[kScTV][kP], tf[kScF];
            const int irr = threadIdx.x + 256 * kScRR * q, itv = threadIdx.x + 256 * kScTV * q,
                      ifw = threadIdx.x + 256 * kScF * q;
#pragma unroll
            for (int u = 0; u < kScRR; ++u) {
                const int i = irr + 256 * u;
                trr[u] = p_rr[i < nrr ? i : 0];
            }
#pragma unroll
            for (int u = 0; u < kScTV; ++u) {
                const int i = itv + 256 * u;
#pragma unroll
                for (int j = 0; j < kP; ++j) ttv[u][j] = pt[(size_t)(i < nb_tv ? i : 0) * kP + j];
            }
#pragma unroll
            for (int u = 0; u < kScF; ++u) {
                const int i = ifw + 256 * u;
                tf[u] = pf[i < nb_fwd ? i : 0];
            }
#pragma unroll
            for (int u = 0; u < kScRR; ++u)
                if (irr + 256 * u < nrr) v[kRR] += trr[u];
#pragma unroll
            for (int u = 0; u < kScTV; ++u)
                if (itv + 256 * u < nb_tv)
#pragma unroll
                    for (int j = 0; j < kP; ++j) v[j] += ttv[u][j];
#pragma unroll
            for (int u = 0; u < kScF; ++u)
                if (ifw + 256 * u < nb_fwd) v[kFwd] += tf[u];
        }
    }
    block_sum<kNV>(v, tot);
    if (stop_now && threadIdx.x == 0) {
        s.stopped = 1;
        s.stop_next = 0;
    }
    if (run && threadIdx.x == 0) {
        if (fresh_rr) s.rr = tot[kRR];
        const double tvf = tot[0], gg = tot[1], gradg = tot[2], ff = tot[4], pp = tot[kFwd];
        const double gh_old = tot[5], gh = tot[6];
        const double den = mu * pp + rho * gradg;
        double c = den > 0.0 ? gg / den : (s.has_prev ? s.c_prev : 0.0);
        // BB1 <s,s>/<s,y> of the last step s = -alpha G_prev, with y the change
        // of the f-gradient at fixed z and lambda, (h - h_prev) + rho grad^T
        // grad s: <s,s> = alpha^2 |G_prev|^2 and <s,y> = alpha (<G_prev, h_prev>
        // - <G_prev, h> + alpha rho |grad G_prev|^2), from this iteration's h;
        // a non-positive <s,y> keeps alpha.  The first step is the exact line
        // search along -G (c).
        double bb1 = s.alpha;
        if (s.has_prev) {
            const double sy = (s.gh_prev - gh_old) + s.alpha * rho * s.gradg_prev;
            if (sy > 0.0) bb1 = s.alpha * s.gg_prev / sy;
        }
        double alpha = s.has_prev ? bb1 : c;
        // BB2 <s,y>/<y,y> of s = -alpha G_prev: den_prev / |mu A^T A G + rho
        // grad^T grad G|^2 (step_rule 1), or the adaptive choice (2): BB2
        // where it is below half the BB1 step; a non-positive <s,y> keeps alpha
        if (want_yy) {
            if (s.den_prev > 0.0) {
                const double yy = tot[kYY];
                const double bb2 = yy > 0.0 ? s.den_prev / yy : bb1;
                alpha = step_rule == 1 ? bb2 : (bb2 / bb1 < 0.5 ? bb2 : bb1);
            } else {
                alpha = s.alpha;
            }
        }
        s.den_prev = den;
        s.gg_prev = gg;
        s.gh_prev = gh;
        s.gradg_prev = gradg;
        // projected steps: BB1 <s,s>/<s,y> of the last step (kept when <s,y> <= 0)
        if (nonneg && s.has_prev) alpha = s.sy > 0.0 ? s.ss / s.sy : s.alpha;
        const double J = tvf + 0.5 * mu * s.rr;
        const double relchg = ff > 0.0 ? alpha * sqrt(gg) / sqrt(ff) : (gg > 0.0 ? INFINITY : 0.0);
        const int64_t k = s.iter;
        int64_t row = k - s.log_base;
        if (log && row >= 0 && row < log_rows) {
            log[row * kLogW + col] = J;
            log[row * kLogW + 2 + col] = alpha;
            log[row * kLogW + 4 + col] = sqrt(tot[3]);
            log[row * kLogW + 6 + col] = sqrt(gg);
        }
        s.J = J;
        s.alpha = alpha;
        s.c_prev = c;
        s.has_prev = 1;
        if (!nonneg) s.relchg = relchg;  // else set from the projected step
        if (!isfinite(J) || !isfinite(alpha) || !isfinite(gg) || !isfinite(pp)) {
            s.nonfinite_iter = (int32_t)(k + 1);
            s.stopped = 1;
            s.alpha = 0.0;
        }
        if (fold && !s.stopped) {  // this iteration's update runs
            s.pending = 1;
            s.iter += 1;
            if (tol > 0.0 && s.relchg < tol) s.stop_next = 1;
        }
    }
    __syncthreads();
}

// ------------------------------------------------ non-negative variant ---
// Chunk bx of 1024 pixels of energy e (fe, fle its f and f_lo; gpad, gpadT
// the interleaved padded layouts).  Projected f-step: t = (f + flo) - alpha
// G, f' = max(t, 0).  The step s = f' - f is kept in FP32 (rounded toward
// zero where the projection clips, so f + s >= 0) and f advances by exactly
// that s, so that r + A s stays the residual of f.  s goes to the transposed
// padded layout (G, in the other layout, is still read by neighbouring
// threads); partials <s,s> and |f|^2 into p_ss_e[bx], p_ff_e[bx].
__device__ __forceinline__ void nn_step_chunk(int bx, int e, float *__restrict__ fe,
                                              float *__restrict__ fle,
                                              const float *__restrict__ gpad,
                                              float *__restrict__ gpadT, double alpha,
                                              double *__restrict__ p_ss_e,
                                              double *__restrict__ p_ff_e, int nx, int ny)
{
    const size_t N = (size_t)nx * ny;
    const int pnx = nx + 2 * kPad, pny = ny + 2 * kPad;
    double v[2] = {0.0, 0.0};
    for (int j = 0; j < 4; ++j) {
        const size_t i = ((size_t)bx * 4 + j) * 256 + threadIdx.x;
        if (i < N) {
            const int r = (int)(i / nx), c = (int)(i % nx);
            const double g = gpad[2 * ((size_t)(r + kPad) * pnx + c + kPad) + e];
            const double fo = (double)fe[i] + (double)fle[i];
            const double t = fo - alpha * g;
            float s32 = t > 0.0 ? (float)(t - fo) : __double2float_rz(-fo);
            if (fo + (double)s32 < 0.0) s32 = __double2float_rz(-fo);
            const double fn = fo + (double)s32;
            const float hi = (float)fn;
            fe[i] = hi;
            fle[i] = (float)(fn - (double)hi);
            gpadT[2 * ((size_t)(c + kPad) * pny + r + kPad) + e] = s32;
            v[0] += (double)s32 * (double)s32;
            v[1] += fo * fo;
        }
    }
    __shared__ double tot[2];
    block_sum<2>(v, tot);
    if (threadIdx.x == 0) {
        p_ss_e[bx] = tot[0];
        p_ff_e[bx] = tot[1];
    }
}

// |grad s|^2 partial of chunk bx (backward differences of Eq. 2) and s copied
// into the normal padded layout, so that the forward projector reads s in both.
__device__ __forceinline__ void nn_grad_chunk(int bx, int e, float *__restrict__ gpad,
                                              const float *__restrict__ gpadT,
                                              double *__restrict__ p_gs_e, int nx, int ny)
{
    const size_t N = (size_t)nx * ny;
    const int pnx = nx + 2 * kPad, pny = ny + 2 * kPad;
    auto sT = [&](int r, int c) { return gpadT[2 * ((size_t)(c + kPad) * pny + r + kPad) + e]; };
    double v[1] = {0.0};
    for (int j = 0; j < 4; ++j) {
        const size_t i = ((size_t)bx * 4 + j) * 256 + threadIdx.x;
        if (i < N) {
            const int r = (int)(i / nx), c = (int)(i % nx);
            const float si = sT(r, c);
            const double gx = c >= 1 ? (double)si - (double)sT(r, c - 1) : 0.0;
            const double gy = r >= 1 ? (double)si - (double)sT(r - 1, c) : 0.0;
            gpad[2 * ((size_t)(r + kPad) * pnx + c + kPad) + e] = si;
            v[0] += gx * gx + gy * gy;
        }
    }
    __shared__ double tot[1];
    block_sum<1>(v, tot);
    if (threadIdx.x == 0) p_gs_e[bx] = tot[0];
}

// Sinogram chunk bx: (r + rlo) += (p + plo) = A s in FP64; partial |r|^2.
__device__ __forceinline__ void nn_resid_chunk(int bx, float *__restrict__ re,
                                               float *__restrict__ rle,
                                               const float *__restrict__ pe,
                                               const float *__restrict__ ple,
                                               double *__restrict__ p_rr_e, int M)
{
    const size_t Ms = (size_t)M;
    double v[1] = {0.0};
    for (int j = 0; j < 4; ++j) {
        const size_t i = ((size_t)bx * 4 + j) * 256 + threadIdx.x;
        if (i < Ms) {
            const double d = ((double)re[i] + (double)rle[i]) + ((double)pe[i] + (double)ple[i]);
            const float hi = (float)d;
            re[i] = hi;
            rle[i] = (float)(d - (double)hi);
            v[0] += d * d;
        }
    }
    __shared__ double tot[1];
    block_sum<1>(v, tot);
    if (threadIdx.x == 0) p_rr_e[bx] = tot[0];
}

// One block per energy: |r|^2, <s,s>, <s,y> = mu |A s|^2 + rho |grad s|^2 and
// |s| / |f| from the partials; counts the iteration, marks the deferred
// multiplier step and applies the relative-change stop rule.
__device__ __forceinline__ void nn_rr_energy(AdmScalars &s, const double *__restrict__ p_rr_e,
                                             int nbs, const double *__restrict__ p_ss_e,
                                             const double *__restrict__ p_ff_e,
                                             const double *__restrict__ p_gs_e, int nbi,
                                             const double *__restrict__ p_as_e, int nb_fwd,
                                             double mu, double rho, double tol)
{
    const bool run = !s.stopped;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (run) {
        for (int i = threadIdx.x; i < nbs; i += 256) v[0] += p_rr_e[i];
        for (int i = threadIdx.x; i < nbi; i += 256) {
            v[1] += p_ss_e[i];
            v[2] += p_ff_e[i];
            v[3] += p_gs_e[i];
        }
        for (int i = threadIdx.x; i < nb_fwd; i += 256) v[4] += p_as_e[i];
    }
    __shared__ double tot[5];
    block_sum<5>(v, tot);
    if (run && threadIdx.x == 0) {
        const double ss = tot[1], ff = tot[2];
        s.rr = tot[0];
        s.ss = ss;
        s.sy = mu * tot[4] + rho * tot[3];
        s.relchg = ff > 0.0 ? sqrt(ss) / sqrt(ff) : (ss > 0.0 ? INFINITY : 0.0);
        s.pending = 1;
        s.iter += 1;
        if (tol > 0.0 && s.relchg < tol) s.stopped = 1;
    }
    __syncthreads();
}

// BB2 / adaptive steps: the partial of |mu A^T A G + rho grad^T grad G|^2 of
// chunk bx of energy e, from the nplanes partial planes ap_e of A^T (A G)
// (summed in plane order) and G in the padded layout (still this
// iteration's G).
__device__ __forceinline__ void yy_chunk(int bx, int e, const float *__restrict__ ap_e,
                                         int nplanes, float mu, const float *__restrict__ gpad,
                                         float rho, double *__restrict__ p_yy_e, int nx, int ny)
{
    const size_t N = (size_t)nx * ny;
    const int pnx = nx + 2 * kPad;
    auto G = [&](int r, int c) { return gpad[2 * ((size_t)(r + kPad) * pnx + c + kPad) + e]; };
    // backward difference along x / y at (r, c) (zero on the first column / row)
    auto gx = [&](int r, int c) { return c >= 1 ? G(r, c) - G(r, c - 1) : 0.f; };
    auto gy = [&](int r, int c) { return r >= 1 ? G(r, c) - G(r - 1, c) : 0.f; };
    double v[1] = {0.0};
    for (int j = 0; j < 4; ++j) {
        const size_t i = ((size_t)bx * 4 + j) * 256 + threadIdx.x;
        if (i < N) {
            const int r = (int)(i / nx), c = (int)(i % nx);
            float a = 0.f;
            for (int q = 0; q < nplanes; ++q) a += ap_e[(size_t)q * N + i];
            float lt = 0.f;  // (grad^T grad G) at (r, c)
            if (c >= 1) lt += gx(r, c);
            if (c + 1 <= nx - 1) lt -= gx(r, c + 1);
            if (r >= 1) lt += gy(r, c);
            if (r + 1 <= ny - 1) lt -= gy(r + 1, c);
            const double y = (double)mu * a + (double)rho * lt;
            v[0] += y * y;
        }
    }
    __shared__ double tot[1];
    block_sum<1>(v, tot);
    if (threadIdx.x == 0) p_yy_e[bx] = tot[0];
}

// ------------------------------------------------------------- update ---
// Chunk bx of 1024 elements: bx < nbi updates the image (f + flo) -= alpha G
// in FP64, split again into f + flo; otherwise sinogram chunk bx - nbi:
// (r + rlo) -= alpha (p + plo) likewise, partial |r|^2 into p_rr[bx - nbi].
// gpad_e: this energy's first element of the interleaved padded G.
__device__ __forceinline__ void update_chunk(int bx, float *__restrict__ fe,
                                             float *__restrict__ fle,
                                             const float *__restrict__ gpad_e,
                                             float *__restrict__ re, float *__restrict__ rle,
                                             const float *__restrict__ pe,
                                             const float *__restrict__ ple,
                                             double *__restrict__ p_rr, double alpha, int nx,
                                             int ny, int M, int nbi)
{
    __shared__ double tot[1];
    const size_t N = (size_t)nx * ny;
    if (bx < nbi) {
        const int pnx = nx + 2 * kPad;
        for (int j = 0; j < 4; ++j) {
            size_t i = ((size_t)bx * 4 + j) * 256 + threadIdx.x;
            if (i < N) {
                int rr = (int)(i / nx), cc = (int)(i % nx);
                const double g = gpad_e[2 * ((size_t)(rr + kPad) * pnx + cc + kPad)];
                const double d = ((double)fe[i] + (double)fle[i]) - alpha * g;
                const float hi = (float)d;
                fe[i] = hi;
                fle[i] = (float)(d - (double)hi);
            }
        }
        return;  // uniform across the block
    }
    const int bs = bx - nbi;
    double acc[1] = {0.0};
    for (int j = 0; j < 4; ++j) {
        size_t i = ((size_t)bs * 4 + j) * 256 + threadIdx.x;
        if ((int)i < M) {
            const double d = ((double)re[i] + (double)rle[i]) -
                             alpha * ((double)pe[i] + (double)ple[i]);
            const float hi = (float)d;
            re[i] = hi;
            rle[i] = (float)(d - (double)hi);
            acc[0] += d * d;
        }
    }
    block_sum<1>(acc, tot);
    if (threadIdx.x == 0) p_rr[bs] = tot[0];
    __syncthreads();
}

// |r|^2 from the residual partials of one energy; after an update
// (step != 0) also counts the iteration, marks the deferred multiplier step
// as pending and applies the relative-change stop rule.
__device__ __forceinline__ void rr_energy(AdmScalars &s, const double *__restrict__ p_rr, int nbs,
                                          int step, double tol)
{
    __shared__ double tot[1];
    const bool run = !(step && s.stopped);
    double v[1] = {0.0};
    if (run)
        for (int i = threadIdx.x; i < nbs; i += 256) v[0] += p_rr[i];
    block_sum<1>(v, tot);
    if (run && threadIdx.x == 0) {
        s.rr = tot[0];
        if (step) {
            s.pending = 1;
            s.iter += 1;
            if (tol > 0.0 && s.relchg < tol) s.stopped = 1;
        }
    }
    __syncthreads();
}

}  // namespace dect
