// Cone-beam Joseph projector pair for the 3-D circular scan (the scanner of
// Sec. 3; the fan-beam path is its central plane) on gfx950.
//
// Source s = R (cos t, sin t, 0); flat panel centred at -(D - R)(cos t, sin t,
// 0), bin b of row j at u_b = (b - (B-1)/2) du + offset along (-sin t, cos t,
// 0) and v_j = (j - (J-1)/2) dv along z.  Volume [nz][ny][nx] of cubic voxels,
// projections [V][J][B].  Each ray steps along the in-plane axis it is more
// aligned with; on every plane of that axis its crossing (in-plane coordinate
// and height) is interpolated bilinearly between the four nearest voxel
// centres, and the samples are scaled by the path length per plane.
//
//   k_cone_pad_x, k_cone_pad_y : two zero-padded permuted copies of the
//                volume, [x][z][y] for x-major rays and [y][z][x] for
//                y-major rays, so that a sample's two in-plane taps are
//                adjacent (borders written as zeros by the same kernels: no
//                memset in the path).
//   k_cone_fwd : one thread per ray (64 adjacent bins of one row per
//                wavefront); the ray's constants are formed in FP64 from the
//                view's cos/sin and turned into 32.32 fixed point (in-plane
//                coordinate and height per plane), stepped by integer adds;
//                FP32 bilinear samples summed in FP64.
//   k_cone_tab, k_cone_scale, k_cone_gather : the transpose in gather form
//                (no atomics, the same result on every run): per-(view, bin)
//                ray constants, projections times each ray's path length,
//                then one thread per voxel column and 4 slices sums over
//                the rays that reach it (see k_cone_gather).
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "volume.h"

namespace dect {
namespace {

constexpr int kCPad = 2;  // zero lines on each side of the padded copies
constexpr double kTwo32c = 4294967296.0;
constexpr float kTwoM32c = 2.3283064365386963e-10f;

struct ConeDev {
    int nx, ny, nz, V, J, B;
    double voxel, bin, row, off, sod, sdd;
    const double *cs;  // [V][2] cos, sin of the view angle
};

struct ConeRay {
    int64_t a, k, az, kz;  // 32.32 in-plane coordinate and height at plane 0, steps
    float L;               // path length per plane
    int xmaj;
};

__device__ __forceinline__ ConeRay cone_ray(const ConeDev &g, int v, int j, int b)
{
    const double ct = g.cs[2 * v], st = g.cs[2 * v + 1];
    const double u = (b - (g.B - 1) / 2.0) * g.bin + g.off;
    const double w = (j - (g.J - 1) / 2.0) * g.row;
    const double sx = g.sod * ct, sy = g.sod * st;
    const double px = -(g.sdd - g.sod) * ct - u * st, py = -(g.sdd - g.sod) * st + u * ct;
    const double dx = px - sx, dy = py - sy, dz = w;
    const double len = sqrt(dx * dx + dy * dy + dz * dz);
    ConeRay r;
    r.xmaj = fabs(dx) >= fabs(dy);
    double a, k, kz, az;
    if (r.xmaj) {
        k = dy / dx;
        kz = dz / dx;
        const double x0 = (0 - (g.nx - 1) / 2.0) * g.voxel;
        a = (sy + (x0 - sx) * k) / g.voxel + (g.ny - 1) / 2.0;
        az = ((x0 - sx) * kz) / g.voxel + (g.nz - 1) / 2.0;
        r.L = (float)(g.voxel * len / fabs(dx));
    } else {
        k = dx / dy;
        kz = dz / dy;
        const double y0 = (0 - (g.ny - 1) / 2.0) * g.voxel;
        a = (sx + (y0 - sy) * k) / g.voxel + (g.nx - 1) / 2.0;
        az = ((y0 - sy) * kz) / g.voxel + (g.nz - 1) / 2.0;
        r.L = (float)(g.voxel * len / fabs(dy));
    }
    // |a|, |az| stay far below 2^31 for validated geometries (rays outside
    // the volume are clamped to a far coordinate and contribute zero)
    a = fmin(fmax(a, -1.0e6), 1.0e6);
    az = fmin(fmax(az, -1.0e6), 1.0e6);
    r.a = __double2ll_rn(a * kTwo32c);
    r.k = __double2ll_rn(k * kTwo32c);
    r.az = __double2ll_rn(az * kTwo32c);
    r.kz = __double2ll_rn(kz * kTwo32c);
    return r;
}

// vol [nz][ny][nx] -> vx [nx][nz+4][ny+4] and vy [ny][nz+4][nx+4], written
// whole (zero borders included).  NE = 2: the two volumes interleaved
// ([..][2]), so that one load carries a tap of both.
//
// k_cone_pad_x: vx is a transpose (y fastest), staged through a 32 x 32
// LDS tile per (x block, padded-y block, padded slice): read along x, write
// along y.  k_cone_pad_y: vy keeps x fastest, one thread per element.
template <int NE>
__global__ __launch_bounds__(256) void k_cone_pad_x(const float *__restrict__ vol0,
                                                    const float *__restrict__ vol1, int nx, int ny,
                                                    int nz, float *__restrict__ vx)
{
    __shared__ float tile[NE][32][33];
    const int pz = nz + 2 * kCPad, py = ny + 2 * kCPad;
    const int x0 = blockIdx.x * 32, yp0 = blockIdx.y * 32, zp = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int z = zp - kCPad;
    const float *vol[2] = {vol0, vol1};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int y = yp0 + ty + 8 * r - kCPad, x = x0 + tx;
        const bool in = x < nx && y >= 0 && y < ny && z >= 0 && z < nz;
#pragma unroll
        for (int e = 0; e < NE; ++e)
            tile[e][ty + 8 * r][tx] = in ? vol[e][((size_t)z * ny + y) * nx + x] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int x = x0 + ty + 8 * r, yp = yp0 + tx;
        if (x < nx && yp < py) {
            const size_t o = ((size_t)x * pz + zp) * py + yp;
#pragma unroll
            for (int e = 0; e < NE; ++e) vx[o * NE + e] = tile[e][tx][ty + 8 * r];
        }
    }
}

template <int NE>
__global__ __launch_bounds__(256) void k_cone_pad_y(const float *__restrict__ vol0,
                                                    const float *__restrict__ vol1, int nx, int ny,
                                                    int nz, float *__restrict__ vy)
{
    const int pz = nz + 2 * kCPad, px = nx + 2 * kCPad;
    const size_t nvy = (size_t)ny * pz * px;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const float *vol[2] = {vol0, vol1};
    if (i < nvy) {  // vy: x fastest
        const int xx = (int)(i % px) - kCPad, zz = (int)(i / px % pz) - kCPad;
        const int y = (int)(i / ((size_t)px * pz));
        const bool in = xx >= 0 && xx < nx && zz >= 0 && zz < nz;
#pragma unroll
        for (int e = 0; e < NE; ++e)
            vy[i * NE + e] = in ? vol[e][((size_t)zz * ny + y) * nx + xx] : 0.f;
    }
}

// four floats at 8-byte alignment: taps h and h + 1 of both volumes
typedef float c4a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef float c2 __attribute__((ext_vector_type(2)));

template <int NE>
__global__ __launch_bounds__(256) void k_cone_fwd(ConeDev g, const float *__restrict__ vx,
                                                  const float *__restrict__ vy,
                                                  float *__restrict__ proj0,
                                                  float *__restrict__ proj1,
                                                  float *__restrict__ lo0,
                                                  float *__restrict__ lo1)
{
    const size_t nray = (size_t)g.V * g.J * g.B;
    const size_t rid = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (rid >= nray) return;
    const int b = (int)(rid % g.B), j = (int)(rid / g.B % g.J), v = (int)(rid / ((size_t)g.B * g.J));
    const ConeRay r = cone_ray(g, v, j, b);
    const int nl = r.xmaj ? g.nx : g.ny, nq = r.xmaj ? g.ny : g.nx;
    const int pq = nq + 2 * kCPad, pz = g.nz + 2 * kCPad;
    const float *base = r.xmaj ? vx : vy;
    int64_t q = r.a, qz = r.az;
    double acc[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) acc[e] = 0.0;
    for (int i0 = 0; i0 < nl; i0 += 4) {
        float s[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) s[e] = 0.f;
        const int i1 = min(nl, i0 + 4);
        for (int i = i0; i < i1; ++i) {
            const int h = min(max((int)(q >> 32), -2), nq);
            const int hz = min(max((int)(qz >> 32), -2), g.nz);
            const float wa = (float)(uint32_t)q * kTwoM32c;
            const float wz = (float)(uint32_t)qz * kTwoM32c;
            const size_t o0 = ((size_t)i * pz + hz + kCPad) * pq + h + kCPad;
            if constexpr (NE == 1) {
                const float *p0 = base + o0;
                const float *p1 = p0 + pq;
                const float lo = fmaf(wa, p0[1] - p0[0], p0[0]);
                const float hi = fmaf(wa, p1[1] - p1[0], p1[0]);
                s[0] += fmaf(wz, hi - lo, lo);
            } else {
                const c4a8 a0 = *(const c4a8 *)(base + 2 * o0);
                const c4a8 a1 = *(const c4a8 *)(base + 2 * (o0 + pq));
                const float lo0 = fmaf(wa, a0.z - a0.x, a0.x), hi0 = fmaf(wa, a1.z - a1.x, a1.x);
                const float lo1 = fmaf(wa, a0.w - a0.y, a0.y), hi1 = fmaf(wa, a1.w - a1.y, a1.y);
                s[0] += fmaf(wz, hi0 - lo0, lo0);
                s[1] += fmaf(wz, hi1 - lo1, lo1);
            }
            q += r.k;
            qz += r.kz;
        }
#pragma unroll
        for (int e = 0; e < NE; ++e) acc[e] += (double)s[e];
    }
    // the FP64 ray sum rounded to FP32; with lo buffers also its rounding
    // error, so that proj + lo carries the sum to about 2^-48
    const double v0 = acc[0] * (double)r.L;
    const float h0 = (float)v0;
    proj0[rid] = h0;
    if (lo0) lo0[rid] = (float)(v0 - (double)h0);
    if constexpr (NE == 2) {
        const double v1 = acc[1] * (double)r.L;
        const float h1 = (float)v1;
        proj1[rid] = h1;
        if (lo1) lo1[rid] = (float)(v1 - (double)h1);
    }
}

// Per (view, bin): the ray's 32.32 in-plane coordinate at plane 0 and its
// step (as in the forward walk), its class, and the height coefficients:
// at plane p the ray's height is qz = w * (g0 + g1 p) + (nz - 1)/2 voxels,
// w the row's height on the panel.
struct ConeTab {
    int64_t a, k;
    double g0, g1;
    int32_t xmaj, pad;
};

__global__ __launch_bounds__(256) void k_cone_tab(ConeDev g, ConeTab *__restrict__ tab)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= g.V * g.B) return;
    const int v = i / g.B, b = i % g.B;
    const ConeRay r = cone_ray(g, v, 0, b);  // in-plane terms do not depend on the row
    const double ct = g.cs[2 * v], st = g.cs[2 * v + 1];
    const double u = (b - (g.B - 1) / 2.0) * g.bin + g.off;
    const double sx = g.sod * ct, sy = g.sod * st;
    const double dx = -(g.sdd - g.sod) * ct - u * st - sx;
    const double dy = -(g.sdd - g.sod) * st + u * ct - sy;
    const double dp = r.xmaj ? dx : dy, sp = r.xmaj ? sx : sy;
    const int np = r.xmaj ? g.nx : g.ny;
    ConeTab t;
    t.a = r.a;
    t.k = r.k;
    t.g0 = ((0 - (np - 1) / 2.0) * g.voxel - sp) / (dp * g.voxel);
    t.g1 = 1.0 / dp;
    t.xmaj = r.xmaj;
    t.pad = 0;
    tab[i] = t;
}

// yl = L * proj (NE = 2: both projections interleaved), L the forward
// walk's path length per plane of each ray.
template <int NE>
__global__ __launch_bounds__(256) void k_cone_scale(ConeDev g, const float *__restrict__ proj0,
                                                    const float *__restrict__ proj1,
                                                    float *__restrict__ yl)
{
    const size_t nray = (size_t)g.V * g.J * g.B;
    const size_t rid = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (rid >= nray) return;
    const int b = (int)(rid % g.B), j = (int)(rid / g.B % g.J), v = (int)(rid / ((size_t)g.B * g.J));
    const float L = cone_ray(g, v, j, b).L;
    yl[rid * NE] = proj0[rid] * L;
    if constexpr (NE == 2) yl[rid * 2 + 1] = proj1[rid] * L;
}

#ifndef DECT_CONE_ZC
#define DECT_CONE_ZC 4
#endif
constexpr int kZC = DECT_CONE_ZC;  // slices per gather thread

// vol = A3^T proj in gather form.  Thread: voxel column (x, y), slices
// [z0, z0 + kZC); lanes along x.  Per view, the rays that can reach the
// column cross the segments (x, y -+ 1) (x-major rays, on plane x) or
// (x -+ 1, y) (y-major rays, on plane y); their bins lie between the
// panel positions of those four points.  Every candidate's in-plane weight
// comes from its exact 32.32 coordinate (the forward's interpolation
// weight); the rows reaching slice z are those whose height on the ray's
// plane lies within one voxel of z, the height taken in FP64 at the first
// such row and stepped in FP32 (a few rows).  Per-view sums in FP32,
// accumulated over views in FP64.
template <int NE>
__global__ __launch_bounds__(256) void k_cone_gather(ConeDev g, const ConeTab *__restrict__ tab,
                                                     const float *__restrict__ yl,
                                                     float *__restrict__ vol0,
                                                     float *__restrict__ vol1)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y;
    const int z0 = (blockIdx.z * 4 + (threadIdx.x >> 6)) * kZC;
    if (x >= g.nx || z0 >= g.nz) return;
    const float vox = (float)g.voxel;
    const float px = (x - (g.nx - 1) * 0.5f) * vox, py = (y - (g.ny - 1) * 0.5f) * vox;
    const float R = (float)g.sod, D = (float)g.sdd;
    const float ibin = (float)(1.0 / g.bin), bc = (float)((g.B - 1) / 2.0 - g.off / g.bin);
    const double cz = (g.nz - 1) / 2.0, jc = (g.J - 1) / 2.0;
    const size_t JB = (size_t)g.J * g.B;
    double acc[kZC][NE];
#pragma unroll
    for (int t = 0; t < kZC; ++t)
#pragma unroll
        for (int e = 0; e < NE; ++e) acc[t][e] = 0.0;
    for (int v = 0; v < g.V; ++v) {
        const float ct = (float)g.cs[2 * v], st = (float)g.cs[2 * v + 1];
        const float sx = R * ct, sy = R * st;
        // continuous bin of the ray through (qx, qy)
        auto bin_of = [&](float qx, float qy) {
            const float rx = qx - sx, ry = qy - sy;
            return -D * (ry * ct - rx * st) / (rx * ct + ry * st) * ibin + bc;
        };
        const float b1 = bin_of(px, py - vox), b2 = bin_of(px, py + vox);
        const float b3 = bin_of(px - vox, py), b4 = bin_of(px + vox, py);
        const float bmin = fminf(fminf(b1, b2), fminf(b3, b4));
        const float bmax = fmaxf(fmaxf(b1, b2), fmaxf(b3, b4));
        // clamped before conversion (bounds only; the exact test below decides)
        const int bl = max(0, (int)ceilf(fminf(fmaxf(bmin - 1e-3f, -1.f), (float)g.B)));
        const int bh = min(g.B - 1, (int)floorf(fminf(fmaxf(bmax + 1e-3f, -1.f), (float)g.B)));
        float part[kZC][NE];
#pragma unroll
        for (int t = 0; t < kZC; ++t)
#pragma unroll
            for (int e = 0; e < NE; ++e) part[t][e] = 0.f;
        const ConeTab *tv = tab + (size_t)v * g.B;
        const float *yv = yl + (size_t)v * JB * NE;
        for (int b = bl; b <= bh; ++b) {
            const ConeTab tb = tv[b];
            const int pl = tb.xmaj ? x : y, c = tb.xmaj ? y : x;
            // bilinear weights are the tent 1 - |q - c| (in-plane, exact in
            // 32.32 as in the forward walk) times 1 - |qz - z| (height)
            const int64_t dq = tb.a + tb.k * pl - ((int64_t)c << 32);
            const uint64_t adq = (uint64_t)(dq < 0 ? -dq : dq);
            if (adq >= (1ull << 32)) continue;
            const float wi = 1.f - (float)(uint32_t)adq * kTwoM32c;
            const double sb = (tb.g0 + tb.g1 * pl) * g.row;  // height step per row (> 0)
            const double qz0 = cz - jc * sb;                  // height of row 0
            const float sbf = (float)sb, isb = 1.f / sbf;
            const float lo0 = (float)(z0 - 1 - qz0) * isb;
            const float *yb = yv + (size_t)b * NE;
#pragma unroll
            for (int t = 0; t < kZC; ++t) {
                // rows with |qz - z| < 1: j in (lo, lo + 2/sb)
                const float lo = lo0 + t * isb, hi = lo + 2.f * isb;
                const int j0 = max(0, (int)floorf(fminf(fmaxf(lo, -1.f), (float)g.J)) + 1);
                const int j1 = min(g.J - 1, (int)ceilf(fminf(fmaxf(hi, -1.f), (float)g.J)) - 1);
                const float e0 = (float)(qz0 + j0 * sb - (z0 + t));  // qz - z at row j0
                float s[NE];
#pragma unroll
                for (int e = 0; e < NE; ++e) s[e] = 0.f;
                for (int j = j0; j <= j1; ++j) {
                    const float w = fmaxf(0.f, 1.f - fabsf(fmaf((float)(j - j0), sbf, e0)));
                    if constexpr (NE == 1) {
                        s[0] = fmaf(w, yb[(size_t)j * g.B], s[0]);
                    } else {
                        const c2 yy = *(const c2 *)(yb + (size_t)j * g.B * 2);
                        s[0] = fmaf(w, yy.x, s[0]);
                        s[1] = fmaf(w, yy.y, s[1]);
                    }
                }
#pragma unroll
                for (int e = 0; e < NE; ++e) part[t][e] = fmaf(wi, s[e], part[t][e]);
            }
        }
#pragma unroll
        for (int t = 0; t < kZC; ++t)
#pragma unroll
            for (int e = 0; e < NE; ++e) acc[t][e] += (double)part[t][e];
    }
    const size_t plane = (size_t)g.nx * g.ny;
#pragma unroll
    for (int t = 0; t < kZC; ++t)
        if (z0 + t < g.nz) {
            const size_t o = (size_t)(z0 + t) * plane + (size_t)y * g.nx + x;
            vol0[o] = (float)acc[t][0];
            if constexpr (NE == 2) vol1[o] = (float)acc[t][1];
        }
}

struct ConeWork {
    DevBuf vx, vy, cs, yl, tab;
    std::vector<double> cs_host;  // what cs holds
};

std::mutex g_cone_mu;
std::vector<std::pair<std::pair<int, hipStream_t>, std::unique_ptr<ConeWork>>> g_cone_ws;

ConeWork *cone_workspace(hipStream_t s)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (auto &p : g_cone_ws)
        if (p.first.first == dev && p.first.second == s) return p.second.get();
    g_cone_ws.emplace_back(std::make_pair(dev, s), std::make_unique<ConeWork>());
    return g_cone_ws.back().second.get();
}

dect_status cone_setup(const dect_cone_geometry *g, ConeDev &d, ConeWork *w, hipStream_t s)
{
    if (!g) return fail(DECT_ERR_INVALID_ARG, "cone geometry is NULL");
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || g->n_views <= 0 || g->n_bins <= 0 ||
        g->n_rows <= 0)
        return fail(DECT_ERR_INVALID_ARG, "cone geometry sizes must be positive");
    if (g->nx > 4096 || g->ny > 4096 || g->nz > 4096 || g->n_bins > 16384 || g->n_rows > 16384 ||
        g->n_views > 65536)
        return fail(DECT_ERR_INVALID_ARG, "cone geometry sizes exceed the supported maximum");
    if (!(g->voxel_mm > 0.0) || !(g->bin_mm > 0.0) || !(g->row_mm > 0.0) ||
        !std::isfinite(g->det_offset_mm))
        return fail(DECT_ERR_INVALID_ARG, "voxel, bin and row sizes must be positive");
    const double hx = 0.5 * g->nx * g->voxel_mm, hy = 0.5 * g->ny * g->voxel_mm;
    if (!(g->sod_mm > std::sqrt(hx * hx + hy * hy)) || !std::isfinite(g->sod_mm))
        return fail(DECT_ERR_GEOMETRY, "source orbit (SOD) must lie outside the volume");
    if (!(g->sdd_mm > g->sod_mm) || !std::isfinite(g->sdd_mm))
        return fail(DECT_ERR_GEOMETRY, "SDD must exceed SOD");
    const double hu = 0.5 * g->n_bins * g->bin_mm + std::fabs(g->det_offset_mm);
    const double hv = 0.5 * g->n_rows * g->row_mm;
    if (!(std::atan(hu / g->sdd_mm) < 0.25 * M_PI))
        return fail(DECT_ERR_GEOMETRY, "fan angle must be below 90 degrees");
    // the height never becomes the driving axis: |dz| < |d_in-plane| on every ray
    if (!(hv < 0.5 * g->sdd_mm))
        return fail(DECT_ERR_GEOMETRY, "cone half-angle must be below atan(1/2)");
    std::vector<double> cs(2 * (size_t)g->n_views);
    for (int v = 0; v < g->n_views; ++v) {
        const double th = g->angles_rad ? g->angles_rad[v] : 2.0 * M_PI * v / g->n_views;
        if (!std::isfinite(th)) return fail(DECT_ERR_INVALID_ARG, "view angles must be finite");
        cs[2 * v] = std::cos(th);
        cs[2 * v + 1] = std::sin(th);
    }
    if (cs != w->cs_host) {
        // kernels in flight on this stream may still read the old table
        DECT_HIP(hipStreamSynchronize(s));
        dect_status st = w->cs.ensure(cs.size() * 8);
        if (st) return st;
        DECT_HIP(hipMemcpy(w->cs.ptr, cs.data(), cs.size() * 8, hipMemcpyHostToDevice));
        w->cs_host = cs;
    }
    d = ConeDev{g->nx, g->ny, g->nz, g->n_views, g->n_rows, g->n_bins, g->voxel_mm, g->bin_mm,
                g->row_mm, g->det_offset_mm, g->sod_mm, g->sdd_mm, (const double *)w->cs.ptr};
    return DECT_OK;
}

// Both projectors for NE volumes (1 or 2) sharing one geometry.
// lo: NULL, or NE buffers for the rounding errors of the FP32 results.
template <int NE>
dect_status cone_project_n(const dect_cone_geometry *g, const float *const *vol,
                           float *const *proj, float *const *lo, hipStream_t s)
{
    for (int e = 0; e < NE; ++e)
        if (!vol[e] || !proj[e]) return fail(DECT_ERR_INVALID_ARG, "dect_cone_project: null buffer");
    std::lock_guard<std::mutex> lk(g_cone_mu);
    ConeWork *w = cone_workspace(s);
    ConeDev d;
    dect_status st = cone_setup(g, d, w, s);
    if (st) return st;
    const size_t pz = d.nz + 2 * kCPad;
    const size_t nxb = (size_t)d.nx * pz * (d.ny + 2 * kCPad) * 4;
    const size_t nyb = (size_t)d.ny * pz * (d.nx + 2 * kCPad) * 4;
    if (w->vx.bytes < nxb * NE || w->vy.bytes < nyb * NE) {
        DECT_HIP(hipStreamSynchronize(s));
        if ((st = w->vx.ensure(nxb * NE)) || (st = w->vy.ensure(nyb * NE))) return st;
    }
    hipLaunchKernelGGL(k_cone_pad_x<NE>,
                       dim3((unsigned)((d.nx + 31) / 32), (unsigned)((d.ny + 2 * kCPad + 31) / 32),
                            (unsigned)pz),
                       dim3(256), 0, s, vol[0], vol[NE - 1], d.nx, d.ny, d.nz, (float *)w->vx.ptr);
    hipLaunchKernelGGL(k_cone_pad_y<NE>, dim3((unsigned)((nyb / 4 + 255) / 256)), dim3(256), 0, s,
                       vol[0], vol[NE - 1], d.nx, d.ny, d.nz, (float *)w->vy.ptr);
    DECT_HIP(hipGetLastError());
    const size_t nray = (size_t)d.V * d.J * d.B;
    hipLaunchKernelGGL(k_cone_fwd<NE>, dim3((unsigned)((nray + 255) / 256)), dim3(256), 0, s, d,
                       (const float *)w->vx.ptr, (const float *)w->vy.ptr, proj[0], proj[NE - 1],
                       lo ? lo[0] : (float *)nullptr, lo ? lo[NE - 1] : (float *)nullptr);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

template <int NE>
dect_status cone_backproject_n(const dect_cone_geometry *g, const float *const *proj,
                               float *const *vol, hipStream_t s)
{
    for (int e = 0; e < NE; ++e)
        if (!vol[e] || !proj[e])
            return fail(DECT_ERR_INVALID_ARG, "dect_cone_backproject: null buffer");
    std::lock_guard<std::mutex> lk(g_cone_mu);
    ConeWork *w = cone_workspace(s);
    ConeDev d;
    dect_status st = cone_setup(g, d, w, s);
    if (st) return st;
    const size_t nray = (size_t)d.V * d.J * d.B;
    const size_t ntab = (size_t)d.V * d.B;
    if (w->yl.bytes < nray * 4 * NE || w->tab.bytes < ntab * sizeof(ConeTab)) {
        DECT_HIP(hipStreamSynchronize(s));
        if ((st = w->yl.ensure(nray * 4 * NE)) || (st = w->tab.ensure(ntab * sizeof(ConeTab))))
            return st;
    }
    hipLaunchKernelGGL(k_cone_tab, dim3((unsigned)((ntab + 255) / 256)), dim3(256), 0, s, d,
                       (ConeTab *)w->tab.ptr);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_cone_scale<NE>, dim3((unsigned)((nray + 255) / 256)), dim3(256), 0, s, d,
                       proj[0], proj[NE - 1], (float *)w->yl.ptr);
    DECT_HIP(hipGetLastError());
    const int nzc = (d.nz + kZC - 1) / kZC;
    hipLaunchKernelGGL(k_cone_gather<NE>, dim3((unsigned)((d.nx + 63) / 64), (unsigned)d.ny,
                                               (unsigned)((nzc + 3) / 4)),
                       dim3(256), 0, s, d, (const ConeTab *)w->tab.ptr, (const float *)w->yl.ptr,
                       vol[0], vol[NE - 1]);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

}  // namespace

dect_status cone_project(const dect_cone_geometry *g, const float *vol, float *proj,
                         hipStream_t s)
{
    return cone_project_n<1>(g, &vol, &proj, nullptr, s);
}

dect_status cone_backproject(const dect_cone_geometry *g, const float *proj, float *vol,
                             hipStream_t s)
{
    return cone_backproject_n<1>(g, &proj, &vol, s);
}

dect_status cone_project2(const dect_cone_geometry *g, const float *const vol[2],
                          float *const proj[2], hipStream_t s)
{
    return cone_project_n<2>(g, vol, proj, nullptr, s);
}

dect_status cone_project2_lo(const dect_cone_geometry *g, const float *const vol[2],
                             float *const proj[2], float *const lo[2], hipStream_t s)
{
    return cone_project_n<2>(g, vol, proj, lo, s);
}

dect_status cone_backproject2(const dect_cone_geometry *g, const float *const proj[2],
                              float *const vol[2], hipStream_t s)
{
    return cone_backproject_n<2>(g, proj, vol, s);
}

void release_cone_work()
{
    std::lock_guard<std::mutex> lk(g_cone_mu);
    g_cone_ws.clear();
}

}  // namespace dect
