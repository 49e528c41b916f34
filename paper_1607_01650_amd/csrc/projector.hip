// Joseph fan-beam projector pair for gfx950.
//
// Forward (A x): one lane per ray; a wavefront holds 64 adjacent bins of one
// view and steps through the driving lines in lockstep, so the two taps of
// all lanes land in one short run of a padded image line (the transposed
// copy for x-major rays): coalesced reads, coalesced sinogram writes.  The
// line coordinate is advanced in exact 32.32 fixed point.
//
// Adjoint (A^T y): output-stationary gather.  A wavefront owns a 64x64 pixel
// tile held in LDS; for x-major rays lane l owns tile column l and walks the
// bins whose rays cross that column inside the tile, for y-major rays lane l
// owns tile row l.  Every weight is recomputed from the same fixed-point line
// coordinate as the forward pass (evaluated exactly in FP64), so the adjoint
// is the exact transpose of the forward matrix.  No atomics: each pixel's sum
// runs in a fixed order (views of a wave, waves of a block, view groups).
#include "common.h"

namespace dect {

namespace {

constexpr int kTile = 64;        // adjoint tile side
constexpr int kTileLd = 65;      // LDS row stride (avoids bank conflicts)
constexpr float kTwoM32 = 2.3283064365386963e-10f;  // 2^-32

// ------------------------------------------------------------ padding ---
// In: img [batch][ny][nx].  Out: pad [batch][ny+4][nx+4] and padT
// [batch][nx+4][ny+4], written whole (zero border of kPad included), so a
// reused buffer never carries another geometry's values.  The grid covers the
// padded domain in 32x32 tiles; padT goes through an LDS transpose.
__global__ __launch_bounds__(256) void k_pad(const float *__restrict__ img,
                                             float *__restrict__ pad,
                                             float *__restrict__ padT, int nx, int ny)
{
    __shared__ float tile[32][33];
    const int e = blockIdx.z;
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;  // padded coordinates
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const size_t in_off = (size_t)e * nx * ny;
    const int pnx = nx + 2 * kPad, pny = ny + 2 * kPad;
    const size_t p_off = (size_t)e * pnx * pny;
    for (int j = ty; j < 32; j += 8) {
        int rp = r0 + j, cp = c0 + tx;
        int r = rp - kPad, c = cp - kPad;
        float v = (r >= 0 && r < ny && c >= 0 && c < nx) ? img[in_off + (size_t)r * nx + c] : 0.f;
        if (rp < pny && cp < pnx) pad[p_off + (size_t)rp * pnx + cp] = v;
        tile[j][tx] = v;
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        int cp = c0 + j, rp = r0 + tx;
        if (rp < pny && cp < pnx) padT[p_off + (size_t)cp * pny + rp] = tile[tx][j];
    }
}

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

template <bool NORM>
__global__ __launch_bounds__(256) void k_fwd(const float *__restrict__ pad,
                                             const float *__restrict__ padT,
                                             const RayFwd *__restrict__ rays,
                                             const float *__restrict__ len,
                                             const Bundle *__restrict__ bundles,
                                             float *__restrict__ sino, int nx, int ny, int V,
                                             int B, int nbundle, float scale,
                                             double *__restrict__ partial)
{
    const int e = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gw = blockIdx.x * 4 + wid;
    const bool wave_ok = gw < V * nbundle;
    float result = 0.f;
    if (wave_ok) {
        const int v = gw / nbundle, j = gw - v * nbundle;
        const int b = j * kBundle + lane;
        const bool act = b < B;
        const size_t ray = (size_t)v * B + (act ? b : 0);
        const RayFwd rf = rays[ray];
        const float L = len[ray];
        const Bundle bu = bundles[(size_t)v * nbundle + j];
        const int pnx = nx + 2 * kPad, pny = ny + 2 * kPad;
        const size_t p_off = (size_t)e * pnx * pny;
        float acc0 = 0.f, acc1 = 0.f;
        const int64_t far = -(int64_t(1000000) << 32);
        const int64_t a = rf.a_fx, k = rf.k_fx;
        // the sign of the stored path length marks the ray class (+ x-major)
        const bool is_x = act && L > 0.f;
        const bool is_y = act && L < 0.f;
        if (bu.x0 <= bu.x1) {
            int64_t q = is_x ? a + k * (int64_t)bu.x0 : far;
            int64_t dq = is_x ? k : 0;
            walk(padT + p_off + (size_t)(bu.x0 + kPad) * pny + kPad, pny, bu.x0, bu.x1, q, dq, ny,
                 acc0, acc1);
        }
        if (bu.y0 <= bu.y1) {
            int64_t q = is_y ? a + k * (int64_t)bu.y0 : far;
            int64_t dq = is_y ? k : 0;
            walk(pad + p_off + (size_t)(bu.y0 + kPad) * pnx + kPad, pnx, bu.y0, bu.y1, q, dq, nx,
                 acc0, acc1);
        }
        result = fabsf(L) * (acc0 + acc1 * kTwoM32) * scale;
        if (act) sino[(size_t)e * V * B + (size_t)v * B + b] = result;
        if (!act) result = 0.f;
    }
    if (NORM) {
        __shared__ double red[256];
        double r2 = (double)result * (double)result;
        red[threadIdx.x] = r2;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(size_t)e * gridDim.x + blockIdx.x] = red[0];
    }
}

// ------------------------------------------------------------ adjoint ---
struct AdjGeo {
    float R, D, inv_du, beta0;  // beta(p) = D (p.e_u) / (R - p.e_s) * inv_du + beta0
    float dl, xoff, yoff;       // pixel centre x = c*dl - xoff, y = r*dl - yoff
    float margin;
};

__device__ __forceinline__ float beta_of(const AdjGeo &g, float ct, float st, float px, float py)
{
    float pu = -px * st + py * ct;
    float ps = px * ct + py * st;
    return g.D * pu / (g.R - ps) * g.inv_du + g.beta0;
}

__global__ __launch_bounds__(256) void k_adj(const float *__restrict__ sino,
                                             const RayAdj *__restrict__ rays,
                                             const float *__restrict__ len,
                                             const ViewInfo *__restrict__ views, AdjGeo geo,
                                             int nx, int ny, int V, int B, int ntx, int nvg,
                                             float *__restrict__ out, float *__restrict__ part,
                                             int *__restrict__ counters, float scale)
{
    __shared__ float acc[4][kTile * kTileLd];
    __shared__ int is_last;
    const int e = blockIdx.z, g = blockIdx.y;
    const int tile = blockIdx.x;
    const int tr0 = (tile / ntx) * kTile, tc0 = (tile % ntx) * kTile;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float *my = acc[wid];
    for (int i = lane; i < kTile * kTileLd; i += 64) my[i] = 0.f;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();

    const int v_begin = (int)((int64_t)V * g / nvg), v_end = (int)((int64_t)V * (g + 1) / nvg);
    const float *y_e = sino + (size_t)e * V * B;
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
    const size_t plane = (size_t)nx * ny;
    const int ntiles = gridDim.x;
    float *dst = out + (size_t)e * plane;
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
    float *tiles = part + ((size_t)e * ntiles + tile) * nvg * (kTile * kTile);
    for (int i = threadIdx.x; i < kTile * kTile; i += 256) {
        int o = (i / kTile) * kTileLd + i % kTile;
        tiles[(size_t)g * (kTile * kTile) + i] = ((acc[0][o] + acc[1][o]) + acc[2][o]) + acc[3][o];
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        int prev = atomicAdd(&counters[e * ntiles + tile], 1);
        is_last = prev == nvg - 1;
    }
    __syncthreads();
    if (!is_last) return;
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
    if (threadIdx.x == 0) counters[e * ntiles + tile] = 0;  // ready for the next launch
}

}  // namespace

// ---------------------------------------------------------- launchers ---
dect_status launch_pad(const GeomTables &t, const float *img, float *pad, float *padT, int batch,
                       hipStream_t s)
{
    const int nx = t.key.nx, ny = t.key.ny;
    dim3 grid((nx + 2 * kPad + 31) / 32, (ny + 2 * kPad + 31) / 32, batch);
    hipLaunchKernelGGL(k_pad, grid, dim3(256), 0, s, img, pad, padT, nx, ny);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

int fwd_blocks(const GeomTables &t) { return (t.key.V * t.nbundle + 3) / 4; }

dect_status launch_fwd(const GeomTables &t, const float *pad, const float *padT, float *sino,
                       int batch, float scale, double *norm_partial, hipStream_t s)
{
    const GeomKey &k = t.key;
    dim3 grid(fwd_blocks(t), batch);
    if (norm_partial)
        hipLaunchKernelGGL(k_fwd<true>, grid, dim3(256), 0, s, pad, padT, t.fwd, t.len,
                           t.bundles, sino, k.nx, k.ny, k.V, k.B, t.nbundle, scale,
                           norm_partial);
    else
        hipLaunchKernelGGL(k_fwd<false>, grid, dim3(256), 0, s, pad, padT, t.fwd, t.len,
                           t.bundles, sino, k.nx, k.ny, k.V, k.B, t.nbundle, scale,
                           (double *)nullptr);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

int adj_groups(const GeomTables &t, int batch)
{
    const int tiles = ((t.key.nx + kTile - 1) / kTile) * ((t.key.ny + kTile - 1) / kTile);
    int want = (512 + tiles * batch - 1) / (tiles * batch);
    int cap = std::max(1, t.key.V / 8);
    return std::max(1, std::min(want, cap));
}

size_t adj_partial_floats(const GeomTables &t, int batch)
{
    const int tiles = ((t.key.nx + kTile - 1) / kTile) * ((t.key.ny + kTile - 1) / kTile);
    const int nvg = adj_groups(t, batch);
    return nvg > 1 ? (size_t)batch * tiles * nvg * kTile * kTile : 0;
}

size_t adj_counters(const GeomTables &t, int batch)
{
    const int tiles = ((t.key.nx + kTile - 1) / kTile) * ((t.key.ny + kTile - 1) / kTile);
    return (size_t)batch * tiles;
}

dect_status launch_adj(const GeomTables &t, const float *sino, float *img, float *partial,
                       int *counters, int batch, float scale, hipStream_t s)
{
    const GeomKey &k = t.key;
    const int ntx = (k.nx + kTile - 1) / kTile, nty = (k.ny + kTile - 1) / kTile;
    const int nvg = adj_groups(t, batch);
    AdjGeo geo;
    geo.R = (float)k.sod;
    geo.D = (float)k.sdd;
    geo.inv_du = (float)(1.0 / k.bin);
    geo.beta0 = (float)((k.B - 1) / 2.0 - k.off / k.bin);
    geo.dl = (float)k.pixel;
    geo.xoff = (float)((k.nx - 1) / 2.0 * k.pixel);
    geo.yoff = (float)((k.ny - 1) / 2.0 * k.pixel);
    geo.margin = 0.5f;
    dim3 grid(ntx * nty, nvg, batch);
    hipLaunchKernelGGL(k_adj, grid, dim3(256), 0, s, sino, t.adj, t.len, t.views, geo, k.nx,
                       k.ny, k.V, k.B, ntx, nvg, img, partial, counters, scale);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

// ----------------------------------------------------- plain entry points ---
static std::mutex g_ws_mu;
static std::vector<std::pair<std::pair<int, hipStream_t>, std::unique_ptr<ProjWork>>> g_ws;

// One workspace per (device, stream): calls on different streams never share
// scratch memory.
static ProjWork *workspace(hipStream_t s)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (auto &p : g_ws)
        if (p.first.first == dev && p.first.second == s) return p.second.get();
    g_ws.emplace_back(std::make_pair(dev, s), std::make_unique<ProjWork>());
    return g_ws.back().second.get();
}

dect_status project(const dect_geometry *g, const float *img, float *sino, int batch,
                    hipStream_t s)
{
    if (!img || !sino || batch <= 0)
        return fail(DECT_ERR_INVALID_ARG, "dect_project: null buffer or batch <= 0");
    GeomTables *t = nullptr;
    dect_status st = get_tables(g, &t);
    if (st != DECT_OK) return st;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    ProjWork *w = workspace(s);
    const size_t padn = (size_t)(g->nx + 2 * kPad) * (g->ny + 2 * kPad) * batch * sizeof(float);
    // the padded copies are reused across calls and geometries; k_pad writes
    // them whole, border included
    if (w->pad.bytes < padn) {
        DECT_HIP(hipStreamSynchronize(s));
        if ((st = w->pad.ensure(padn)) != DECT_OK) return st;
        if ((st = w->padT.ensure(padn)) != DECT_OK) return st;
    }
    if ((st = launch_pad(*t, img, (float *)w->pad.ptr, (float *)w->padT.ptr, batch, s)) != DECT_OK)
        return st;
    return launch_fwd(*t, (const float *)w->pad.ptr, (const float *)w->padT.ptr, sino, batch, 1.0f,
                      nullptr, s);
}

dect_status backproject(const dect_geometry *g, const float *sino, float *img, int batch,
                        hipStream_t s)
{
    if (!img || !sino || batch <= 0)
        return fail(DECT_ERR_INVALID_ARG, "dect_backproject: null buffer or batch <= 0");
    GeomTables *t = nullptr;
    dect_status st = get_tables(g, &t);
    if (st != DECT_OK) return st;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    ProjWork *w = workspace(s);
    const size_t need = adj_partial_floats(*t, batch) * sizeof(float);
    const size_t ncnt = adj_counters(*t, batch) * sizeof(int);
    if (w->partial.bytes < need || w->norm.bytes < ncnt) {
        DECT_HIP(hipStreamSynchronize(s));
        if ((st = w->partial.ensure(need)) != DECT_OK) return st;
        if ((st = w->norm.ensure(ncnt, true)) != DECT_OK) return st;  // counters start at zero
    }
    return launch_adj(*t, sino, img, (float *)w->partial.ptr, (int *)w->norm.ptr, batch, 1.0f, s);
}

}  // namespace dect
