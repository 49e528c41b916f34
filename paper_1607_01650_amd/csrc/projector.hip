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
#include "proj_device.h"
#include "xcd.h"

namespace dect {

namespace {

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
template <bool NORM>
__global__ __launch_bounds__(256) void k_fwd(const float *__restrict__ pad,
                                             const float *__restrict__ padT,
                                             const RayFwd *__restrict__ rays,
                                             const float *__restrict__ len,
                                             const Bundle *__restrict__ bundles,
                                             float *__restrict__ sino, int nx, int ny, int V,
                                             int B, int nbundle, float scale,
                                             double *__restrict__ partial,
                                             const float *__restrict__ sub0,
                                             const float *__restrict__ sub1, double ss0, double ss1,
                                             float *__restrict__ lo)
{
    __shared__ FwdShared sh;
    // (view, bundle) blocks in XCD order: each XCD works on one energy's
    // image, which then fits its L2
    const unsigned item = xcd_order(block_linear(), grid_blocks());
    const int e = (int)(item / gridDim.x), vb = (int)(item % gridDim.x);
    const size_t p_off = (size_t)e * (nx + 2 * kPad) * (ny + 2 * kPad);
    const double result =
        fwd_block(sh, pad + p_off, padT + p_off, rays, len, bundles, sino + (size_t)e * V * B, nx,
                  ny, B, nbundle, vb, scale, e == 0 ? sub0 : e == 1 ? sub1 : nullptr,
                  e == 0 ? ss0 : ss1, lo ? lo + (size_t)e * V * B : nullptr);
    if (NORM) {
        __shared__ double red[256];
        double tot = block_sum_256(result * result, red);
        if (threadIdx.x == 0) partial[(size_t)e * gridDim.x + vb] = tot;
    }
}

// ------------------------------------------------------------ adjoint ---
// grid (strips of both classes, view groups, batch); part: [batch][2][nvg]
// planes of nx*ny floats.
__global__ __launch_bounds__(kAdjThreads) void k_adj(const float *__restrict__ sino,
                                             const RayAdj *__restrict__ rays,
                                             const float *__restrict__ len,
                                             const BinRange *__restrict__ bins, int nx, int ny,
                                             int V, int B, int nvg, float *__restrict__ part)
{
    __shared__ AdjShared sh;
    // (strip, view group, item) blocks in XCD order: the blocks of one XCD
    // share a view group's rays and sinogram rows
    const unsigned item = xcd_order(block_linear(), grid_blocks());
    const int strip = (int)(item % gridDim.x), g = (int)(item / gridDim.x % gridDim.y);
    const int e = (int)(item / (gridDim.x * gridDim.y));
    const int nsx = adj_strips_x(nx, ny);
    const size_t plane = (size_t)nx * ny;
    const int cls = strip < nsx ? 0 : 1;
    adj_block(sh, sino + (size_t)e * V * B, rays, len, bins, nx, ny, V, B, strip, g, nvg,
              part + ((size_t)e * 2 * nvg + (size_t)cls * nvg + g) * plane);
}

__global__ __launch_bounds__(256) void k_adj_sum(const float *__restrict__ part, int nvg,
                                                 size_t plane, float *__restrict__ out,
                                                 float scale)
{
    const int e = blockIdx.y;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= plane) return;
    out[(size_t)e * plane + i] =
        adj_sum_pixel(part + (size_t)e * 2 * nvg * plane, plane, nvg, i) * scale;
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

int fwd_blocks(const GeomTables &t) { return t.key.V * t.nbundle; }

dect_status launch_fwd(const GeomTables &t, const float *pad, const float *padT, float *sino,
                       int batch, float scale, double *norm_partial, hipStream_t s,
                       const float *sub0, const float *sub1, double ss0, double ss1,
                       float *lo)
{
    const GeomKey &k = t.key;
    dim3 grid(fwd_blocks(t), batch);
    if (norm_partial)
        hipLaunchKernelGGL(k_fwd<true>, grid, dim3(256), 0, s, pad, padT, t.fwd, t.len,
                           t.bundles, sino, k.nx, k.ny, k.V, k.B, t.nbundle, scale,
                           norm_partial, sub0, sub1, ss0, ss1, lo);
    else
        hipLaunchKernelGGL(k_fwd<false>, grid, dim3(256), 0, s, pad, padT, t.fwd, t.len,
                           t.bundles, sino, k.nx, k.ny, k.V, k.B, t.nbundle, scale,
                           (double *)nullptr, sub0, sub1, ss0, ss1, lo);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

// View groups per strip: enough blocks to fill the chip (kAdjBlocks), but
// at least 8 views per group.
int adj_groups(const GeomTables &t, int batch)
{
    const int strips = adj_strips(t.key.nx, t.key.ny);
    int want = (kAdjBlocks + strips * batch - 1) / (strips * batch);
    int cap = std::max(1, t.key.V / 8);
    return std::max(1, std::min(want, cap));
}

size_t adj_partial_floats(const GeomTables &t, int batch, int nvg)
{
    if (nvg <= 0) nvg = adj_groups(t, batch);
    return (size_t)batch * 2 * nvg * t.key.nx * t.key.ny;
}

dect_status launch_adj(const GeomTables &t, const float *sino, float *img, float *partial,
                       int batch, float scale, hipStream_t s, int nvg)
{
    const GeomKey &k = t.key;
    if (nvg <= 0) nvg = adj_groups(t, batch);
    const size_t plane = (size_t)k.nx * k.ny;
    hipLaunchKernelGGL(k_adj, dim3(adj_strips(k.nx, k.ny), nvg, batch), dim3(kAdjThreads), 0, s,
                       sino,
                       t.adj, t.len, t.adj_bins, k.nx, k.ny, k.V, k.B, nvg, partial);
    DECT_HIP(hipGetLastError());
    if (!img) return DECT_OK;  // the caller consumes the partial planes itself
    hipLaunchKernelGGL(k_adj_sum, dim3((unsigned)((plane + 255) / 256), batch), dim3(256), 0, s,
                       (const float *)partial, nvg, plane, img, scale);
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
    if (w->partial.bytes < need) {
        DECT_HIP(hipStreamSynchronize(s));
        if ((st = w->partial.ensure(need)) != DECT_OK) return st;
    }
    return launch_adj(*t, sino, img, (float *)w->partial.ptr, batch, 1.0f, s);
}

}  // namespace dect
