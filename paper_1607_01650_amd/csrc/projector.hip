// Joseph fan-beam projector pair for gfx950.
//
// Both directions work on pairs of images with one geometry (the two
// energies of a slice, or consecutive batch items).  The padded images are
// stored interleaved, both images' values of a pixel side by side, so one
// load fetches the two taps of both images.
//
// Forward (A x): one lane per ray; a wavefront holds 16 adjacent bins of 4
// adjacent views and the block's wavefronts step through shares of the
// driving lines in lockstep, so the taps of all lanes land in one short run
// of a padded image line (the transposed copy for x-major rays).  The line
// coordinate is advanced in exact 32.32 fixed point.
//
// Adjoint (A^T y): output-stationary gather on strips.  x-major rays are
// gathered on strips of kSW rows x 64 columns (lane = column), y-major rays
// on strips of kSW columns x 64 rows (lane = row); each wavefront holds the
// strip in LDS and walks, view by view, the bins whose rays put a tap on its
// lanes' lines (each lane its own bins, from exact per-lane ranges).  Every
// weight is recomputed from the same fixed-point line coordinate as the
// forward pass, so the adjoint is the exact transpose of the forward matrix.
// No atomics: each pixel's sum runs in a fixed order (bins and views of a
// wave, waves of a block, view groups).
#include "proj_device.h"
#include "xcd.h"

namespace dect {

namespace {

// ------------------------------------------------------------ padding ---
// In: img [batch][ny][nx].  Out, per pair p of items (2p, 2p + 1; the second
// reads as zero when batch is odd): pad2 [p][ny+4][nx+4][2] and padT2
// [p][nx+4][ny+4][2], written whole (zero border of kPad included), so a
// reused buffer never carries another geometry's values.  The grid covers the
// padded domain in 32x32 tiles; padT2 goes through an LDS transpose.
__global__ __launch_bounds__(256) void k_pad(const float *__restrict__ img, int batch,
                                             f2v *__restrict__ pad2, f2v *__restrict__ padT2,
                                             int nx, int ny)
{
    __shared__ f2v tile[32][33];
    const int pr = blockIdx.z;
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;  // padded coordinates
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const size_t N = (size_t)nx * ny;
    const float *im0 = img + (size_t)(2 * pr) * N;
    const float *im1 = 2 * pr + 1 < batch ? im0 + N : nullptr;
    const int pnx = nx + 2 * kPad, pny = ny + 2 * kPad;
    const size_t p_off = (size_t)pr * pnx * pny;
    for (int j = ty; j < 32; j += 8) {
        int rp = r0 + j, cp = c0 + tx;
        int r = rp - kPad, c = cp - kPad;
        f2v v = f2v(0.f);
        if (r >= 0 && r < ny && c >= 0 && c < nx) {
            const size_t i = (size_t)r * nx + c;
            v.x = im0[i];
            v.y = im1 ? im1[i] : 0.f;
        }
        if (rp < pny && cp < pnx) pad2[p_off + (size_t)rp * pnx + cp] = v;
        tile[j][tx] = v;
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        int cp = c0 + j, rp = r0 + tx;
        if (rp < pny && cp < pnx) padT2[p_off + (size_t)cp * pny + rp] = tile[tx][j];
    }
}

// ------------------------------------------------------------ forward ---
// grid ((view, bundle) blocks, pairs); items 2p, 2p + 1 of `batch`.
template <bool NORM, bool SID>
__global__ __launch_bounds__(kFwdThreads) void k_fwd(const float *__restrict__ pad2,
                                             const float *__restrict__ padT2,
                                             const RayFwd *__restrict__ rays,
                                             const float *__restrict__ len,
                                             const SidW *__restrict__ sid,
                                             const Bundle *__restrict__ bundles,
                                             float *__restrict__ sino, int batch, int nx, int ny,
                                             int V, int B, int nbundle, float scale,
                                             double *__restrict__ partial,
                                             const float *__restrict__ sub0,
                                             const float *__restrict__ sub1, double ss0, double ss1,
                                             float *__restrict__ lo)
{
    __shared__ FwdShared sh;
    // (view, bundle) blocks in XCD order: neighbouring views and bundles,
    // which read the same image lines, share an XCD's L2
    const unsigned item = xcd_order(block_linear(), grid_blocks());
    const int pr = (int)(item / gridDim.x), vb = (int)(item % gridDim.x);
    const size_t p_off = (size_t)pr * 2 * (nx + 2 * kPad) * (ny + 2 * kPad);
    const size_t M = (size_t)V * B;
    const int e0 = 2 * pr;
    const bool two = e0 + 1 < batch;
    FwdOut o;
    o.sino[0] = sino + e0 * M;
    o.sino[1] = two ? sino + (e0 + 1) * M : nullptr;
    o.lo[0] = lo ? lo + e0 * M : nullptr;
    o.lo[1] = lo && two ? lo + (e0 + 1) * M : nullptr;
    o.sub[0] = e0 == 0 ? sub0 : nullptr;  // the subtrahends belong to items 0 and 1
    o.sub[1] = e0 == 0 ? sub1 : nullptr;
    o.sub_scale[0] = ss0;
    o.sub_scale[1] = ss1;
    double res[2];
    fwd_block<SID>(sh, pad2 + p_off, padT2 + p_off, rays, len, sid, bundles, o, nx, ny, V, B,
                   nbundle, vb, scale, res);
    if (NORM && threadIdx.x < 64) {  // the values live in wavefront 0
        const double t0 = lane_sum(res[0] * res[0]);
        const double t1 = lane_sum(res[1] * res[1]);
        if (threadIdx.x == 0) {
            partial[(size_t)e0 * gridDim.x + vb] = t0;
            if (two) partial[(size_t)(e0 + 1) * gridDim.x + vb] = t1;
        }
    }
}

// ------------------------------------------------------------ adjoint ---
// grid (strips of both classes, view groups, groups of NE items starting at
// item0); part: [batch][2][nvg] planes of nx*ny floats.
template <int NE, bool SID>
__global__ __launch_bounds__(kAdjThreads) void k_adj(const float *__restrict__ sino,
                                                     const RayFwd *__restrict__ rays_fx,
                                                     const float *__restrict__ len,
                                                     const SidW *__restrict__ sid,
                                                     const BinRange *__restrict__ bins,
                                                     const LaneRange *__restrict__ lanes, int nx,
                                                     int ny, int V, int B, int nvg, int item0,
                                                     float *__restrict__ part)
{
    __shared__ AdjShared<NE> sh;
    __shared__ AdjStage stage;
    __shared__ SidW sid_stage[SID ? kStageSlots : 1];
    // (strip, view group, items) blocks in XCD order: the blocks of one XCD
    // share a view group's rays and sinogram rows
    const unsigned item = xcd_order(block_linear(), grid_blocks());
    const int strip = (int)(item % gridDim.x), g = (int)(item / gridDim.x % gridDim.y);
    const int e0 = item0 + NE * (int)(item / (gridDim.x * gridDim.y));
    const int nsx = adj_strips_x(nx, ny);
    const size_t plane = (size_t)nx * ny, M = (size_t)V * B;
    const int cls = strip < nsx ? 0 : 1;
    const float *s[NE];
    float *p[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        s[i] = sino + (size_t)(e0 + i) * M;
        p[i] = part + ((size_t)(e0 + i) * 2 * nvg + (size_t)cls * nvg + g) * plane;
    }
    adj_block<NE, SID>(sh, s, rays_fx, len, sid, bins, lanes, nx, ny, V, B, strip, g, nvg, p,
                       stage, sid_stage);
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
int pairs_of(int batch) { return (batch + 1) / 2; }

dect_status launch_pad(const GeomTables &t, const float *img, float *pad2, float *padT2, int batch,
                       hipStream_t s)
{
    const int nx = t.key.nx, ny = t.key.ny;
    dim3 grid((nx + 2 * kPad + 31) / 32, (ny + 2 * kPad + 31) / 32, pairs_of(batch));
    hipLaunchKernelGGL(k_pad, grid, dim3(256), 0, s, img, batch, (f2v *)pad2, (f2v *)padT2, nx,
                       ny);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

int fwd_blocks(const GeomTables &t)
{
    return (t.key.V + kFwdViews - 1) / kFwdViews * t.nbundle;
}

dect_status launch_fwd(const GeomTables &t, const float *pad2, const float *padT2, float *sino,
                       int batch, float scale, double *norm_partial, hipStream_t s,
                       const float *sub0, const float *sub1, double ss0, double ss1,
                       float *lo)
{
    const GeomKey &k = t.key;
    dim3 grid(fwd_blocks(t), pairs_of(batch));
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(kFwdThreads), 0, s, pad2, padT2, t.fwd, t.len, t.sid,
                           t.bundles, sino, batch, k.nx, k.ny, k.V, k.B, t.nbundle, scale,
                           norm_partial, sub0, sub1, ss0, ss1, lo);
    };
    const bool sid = k.model == DECT_SIDDON;
    if (norm_partial) {
        if (sid) go(k_fwd<true, true>);
        else go(k_fwd<true, false>);
    } else {
        if (sid) go(k_fwd<false, true>);
        else go(k_fwd<false, false>);
    }
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

// View groups per strip: enough blocks to fill the chip (kAdjBlocks), but
// at least 8 views per group.  A block carries a pair of items.
int adj_groups(const GeomTables &t, int batch)
{
    const int strips = adj_strips(t.key.nx, t.key.ny);
    const int units = strips * pairs_of(batch);
    int want = (kAdjBlocks + units - 1) / units;
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
    const unsigned strips = (unsigned)adj_strips(k.nx, k.ny);
    auto go = [&](auto kern, unsigned items, int item0) {
        hipLaunchKernelGGL(kern, dim3(strips, nvg, items), dim3(kAdjThreads), 0, s, sino,
                           t.fwd, t.len, t.sid, t.adj_bins, t.adj_lanes, k.nx, k.ny, k.V, k.B, nvg,
                           item0, partial);
    };
    const bool sid = k.model == DECT_SIDDON;
    if (batch >= 2) {
        if (sid) go(k_adj<2, true>, batch / 2, 0);
        else go(k_adj<2, false>, batch / 2, 0);
    }
    if (batch % 2) {  // the last item of an odd batch on its own
        if (sid) go(k_adj<1, true>, 1, batch - 1);
        else go(k_adj<1, false>, 1, batch - 1);
    }
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

// Bytes of one interleaved padded layout of `batch` images (pairs).
static size_t pad_bytes(const dect_geometry *g, int batch)
{
    return (size_t)(g->nx + 2 * kPad) * (g->ny + 2 * kPad) * 2 * pairs_of(batch) * sizeof(float);
}

// The work buffers dect_project and dect_backproject allocate for `batch`
// images on one stream, for a dry run under a SizingScope.
dect_status proj_size_run(const dect_geometry *g, int batch)
{
    GeomTables *t = nullptr;
    dect_status st = get_tables(g, &t);
    if (st) return st;
    ProjWork w;
    if ((st = w.pad.ensure(pad_bytes(g, batch))) || (st = w.padT.ensure(pad_bytes(g, batch))) ||
        (st = w.partial.ensure(adj_partial_floats(*t, batch) * sizeof(float))))
        return st;
    return DECT_OK;
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
    const size_t padn = pad_bytes(g, batch);
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

void release_proj_work()
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    g_ws.clear();
}

}  // namespace dect
