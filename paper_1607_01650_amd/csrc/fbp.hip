// Fan-beam filtered back-projection on gfx950: the analytic reconstruction
// the paper compares its method with (Sec. 3), for the flat detector over a
// full turn of equally spaced views, in the textbook form for equally spaced
// collinear detectors:
//   k_fbp_filter : per (64-bin chunk, view, pair) block.  Both images' rows are weighted by
//                  R / sqrt(R^2 + s_b^2) (s_b the bin position scaled to a
//                  virtual detector through the isocentre, spacing ds =
//                  du R / D) into LDS, then convolved with the band-limited
//                  ramp kernel of spacing ds and halved (a full turn sees
//                  every line twice).  Output: the pair's filtered views,
//                  interleaved and zero-padded by kQPad bins on each side.
//   k_fbp_bp     : one thread per pixel of a pair, all views: the filtered
//                  views at the virtual-detector position where the ray from
//                  the source through the pixel meets it (linear
//                  interpolation, one 16-byte load for both taps of both
//                  images), weighted by R^2 / (R - p . e_s)^2, times 2 pi / V.
// Both are gathers with no atomics; the filter reads its row from LDS, the
// back-projection reads the ~1 MB of filtered views per image from L2.
#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"
#include "proj_device.h"
#include "xcd.h"

namespace dect {
namespace {

constexpr int kQPad = 2;           // zero bins on each side of a filtered view
constexpr int kFbpMaxBins = 6144;  // the filter's LDS (2.5 floats per bin) stays under 64 KB

// grid (output chunks of 64 bins, V, pairs), 256 threads; dynamic LDS:
// 2 * B weighted samples (interleaved) + B / 2 + 1 kernel values.  Wavefront
// w of a block sums the w-th quarter of the odd kernel taps for the chunk's
// 64 outputs (lane = output); the four partial sums are added in wave order.
__global__ __launch_bounds__(256) void k_fbp_filter(const float *__restrict__ sino, int batch,
                                                    int V, int B, float r_sod, float u_to_s,
                                                    float u0, float du_v, float inv2ds,
                                                    f2v *__restrict__ q)
{
    extern __shared__ float lds[];
    __shared__ double part[4][2][64];
    f2v *row = (f2v *)lds;         // [B]
    float *hk = lds + 2 * B;       // [B / 2 + 1]: 1 / (pi^2 k^2), k = 2j + 1
    const int v = blockIdx.y, pr = blockIdx.z;
    const int e0 = 2 * pr;
    const bool two = e0 + 1 < batch;
    const size_t M = (size_t)V * B;
    const float *s0 = sino + (size_t)e0 * M + (size_t)v * B;
    const float *s1 = two ? s0 + M : nullptr;
    for (int b = threadIdx.x; b < B; b += 256) {
        // virtual-detector position s_b = u_b R / D, weight R / sqrt(R^2 + s_b^2)
        const float s = (u0 + b * du_v) * u_to_s;
        const float w = r_sod * rsqrtf(fmaf(s, s, r_sod * r_sod));
        f2v t;
        t.x = w * s0[b];
        t.y = two ? w * s1[b] : 0.f;
        row[b] = t;
    }
    const double kPi2 = 9.869604401089358;  // pi^2
    for (int j = threadIdx.x; j <= B / 2; j += 256) {
        const double k = 2.0 * j + 1.0;
        hk[j] = (float)(1.0 / (kPi2 * k * k));
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int b = blockIdx.x * 64 + lane;  // padded output index
    const int c = b - kQPad;               // the bin it holds
    const int nk = B / 2;                  // odd taps k = 2j + 1 < B
    const int j0 = nk * wid / 4, j1 = nk * (wid + 1) / 4;
    double ax = 0.0, ay = 0.0;
    if (c >= 0 && c < B)
        for (int j = j0; j < j1; ++j) {
            const int k = 2 * j + 1;
            f2v t = f2v(0.f);
            if (c - k >= 0) t += row[c - k];
            if (c + k < B) t += row[c + k];
            const float h = hk[j];
            ax = fma((double)h, (double)t.x, ax);
            ay = fma((double)h, (double)t.y, ay);
        }
    part[wid][0][lane] = ax;
    part[wid][1][lane] = ay;
    __syncthreads();
    if (wid == 0 && b < B + 2 * kQPad) {
        f2v r = f2v(0.f);
        if (c >= 0 && c < B) {
            ax = part[0][0][lane] + part[1][0][lane] + part[2][0][lane] + part[3][0][lane];
            ay = part[0][1][lane] + part[1][1][lane] + part[2][1][lane] + part[3][1][lane];
            const f2v p = row[c];
            r.x = (float)((0.25 * (double)p.x - ax) * (double)inv2ds);
            r.y = (float)((0.25 * (double)p.y - ay) * (double)inv2ds);
        }
        q[((size_t)pr * V + v) * (B + 2 * kQPad) + b] = r;
    }
}

// grid (tiles, pairs) of 16 x 16 pixels, XCD-ordered.
__global__ __launch_bounds__(256) void k_fbp_bp(const f2v *__restrict__ q,
                                                const ViewInfo *__restrict__ views, int batch,
                                                int nx, int ny, int V, int B, float pixel,
                                                float sod, float sdd_over_du, float b0,
                                                float scale, float *__restrict__ img)
{
    const unsigned item = xcd_order(block_linear(), grid_blocks());
    const int ntx = (nx + 15) / 16, nty = (ny + 15) / 16;
    const int pr = (int)(item / (unsigned)(ntx * nty));
    const int tile = (int)(item % (unsigned)(ntx * nty));
    const int c = (tile % ntx) * 16 + (threadIdx.x & 15);
    const int r = (tile / ntx) * 16 + (threadIdx.x >> 4);
    if (c >= nx || r >= ny) return;
    const float x = (c - 0.5f * (nx - 1)) * pixel, y = (r - 0.5f * (ny - 1)) * pixel;
    const int stride = B + 2 * kQPad;
    const char *base = (const char *)(q + (size_t)pr * V * stride);
    // one view: its contribution to both images
    auto view = [&](int v, float &s0, float &s1) {
        const ViewInfo vi = views[v];
        const float dist = sod - fmaf(x, vi.ct, y * vi.st);
        const float inv = __builtin_amdgcn_rcpf(dist);
        const float pu = fmaf(-x, vi.st, y * vi.ct);
        const float bf = fmaf(pu * inv, sdd_over_du, b0);
        const float fl = floorf(bf);
        // taps h, h + 1 of the padded row; beyond the detector both are zero
        const int h = (int)fminf(fmaxf(fl, (float)-kQPad), (float)B);
        const float w = bf - fl;
        const char *rowp = base + (size_t)v * stride * 8;
        const f4a8 t = *(const f4a8 *)(rowp + (unsigned)(h + kQPad) * 8u);
        const float g = (sod * inv) * (sod * inv);
        s0 = fmaf(g, fmaf(w, t.z - t.x, t.x), s0);
        s1 = fmaf(g, fmaf(w, t.w - t.y, t.y), s1);
    };
    // groups of 8 views (their loads in flight together) summed in FP32,
    // the group sums in FP64
    double acc0 = 0.0, acc1 = 0.0;
    int v0 = 0;
    for (; v0 + 8 <= V; v0 += 8) {
        float s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int u = 0; u < 8; ++u) view(v0 + u, s0, s1);
        acc0 += (double)s0;
        acc1 += (double)s1;
    }
    float s0 = 0.f, s1 = 0.f;
    for (; v0 < V; ++v0) view(v0, s0, s1);
    acc0 += (double)s0;
    acc1 += (double)s1;
    const size_t N = (size_t)nx * ny, i = (size_t)r * nx + c;
    const int e0 = 2 * pr;
    img[(size_t)e0 * N + i] = (float)(acc0 * (double)scale);
    if (e0 + 1 < batch) img[(size_t)(e0 + 1) * N + i] = (float)(acc1 * (double)scale);
}

std::mutex g_fbp_mu;
std::vector<std::pair<std::pair<int, hipStream_t>, std::unique_ptr<DevBuf>>> g_fbp_ws;

DevBuf *fbp_workspace(hipStream_t s)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (auto &p : g_fbp_ws)
        if (p.first.first == dev && p.first.second == s) return p.second.get();
    g_fbp_ws.emplace_back(std::make_pair(dev, s), std::make_unique<DevBuf>());
    return g_fbp_ws.back().second.get();
}

}  // namespace

// Bytes of the filtered, padded sinograms of `batch` items (pairs).
static size_t fbp_work_bytes(const dect_geometry *g, int batch)
{
    return (size_t)pairs_of(batch) * g->n_views * (g->n_bins + 2 * kQPad) * sizeof(f2v);
}

// The work buffer dect_fbp allocates for `batch` sinograms on one stream,
// for a dry run under a SizingScope.
dect_status fbp_size_run(const dect_geometry *g, int batch)
{
    DevBuf w;
    return w.ensure(fbp_work_bytes(g, batch));
}

dect_status fbp(const dect_geometry *g, const float *sino, float *img, int batch, hipStream_t s)
{
    if (!sino || !img || batch <= 0)
        return fail(DECT_ERR_INVALID_ARG, "dect_fbp: null buffer or batch <= 0");
    dect_status st = validate_geometry(g);
    if (st != DECT_OK) return st;
    if (g->angles_rad)
        return fail(DECT_ERR_INVALID_ARG, "dect_fbp: needs the equally spaced full turn (angles_rad NULL)");
    if (g->n_bins > kFbpMaxBins)
        return fail(DECT_ERR_INVALID_ARG, "dect_fbp: at most 6144 detector bins");
    GeomTables *t = nullptr;
    if ((st = get_tables(g, &t)) != DECT_OK) return st;
    const int V = g->n_views, B = g->n_bins, pairs = pairs_of(batch);
    const size_t qbytes = fbp_work_bytes(g, batch);
    std::lock_guard<std::mutex> lk(g_fbp_mu);
    DevBuf *w = fbp_workspace(s);
    if (w->bytes < qbytes) {
        DECT_HIP(hipStreamSynchronize(s));
        if ((st = w->ensure(qbytes)) != DECT_OK) return st;
    }
    const double R = g->sod_mm, D = g->sdd_mm, du = g->bin_mm;
    const double ds = du * R / D;
    const size_t lds = (size_t)(2 * B + B / 2 + 1) * sizeof(float);
    const unsigned chunks = (unsigned)((B + 2 * kQPad + 63) / 64);
    hipLaunchKernelGGL(k_fbp_filter, dim3(chunks, V, pairs), dim3(256), lds, s, sino, batch, V, B,
                       (float)R, (float)(R / D), (float)(-(B - 1) / 2.0 * du + g->det_offset_mm),
                       (float)du, (float)(0.5 / ds), (f2v *)w->ptr);
    DECT_HIP(hipGetLastError());
    const int ntx = (g->nx + 15) / 16, nty = (g->ny + 15) / 16;
    const float b0 = (float)((B - 1) / 2.0 - g->det_offset_mm / du);
    hipLaunchKernelGGL(k_fbp_bp, dim3(ntx * nty, pairs), dim3(256), 0, s, (const f2v *)w->ptr,
                       (const ViewInfo *)t->views, batch, g->nx, g->ny, V, B, (float)g->pixel_mm,
                       (float)R, (float)(D / du), b0, (float)(2.0 * M_PI / V), img);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

void release_fbp_work()
{
    std::lock_guard<std::mutex> lk(g_fbp_mu);
    g_fbp_ws.clear();
}

}  // namespace dect
