// One unrolled ADM-TV step (Eq. 10 with a given step alpha in place of the
// BB step) and its vector-Jacobian product, for a batch of images that
// share one size.  The data term h = mu A^T (A f - g) comes from the
// projector pair (the caller forms A f, r = A f - g with k_unr_resid, and
// A^T r); everything else runs here:
//   z  = shrink(grad f - lambda / rho, 1 / rho)                      (Eq. 8)
//   G  = mu hb + grad^T (rho (grad f - z) - lambda)                  (Eq. 9)
//   f' = f - alpha G
//   lambda' = lambda - xi (grad f' - z)                              (Eq. 7)
// with grad the backward differences of Eq. 2 (zero on the first column and
// row), grad^T its exact adjoint and shrink the isotropic shrinkage with
// |v| evaluated as sqrt(max(|v|^2, 1e-30)) so that value and derivative stay
// finite at v = 0.  Images are [batch][ny][nx] FP32; (mu, rho, xi, alpha)
// are read from device memory, so learnable step parameters never leave the
// device.  Per-pixel arithmetic in FP32; the parameter gradients are FP64
// per-block partial sums reduced in a fixed order by one block (bitwise
// reproducible).
#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"

namespace dect {
namespace {

constexpr int kUnrBlocks = 2048;  // grid of the element-wise kernels (grid-stride)
enum { P_MU, P_RHO, P_XI, P_ALPHA, P_COUNT };

struct Img {
    int nx, ny;
    size_t N, T;  // pixels per image, pixels of the batch
};

struct Prm {
    float mu, rho, xi, alpha;
};

__device__ __forceinline__ Prm load_prm(const float *__restrict__ p)
{
    return Prm{p[0], p[1], p[2], p[3]};
}

// Backward differences of Eq. 2 at pixel i (column c, row r) of image x.
__device__ __forceinline__ void grad_at(const Img &d, const float *__restrict__ x, size_t i, int c,
                                        int r, float &gx, float &gy)
{
    const float xi = x[i];
    gx = c >= 1 ? xi - x[i - 1] : 0.f;
    gy = r >= 1 ? xi - x[i - d.nx] : 0.f;
}

// The z-step at pixel i: v = grad f - lambda / rho, n = |v| (floored), the
// shrink factor s and z = s v; also W = rho (grad f - z) - lambda.
struct ZW {
    float dx, dy, vx, vy, n, s, zx, zy, wx, wy;
};

__device__ __forceinline__ ZW zstep(const Img &d, const float *__restrict__ f,
                                    const float *__restrict__ lx, const float *__restrict__ ly,
                                    size_t i, int c, int r, float rho)
{
    ZW o;
    grad_at(d, f, i, c, r, o.dx, o.dy);
    const float lxi = lx[i], lyi = ly[i];
    o.vx = o.dx - lxi / rho;
    o.vy = o.dy - lyi / rho;
    o.n = sqrtf(fmaxf(o.vx * o.vx + o.vy * o.vy, 1e-30f));
    const float t = 1.0f / rho;
    o.s = fmaxf(o.n - t, 0.f) / o.n;
    o.zx = o.s * o.vx;
    o.zy = o.s * o.vy;
    o.wx = rho * (o.dx - o.zx) - lxi;
    o.wy = rho * (o.dy - o.zy) - lyi;
    return o;
}

__device__ __forceinline__ void pix(const Img &d, size_t i, int &c, int &r)
{
    const size_t p = i % d.N;
    c = (int)(p % d.nx);
    r = (int)(p / d.nx);
}

// G at pixel i: mu hb + grad^T W, W formed at i and at its successors
// i + 1 and i + nx (the adjoint of the backward differences).
__device__ __forceinline__ float g_at(const Img &d, const float *__restrict__ f,
                                      const float *__restrict__ lx, const float *__restrict__ ly,
                                      const float *__restrict__ hb, size_t i, int c, int r,
                                      const Prm &p, ZW &own)
{
    own = zstep(d, f, lx, ly, i, c, r, p.rho);
    float s = 0.f;
    if (c >= 1) s += own.wx;
    if (c + 1 <= d.nx - 1) s -= zstep(d, f, lx, ly, i + 1, c + 1, r, p.rho).wx;
    if (r >= 1) s += own.wy;
    if (r + 1 <= d.ny - 1) s -= zstep(d, f, lx, ly, i + d.nx, c, r + 1, p.rho).wy;
    return p.mu * hb[i] + s;
}

__device__ __forceinline__ void block_sum(double v, double *out)
{
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
    __syncthreads();
}

#define UNR_LOOP(d) \
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < (d).T; i += (size_t)gridDim.x * 256)

// r = p - g (r may be p)
__global__ __launch_bounds__(256) void k_unr_resid(const float *p, const float *__restrict__ g,
                                                   size_t n, float *r)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        r[i] = p[i] - g[i];
}

// Forward, first pass: f' = f - alpha G; z into the lambda outputs (the
// second pass turns it into lambda').
__global__ __launch_bounds__(256) void k_unr_fwd_a(Img d, const float *__restrict__ f,
                                                   const float *__restrict__ lx,
                                                   const float *__restrict__ ly,
                                                   const float *__restrict__ hb,
                                                   const float *__restrict__ prm,
                                                   float *__restrict__ fo, float *__restrict__ zx,
                                                   float *__restrict__ zy)
{
    const Prm p = load_prm(prm);
    UNR_LOOP(d) {
        int c, r;
        pix(d, i, c, r);
        ZW own;
        const float G = g_at(d, f, lx, ly, hb, i, c, r, p, own);
        fo[i] = f[i] - p.alpha * G;
        zx[i] = own.zx;
        zy[i] = own.zy;
    }
}

// Forward, second pass: lambda' = lambda - xi (grad f' - z), z read from the
// outputs it replaces.
__global__ __launch_bounds__(256) void k_unr_fwd_b(Img d, const float *__restrict__ fo,
                                                   const float *__restrict__ lx,
                                                   const float *__restrict__ ly,
                                                   const float *__restrict__ prm,
                                                   float *__restrict__ lxo, float *__restrict__ lyo)
{
    const float xi = prm[P_XI];
    UNR_LOOP(d) {
        int c, r;
        pix(d, i, c, r);
        float gx, gy;
        grad_at(d, fo, i, c, r, gx, gy);
        lxo[i] = lx[i] - xi * (gx - lxo[i]);
        lyo[i] = ly[i] - xi * (gy - lyo[i]);
    }
}

// Backward, pass 1: G and f' recomputed (bitwise as in the forward).
__global__ __launch_bounds__(256) void k_unr_bwd_g(Img d, const float *__restrict__ f,
                                                   const float *__restrict__ lx,
                                                   const float *__restrict__ ly,
                                                   const float *__restrict__ hb,
                                                   const float *__restrict__ prm,
                                                   float *__restrict__ G, float *__restrict__ fo)
{
    const Prm p = load_prm(prm);
    UNR_LOOP(d) {
        int c, r;
        pix(d, i, c, r);
        ZW own;
        const float g = g_at(d, f, lx, ly, hb, i, c, r, p, own);
        G[i] = g;
        fo[i] = f[i] - p.alpha * g;
    }
}

// Backward, pass 2, given the cotangents gfo of f' and glx, gly of lambda':
//   the multiplier step: d(grad f')~ = -xi glam', xi~ = -<glam', grad f' - z>;
//   f'~ = gfo + grad^T d(grad f')~ (kept in ftot);
//   G~ = -alpha f'~, alpha~ = -<f'~, G>; hb~ = mu G~, mu~ = <G~, hb>.
__global__ __launch_bounds__(256) void k_unr_bwd_f(Img d, const float *__restrict__ f,
                                                   const float *__restrict__ lx,
                                                   const float *__restrict__ ly,
                                                   const float *__restrict__ hb,
                                                   const float *__restrict__ prm,
                                                   const float *__restrict__ G,
                                                   const float *__restrict__ fo,
                                                   const float *__restrict__ gfo,
                                                   const float *__restrict__ glx,
                                                   const float *__restrict__ gly,
                                                   float *__restrict__ ftot, float *__restrict__ Gb,
                                                   float *__restrict__ ghb,
                                                   double *__restrict__ part, size_t stride)
{
    const Prm p = load_prm(prm);
    double sxi = 0.0, salpha = 0.0, smu = 0.0;
    UNR_LOOP(d) {
        int c, r;
        pix(d, i, c, r);
        const ZW z = zstep(d, f, lx, ly, i, c, r, p.rho);
        float gx, gy;
        grad_at(d, fo, i, c, r, gx, gy);
        const float ax = glx[i], ay = gly[i];
        sxi -= (double)ax * (gx - z.zx) + (double)ay * (gy - z.zy);
        // grad^T of -xi glam' at i
        float t = 0.f;
        if (c >= 1) t += -p.xi * ax;
        if (c + 1 <= d.nx - 1) t -= -p.xi * glx[i + 1];
        if (r >= 1) t += -p.xi * ay;
        if (r + 1 <= d.ny - 1) t -= -p.xi * gly[i + d.nx];
        const float ft = gfo[i] + t;
        ftot[i] = ft;
        const float gb = -p.alpha * ft;
        Gb[i] = gb;
        ghb[i] = p.mu * gb;
        salpha -= (double)ft * G[i];
        smu += (double)gb * hb[i];
    }
    block_sum(smu, part + P_MU * stride + blockIdx.x);
    block_sum(sxi, part + P_XI * stride + blockIdx.x);
    block_sum(salpha, part + P_ALPHA * stride + blockIdx.x);
}

// Backward, pass 3: W~ = grad G~ (grad^T's adjoint), then through W = rho
// (d - z) - lambda, the shrinkage and v = d - lambda / rho:
//   z~ = xi glam' - rho W~;
//   v~ = z~ - t (z~ / n - v <v, z~> / n^3), t~ = -<z~, v> / n  where n > t
//        (z = v - t v / n), else 0;
//   d~ = rho W~ + v~ (kept in db), lambda~ = glam' - W~ - v~ / rho;
//   rho~ = <W~, d - z> + <v~, lambda> / rho^2 - t~ / rho^2.
__global__ __launch_bounds__(256) void k_unr_bwd_z(Img d, const float *__restrict__ f,
                                                   const float *__restrict__ lx,
                                                   const float *__restrict__ ly,
                                                   const float *__restrict__ prm,
                                                   const float *__restrict__ Gb,
                                                   const float *__restrict__ glx,
                                                   const float *__restrict__ gly,
                                                   float *__restrict__ dbx, float *__restrict__ dby,
                                                   float *__restrict__ glx_in,
                                                   float *__restrict__ gly_in,
                                                   double *__restrict__ part, size_t stride)
{
    const Prm p = load_prm(prm);
    const float t = 1.0f / p.rho;
    double srho = 0.0;
    UNR_LOOP(d) {
        int c, r;
        pix(d, i, c, r);
        const ZW z = zstep(d, f, lx, ly, i, c, r, p.rho);
        float wbx, wby;
        grad_at(d, Gb, i, c, r, wbx, wby);
        const float ax = glx[i], ay = gly[i];
        const float zbx = p.xi * ax - p.rho * wbx, zby = p.xi * ay - p.rho * wby;
        float vbx = 0.f, vby = 0.f, tb = 0.f;
        if (z.n > t) {
            const float vz = z.vx * zbx + z.vy * zby;
            const float n3 = z.n * z.n * z.n;
            vbx = zbx - t * (zbx / z.n - z.vx * vz / n3);
            vby = zby - t * (zby / z.n - z.vy * vz / n3);
            tb = -vz / z.n;
        }
        dbx[i] = p.rho * wbx + vbx;
        dby[i] = p.rho * wby + vby;
        const float lxi = lx[i], lyi = ly[i];
        glx_in[i] = ax - wbx - vbx / p.rho;
        gly_in[i] = ay - wby - vby / p.rho;
        const double r2 = (double)p.rho * p.rho;
        srho += (double)wbx * (z.dx - z.zx) + (double)wby * (z.dy - z.zy) +
                ((double)vbx * lxi + (double)vby * lyi) / r2 - (double)tb / r2;
    }
    block_sum(srho, part + P_RHO * stride + blockIdx.x);
}

// Backward, pass 4: f~ = f'~ + grad^T d~.
__global__ __launch_bounds__(256) void k_unr_bwd_out(Img d, const float *__restrict__ ftot,
                                                     const float *__restrict__ dbx,
                                                     const float *__restrict__ dby,
                                                     float *__restrict__ gf)
{
    UNR_LOOP(d) {
        int c, r;
        pix(d, i, c, r);
        float s = 0.f;
        if (c >= 1) s += dbx[i];
        if (c + 1 <= d.nx - 1) s -= dbx[i + 1];
        if (r >= 1) s += dby[i];
        if (r + 1 <= d.ny - 1) s -= dby[i + d.nx];
        gf[i] = ftot[i] + s;
    }
}

// The four parameter gradients (mu, rho, xi, alpha) from the partial sums,
// each in a fixed order, rounded to FP32.
__global__ __launch_bounds__(256) void k_unr_bwd_prm(const double *__restrict__ part,
                                                     size_t stride, int nb,
                                                     float *__restrict__ gprm)
{
    __shared__ double red[256];
    for (int q = 0; q < P_COUNT; ++q) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nb; b += 256) v += part[q * stride + b];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) gprm[q] = (float)red[0];
        __syncthreads();
    }
}

struct UnrWork {
    DevBuf G, fo, ftot, Gb, dbx, dby, part;
};

std::mutex g_unr_mu;
std::vector<std::pair<int, std::unique_ptr<UnrWork>>> g_unr;

UnrWork *unr_work()
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (auto &p : g_unr)
        if (p.first == dev) return p.second.get();
    g_unr.emplace_back(dev, std::make_unique<UnrWork>());
    return g_unr.back().second.get();
}

dect_status check_img(int nx, int ny, int batch, Img &d)
{
    if (nx <= 0 || ny <= 0 || batch < 0 || (int64_t)nx * ny > (int64_t)1 << 30 ||
        (int64_t)nx * ny * batch > (int64_t)1 << 34)
        return fail(DECT_ERR_INVALID_ARG, "unrolled step: bad image size or batch");
    d.nx = nx;
    d.ny = ny;
    d.N = (size_t)nx * ny;
    d.T = d.N * (size_t)batch;
    return DECT_OK;
}

unsigned grid_of(size_t n) { return (unsigned)std::min<size_t>(kUnrBlocks, (n + 255) / 256); }

bool overlaps(const void *a, const void *b, size_t bytes)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + bytes && y < x + bytes;
}

}  // namespace

void release_unrolled_work()
{
    std::lock_guard<std::mutex> lk(g_unr_mu);
    g_unr.clear();
}

dect_status unrolled_residual(int64_t n, const float *p, const float *g, float *r, hipStream_t s)
{
    if (n < 0) return fail(DECT_ERR_INVALID_ARG, "dect_unrolled_residual: n < 0");
    if (n == 0) return DECT_OK;
    if (!p || !g || !r) return fail(DECT_ERR_INVALID_ARG, "dect_unrolled_residual: null buffer");
    hipLaunchKernelGGL(k_unr_resid, dim3(grid_of((size_t)n)), dim3(256), 0, s, p, g, (size_t)n,
                       r);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status unrolled_step(int nx, int ny, int batch, const float *f, const float *lx,
                          const float *ly, const float *hb, const float *prm, float *fo,
                          float *lxo, float *lyo, hipStream_t s)
{
    Img d;
    dect_status st = check_img(nx, ny, batch, d);
    if (st) return st;
    if (d.T == 0) return DECT_OK;
    if (!f || !lx || !ly || !hb || !prm || !fo || !lxo || !lyo)
        return fail(DECT_ERR_INVALID_ARG, "dect_unrolled_step: null buffer");
    const size_t bytes = d.T * 4;
    const void *in[4] = {f, lx, ly, hb};
    const void *out[3] = {fo, lxo, lyo};
    for (const void *o : out)
        for (const void *i : in)
            if (overlaps(o, i, bytes))
                return fail(DECT_ERR_INVALID_ARG, "dect_unrolled_step: outputs overlap inputs");
    if (overlaps(fo, lxo, bytes) || overlaps(fo, lyo, bytes) || overlaps(lxo, lyo, bytes))
        return fail(DECT_ERR_INVALID_ARG, "dect_unrolled_step: outputs overlap each other");
    const unsigned g = grid_of(d.T);
    hipLaunchKernelGGL(k_unr_fwd_a, dim3(g), dim3(256), 0, s, d, f, lx, ly, hb, prm, fo, lxo, lyo);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_unr_fwd_b, dim3(g), dim3(256), 0, s, d, (const float *)fo, lx, ly, prm,
                       lxo, lyo);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status unrolled_step_backward(int nx, int ny, int batch, const float *f, const float *lx,
                                   const float *ly, const float *hb, const float *prm,
                                   const float *gfo, const float *glxo, const float *glyo,
                                   float *gf, float *glx, float *gly, float *ghb, float *gprm,
                                   hipStream_t s)
{
    Img d;
    dect_status st = check_img(nx, ny, batch, d);
    if (st) return st;
    if (!gprm) return fail(DECT_ERR_INVALID_ARG, "dect_unrolled_step_backward: gprm is NULL");
    if (d.T == 0) {  // an empty batch: zero parameter gradients
        hipLaunchKernelGGL(k_unr_bwd_prm, dim3(1), dim3(256), 0, s, (const double *)nullptr,
                           (size_t)0, 0, gprm);
        DECT_HIP(hipGetLastError());
        return DECT_OK;
    }
    if (!f || !lx || !ly || !hb || !prm || !gfo || !glxo || !glyo || !gf || !glx || !gly || !ghb)
        return fail(DECT_ERR_INVALID_ARG, "dect_unrolled_step_backward: null buffer");
    const size_t bytes = d.T * 4;
    const void *in[8] = {f, lx, ly, hb, gfo, glxo, glyo, prm};
    const void *out[4] = {gf, glx, gly, ghb};
    for (const void *o : out)
        for (int k = 0; k < 8; ++k)
            if (overlaps(o, in[k], k == 7 ? 16 : bytes))
                return fail(DECT_ERR_INVALID_ARG,
                            "dect_unrolled_step_backward: outputs overlap inputs");
    for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b)
            if (overlaps(out[a], out[b], bytes))
                return fail(DECT_ERR_INVALID_ARG,
                            "dect_unrolled_step_backward: outputs overlap each other");
    const unsigned g = grid_of(d.T);
    std::lock_guard<std::mutex> lk(g_unr_mu);
    UnrWork *w = unr_work();
    if ((st = w->G.ensure(bytes)) || (st = w->fo.ensure(bytes)) || (st = w->ftot.ensure(bytes)) ||
        (st = w->Gb.ensure(bytes)) || (st = w->dbx.ensure(bytes)) || (st = w->dby.ensure(bytes)) ||
        (st = w->part.ensure((size_t)P_COUNT * g * 8)))
        return st;
    float *G = (float *)w->G.ptr, *fo = (float *)w->fo.ptr, *ftot = (float *)w->ftot.ptr;
    float *Gb = (float *)w->Gb.ptr, *dbx = (float *)w->dbx.ptr, *dby = (float *)w->dby.ptr;
    double *part = (double *)w->part.ptr;
    hipLaunchKernelGGL(k_unr_bwd_g, dim3(g), dim3(256), 0, s, d, f, lx, ly, hb, prm, G, fo);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_unr_bwd_f, dim3(g), dim3(256), 0, s, d, f, lx, ly, hb, prm,
                       (const float *)G, (const float *)fo, gfo, glxo, glyo, ftot, Gb, ghb, part,
                       (size_t)g);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_unr_bwd_z, dim3(g), dim3(256), 0, s, d, f, lx, ly, prm,
                       (const float *)Gb, glxo, glyo, dbx, dby, glx, gly, part, (size_t)g);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_unr_bwd_out, dim3(g), dim3(256), 0, s, d, (const float *)ftot,
                       (const float *)dbx, (const float *)dby, gf);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_unr_bwd_prm, dim3(1), dim3(256), 0, s, (const double *)part, (size_t)g,
                       (int)g, gprm);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

}  // namespace dect
