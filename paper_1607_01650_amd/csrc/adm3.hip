// ADM-TV on a volume (Eq. 10 with Eq. 2's TV over backward differences in
// x, y and z, the isotropic shrinkage of Eq. 8 on the 3-vector, the
// deferred multiplier step of Eq. 7 and the BB1 step of Eq. 9), with the
// cone-beam projector pair as A.  The two energies advance together (each
// with its own state, step and partial sums) so that every projector call
// walks both volumes at once.  The iterate f and the residual r = A f -
// beta m are unevaluated sums of two FP32 values (f + flo, r + rlo, the low
// part within half an ulp of the high one), updated in FP64; the other
// state is FP32.  Every reduction is FP64 from per-block partial sums
// reduced in a fixed order by one block; scalars and the log stay on the
// device.
//
// Set-up: f + flo = beta x0 (or 0), lambda = z = 0, r + rlo = A f - beta m
// (the projector's FP64 ray sums, minus beta m in FP64), h = mu A^T r.
// Iteration k (element-wise kernels: grid-stride loops over at most 2048
// blocks, so the one-block reductions read few partial sums):
//   k3_tv     lambda -= xi (grad f - z) (k > 0: the previous iteration's
//             multiplier step, grad f being the new image's), z = shrink(
//             grad f - lambda / rho, 1 / rho), W = rho (grad f - z) - lambda;
//             partials TV(f), |grad f - z|^2
//   k3_g      G = grad^T W + h; partial |G|^2   (k = 0 also |grad G|^2)
//   A G       p + plo, the FP64 ray sums of G split in two FP32 parts
//   k3_scalar (k = 0) the exact line search along -G; then log row k
//   k3_step   s = -alpha G, f += s in FP64; partials |f^k|^2, <s,s>
//             (DECT_NONNEG: s the step to max(f - alpha G, 0), in FP32)
//   k3_rupd   r -= alpha (p + plo) in FP64, so that r stays A f - beta m
//             without projecting f (DECT_NONNEG: r += A s, projecting s;
//             A G is then formed for the first step only); partial |r|^2
//   A^T r     h' = mu A^T r, y = h' - h + rho grad^T grad s, h = h';
//             partials <s,y>, <y,y>
//   k3_scalar alpha = <s,s>/<s,y> (BB1), <s,y>/<y,y> (BB2) or the adaptive
//             choice when <s,y> > 0, relative change
// DECT_COUPLED_TV: k3_tv_coupled takes the z-step of both energies at once,
// shrinking the 6-vector of their gradients (a fixed iteration count).
// With a tolerance the host reads both relative changes after every
// iteration and stops an energy at the first one below it (the stop rule of
// Sec. 3); the other energy runs on alone.
#include <cmath>
#include <memory>
#include <mutex>
#include <vector>

#include "volume.h"

namespace dect {
namespace {

enum { Q_TV, Q_PRES, Q_GG, Q_GRADG, Q_PP, Q_FF, Q_RR, Q_SS, Q_SY, Q_YY, Q_COUNT };

struct Dims {
    int nx, ny, nz;
    size_t N;
};

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
}

// Backward differences of f + flo: each part differenced in FP32 (exact for
// neighbouring values within a factor of two of each other) and the two
// differences added.
__device__ __forceinline__ void grad2_at(const Dims &d, const float *__restrict__ f,
                                         const float *__restrict__ flo, size_t i, int c, int r,
                                         int z, float &gx, float &gy, float &gz)
{
    const float fi = f[i], li = flo[i];
    const size_t P = (size_t)d.nx * d.ny;
    gx = c >= 1 ? (fi - f[i - 1]) + (li - flo[i - 1]) : 0.f;
    gy = r >= 1 ? (fi - f[i - d.nx]) + (li - flo[i - d.nx]) : 0.f;
    gz = z >= 1 ? (fi - f[i - P]) + (li - flo[i - P]) : 0.f;
}

__device__ __forceinline__ void grad_at(const Dims &d, const float *__restrict__ f, size_t i,
                                        int c, int r, int z, float &gx, float &gy, float &gz)
{
    const float fi = f[i];
    const size_t P = (size_t)d.nx * d.ny;
    gx = c >= 1 ? fi - f[i - 1] : 0.f;
    gy = r >= 1 ? fi - f[i - d.nx] : 0.f;
    gz = z >= 1 ? fi - f[i - P] : 0.f;
}

__device__ __forceinline__ void coords(const Dims &d, size_t i, int &c, int &r, int &z)
{
    c = (int)(i % d.nx);
    r = (int)(i / d.nx % d.ny);
    z = (int)(i / ((size_t)d.nx * d.ny));
}

constexpr int kMaxBlk = 2048;  // grid of the element-wise kernels (grid-stride loops)

// One energy's state at the z-step.
struct TvSet {
    const float *f, *flo;
    float *lam, *zz, *W;
    double *part;
};

// grad f at voxel i, the deferred multiplier step (k > 0) and v = grad f -
// lambda / rho of one energy.
__device__ __forceinline__ void tv_pre(const Dims &d, const TvSet &S, size_t i, int c, int r,
                                       int z, int first, float xi, float rho, float g[3],
                                       float l[3], float v[3])
{
    grad2_at(d, S.f, S.flo, i, c, r, z, g[0], g[1], g[2]);
    for (int a = 0; a < 3; ++a) {
        l[a] = S.lam[a * d.N + i];
        if (!first) l[a] -= xi * (g[a] - S.zz[a * d.N + i]);
        v[a] = g[a] - l[a] / rho;
    }
}

// z = sh v, W = rho (grad f - z) - lambda, lambda stored; returns
// |grad f - z|^2 at voxel i.
__device__ __forceinline__ double tv_post(const Dims &d, const TvSet &S, size_t i, float sh,
                                          float rho, const float g[3], const float l[3],
                                          const float v[3])
{
    double pres = 0.0;
    for (int a = 0; a < 3; ++a) {
        const float za = sh * v[a];
        S.lam[a * d.N + i] = l[a];
        S.zz[a * d.N + i] = za;
        S.W[a * d.N + i] = rho * (g[a] - za) - l[a];
        pres += (double)(g[a] - za) * (g[a] - za);
    }
    return pres;
}

__device__ __forceinline__ float shrink_factor(float mag, float rho)
{
    const float t = 1.f / rho;
    return mag > t ? (mag - t) / mag : 0.f;
}

__global__ __launch_bounds__(256) void k3_tv(Dims d, TvSet S, int first, float xi, float rho,
                                             size_t stride)
{
    double tv = 0.0, pres = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < d.N; i += (size_t)gridDim.x * 256) {
        int c, r, z;
        coords(d, i, c, r, z);
        float g[3], l[3], v[3];
        tv_pre(d, S, i, c, r, z, first, xi, rho, g, l, v);
        const float sh = shrink_factor(sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]), rho);
        pres += tv_post(d, S, i, sh, rho, g, l, v);
        tv += sqrt((double)g[0] * g[0] + (double)g[1] * g[1] + (double)g[2] * g[2]);
    }
    block_sum(tv, S.part + Q_TV * stride + blockIdx.x);
    block_sum(pres, S.part + Q_PRES * stride + blockIdx.x);
}

// The z-step with the TV coupled across the energies: one shrinkage of the
// 6-vector (v_high, v_low) at every voxel, its squared norm summed over the
// high energy's three components and then the low energy's.  The joint TV
// goes to the high energy's partials, zero to the low energy's.
__global__ __launch_bounds__(256) void k3_tv_coupled(Dims d, TvSet S0, TvSet S1, int first,
                                                     float xi, float rho, size_t stride)
{
    double tv = 0.0, pr0 = 0.0, pr1 = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < d.N; i += (size_t)gridDim.x * 256) {
        int c, r, z;
        coords(d, i, c, r, z);
        float g0[3], l0[3], v0[3], g1[3], l1[3], v1[3];
        tv_pre(d, S0, i, c, r, z, first, xi, rho, g0, l0, v0);
        tv_pre(d, S1, i, c, r, z, first, xi, rho, g1, l1, v1);
        const float sh = shrink_factor(sqrtf(v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2] +
                                             v1[0] * v1[0] + v1[1] * v1[1] + v1[2] * v1[2]),
                                       rho);
        pr0 += tv_post(d, S0, i, sh, rho, g0, l0, v0);
        pr1 += tv_post(d, S1, i, sh, rho, g1, l1, v1);
        tv += sqrt((double)g0[0] * g0[0] + (double)g0[1] * g0[1] + (double)g0[2] * g0[2] +
                   (double)g1[0] * g1[0] + (double)g1[1] * g1[1] + (double)g1[2] * g1[2]);
    }
    block_sum(tv, S0.part + Q_TV * stride + blockIdx.x);
    block_sum(pr0, S0.part + Q_PRES * stride + blockIdx.x);
    block_sum(pr1, S1.part + Q_PRES * stride + blockIdx.x);
    if (threadIdx.x == 0) S1.part[Q_TV * stride + blockIdx.x] = 0.0;
}

// TV(f) alone (the last log row); with a second energy (f1 != NULL) the
// joint TV into part0 and zero into part1.
__global__ __launch_bounds__(256) void k3_tvonly(Dims d, const float *__restrict__ f,
                                                 const float *__restrict__ flo,
                                                 const float *__restrict__ f1,
                                                 const float *__restrict__ flo1,
                                                 double *__restrict__ part,
                                                 double *__restrict__ part1, size_t stride)
{
    double tv = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < d.N; i += (size_t)gridDim.x * 256) {
        int c, r, z;
        coords(d, i, c, r, z);
        float g[3];
        grad2_at(d, f, flo, i, c, r, z, g[0], g[1], g[2]);
        double q = (double)g[0] * g[0] + (double)g[1] * g[1] + (double)g[2] * g[2];
        if (f1) {
            grad2_at(d, f1, flo1, i, c, r, z, g[0], g[1], g[2]);
            q += (double)g[0] * g[0] + (double)g[1] * g[1] + (double)g[2] * g[2];
        }
        tv += sqrt(q);
    }
    block_sum(tv, part + Q_TV * stride + blockIdx.x);
    if (f1 && threadIdx.x == 0) part1[Q_TV * stride + blockIdx.x] = 0.0;
}

// grad^T of a 3-component field at voxel i (exact adjoint of grad_at).
__device__ __forceinline__ float gradT_at(const Dims &d, const float *__restrict__ W, size_t i,
                                          int c, int r, int z)
{
    const size_t P = (size_t)d.nx * d.ny, N = d.N;
    float s = 0.f;
    if (c >= 1) s += W[i];
    if (c + 1 <= d.nx - 1) s -= W[i + 1];
    if (r >= 1) s += W[N + i];
    if (r + 1 <= d.ny - 1) s -= W[N + i + d.nx];
    if (z >= 1) s += W[2 * N + i];
    if (z + 1 <= d.nz - 1) s -= W[2 * N + i + P];
    return s;
}

__global__ __launch_bounds__(256) void k3_g(Dims d, const float *__restrict__ W,
                                            const float *__restrict__ h, float *__restrict__ G,
                                            double *__restrict__ part, size_t stride)
{
    double gg = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < d.N; i += (size_t)gridDim.x * 256) {
        int c, r, z;
        coords(d, i, c, r, z);
        const float g = gradT_at(d, W, i, c, r, z) + h[i];
        G[i] = g;
        gg += (double)g * g;
    }
    block_sum(gg, part + Q_GG * stride + blockIdx.x);
}

// |grad G|^2 (first step's exact line search).
__global__ __launch_bounds__(256) void k3_gradnorm(Dims d, const float *__restrict__ G,
                                                   double *__restrict__ part, size_t stride)
{
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < d.N; i += (size_t)gridDim.x * 256) {
        int c, r, z;
        coords(d, i, c, r, z);
        float g[3];
        grad_at(d, G, i, c, r, z, g[0], g[1], g[2]);
        s += (double)g[0] * g[0] + (double)g[1] * g[1] + (double)g[2] * g[2];
    }
    block_sum(s, part + Q_GRADG * stride + blockIdx.x);
}

// sum of squares of a length-n vector into quantity q.
__global__ __launch_bounds__(256) void k3_sumsq(const float *__restrict__ p, size_t n, int q,
                                                double *__restrict__ part, size_t stride)
{
    double ss = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        ss += (double)p[i] * p[i];
    block_sum(ss, part + q * stride + blockIdx.x);
}

struct Scal3 {
    double alpha, relchg, rr;
};

// s = -alpha G and (f + flo) += s in FP64, split again; partials |f^k|^2
// (the image before the step) and <s,s>, both in FP64.  nonneg: the step is
// projected onto f >= 0, s = max(f - alpha G, 0) - f rounded toward zero to
// FP32 (so that f + s >= 0), and f advances by exactly that s, so that the
// residual recurrence r += A s stays the residual of f.
__global__ __launch_bounds__(256) void k3_step(Dims d, const float *__restrict__ G,
                                               float *__restrict__ f, float *__restrict__ flo,
                                               float *__restrict__ s, const Scal3 *__restrict__ sc,
                                               int nonneg, double *__restrict__ part,
                                               size_t stride)
{
    const double alpha = sc->alpha;
    double ff = 0.0, ss = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < d.N; i += (size_t)gridDim.x * 256) {
        const double fo = (double)f[i] + (double)flo[i];
        double sd = -alpha * (double)G[i];
        float sf;
        if (nonneg) {
            const double t = fo + sd;
            sf = __double2float_rz((t > 0.0 ? t : 0.0) - fo);
            sd = (double)sf;
        } else {
            sf = (float)sd;
        }
        const double fn = fo + sd;
        const float hi = (float)fn;
        f[i] = hi;
        flo[i] = (float)(fn - (double)hi);
        s[i] = sf;
        ff += fo * fo;
        ss += sd * sd;
    }
    block_sum(ff, part + Q_FF * stride + blockIdx.x);
    block_sum(ss, part + Q_SS * stride + blockIdx.x);
}

// (r + rlo) += c (p + plo) in FP64, split again; partial |r|^2.  c = -alpha
// with p + plo = A G (plain step), or c = 1 with p + plo = A s (projected
// step).
__global__ __launch_bounds__(256) void k3_rupd(float *__restrict__ r, float *__restrict__ rlo,
                                               const float *__restrict__ p,
                                               const float *__restrict__ plo,
                                               const Scal3 *__restrict__ sc, int by_step,
                                               size_t M, double *__restrict__ part, size_t stride)
{
    const double coef = by_step ? 1.0 : -sc->alpha;
    double rr = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < M; i += (size_t)gridDim.x * 256) {
        const double v = ((double)r[i] + (double)rlo[i]) + coef * ((double)p[i] + (double)plo[i]);
        const float hi = (float)v;
        r[i] = hi;
        rlo[i] = (float)(v - (double)hi);
        rr += v * v;
    }
    block_sum(rr, part + Q_RR * stride + blockIdx.x);
}

// r + rlo = (p + plo) - beta m in FP64 (p == NULL: a zero image, A f = 0);
// partial |r|^2.
__global__ __launch_bounds__(256) void k3_rinit(const float *__restrict__ p,
                                                const float *__restrict__ plo,
                                                const float *__restrict__ m, double beta, size_t M,
                                                float *__restrict__ r, float *__restrict__ rlo,
                                                double *__restrict__ part, size_t stride)
{
    double rr = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < M; i += (size_t)gridDim.x * 256) {
        const double af = p ? (double)p[i] + (double)plo[i] : 0.0;
        const double v = af - beta * (double)m[i];
        const float hi = (float)v;
        r[i] = hi;
        rlo[i] = (float)(v - (double)hi);
        rr += v * v;
    }
    block_sum(rr, part + Q_RR * stride + blockIdx.x);
}

// f + flo = beta x0 (x0 == NULL: zero).
__global__ __launch_bounds__(256) void k3_start(const float *__restrict__ x0, double beta,
                                                size_t n, float *__restrict__ f,
                                                float *__restrict__ flo)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const double v = x0 ? beta * (double)x0[i] : 0.0;
        const float hi = (float)v;
        f[i] = hi;
        flo[i] = (float)(v - (double)hi);
    }
}

// h' = mu hb; y = h' - h + rho grad^T grad s; h = h'; partials <s,y> and
// <y,y>.  With s == NULL only h is formed (the start).
__global__ __launch_bounds__(256) void k3_y(Dims d, const float *__restrict__ hb,
                                            float *__restrict__ h, const float *__restrict__ s,
                                            float mu, float rho, double *__restrict__ part,
                                            size_t stride)
{
    double sy = 0.0, yy = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < d.N; i += (size_t)gridDim.x * 256) {
        const float hn = mu * hb[i];
        if (s) {
            int c, r, z;
            coords(d, i, c, r, z);
            // grad^T grad s at i: per axis, (s_i - s_prev) when i has a
            // predecessor minus (s_next - s_i) when it has a successor
            const size_t P = (size_t)d.nx * d.ny;
            const float si = s[i];
            float l = 0.f;
            if (c >= 1) l += si - s[i - 1];
            if (c + 1 <= d.nx - 1) l -= s[i + 1] - si;
            if (r >= 1) l += si - s[i - d.nx];
            if (r + 1 <= d.ny - 1) l -= s[i + d.nx] - si;
            if (z >= 1) l += si - s[i - P];
            if (z + 1 <= d.nz - 1) l -= s[i + P] - si;
            const float y = (hn - h[i]) + rho * l;
            sy += (double)si * y;
            yy += (double)y * y;
        }
        h[i] = hn;
    }
    if (s) {
        block_sum(sy, part + Q_SY * stride + blockIdx.x);
        block_sum(yy, part + Q_YY * stride + blockIdx.x);
    }
}

__device__ double reduce_q(const double *__restrict__ part, size_t stride, int q, int nb)
{
    __shared__ double red[256];
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) v += part[q * stride + b];
    __syncthreads();
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

// phase 0: first step's line search (alpha = |G|^2 / (mu |A G|^2 + rho |grad G|^2))
// phase 1: log row k (J, alpha, ...) before the f-step
// phase 2: the BB step (step_rule 0 BB1, 1 BB2, 2 adaptive) and the relative
//          change after the f-step
// phase 3: last log row
__global__ __launch_bounds__(256) void k3_scalar(Scal3 *sc, const double *__restrict__ part,
                                                 size_t stride, int nbN, int nbM, int phase,
                                                 double mu, double rho, int step_rule,
                                                 double *log_row)
{
    if (phase == 0) {
        const double gg = reduce_q(part, stride, Q_GG, nbN);
        const double pp = reduce_q(part, stride, Q_PP, nbM);
        const double gd = reduce_q(part, stride, Q_GRADG, nbN);
        if (threadIdx.x == 0) {
            const double den = mu * pp + rho * gd;
            sc->alpha = den > 0.0 ? gg / den : 0.0;
        }
    } else if (phase == 1 || phase == 3) {
        const double tv = reduce_q(part, stride, Q_TV, nbN);
        const double gg = phase == 1 ? reduce_q(part, stride, Q_GG, nbN) : 0.0;
        const double pr = phase == 1 ? reduce_q(part, stride, Q_PRES, nbN) : 0.0;
        if (threadIdx.x == 0 && log_row) {
            log_row[0] = tv + 0.5 * mu * sc->rr;
            log_row[1] = sc->alpha;
            log_row[2] = sqrt(pr);
            log_row[3] = sc->relchg;
            log_row[4] = sqrt(gg);
        }
    } else {
        const double rr = reduce_q(part, stride, Q_RR, nbM);
        const double ss = reduce_q(part, stride, Q_SS, nbN);
        const double sy = reduce_q(part, stride, Q_SY, nbN);
        const double yy = reduce_q(part, stride, Q_YY, nbN);
        const double ff = reduce_q(part, stride, Q_FF, nbN);
        if (threadIdx.x == 0) {
            sc->rr = rr;
            if (sy > 0.0) {  // BB1, BB2 or the adaptive choice; else keep alpha
                const double bb1 = ss / sy, bb2 = yy > 0.0 ? sy / yy : bb1;
                sc->alpha = step_rule == 1 ? bb2 : step_rule == 2 ? (bb2 / bb1 < 0.5 ? bb2 : bb1)
                                                                   : bb1;
            }
            const double fn = sqrt(ff);
            sc->relchg = fn > 0.0 ? sqrt(ss) / fn : (ss > 0.0 ? INFINITY : 0.0);
        }
    }
}

__global__ void k3_init(Scal3 *sc, const double *__restrict__ part, size_t stride, int nbM)
{
    const double rr = reduce_q(part, stride, Q_RR, nbM);
    if (threadIdx.x == 0) {
        sc->alpha = 0.0;
        sc->relchg = 0.0;
        sc->rr = rr;
    }
}

__global__ __launch_bounds__(256) void k3_zero(float *__restrict__ p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        p[i] = 0.f;
}

// x = (f + flo) / beta
__global__ __launch_bounds__(256) void k3_out(const float *__restrict__ f,
                                              const float *__restrict__ flo, double beta, size_t n,
                                              float *__restrict__ x)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        x[i] = (float)(((double)f[i] + (double)flo[i]) / beta);
}

unsigned nblk(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

struct Adm3Work {
    DevBuf buf[2][13], bpart[2], bsc, blog;
};

static std::mutex g_adm3_mu;
static std::vector<std::pair<int, std::unique_ptr<Adm3Work>>> g_adm3;

static Adm3Work *adm3_work()
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (auto &p : g_adm3)
        if (p.first == dev) return p.second.get();
    g_adm3.emplace_back(dev, std::make_unique<Adm3Work>());
    return g_adm3.back().second.get();
}

void release_adm3_work()
{
    std::lock_guard<std::mutex> lk(g_adm3_mu);
    g_adm3.clear();
}

dect_status adm_tv3(const dect_cone_geometry *g, const float *m_high, const float *m_low,
                    const dect_adm_params *p, float *x_high, float *x_low, dect_report *rep,
                    hipStream_t s)
{
    if (!g || !p || !m_high || !m_low || !x_high || !x_low)
        return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv3: null argument");
    if (p->flags & ~(DECT_WARM_START | DECT_NONNEG | DECT_COUPLED_TV | DECT_STEP_BB2 | DECT_STEP_ABB))
        return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv3: unknown flag");
    if ((p->flags & DECT_COUPLED_TV) && (p->flags & (DECT_STEP_BB2 | DECT_STEP_ABB)))
        return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv3: coupled TV takes the BB1 step only");
    if ((p->flags & DECT_COUPLED_TV) && p->tol != 0.0)
        return fail(DECT_ERR_INVALID_ARG,
                    "dect_adm_tv3: coupled TV runs a fixed iteration count (tol 0)");
    if ((p->flags & DECT_STEP_BB2) && (p->flags & DECT_STEP_ABB))
        return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv3: DECT_STEP_BB2 and DECT_STEP_ABB exclude each other");
    if (!(p->tol >= 0.0) || !std::isfinite(p->tol))
        return fail(DECT_ERR_INVALID_ARG, "tol must be finite and >= 0");
    if (p->max_iter < 0 || p->max_iter > 1000000)
        return fail(DECT_ERR_INVALID_ARG, "max_iter out of range");
    if (!(p->mu > 0.0) || !(p->rho > 0.0) || !(p->xi >= 0.0) || !(p->beta_high > 0.0) ||
        !(p->beta_low > 0.0))
        return fail(DECT_ERR_INVALID_ARG, "mu, rho, beta must be positive and xi >= 0");
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || g->n_views <= 0 || g->n_rows <= 0 ||
        g->n_bins <= 0)
        return fail(DECT_ERR_INVALID_ARG, "cone geometry sizes must be positive");
    const Dims d{g->nx, g->ny, g->nz, (size_t)g->nx * g->ny * g->nz};
    const size_t M = (size_t)g->n_views * g->n_rows * g->n_bins;
    const int K = p->max_iter;
    const bool warm = (p->flags & DECT_WARM_START) != 0;
    const int nonneg = (p->flags & DECT_NONNEG) ? 1 : 0;
    const bool coupled = (p->flags & DECT_COUPLED_TV) != 0;
    const int step_rule = (p->flags & DECT_STEP_BB2) ? 1 : (p->flags & DECT_STEP_ABB) ? 2 : 0;
    const int nbN = (int)std::min<size_t>(kMaxBlk, nblk(d.N));
    const int nbM = (int)std::min<size_t>(kMaxBlk, nblk(M));
    const size_t stride = (size_t)std::max(nbN, nbM);

    // library-owned work buffers (one set per device, grown to the problem
    // and kept between calls), one set per energy; the two energies advance
    // together so that every projector call walks both volumes at once
    std::lock_guard<std::mutex> lk(g_adm3_mu);
    Adm3Work *w3 = adm3_work();
    auto &buf = w3->buf;
    auto &bpart = w3->bpart;
    auto &bsc = w3->bsc;
    auto &blog = w3->blog;
    enum { B_F, B_FLO, B_S, B_G, B_H, B_HB, B_LAM, B_Z, B_W, B_R, B_RLO, B_P, B_PLO, B_COUNT };
    const size_t vsz[B_COUNT] = {d.N, d.N, d.N, d.N, d.N, d.N, 3 * d.N, 3 * d.N, 3 * d.N,
                                 M,   M,   M,   M};
    dect_status st;
    for (int e = 0; e < 2; ++e) {
        for (int a = 0; a < B_COUNT; ++a)
            if ((st = buf[e][a].ensure(vsz[a] * 4))) return st;
        if ((st = bpart[e].ensure(Q_COUNT * stride * 8))) return st;
    }
    if ((st = bsc.ensure(2 * sizeof(Scal3))) || (st = blog.ensure((size_t)(K + 1) * 5 * 8 * 2)))
        return st;
    float *V[2][B_COUNT];
    double *part[2];
    for (int e = 0; e < 2; ++e) {
        for (int a = 0; a < B_COUNT; ++a) V[e][a] = (float *)buf[e][a].ptr;
        part[e] = (double *)bpart[e].ptr;
    }
    double *dlog = (double *)blog.ptr;
    Scal3 *sc = (Scal3 *)bsc.ptr;
    const float mu = (float)p->mu, rho = (float)p->rho, xi = (float)p->xi;
    const float *ms[2] = {m_high, m_low};
    float *xs[2] = {x_high, x_low};
    const double betas[2] = {p->beta_high, p->beta_low};
    const float *cf[2] = {V[0][B_F], V[1][B_F]}, *cG[2] = {V[0][B_G], V[1][B_G]};
    const float *cr[2] = {V[0][B_R], V[1][B_R]};
    float *pp[2] = {V[0][B_P], V[1][B_P]}, *plo[2] = {V[0][B_PLO], V[1][B_PLO]};
    float *hb[2] = {V[0][B_HB], V[1][B_HB]};

    // set-up: f + flo = beta x0 (or 0), lambda = z = 0, r = A f - beta m,
    // h = mu A^T r
    for (int e = 0; e < 2; ++e) {
        hipLaunchKernelGGL(k3_start, dim3(nbN), dim3(256), 0, s,
                           warm ? (const float *)xs[e] : (const float *)nullptr, betas[e], d.N,
                           V[e][B_F], V[e][B_FLO]);
        hipLaunchKernelGGL(k3_zero, dim3(nbN), dim3(256), 0, s, V[e][B_LAM], 3 * d.N);
        hipLaunchKernelGGL(k3_zero, dim3(nbN), dim3(256), 0, s, V[e][B_Z], 3 * d.N);
    }
    DECT_HIP(hipGetLastError());
    // A f of the high parts (flo, below half an ulp of f, is not projected)
    if (warm && (st = cone_project2_lo(g, cf, pp, plo, s))) return st;
    for (int e = 0; e < 2; ++e)
        hipLaunchKernelGGL(k3_rinit, dim3(nbM), dim3(256), 0, s,
                           warm ? (const float *)pp[e] : (const float *)nullptr,
                           (const float *)plo[e], ms[e], betas[e], M, V[e][B_R], V[e][B_RLO],
                           part[e], stride);
    if ((st = cone_backproject2(g, cr, hb, s))) return st;
    for (int e = 0; e < 2; ++e) {
        hipLaunchKernelGGL(k3_y, dim3(nbN), dim3(256), 0, s, d, (const float *)hb[e], V[e][B_H],
                           (const float *)nullptr, mu, rho, part[e], stride);
        hipLaunchKernelGGL(k3_init, dim3(1), dim3(256), 0, s, sc + e, part[e], stride, nbM);
    }
    DECT_HIP(hipGetLastError());

    auto tvset = [&](int e) {
        return TvSet{V[e][B_F], V[e][B_FLO], V[e][B_LAM], V[e][B_Z], V[e][B_W], part[e]};
    };

    // each energy runs until max_iter or, with a tolerance, until its
    // relative change first falls below it; stop[e] = its iteration count
    int stop[2] = {K, K};
    bool done[2] = {false, false};
    for (int k = 0; k < K && !(done[0] && done[1]); ++k) {
        DECT_TRACE("adm3 iteration");
        // coupled: one joint z-step (tol is 0, so neither energy stops early)
        if (coupled)
            hipLaunchKernelGGL(k3_tv_coupled, dim3(nbN), dim3(256), 0, s, d, tvset(0), tvset(1),
                               k == 0 ? 1 : 0, xi, rho, stride);
        for (int e = 0; e < 2; ++e) {
            if (done[e]) continue;
            if (!coupled)
                hipLaunchKernelGGL(k3_tv, dim3(nbN), dim3(256), 0, s, d, tvset(e), k == 0 ? 1 : 0,
                                   xi, rho, stride);
            hipLaunchKernelGGL(k3_g, dim3(nbN), dim3(256), 0, s, d, (const float *)V[e][B_W],
                               (const float *)V[e][B_H], V[e][B_G], part[e], stride);
        }
        // p + plo = A G (a stopped energy's G is stale and its p unused); the
        // projected iteration needs it for the first (Cauchy) step only
        if ((!nonneg || k == 0) && (st = cone_project2_lo(g, cG, pp, plo, s))) return st;
        for (int e = 0; e < 2; ++e) {
            if (done[e]) continue;
            if (k == 0) {
                hipLaunchKernelGGL(k3_sumsq, dim3(nbM), dim3(256), 0, s, (const float *)pp[e], M,
                                   (int)Q_PP, part[e], stride);
                hipLaunchKernelGGL(k3_gradnorm, dim3(nbN), dim3(256), 0, s, d,
                                   (const float *)V[e][B_G], part[e], stride);
                hipLaunchKernelGGL(k3_scalar, dim3(1), dim3(256), 0, s, sc + e, part[e], stride,
                                   nbN, nbM, 0, p->mu, p->rho, step_rule, (double *)nullptr);
            }
            hipLaunchKernelGGL(k3_scalar, dim3(1), dim3(256), 0, s, sc + e, part[e], stride, nbN,
                               nbM, 1, p->mu, p->rho, step_rule, dlog + ((size_t)e * (K + 1) + k) * 5);
            hipLaunchKernelGGL(k3_step, dim3(nbN), dim3(256), 0, s, d, (const float *)V[e][B_G],
                               V[e][B_F], V[e][B_FLO], V[e][B_S], sc + e, nonneg, part[e], stride);
            if (!nonneg)
                hipLaunchKernelGGL(k3_rupd, dim3(nbM), dim3(256), 0, s, V[e][B_R], V[e][B_RLO],
                                   (const float *)pp[e], (const float *)plo[e], sc + e, 0, M,
                                   part[e], stride);
        }
        if (nonneg) {  // r += A s of the projected step
            const float *cs[2] = {V[0][B_S], V[1][B_S]};
            if ((st = cone_project2_lo(g, cs, pp, plo, s))) return st;
            for (int e = 0; e < 2; ++e)
                if (!done[e])
                    hipLaunchKernelGGL(k3_rupd, dim3(nbM), dim3(256), 0, s, V[e][B_R],
                                       V[e][B_RLO], (const float *)pp[e], (const float *)plo[e],
                                       sc + e, 1, M, part[e], stride);
        }
        if ((st = cone_backproject2(g, cr, hb, s))) return st;
        for (int e = 0; e < 2; ++e) {
            if (done[e]) continue;
            hipLaunchKernelGGL(k3_y, dim3(nbN), dim3(256), 0, s, d, (const float *)hb[e],
                               V[e][B_H], (const float *)V[e][B_S], mu, rho, part[e], stride);
            hipLaunchKernelGGL(k3_scalar, dim3(1), dim3(256), 0, s, sc + e, part[e], stride, nbN,
                               nbM, 2, p->mu, p->rho, step_rule, (double *)nullptr);
        }
        DECT_HIP(hipGetLastError());
        if (p->tol > 0.0) {
            Scal3 hs[2];
            DECT_HIP(hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, s));
            DECT_HIP(hipStreamSynchronize(s));
            for (int e = 0; e < 2; ++e)
                if (!done[e] && hs[e].relchg < p->tol) {
                    done[e] = true;
                    stop[e] = k + 1;
                }
        }
    }
    if (coupled)
        hipLaunchKernelGGL(k3_tvonly, dim3(nbN), dim3(256), 0, s, d, (const float *)V[0][B_F],
                           (const float *)V[0][B_FLO], (const float *)V[1][B_F],
                           (const float *)V[1][B_FLO], part[0], part[1], stride);
    for (int e = 0; e < 2; ++e) {
        if (!coupled)
            hipLaunchKernelGGL(k3_tvonly, dim3(nbN), dim3(256), 0, s, d, (const float *)V[e][B_F],
                               (const float *)V[e][B_FLO], (const float *)nullptr,
                               (const float *)nullptr, part[e], (double *)nullptr, stride);
        hipLaunchKernelGGL(k3_scalar, dim3(1), dim3(256), 0, s, sc + e, part[e], stride, nbN, nbM,
                           3, p->mu, p->rho, step_rule, dlog + ((size_t)e * (K + 1) + stop[e]) * 5);
        hipLaunchKernelGGL(k3_out, dim3(nbN), dim3(256), 0, s, (const float *)V[e][B_F],
                           (const float *)V[e][B_FLO], betas[e], d.N, xs[e]);
    }
    DECT_HIP(hipGetLastError());
    std::vector<double> hlog((size_t)(K + 1) * 5 * 2);
    DECT_HIP(hipMemcpyAsync(hlog.data(), dlog, hlog.size() * 8, hipMemcpyDeviceToHost, s));
    DECT_HIP(hipStreamSynchronize(s));
    auto row = [&](int e, int k) { return &hlog[((size_t)e * (K + 1) + k) * 5]; };
    // J and the step must stay finite (the relative change after the first
    // step of a zero start is infinite by definition)
    bool finite = true;
    for (int e = 0; e < 2; ++e)
        for (int k = 0; k <= stop[e]; ++k)
            finite = finite && std::isfinite(row(e, k)[0]) && std::isfinite(row(e, k)[1]);
    for (int k = 0; k <= K; ++k)
        for (int e = 0; e < 2; ++e) {  // rows after an energy's stop hold zeros
            const bool in = k <= stop[e];
            if (p->log) {
                p->log[k * 4 + e] = in ? row(e, k)[0] : 0.0;
                p->log[k * 4 + 2 + e] = in ? row(e, k)[1] : 0.0;
            }
            if (p->log_aux) {
                p->log_aux[k * 4 + e] = in ? row(e, k)[2] : 0.0;
                p->log_aux[k * 4 + 2 + e] = in ? row(e, k)[4] : 0.0;
            }
        }
    if (rep) {
        rep->iters = std::max(stop[0], stop[1]);
        rep->objective = row(0, stop[0])[0] + row(1, stop[1])[0];
        rep->rel_change = std::max(row(0, stop[0])[3], row(1, stop[1])[3]);
        rep->pcg_residual = 0.0;
        rep->status = finite ? DECT_OK : DECT_ERR_NONFINITE;
    }
    if (!finite) return fail(DECT_ERR_NONFINITE, "non-finite objective or step");
    return DECT_OK;
}

}  // namespace dect
