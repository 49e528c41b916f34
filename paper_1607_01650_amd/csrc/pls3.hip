// PLS decomposition of volumes (Eqs. 11-15 with R of Eq. 14 over the six
// face neighbours): D^{-1} per voxel (Eq. 12), the 3-D Prewitt edge map of
// x_low (per axis, the 3 x 3 face sum at +1 minus the one at -1, borders
// replicated; FP32 in a fixed order, since the map is a threshold
// decision), the pair weights, then Jacobi-PCG on (I + gamma L) u = D^{-1} x
// per material (FP32 vectors, FP64 dot products, scalars on the device), or
// in the attenuation-space mode the coupled system of |x - D u|^2 + gamma
// R(u) (FP64).
//
// Element-wise kernels use a grid of at most kMaxBlocks blocks with
// grid-stride loops, so per-block partial sums stay few and one block
// reduces them in a fixed order.
#include <algorithm>
#include <cmath>
#include <memory>
#include <mutex>
#include <vector>

#include "volume.h"

namespace dect {
namespace {

constexpr int kMaxBlocks = 2048;

struct Vol {
    int nx, ny, nz;
    size_t N, P;
};

__device__ __forceinline__ double block_sum3(double v)
{
    __shared__ double red[256];
    __syncthreads();
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

__device__ __forceinline__ float block_max3(float v)
{
    __shared__ float red[256];
    __syncthreads();
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    return red[0];
}

__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v > n - 1 ? n - 1 : v); }

// b1, b2 = D^{-1} (x_high, x_low) per voxel (Eq. 12), formed in FP64.
__global__ __launch_bounds__(256) void kp3_dinv(Vol v, const float *__restrict__ xh,
                                                const float *__restrict__ xl, double e1h, double e2h,
                                                double e1l, double e2l, float *__restrict__ b1,
                                                float *__restrict__ b2)
{
    const double det = e1h * e2l - e2h * e1l;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < v.N; i += (size_t)gridDim.x * 256) {
        const double h = xh[i], l = xl[i];
        b1[i] = (float)((e2l * h - e2h * l) / det);
        b2[i] = (float)((e1h * l - e1l * h) / det);
    }
}

// m2 = |3-D Prewitt|^2 of x (FP32, the fixed order above); per-block max.
__global__ __launch_bounds__(256) void kp3_m2(Vol v, const float *__restrict__ x,
                                              float *__restrict__ m2, float *__restrict__ bmax)
{
    float mx = 0.f;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < v.N; i += (size_t)gridDim.x * 256) {
        const int c = (int)(i % v.nx), r = (int)(i / v.nx % v.ny), z = (int)(i / v.P);
        auto X = [&](int zz, int rr, int cc) {
            return x[(size_t)clampi(zz, v.nz) * v.P + (size_t)clampi(rr, v.ny) * v.nx +
                     clampi(cc, v.nx)];
        };
        float xp = 0.f, xm = 0.f, yp = 0.f, ym = 0.f, zp = 0.f, zm = 0.f;
        bool first = true;
        for (int a = -1; a <= 1; ++a)
            for (int b = -1; b <= 1; ++b) {
                const float vxp = X(z + a, r + b, c + 1), vxm = X(z + a, r + b, c - 1);
                const float vyp = X(z + a, r + 1, c + b), vym = X(z + a, r - 1, c + b);
                const float vzp = X(z + 1, r + a, c + b), vzm = X(z - 1, r + a, c + b);
                if (first) {
                    xp = vxp; xm = vxm; yp = vyp; ym = vym; zp = vzp; zm = vzm;
                    first = false;
                } else {
                    xp += vxp; xm += vxm; yp += vyp; ym += vym; zp += vzp; zm += vzm;
                }
            }
        const float gx = xp - xm, gy = yp - ym, gz = zp - zm;
        const float val = fmaf(gx, gx, fmaf(gy, gy, gz * gz));
        m2[i] = val;
        mx = fmaxf(mx, val);
    }
    const float bm = block_max3(mx);
    if (threadIdx.x == 0) bmax[blockIdx.x] = bm;
}

__global__ __launch_bounds__(256) void kp3_thr(const float *__restrict__ bmax, int nb, float tau2,
                                               float *__restrict__ thr)
{
    float mx = 0.f;
    for (int b = threadIdx.x; b < nb; b += 256) mx = fmaxf(mx, bmax[b]);
    const float m = block_max3(mx);
    if (threadIdx.x == 0) *thr = tau2 * m;
}

// pair weights: eps where either voxel is an edge, 1 otherwise, 0 beyond.
__global__ __launch_bounds__(256) void kp3_w(Vol v, const float *__restrict__ m2,
                                             const float *__restrict__ thr, float eps,
                                             float *__restrict__ ex, float *__restrict__ ey,
                                             float *__restrict__ ez)
{
    const float t = *thr;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < v.N; i += (size_t)gridDim.x * 256) {
        const int c = (int)(i % v.nx), r = (int)(i / v.nx % v.ny), z = (int)(i / v.P);
        const bool e = m2[i] > t;
        ex[i] = c + 1 < v.nx ? ((e || m2[i + 1] > t) ? eps : 1.f) : 0.f;
        ey[i] = r + 1 < v.ny ? ((e || m2[i + v.nx] > t) ? eps : 1.f) : 0.f;
        ez[i] = z + 1 < v.nz ? ((e || m2[i + v.P] > t) ? eps : 1.f) : 0.f;
    }
}

struct PW {
    const float *ex, *ey, *ez;
};

// (L u)_i over the six face neighbours and the weight sum d_i.
__device__ __forceinline__ float lap(const Vol &v, const PW &w, const float *__restrict__ u,
                                     size_t i, float &dsum)
{
    const int c = (int)(i % v.nx), r = (int)(i / v.nx % v.ny), z = (int)(i / v.P);
    const float ui = u[i];
    float s = 0.f, d = 0.f;
    if (c + 1 < v.nx) { s += w.ex[i] * (ui - u[i + 1]); d += w.ex[i]; }
    if (c >= 1) { s += w.ex[i - 1] * (ui - u[i - 1]); d += w.ex[i - 1]; }
    if (r + 1 < v.ny) { s += w.ey[i] * (ui - u[i + v.nx]); d += w.ey[i]; }
    if (r >= 1) { s += w.ey[i - v.nx] * (ui - u[i - v.nx]); d += w.ey[i - v.nx]; }
    if (z + 1 < v.nz) { s += w.ez[i] * (ui - u[i + v.P]); d += w.ez[i]; }
    if (z >= 1) { s += w.ez[i - v.P] * (ui - u[i - v.P]); d += w.ez[i - v.P]; }
    dsum = d;
    return s;
}

struct PState {
    double rz, a, beta, bn, rn, tol;
    int it, done;
};

enum { R_BB, R_RR, R_RZ, R_PQ, R_COUNT };

// u = b; res = b - (u + gamma L u); dinv; z = dinv res; p = z; partials.
__global__ __launch_bounds__(256) void kp3_setup(Vol v, PW w, float gamma, const float *__restrict__ b,
                                                 float *__restrict__ u, float *__restrict__ res,
                                                 float *__restrict__ dinv, float *__restrict__ p,
                                                 double *__restrict__ part)
{
    double bb = 0.0, rr = 0.0, rz = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < v.N; i += (size_t)gridDim.x * 256) {
        float d;
        const float lu = lap(v, w, b, i, d);
        const float bi = b[i];
        const float ri = bi - (bi + gamma * lu);
        const float di = 1.f / (1.f + gamma * d);
        u[i] = bi;
        res[i] = ri;
        dinv[i] = di;
        p[i] = di * ri;
        bb += (double)bi * bi;
        rr += (double)ri * ri;
        rz += (double)ri * (di * ri);
    }
    const double s0 = block_sum3(bb), s1 = block_sum3(rr), s2 = block_sum3(rz);
    if (threadIdx.x == 0) {
        part[R_BB * kMaxBlocks + blockIdx.x] = s0;
        part[R_RR * kMaxBlocks + blockIdx.x] = s1;
        part[R_RZ * kMaxBlocks + blockIdx.x] = s2;
    }
}

__global__ __launch_bounds__(256) void kp3_apply(Vol v, PW w, float gamma,
                                                 const float *__restrict__ p, float *__restrict__ q,
                                                 const PState *__restrict__ ps,
                                                 double *__restrict__ part)
{
    if (ps->done) return;
    double pq = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < v.N; i += (size_t)gridDim.x * 256) {
        float d;
        const float qi = p[i] + gamma * lap(v, w, p, i, d);
        q[i] = qi;
        pq += (double)p[i] * qi;
    }
    const double s = block_sum3(pq);
    if (threadIdx.x == 0) part[R_PQ * kMaxBlocks + blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void kp3_update(Vol v, const float *__restrict__ p,
                                                  const float *__restrict__ q,
                                                  const float *__restrict__ dinv,
                                                  float *__restrict__ u, float *__restrict__ res,
                                                  float *__restrict__ zv,
                                                  const PState *__restrict__ ps,
                                                  double *__restrict__ part)
{
    if (ps->done) return;
    const float a = (float)ps->a;
    double rr = 0.0, rz = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < v.N; i += (size_t)gridDim.x * 256) {
        u[i] += a * p[i];
        const float ri = res[i] - a * q[i];
        res[i] = ri;
        const float zi = dinv[i] * ri;
        zv[i] = zi;
        rr += (double)ri * ri;
        rz += (double)ri * zi;
    }
    const double s1 = block_sum3(rr), s2 = block_sum3(rz);
    if (threadIdx.x == 0) {
        part[R_RR * kMaxBlocks + blockIdx.x] = s1;
        part[R_RZ * kMaxBlocks + blockIdx.x] = s2;
    }
}

__global__ __launch_bounds__(256) void kp3_dir(Vol v, const float *__restrict__ zv,
                                               float *__restrict__ p, const PState *__restrict__ ps)
{
    if (ps->done) return;
    const float beta = (float)ps->beta;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < v.N; i += (size_t)gridDim.x * 256)
        p[i] = zv[i] + beta * p[i];
}

__device__ double reduce_part(const double *__restrict__ part, int q, int nb)
{
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[q * kMaxBlocks + b];
    return block_sum3(s);
}

// phase 0: start (bn, rn, rz; done when rn <= tol bn); 1: step a = rz / pq
// (done when pq <= 0); 2: after the update (it, rn, beta; done when
// rn <= tol bn or it reaches max_iter).
__global__ __launch_bounds__(256) void kp3_scalar(PState *ps, const double *__restrict__ part, int nb,
                                                  int phase, double tol, int max_iter)
{
    const int done = ps->done;
    if (phase == 0) {
        const double bb = reduce_part(part, R_BB, nb), rr = reduce_part(part, R_RR, nb),
                     rz = reduce_part(part, R_RZ, nb);
        if (threadIdx.x == 0) {
            double bn = sqrt(bb), rn = sqrt(rr);
            if (bn == 0.0) {  // b = 0: u = b = 0 already
                bn = 1.0;
                rn = 0.0;
            }
            ps->bn = bn;
            ps->rn = rn;
            ps->rz = rz;
            ps->tol = tol;
            ps->it = 0;
            ps->done = (rn <= tol * bn || max_iter <= 0) ? 1 : 0;
        }
    } else if (phase == 1) {
        if (done) return;
        const double pq = reduce_part(part, R_PQ, nb);
        if (threadIdx.x == 0) {
            if (pq <= 0.0) ps->done = 1;
            else ps->a = ps->rz / pq;
        }
    } else {
        if (done) return;
        const double rr = reduce_part(part, R_RR, nb), rz2 = reduce_part(part, R_RZ, nb);
        if (threadIdx.x == 0) {
            ps->it += 1;
            ps->rn = sqrt(rr);
            ps->beta = rz2 / ps->rz;
            ps->rz = rz2;
            if (ps->rn <= ps->tol * ps->bn || ps->it >= max_iter) ps->done = 1;
        }
    }
}

// ------------------------------------------- attenuation-space system ---
// (D^T D (x) I + gamma I (x) L) u = D^T x over both materials at once
// (|x - D u|^2 + gamma R(u)), Jacobi-preconditioned with the 2 x 2 block
// D^T D + gamma diag(L) per voxel, from u = D^{-1} x.  D^T D has condition
// number about 740 for water and bone, which FP32 CG cannot resolve, so the
// vectors and the arithmetic are FP64 ([2][N]: material-major).
struct AttK {
    double e1h, e2h, e1l, e2l, g11, g12, g22, det;
};

// D^{-1} x at voxel j (Eq. 12) in FP64.
__device__ __forceinline__ void att_dinv(const AttK &k, const float *__restrict__ xh,
                                         const float *__restrict__ xl, size_t j, double &a,
                                         double &b)
{
    const double h = xh[j], l = xl[j];
    a = (k.e2l * h - k.e2h * l) / k.det;
    b = (k.e1h * l - k.e1l * h) / k.det;
}

// (L u)_i of both materials of a [2][N] FP64 vector over the six face
// neighbours, and the weight sum d_i.
__device__ __forceinline__ void lap2(const Vol &v, const PW &w, const double *__restrict__ u,
                                     size_t i, double (&out)[2], double &dsum)
{
    const int c = (int)(i % v.nx), r = (int)(i / v.nx % v.ny), z = (int)(i / v.P);
    const size_t N = v.N;
    double s0 = 0.0, s1 = 0.0, d = 0.0;
    auto add = [&](double wt, size_t k) {
        s0 += wt * (u[i] - u[k]);
        s1 += wt * (u[N + i] - u[N + k]);
        d += wt;
    };
    if (c + 1 < v.nx) add(w.ex[i], i + 1);
    if (c >= 1) add(w.ex[i - 1], i - 1);
    if (r + 1 < v.ny) add(w.ey[i], i + v.nx);
    if (r >= 1) add(w.ey[i - v.nx], i - v.nx);
    if (z + 1 < v.nz) add(w.ez[i], i + v.P);
    if (z >= 1) add(w.ez[i - v.P], i - v.P);
    out[0] = s0;
    out[1] = s1;
    dsum = d;
}

__device__ __forceinline__ void att_prec(const AttK &k, double gamma, double d,
                                         const double (&rs)[2], double (&z)[2])
{
    const double a11 = k.g11 + gamma * d, a22 = k.g22 + gamma * d;
    const double dt = a11 * a22 - k.g12 * k.g12;
    z[0] = (a22 * rs[0] - k.g12 * rs[1]) / dt;
    z[1] = (a11 * rs[1] - k.g12 * rs[0]) / dt;
}

// u = D^{-1} x (first pass: the stencil of the second reads neighbours' u).
__global__ __launch_bounds__(256) void kp3a_init(Vol v, AttK k, const float *__restrict__ xh,
                                                 const float *__restrict__ xl,
                                                 double *__restrict__ u)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < v.N; i += (size_t)gridDim.x * 256) {
        double a, b;
        att_dinv(k, xh, xl, i, a, b);
        u[i] = a;
        u[v.N + i] = b;
    }
}

// res = D^T x - (D^T D u + gamma L u), z = P^{-1} res, p = z; partials
// |D^T x|^2, |res|^2, <res, z>.
__global__ __launch_bounds__(256) void kp3a_setup(Vol v, PW w, double gamma, AttK k,
                                                  const float *__restrict__ xh,
                                                  const float *__restrict__ xl,
                                                  const double *__restrict__ u,
                                                  double *__restrict__ res, double *__restrict__ zv,
                                                  double *__restrict__ p,
                                                  double *__restrict__ part)
{
    double bb = 0.0, rr = 0.0, rz = 0.0;
    const size_t N = v.N;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (size_t)gridDim.x * 256) {
        double lu[2], d;
        lap2(v, w, u, i, lu, d);
        const double a = u[i], b = u[N + i];
        const double h = xh[i], l = xl[i];
        const double c0 = k.e1h * h + k.e1l * l, c1 = k.e2h * h + k.e2l * l;
        const double rs[2] = {c0 - (k.g11 * a + k.g12 * b + gamma * lu[0]),
                              c1 - (k.g12 * a + k.g22 * b + gamma * lu[1])};
        double z[2];
        att_prec(k, gamma, d, rs, z);
        res[i] = rs[0];
        res[N + i] = rs[1];
        zv[i] = z[0];
        zv[N + i] = z[1];
        p[i] = z[0];
        p[N + i] = z[1];
        bb += c0 * c0 + c1 * c1;
        rr += rs[0] * rs[0] + rs[1] * rs[1];
        rz += rs[0] * z[0] + rs[1] * z[1];
    }
    const double s0 = block_sum3(bb), s1 = block_sum3(rr), s2 = block_sum3(rz);
    if (threadIdx.x == 0) {
        part[R_BB * kMaxBlocks + blockIdx.x] = s0;
        part[R_RR * kMaxBlocks + blockIdx.x] = s1;
        part[R_RZ * kMaxBlocks + blockIdx.x] = s2;
    }
}

// q = D^T D p + gamma L p; partial <p, q>.
__global__ __launch_bounds__(256) void kp3a_apply(Vol v, PW w, double gamma, AttK k,
                                                  const double *__restrict__ p,
                                                  double *__restrict__ q,
                                                  const PState *__restrict__ ps,
                                                  double *__restrict__ part)
{
    if (ps->done) return;
    double pq = 0.0;
    const size_t N = v.N;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (size_t)gridDim.x * 256) {
        double lp[2], d;
        lap2(v, w, p, i, lp, d);
        const double a = p[i], b = p[N + i];
        const double q0 = k.g11 * a + k.g12 * b + gamma * lp[0];
        const double q1 = k.g12 * a + k.g22 * b + gamma * lp[1];
        q[i] = q0;
        q[N + i] = q1;
        pq += a * q0 + b * q1;
    }
    const double s = block_sum3(pq);
    if (threadIdx.x == 0) part[R_PQ * kMaxBlocks + blockIdx.x] = s;
}

// u += a p, res -= a q, z = P^{-1} res; partials |res|^2, <res, z>.
__global__ __launch_bounds__(256) void kp3a_update(Vol v, PW w, double gamma, AttK k,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ q,
                                                   double *__restrict__ u,
                                                   double *__restrict__ res,
                                                   double *__restrict__ zv,
                                                   const PState *__restrict__ ps,
                                                   double *__restrict__ part)
{
    if (ps->done) return;
    const double a = ps->a;
    const size_t N = v.N;
    double rr = 0.0, rz = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (size_t)gridDim.x * 256) {
        const int c = (int)(i % v.nx), r = (int)(i / v.nx % v.ny), zz = (int)(i / v.P);
        double d = 0.0;
        if (c + 1 < v.nx) d += w.ex[i];
        if (c >= 1) d += w.ex[i - 1];
        if (r + 1 < v.ny) d += w.ey[i];
        if (r >= 1) d += w.ey[i - v.nx];
        if (zz + 1 < v.nz) d += w.ez[i];
        if (zz >= 1) d += w.ez[i - v.P];
        u[i] += a * p[i];
        u[N + i] += a * p[N + i];
        const double rs[2] = {res[i] - a * q[i], res[N + i] - a * q[N + i]};
        double z[2];
        att_prec(k, gamma, d, rs, z);
        res[i] = rs[0];
        res[N + i] = rs[1];
        zv[i] = z[0];
        zv[N + i] = z[1];
        rr += rs[0] * rs[0] + rs[1] * rs[1];
        rz += rs[0] * z[0] + rs[1] * z[1];
    }
    const double s1 = block_sum3(rr), s2 = block_sum3(rz);
    if (threadIdx.x == 0) {
        part[R_RR * kMaxBlocks + blockIdx.x] = s1;
        part[R_RZ * kMaxBlocks + blockIdx.x] = s2;
    }
}

// p = z + beta p over both materials.
__global__ __launch_bounds__(256) void kp3a_dir(Vol v, const double *__restrict__ zv,
                                                double *__restrict__ p,
                                                const PState *__restrict__ ps)
{
    if (ps->done) return;
    const double beta = ps->beta;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < 2 * v.N;
         i += (size_t)gridDim.x * 256)
        p[i] = zv[i] + beta * p[i];
}

__global__ __launch_bounds__(256) void kp3a_out(Vol v, const double *__restrict__ u,
                                                float *__restrict__ u1, float *__restrict__ u2)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < v.N; i += (size_t)gridDim.x * 256) {
        u1[i] = (float)u[i];
        u2[i] = (float)u[v.N + i];
    }
}

// Work buffers of the 3-D decomposition, one set per device, grown on
// demand and kept between calls (the a_* FP64 vectors only for the
// attenuation-space system).
struct Pls3Work {
    DevBuf b1, b2, m2, w, res, dinv, p, q, z, part, bmax, thr, ps;
    DevBuf a_u, a_res, a_z, a_p, a_q;
};

std::mutex g_pls3_mu;
std::vector<std::pair<int, std::unique_ptr<Pls3Work>>> g_pls3;

Pls3Work *pls3_work()
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (auto &p : g_pls3)
        if (p.first == dev) return p.second.get();
    g_pls3.emplace_back(dev, std::make_unique<Pls3Work>());
    return g_pls3.back().second.get();
}

dect_status check_vol(int nx, int ny, int nz, const char *who)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || nx > 16384 || ny > 16384 || nz > 16384)
        return fail(DECT_ERR_INVALID_ARG, std::string(who) + ": volume sizes must be in [1, 16384]");
    return DECT_OK;
}

// The 3-D Prewitt map of x and the pair weights [3][N] into w.
dect_status edges3_into(const Vol &v, const float *x, double tau, double eps, float *w,
                        Pls3Work *W, hipStream_t s)
{
    const int nb = (int)std::min<size_t>(kMaxBlocks, (v.N + 255) / 256);
    dect_status st;
    if ((st = W->m2.ensure(v.N * 4)) || (st = W->bmax.ensure(kMaxBlocks * 4)) ||
        (st = W->thr.ensure(4)))
        return st;
    hipLaunchKernelGGL(kp3_m2, dim3(nb), dim3(256), 0, s, v, x, (float *)W->m2.ptr,
                       (float *)W->bmax.ptr);
    const float tau2 = (float)(tau * tau);
    hipLaunchKernelGGL(kp3_thr, dim3(1), dim3(256), 0, s, (const float *)W->bmax.ptr, nb, tau2,
                       (float *)W->thr.ptr);
    hipLaunchKernelGGL(kp3_w, dim3(nb), dim3(256), 0, s, v, (const float *)W->m2.ptr,
                       (const float *)W->thr.ptr, (float)eps, w, w + v.N, w + 2 * v.N);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

}  // namespace

dect_status pls_edge_weights3(int nx, int ny, int nz, const float *x, double tau, double eps,
                              float *w, hipStream_t s)
{
    if (!x || !w) return fail(DECT_ERR_INVALID_ARG, "dect_pls_edge_weights3: null argument");
    dect_status st = check_vol(nx, ny, nz, "dect_pls_edge_weights3");
    if (st) return st;
    if (!(tau >= 0.0) || !std::isfinite(tau) || !std::isfinite(eps))
        return fail(DECT_ERR_INVALID_ARG, "dect_pls_edge_weights3: bad tau/eps");
    const Vol v{nx, ny, nz, (size_t)nx * ny * nz, (size_t)nx * ny};
    std::lock_guard<std::mutex> lk(g_pls3_mu);
    return edges3_into(v, x, tau, eps, w, pls3_work(), s);
}

dect_status pls_decompose3(int nx, int ny, int nz, const float *xh, const float *xl,
                           const dect_pls_params *p, const float *ew, float *u1, float *u2,
                           dect_report *rep, hipStream_t s)
{
    if (!xh || !xl || !p || !u1 || !u2)
        return fail(DECT_ERR_INVALID_ARG, "dect_pls_decompose3: null argument");
    dect_status st = check_vol(nx, ny, nz, "dect_pls_decompose3");
    if (st) return st;
    if (p->mode != DECT_PLS_IMAGE && p->mode != DECT_PLS_ATTENUATION)
        return fail(DECT_ERR_INVALID_ARG, "dect_pls_decompose3: unknown mode");
    if (!(p->gamma >= 0.0) || !(p->edge_eps > 0.0) || !(p->edge_tau >= 0.0) || p->max_iter < 0 ||
        !(p->tol >= 0.0))
        return fail(DECT_ERR_INVALID_ARG, "gamma, tau, tol >= 0, eps > 0 and max_iter >= 0");
    const double det = p->eta_water_high * p->eta_bone_low - p->eta_bone_high * p->eta_water_low;
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det))
        return fail(DECT_ERR_INVALID_ARG, "the material matrix of Eq. 12 is singular");
    const Vol v{nx, ny, nz, (size_t)nx * ny * nz, (size_t)nx * ny};
    const int nb = (int)std::min<size_t>(kMaxBlocks, (v.N + 255) / 256);
    std::lock_guard<std::mutex> lk(g_pls3_mu);
    Pls3Work *W = pls3_work();
    const bool att = p->mode == DECT_PLS_ATTENUATION;
    if ((st = W->part.ensure((size_t)R_COUNT * kMaxBlocks * 8)) ||
        (st = W->ps.ensure(sizeof(PState))))
        return st;
    if (!att && ((st = W->b1.ensure(v.N * 4)) || (st = W->b2.ensure(v.N * 4)) ||
                 (st = W->res.ensure(v.N * 4)) || (st = W->dinv.ensure(v.N * 4)) ||
                 (st = W->p.ensure(v.N * 4)) || (st = W->q.ensure(v.N * 4)) ||
                 (st = W->z.ensure(v.N * 4))))
        return st;
    float *b[2] = {(float *)W->b1.ptr, (float *)W->b2.ptr};
    float *us[2] = {u1, u2};
    double *part = (double *)W->part.ptr;
    PState *ps = (PState *)W->ps.ptr;
    if (!att) {
        hipLaunchKernelGGL(kp3_dinv, dim3(nb), dim3(256), 0, s, v, xh, xl, p->eta_water_high,
                           p->eta_bone_high, p->eta_water_low, p->eta_bone_low, b[0], b[1]);
        DECT_HIP(hipGetLastError());
    }
    const float *wp = ew;
    if (!wp) {
        if ((st = W->w.ensure(3 * v.N * 4))) return st;
        if ((st = edges3_into(v, xl, p->edge_tau, p->edge_eps, (float *)W->w.ptr, W, s)))
            return st;
        wp = (const float *)W->w.ptr;
    }
    const PW w{wp, wp + v.N, wp + 2 * v.N};
    if (att) {
        const double e1h = p->eta_water_high, e2h = p->eta_bone_high, e1l = p->eta_water_low,
                     e2l = p->eta_bone_low;
        const AttK k{e1h, e2h, e1l, e2l, e1h * e1h + e1l * e1l, e1h * e2h + e1l * e2l,
                     e2h * e2h + e2l * e2l, det};
        const size_t vb = 2 * v.N * 8;
        if ((st = W->a_u.ensure(vb)) || (st = W->a_res.ensure(vb)) || (st = W->a_z.ensure(vb)) ||
            (st = W->a_p.ensure(vb)) || (st = W->a_q.ensure(vb)))
            return st;
        double *u = (double *)W->a_u.ptr, *res = (double *)W->a_res.ptr,
               *zv = (double *)W->a_z.ptr, *pp = (double *)W->a_p.ptr, *q = (double *)W->a_q.ptr;
        const double gamma = p->gamma;
        hipLaunchKernelGGL(kp3a_init, dim3(nb), dim3(256), 0, s, v, k, xh, xl, u);
        hipLaunchKernelGGL(kp3a_setup, dim3(nb), dim3(256), 0, s, v, w, gamma, k, xh, xl,
                           (const double *)u, res, zv, pp, part);
        hipLaunchKernelGGL(kp3_scalar, dim3(1), dim3(256), 0, s, ps, part, nb, 0, p->tol,
                           p->max_iter);
        DECT_HIP(hipGetLastError());
        PState h{};
        for (int it = 0; it < p->max_iter; ++it) {
            hipLaunchKernelGGL(kp3a_apply, dim3(nb), dim3(256), 0, s, v, w, gamma, k,
                               (const double *)pp, q, ps, part);
            hipLaunchKernelGGL(kp3_scalar, dim3(1), dim3(256), 0, s, ps, part, nb, 1, p->tol,
                               p->max_iter);
            hipLaunchKernelGGL(kp3a_update, dim3(nb), dim3(256), 0, s, v, w, gamma, k,
                               (const double *)pp, (const double *)q, u, res, zv, ps, part);
            hipLaunchKernelGGL(kp3_scalar, dim3(1), dim3(256), 0, s, ps, part, nb, 2, p->tol,
                               p->max_iter);
            hipLaunchKernelGGL(kp3a_dir, dim3(nb), dim3(256), 0, s, v, (const double *)zv, pp, ps);
            DECT_HIP(hipGetLastError());
            if (it % 8 == 7) {  // look at the device flag now and then
                DECT_HIP(hipMemcpyAsync(&h, ps, sizeof(PState), hipMemcpyDeviceToHost, s));
                DECT_HIP(hipStreamSynchronize(s));
                if (h.done) break;
            }
        }
        hipLaunchKernelGGL(kp3a_out, dim3(nb), dim3(256), 0, s, v, (const double *)u, u1, u2);
        DECT_HIP(hipGetLastError());
        DECT_HIP(hipMemcpyAsync(&h, ps, sizeof(PState), hipMemcpyDeviceToHost, s));
        DECT_HIP(hipStreamSynchronize(s));
        const bool capped = h.it >= p->max_iter && !(h.rn <= p->tol * h.bn);
        if (rep) {
            rep->iters = h.it;
            rep->objective = 0.0;
            rep->rel_change = 0.0;
            rep->pcg_residual = h.rn / h.bn;
            rep->status = capped ? DECT_WARN_MAXITER : DECT_OK;
        }
        if (capped)
            return fail(DECT_WARN_MAXITER, "dect_pls_decompose3: PCG reached max_iter above tolerance");
        return DECT_OK;
    }
    const float gamma = (float)p->gamma;
    int iters[2] = {0, 0};
    double relres[2] = {0.0, 0.0};
    bool capped = false;
    for (int m = 0; m < 2; ++m) {
        float *res = (float *)W->res.ptr, *dinv = (float *)W->dinv.ptr, *pp = (float *)W->p.ptr,
              *q = (float *)W->q.ptr, *zv = (float *)W->z.ptr;
        hipLaunchKernelGGL(kp3_setup, dim3(nb), dim3(256), 0, s, v, w, gamma, b[m], us[m], res,
                           dinv, pp, part);
        hipLaunchKernelGGL(kp3_scalar, dim3(1), dim3(256), 0, s, ps, part, nb, 0, p->tol,
                           p->max_iter);
        DECT_HIP(hipGetLastError());
        PState h{};
        for (int it = 0; it < p->max_iter; ++it) {
            hipLaunchKernelGGL(kp3_apply, dim3(nb), dim3(256), 0, s, v, w, gamma, pp, q, ps, part);
            hipLaunchKernelGGL(kp3_scalar, dim3(1), dim3(256), 0, s, ps, part, nb, 1, p->tol,
                               p->max_iter);
            hipLaunchKernelGGL(kp3_update, dim3(nb), dim3(256), 0, s, v, pp, q, dinv, us[m], res,
                               zv, ps, part);
            hipLaunchKernelGGL(kp3_scalar, dim3(1), dim3(256), 0, s, ps, part, nb, 2, p->tol,
                               p->max_iter);
            hipLaunchKernelGGL(kp3_dir, dim3(nb), dim3(256), 0, s, v, zv, pp, ps);
            DECT_HIP(hipGetLastError());
            if (it % 8 == 7) {  // look at the device flag now and then
                DECT_HIP(hipMemcpyAsync(&h, ps, sizeof(PState), hipMemcpyDeviceToHost, s));
                DECT_HIP(hipStreamSynchronize(s));
                if (h.done) break;
            }
        }
        DECT_HIP(hipMemcpyAsync(&h, ps, sizeof(PState), hipMemcpyDeviceToHost, s));
        DECT_HIP(hipStreamSynchronize(s));
        iters[m] = h.it;
        relres[m] = h.rn / h.bn;
        capped = capped || (h.it >= p->max_iter && !(h.rn <= p->tol * h.bn));
    }
    if (rep) {
        rep->iters = std::max(iters[0], iters[1]);
        rep->objective = 0.0;
        rep->rel_change = 0.0;
        rep->pcg_residual = std::max(relres[0], relres[1]);
        rep->status = capped ? DECT_WARN_MAXITER : DECT_OK;
    }
    if (capped)
        return fail(DECT_WARN_MAXITER, "dect_pls_decompose3: PCG reached max_iter above tolerance");
    return DECT_OK;
}

void release_pls3_work()
{
    std::lock_guard<std::mutex> lk(g_pls3_mu);
    g_pls3.clear();
}

}  // namespace dect
