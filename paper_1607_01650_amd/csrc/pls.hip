// Penalised least-squares image-domain decomposition (Eqs. 11-15) on gfx950.
//
//   dinv   : b = D^{-1} x per pixel (closed-form 2x2, Eq. 12); u starts at b.
//   prewitt: m2 = fmaf(gx, gx, gy*gy) of the Prewitt responses (fixed FP32
//            operation order, no contraction), per-block maxima.
//   weights: e_ik = eps where either pixel is an edge (m2 > tau^2 max m2),
//            1 otherwise (Eq. 14's edge weights after Sec. 2.3).
//   PCG    : (I + gamma L) u = b per material (Eq. 15 with grad R = 2L),
//            Jacobi preconditioner, two kernels per iteration, both materials
//            per launch.  Scalars are reduced redundantly by every block in
//            a fixed order, so every block takes the same decision.
#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"

namespace dect {
namespace {

constexpr int kPix = 4;  // pixels per thread in the streaming kernels

__device__ __forceinline__ double wave_sum_d(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int NV>
__device__ __forceinline__ void bsum(double (&v)[NV], double *out)
{
    __shared__ double sh[4][NV];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum_d(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[wid][i] = v[i];
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        int t = threadIdx.x;
        out[t] = ((sh[0][t] + sh[1][t]) + sh[2][t]) + sh[3][t];
    }
    __syncthreads();
}

// Sum of n doubles in a fixed order, result broadcast through LDS.
__device__ __forceinline__ double reduce_array(const double *__restrict__ a, int n)
{
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += 256) v[0] += a[i];
    __shared__ double out[1];
    bsum<1>(v, out);
    return out[0];
}

struct PlsCoef {
    float i11, i12, i21, i22;  // D^{-1} = [[i11, i12], [i21, i22]]
};

__global__ __launch_bounds__(256) void k_dinv(const float *__restrict__ xh,
                                              const float *__restrict__ xl, PlsCoef c,
                                              float *__restrict__ u1, float *__restrict__ u2,
                                              float *__restrict__ b, size_t N)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    float h = xh[i], l = xl[i];
    float a = c.i11 * h + c.i12 * l;
    float d = c.i21 * h + c.i22 * l;
    u1[i] = a;
    u2[i] = d;
    b[i] = a;
    b[N + i] = d;
}

__global__ __launch_bounds__(256) void k_prewitt(const float *__restrict__ x,
                                                 float *__restrict__ m2,
                                                 float *__restrict__ pmax, int nx, int ny)
{
#pragma clang fp contract(off)
    const size_t N = (size_t)nx * ny;
    float mx = 0.f;
    for (int j = 0; j < kPix; ++j) {
        size_t i = ((size_t)blockIdx.x * kPix + j) * 256 + threadIdx.x;
        if (i < N) {
            int r = (int)(i / nx), c = (int)(i % nx);
            int ru = r > 0 ? r - 1 : 0, rd = r < ny - 1 ? r + 1 : ny - 1;
            int cl = c > 0 ? c - 1 : 0, cr = c < nx - 1 ? c + 1 : nx - 1;
#define X(rr, cc) x[(size_t)(rr) * nx + (cc)]
            float right = (X(ru, cr) + X(r, cr)) + X(rd, cr);
            float left = (X(ru, cl) + X(r, cl)) + X(rd, cl);
            float down = (X(rd, cl) + X(rd, c)) + X(rd, cr);
            float up = (X(ru, cl) + X(ru, c)) + X(ru, cr);
#undef X
            float gx = right - left, gy = down - up;
            float v = fmaf(gx, gx, gy * gy);
            m2[i] = v;
            mx = fmaxf(mx, v);
        }
    }
    __shared__ float sh[256];
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) pmax[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_weights(const float *__restrict__ m2,
                                                 const float *__restrict__ pmax, int nblk,
                                                 float tau2, float eps, float *__restrict__ w,
                                                 int nx, int ny)
{
    __shared__ float sh[256];
    float mx = 0.f;
    for (int i = threadIdx.x; i < nblk; i += 256) mx = fmaxf(mx, pmax[i]);
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const float thr = tau2 * sh[0];
    const size_t N = (size_t)nx * ny;
    for (int j = 0; j < kPix; ++j) {
        size_t i = ((size_t)blockIdx.x * kPix + j) * 256 + threadIdx.x;
        if (i < N) {
            int r = (int)(i / nx), c = (int)(i % nx);
            bool ei = m2[i] > thr;
            float wr = 0.f, wd = 0.f;
            if (c + 1 < nx) wr = (ei || m2[i + 1] > thr) ? eps : 1.0f;
            if (r + 1 < ny) wd = (ei || m2[i + nx] > thr) ? eps : 1.0f;
            w[i] = wr;
            w[N + i] = wd;
        }
    }
}

// Jacobi preconditioner 1 / (1 + gamma sum_k e_ik).
__device__ __forceinline__ float lap_diag(const float *__restrict__ er,
                                          const float *__restrict__ ed, size_t i, int r, int c,
                                          int nx, int ny)
{
    float d = 0.f;
    if (c + 1 < nx) d += er[i];
    if (c >= 1) d += er[i - 1];
    if (r + 1 < ny) d += ed[i];
    if (r >= 1) d += ed[i - nx];
    return d;
}

struct PcgStatus {
    int32_t done, iters;
    double relres;
};

// Setup: res = b - (I + gamma L) b (u starts at b), z = M^{-1} res, p_old = 0,
// partials rz, |res|^2, |b|^2.
__global__ __launch_bounds__(256) void k_pcg_setup(
    const float *__restrict__ b, const float *__restrict__ w, float gamma,
    float *__restrict__ res, float *__restrict__ z, float *__restrict__ pold,
    float *__restrict__ minv, double *__restrict__ p_rz, double *__restrict__ p_rr,
    double *__restrict__ p_bb, PcgStatus *__restrict__ stat, int nx, int ny, int nblk)
{
    const int m = blockIdx.y;
    const size_t N = (size_t)nx * ny;
    const float *er = w, *ed = w + N;
    const float *bm = b + m * N;
    double v[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < kPix; ++j) {
        size_t i = ((size_t)blockIdx.x * kPix + j) * 256 + threadIdx.x;
        if (i < N) {
            int r = (int)(i / nx), c = (int)(i % nx);
            float ui = bm[i];
            float lu = 0.f;
            if (c + 1 < nx) lu += er[i] * (ui - bm[i + 1]);
            if (c >= 1) lu += er[i - 1] * (ui - bm[i - 1]);
            if (r + 1 < ny) lu += ed[i] * (ui - bm[i + nx]);
            if (r >= 1) lu += ed[i - nx] * (ui - bm[i - nx]);
            float rs = ui - (ui + gamma * lu);
            float mi = 1.0f / (1.0f + gamma * lap_diag(er, ed, i, r, c, nx, ny));
            float zz = mi * rs;
            res[m * N + i] = rs;
            z[m * N + i] = zz;
            pold[m * N + i] = 0.f;
            if (m == 0) minv[i] = mi;
            v[0] += (double)rs * zz;
            v[1] += (double)rs * rs;
            v[2] += (double)ui * ui;
        }
    }
    __shared__ double out[3];
    bsum<3>(v, out);
    if (threadIdx.x == 0) {
        p_rz[(size_t)m * nblk + blockIdx.x] = out[0];
        p_rr[(size_t)m * nblk + blockIdx.x] = out[1];
        p_bb[(size_t)m * nblk + blockIdx.x] = out[2];
        if (blockIdx.x == 0) {
            stat[m].done = 0;
            stat[m].iters = 0;
            stat[m].relres = 0.0;
        }
    }
}

// Iteration it, part A: convergence test on the previous residual, beta,
// p_new = z + beta p_old, q = (I + gamma L) p_new, partial <p_new, q>.
// rz_cur: partials of <res, z> of this iteration; rz_prev of the previous.
__global__ __launch_bounds__(256) void k_pcg_a(
    const float *__restrict__ z, const float *__restrict__ pold, float *__restrict__ pnew,
    float *__restrict__ q, const float *__restrict__ w, float gamma,
    const double *__restrict__ rz_cur, const double *__restrict__ rz_prev,
    const double *__restrict__ p_rr, const double *__restrict__ p_bb,
    double *__restrict__ p_pq, PcgStatus *__restrict__ stat, int it, double tol, int nx, int ny,
    int nblk)
{
    const int m = blockIdx.y;
    if (stat[m].done) return;
    const double rr = reduce_array(p_rr + (size_t)m * nblk, nblk);
    const double bb = reduce_array(p_bb + (size_t)m * nblk, nblk);
    const double bn = bb > 0.0 ? sqrt(bb) : 1.0;
    const double rn = bb > 0.0 ? sqrt(rr) : 0.0;
    if (rn <= tol * bn) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            stat[m].done = 1;
            stat[m].iters = it;
            stat[m].relres = rn / bn;
        }
        return;
    }
    float beta = 0.f;
    if (it > 0) {
        const double a = reduce_array(rz_cur + (size_t)m * nblk, nblk);
        const double b = reduce_array(rz_prev + (size_t)m * nblk, nblk);
        beta = (float)(a / b);
    }
    const size_t N = (size_t)nx * ny;
    const float *er = w, *ed = w + N;
    const float *zm = z + m * N, *pm = pold + m * N;
    double v[1] = {0.0};
    for (int j = 0; j < kPix; ++j) {
        size_t i = ((size_t)blockIdx.x * kPix + j) * 256 + threadIdx.x;
        if (i < N) {
            int r = (int)(i / nx), c = (int)(i % nx);
            float pi = zm[i] + beta * pm[i];
            float lp = 0.f;
            if (c + 1 < nx) lp += er[i] * (pi - (zm[i + 1] + beta * pm[i + 1]));
            if (c >= 1) lp += er[i - 1] * (pi - (zm[i - 1] + beta * pm[i - 1]));
            if (r + 1 < ny) lp += ed[i] * (pi - (zm[i + nx] + beta * pm[i + nx]));
            if (r >= 1) lp += ed[i - nx] * (pi - (zm[i - nx] + beta * pm[i - nx]));
            float qi = pi + gamma * lp;
            pnew[m * N + i] = pi;
            q[m * N + i] = qi;
            v[0] += (double)pi * qi;
        }
    }
    __shared__ double out[1];
    bsum<1>(v, out);
    if (threadIdx.x == 0) p_pq[(size_t)m * nblk + blockIdx.x] = out[0];
}

// Part B: a = rz / <p, q>, u += a p, res -= a q, z = M^{-1} res; partials of
// the next <res, z> and |res|^2.
__global__ __launch_bounds__(256) void k_pcg_b(
    float *__restrict__ u1, float *__restrict__ u2, float *__restrict__ res,
    float *__restrict__ z, const float *__restrict__ pnew, const float *__restrict__ q,
    const float *__restrict__ minv, const double *__restrict__ rz_cur,
    const double *__restrict__ p_pq, double *__restrict__ rz_next, double *__restrict__ p_rr,
    PcgStatus *__restrict__ stat, int nx, int ny, int nblk)
{
    const int m = blockIdx.y;
    if (stat[m].done) return;
    const double pq = reduce_array(p_pq + (size_t)m * nblk, nblk);
    const double rz = reduce_array(rz_cur + (size_t)m * nblk, nblk);
    if (!(pq > 0.0)) {  // breakdown: stop with the current iterate
        if (blockIdx.x == 0 && threadIdx.x == 0) stat[m].done = 2;
        return;
    }
    const float a = (float)(rz / pq);
    const size_t N = (size_t)nx * ny;
    float *um = m == 0 ? u1 : u2;
    double v[2] = {0.0, 0.0};
    for (int j = 0; j < kPix; ++j) {
        size_t i = ((size_t)blockIdx.x * kPix + j) * 256 + threadIdx.x;
        if (i < N) {
            um[i] += a * pnew[m * N + i];
            float rs = res[m * N + i] - a * q[m * N + i];
            float zz = minv[i] * rs;
            res[m * N + i] = rs;
            z[m * N + i] = zz;
            v[0] += (double)rs * zz;
            v[1] += (double)rs * rs;
        }
    }
    __shared__ double out[2];
    bsum<2>(v, out);
    if (threadIdx.x == 0) {
        rz_next[(size_t)m * nblk + blockIdx.x] = out[0];
        p_rr[(size_t)m * nblk + blockIdx.x] = out[1];
    }
}

// After the last iteration: final residual of materials still running.
__global__ __launch_bounds__(256) void k_pcg_final(const double *__restrict__ p_rr,
                                                   const double *__restrict__ p_bb,
                                                   PcgStatus *__restrict__ stat, int iters,
                                                   double tol, int nblk)
{
    const int m = blockIdx.x;
    if (stat[m].done) return;
    const double rr = reduce_array(p_rr + (size_t)m * nblk, nblk);
    const double bb = reduce_array(p_bb + (size_t)m * nblk, nblk);
    if (threadIdx.x != 0) return;
    const double bn = bb > 0.0 ? sqrt(bb) : 1.0;
    const double rn = bb > 0.0 ? sqrt(rr) : 0.0;
    stat[m].iters = iters;
    stat[m].relres = rn / bn;
    stat[m].done = rn <= tol * bn ? 1 : 3;  // 3: stopped at the cap
}

// ---------------------------------------------- attenuation-space PLS ---
// (D^T D (x) I + gamma I (x) L) u = D^T x (|x - Du|^2 + gamma R(u)): both
// materials of a pixel in one thread, so the per-pixel 2 x 2 coupling D^T D
// and the block-Jacobi preconditioner (D^T D + gamma diag(L)) apply in place;
// joint scalars over both materials.  D^T D has the condition number of D
// squared (~740 for water and bone), so vectors and arithmetic are FP64.
struct AttCoef {
    double g11, g12, g22;       // D^T D
    double e1h, e2h, e1l, e2l;  // D
};

// (A v)_m at pixel i for the two-material FP64 vector v ([2][N]).
__device__ __forceinline__ void att_apply(const double *__restrict__ v,
                                          const float *__restrict__ er,
                                          const float *__restrict__ ed, const AttCoef &k,
                                          double gamma, size_t i, int r, int c, int nx, int ny,
                                          size_t N, double (&out)[2])
{
    double lv[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const double *vm = v + m * N;
        const double vi = vm[i];
        double l = 0.0;
        if (c + 1 < nx) l += (double)er[i] * (vi - vm[i + 1]);
        if (c >= 1) l += (double)er[i - 1] * (vi - vm[i - 1]);
        if (r + 1 < ny) l += (double)ed[i] * (vi - vm[i + nx]);
        if (r >= 1) l += (double)ed[i - nx] * (vi - vm[i - nx]);
        lv[m] = l;
    }
    const double a = v[i], b = v[N + i];
    out[0] = k.g11 * a + k.g12 * b + gamma * lv[0];
    out[1] = k.g12 * a + k.g22 * b + gamma * lv[1];
}

// z = P^{-1} res at one pixel, P = D^T D + gamma diag(L) I.
__device__ __forceinline__ void att_precond(const AttCoef &k, double gamma, double d,
                                            const double (&rs)[2], double (&z)[2])
{
    const double a11 = k.g11 + gamma * d, a22 = k.g22 + gamma * d;
    const double dt = a11 * a22 - k.g12 * k.g12;
    z[0] = (a22 * rs[0] - k.g12 * rs[1]) / dt;
    z[1] = (a11 * rs[1] - k.g12 * rs[0]) / dt;
}

// Setup from u = D^{-1} x (u1, u2): u64 = u, res = D^T x - A u, z = P^{-1} res,
// p_old = 0; partials <res, z>, |res|^2, |D^T x|^2 in slot 0.
__global__ __launch_bounds__(256) void k_apcg_setup(
    const float *__restrict__ xh, const float *__restrict__ xl, const float *__restrict__ u1,
    const float *__restrict__ u2, const float *__restrict__ w, double gamma, AttCoef k,
    double *__restrict__ u, double *__restrict__ res, double *__restrict__ z,
    double *__restrict__ pold, double *__restrict__ p_rz, double *__restrict__ p_rr,
    double *__restrict__ p_bb, PcgStatus *__restrict__ stat, int nx, int ny)
{
    const size_t N = (size_t)nx * ny;
    const float *er = w, *ed = w + N;
    // u64 first, block by block: the stencil below reads neighbours' values
    // from the float inputs, so no ordering between blocks is needed
    double v[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < kPix; ++j) {
        size_t i = ((size_t)blockIdx.x * kPix + j) * 256 + threadIdx.x;
        if (i < N) {
            const int r = (int)(i / nx), c = (int)(i % nx);
            double lu[2];
            const float *um[2] = {u1, u2};
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const double ui = um[m][i];
                double l = 0.0;
                if (c + 1 < nx) l += (double)er[i] * (ui - (double)um[m][i + 1]);
                if (c >= 1) l += (double)er[i - 1] * (ui - (double)um[m][i - 1]);
                if (r + 1 < ny) l += (double)ed[i] * (ui - (double)um[m][i + nx]);
                if (r >= 1) l += (double)ed[i - nx] * (ui - (double)um[m][i - nx]);
                lu[m] = l;
            }
            const double a = u1[i], b = u2[i];
            const double h = xh[i], l = xl[i];
            const double c0 = k.e1h * h + k.e1l * l, c1 = k.e2h * h + k.e2l * l;
            double rs[2] = {c0 - (k.g11 * a + k.g12 * b + gamma * lu[0]),
                            c1 - (k.g12 * a + k.g22 * b + gamma * lu[1])};
            double zz[2];
            att_precond(k, gamma, (double)lap_diag(er, ed, i, r, c, nx, ny), rs, zz);
            u[i] = a;
            u[N + i] = b;
            res[i] = rs[0];
            res[N + i] = rs[1];
            z[i] = zz[0];
            z[N + i] = zz[1];
            pold[i] = 0.0;
            pold[N + i] = 0.0;
            v[0] += rs[0] * zz[0] + rs[1] * zz[1];
            v[1] += rs[0] * rs[0] + rs[1] * rs[1];
            v[2] += c0 * c0 + c1 * c1;
        }
    }
    __shared__ double out[3];
    bsum<3>(v, out);
    if (threadIdx.x == 0) {
        p_rz[blockIdx.x] = out[0];
        p_rr[blockIdx.x] = out[1];
        p_bb[blockIdx.x] = out[2];
        if (blockIdx.x == 0) {
            stat[0].done = 0;
            stat[0].iters = 0;
            stat[0].relres = 0.0;
        }
    }
}

// Part A: convergence test, beta, p_new = z + beta p_old, q = A p_new,
// partial <p_new, q>.  p_new is formed first by every block for its own
// pixels in a separate pass (k_apcg_p) so that q's stencil can read it.
__global__ __launch_bounds__(256) void k_apcg_p(
    const double *__restrict__ z, const double *__restrict__ pold, double *__restrict__ pnew,
    const double *__restrict__ rz_cur, const double *__restrict__ rz_prev,
    const double *__restrict__ p_rr, const double *__restrict__ p_bb,
    PcgStatus *__restrict__ stat, int it, double tol, int nx, int ny, int nblk)
{
    if (stat[0].done) return;
    const double rr = reduce_array(p_rr, nblk);
    const double bb = reduce_array(p_bb, nblk);
    const double bn = bb > 0.0 ? sqrt(bb) : 1.0;
    const double rn = bb > 0.0 ? sqrt(rr) : 0.0;
    if (rn <= tol * bn) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            stat[0].done = 1;
            stat[0].iters = it;
            stat[0].relres = rn / bn;
        }
        return;
    }
    double beta = 0.0;
    if (it > 0) beta = reduce_array(rz_cur, nblk) / reduce_array(rz_prev, nblk);
    const size_t N = (size_t)nx * ny;
    for (int j = 0; j < kPix; ++j) {
        size_t i = ((size_t)blockIdx.x * kPix + j) * 256 + threadIdx.x;
        if (i < N) {
            pnew[i] = z[i] + beta * pold[i];
            pnew[N + i] = z[N + i] + beta * pold[N + i];
        }
    }
}

__global__ __launch_bounds__(256) void k_apcg_q(
    const double *__restrict__ pnew, double *__restrict__ q, const float *__restrict__ w,
    double gamma, AttCoef k, double *__restrict__ p_pq, PcgStatus *__restrict__ stat, int nx,
    int ny)
{
    if (stat[0].done) return;
    const size_t N = (size_t)nx * ny;
    const float *er = w, *ed = w + N;
    double v[1] = {0.0};
    for (int j = 0; j < kPix; ++j) {
        size_t i = ((size_t)blockIdx.x * kPix + j) * 256 + threadIdx.x;
        if (i < N) {
            const int r = (int)(i / nx), c = (int)(i % nx);
            double qq[2];
            att_apply(pnew, er, ed, k, gamma, i, r, c, nx, ny, N, qq);
            q[i] = qq[0];
            q[N + i] = qq[1];
            v[0] += pnew[i] * qq[0] + pnew[N + i] * qq[1];
        }
    }
    __shared__ double out[1];
    bsum<1>(v, out);
    if (threadIdx.x == 0) p_pq[blockIdx.x] = out[0];
}

// Part B: a = rz / <p, q>, u += a p, res -= a q, z = P^{-1} res; partials of
// the next <res, z> and |res|^2.
__global__ __launch_bounds__(256) void k_apcg_b(
    double *__restrict__ u, double *__restrict__ res, double *__restrict__ z,
    const double *__restrict__ pnew, const double *__restrict__ q, const float *__restrict__ w,
    double gamma, AttCoef k, const double *__restrict__ rz_cur, const double *__restrict__ p_pq,
    double *__restrict__ rz_next, double *__restrict__ p_rr, PcgStatus *__restrict__ stat,
    int nx, int ny, int nblk)
{
    if (stat[0].done) return;
    const double pq = reduce_array(p_pq, nblk);
    const double rz = reduce_array(rz_cur, nblk);
    if (!(pq > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) stat[0].done = 2;
        return;
    }
    const double a = rz / pq;
    const size_t N = (size_t)nx * ny;
    const float *er = w, *ed = w + N;
    double v[2] = {0.0, 0.0};
    for (int j = 0; j < kPix; ++j) {
        size_t i = ((size_t)blockIdx.x * kPix + j) * 256 + threadIdx.x;
        if (i < N) {
            const int r = (int)(i / nx), c = (int)(i % nx);
            u[i] += a * pnew[i];
            u[N + i] += a * pnew[N + i];
            double rs[2] = {res[i] - a * q[i], res[N + i] - a * q[N + i]};
            double zz[2];
            att_precond(k, gamma, (double)lap_diag(er, ed, i, r, c, nx, ny), rs, zz);
            res[i] = rs[0];
            res[N + i] = rs[1];
            z[i] = zz[0];
            z[N + i] = zz[1];
            v[0] += rs[0] * zz[0] + rs[1] * zz[1];
            v[1] += rs[0] * rs[0] + rs[1] * rs[1];
        }
    }
    __shared__ double out[2];
    bsum<2>(v, out);
    if (threadIdx.x == 0) {
        rz_next[blockIdx.x] = out[0];
        p_rr[blockIdx.x] = out[1];
    }
}

__global__ __launch_bounds__(256) void k_apcg_out(const double *__restrict__ u,
                                                  float *__restrict__ u1, float *__restrict__ u2,
                                                  size_t N)
{
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    u1[i] = (float)u[i];
    u2[i] = (float)u[N + i];
}

struct PlsWork {
    DevBuf b, res, z, p0, p1, q, minv, w, m2, pmax, prz0, prz1, prr, pbb, ppq, stat, u64;
};

// Device buffers of one image-space decomposition of N pixels (nblk
// reduction blocks): D^{-1} x (both materials), PCG vectors, the Jacobi
// inverse, edge weights and the Prewitt map, per-block partial sums.
struct PlsBufs {
    float *b, *res, *z, *p0, *p1, *q, *minv, *w, *m2, *pmax;
    double *prz0, *prz1, *prr, *pbb, *ppq;
    PcgStatus *stat;
};

std::mutex g_pls_mu;
std::vector<std::pair<int, std::unique_ptr<PlsWork>>> g_pls;

PlsWork *pls_work()
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (auto &p : g_pls)
        if (p.first == dev) return p.second.get();
    g_pls.emplace_back(dev, std::make_unique<PlsWork>());
    return g_pls.back().second.get();
}

dect_status edges_run(int nx, int ny, const float *x, double tau, double eps, float *w,
                      float *m2, float *pmax, hipStream_t s)
{
    const size_t N = (size_t)nx * ny;
    const int nblk = (int)((N + 256 * kPix - 1) / (256 * kPix));
    hipLaunchKernelGGL(k_prewitt, dim3(nblk), dim3(256), 0, s, x, m2, pmax, nx, ny);
    DECT_HIP(hipGetLastError());
    const float tau2 = (float)(tau * tau);
    hipLaunchKernelGGL(k_weights, dim3(nblk), dim3(256), 0, s, (const float *)m2,
                       (const float *)pmax, nblk, tau2, (float)eps, w, nx, ny);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

dect_status edges_into(int nx, int ny, const float *x, double tau, double eps, float *w,
                       PlsWork *W, hipStream_t s)
{
    const size_t N = (size_t)nx * ny;
    const int nblk = (int)((N + 256 * kPix - 1) / (256 * kPix));
    dect_status st;
    if ((st = W->m2.ensure(N * 4)) || (st = W->pmax.ensure((size_t)nblk * 4))) return st;
    return edges_run(nx, ny, x, tau, eps, w, (float *)W->m2.ptr, (float *)W->pmax.ptr, s);
}

dect_status check_pls_args(int nx, int ny, const float *xh, const float *xl,
                           const dect_pls_params *P, float *u1, float *u2, const char *who)
{
    if (nx <= 0 || ny <= 0 || !xh || !xl || !P || !u1 || !u2)
        return fail(DECT_ERR_INVALID_ARG, std::string(who) + ": bad size or null argument");
    const double det = P->eta_water_high * P->eta_bone_low - P->eta_bone_high * P->eta_water_low;
    if (!std::isfinite(det) || det == 0.0)
        return fail(DECT_ERR_INVALID_ARG, std::string(who) + ": singular decomposition matrix");
    if (!(P->gamma >= 0.0) || !std::isfinite(P->gamma) || P->max_iter < 0 || !(P->tol >= 0.0))
        return fail(DECT_ERR_INVALID_ARG, std::string(who) + ": bad gamma/max_iter/tol");
    if (P->mode != DECT_PLS_IMAGE && P->mode != DECT_PLS_ATTENUATION)
        return fail(DECT_ERR_INVALID_ARG, std::string(who) + ": unknown mode");
    return DECT_OK;
}

// D^{-1} x into u1, u2 and B.b (both materials).
void dinv_run(int nx, int ny, const float *xh, const float *xl, const dect_pls_params *P,
              float *u1, float *u2, float *b, hipStream_t s)
{
    const size_t N = (size_t)nx * ny;
    const double det = P->eta_water_high * P->eta_bone_low - P->eta_bone_high * P->eta_water_low;
    PlsCoef c;
    c.i11 = (float)(P->eta_bone_low / det);
    c.i12 = (float)(-P->eta_bone_high / det);
    c.i21 = (float)(-P->eta_water_low / det);
    c.i22 = (float)(P->eta_water_high / det);
    hipLaunchKernelGGL(k_dinv, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, xh, xl, c, u1,
                       u2, b, N);
}

// Jacobi-PCG of the image-space system (I + gamma L) u_m = b_m for both
// materials, from u = b (already in u1, u2), on the pair weights w.
dect_status pcg_image_run(int nx, int ny, const dect_pls_params *P, const float *w, float *u1,
                          float *u2, dect_report *rep, const PlsBufs &B, hipStream_t s)
{
    const size_t N = (size_t)nx * ny;
    const int nblk = (int)((N + 256 * kPix - 1) / (256 * kPix));
    const float gamma = (float)P->gamma;
    PcgStatus *stat = B.stat;
    float *pbuf[2] = {B.p0, B.p1};
    double *rzb[2] = {B.prz0, B.prz1};
    hipLaunchKernelGGL(k_pcg_setup, dim3(nblk, 2), dim3(256), 0, s, (const float *)B.b, w, gamma,
                       B.res, B.z, pbuf[0], B.minv, rzb[0], B.prr, B.pbb, stat, nx, ny, nblk);
    DECT_HIP(hipGetLastError());
    int it = 0;
    const int check_every = 16;
    for (; it < P->max_iter; ++it) {
        float *pold = pbuf[it & 1], *pnew = pbuf[(it + 1) & 1];
        const double *rz_prev = rzb[(it + 1) & 1];
        hipLaunchKernelGGL(k_pcg_a, dim3(nblk, 2), dim3(256), 0, s, (const float *)B.z,
                           (const float *)pold, pnew, B.q, w, gamma, (const double *)rzb[it & 1],
                           rz_prev, (const double *)B.prr, (const double *)B.pbb, B.ppq, stat, it,
                           P->tol, nx, ny, nblk);
        DECT_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_pcg_b, dim3(nblk, 2), dim3(256), 0, s, u1, u2, B.res, B.z,
                           (const float *)pnew, (const float *)B.q, (const float *)B.minv,
                           (const double *)rzb[it & 1], (const double *)B.ppq, rzb[(it + 1) & 1],
                           B.prr, stat, nx, ny, nblk);
        DECT_HIP(hipGetLastError());
        if ((it + 1) % check_every == 0) {
            PcgStatus hs[2];
            DECT_HIP(hipMemcpyAsync(hs, stat, sizeof(hs), hipMemcpyDeviceToHost, s));
            DECT_HIP(hipStreamSynchronize(s));
            if (hs[0].done && hs[1].done) {
                ++it;
                break;
            }
        }
    }
    hipLaunchKernelGGL(k_pcg_final, dim3(2), dim3(256), 0, s, (const double *)B.prr,
                       (const double *)B.pbb, stat, it, P->tol, nblk);
    DECT_HIP(hipGetLastError());
    if (rep) {
        PcgStatus hs[2];
        DECT_HIP(hipMemcpyAsync(hs, stat, sizeof(hs), hipMemcpyDeviceToHost, s));
        DECT_HIP(hipStreamSynchronize(s));
        rep->iters = std::max(hs[0].iters, hs[1].iters);
        rep->pcg_residual = std::max(hs[0].relres, hs[1].relres);
        rep->objective = 0.0;
        rep->rel_change = 0.0;
        rep->status = (hs[0].done == 3 || hs[1].done == 3) ? DECT_WARN_MAXITER : DECT_OK;
        if (rep->status == DECT_WARN_MAXITER) {
            set_error("dect_pls_decompose: PCG reached max_iter above tolerance");
            return DECT_WARN_MAXITER;
        }
    }
    return DECT_OK;
}

}  // namespace

dect_status pls_edge_weights(int nx, int ny, const float *x, double tau, double eps, float *w,
                             hipStream_t s)
{
    if (nx <= 0 || ny <= 0 || !x || !w)
        return fail(DECT_ERR_INVALID_ARG, "dect_pls_edge_weights: bad size or null buffer");
    if (!(tau >= 0.0) || !std::isfinite(tau) || !std::isfinite(eps))
        return fail(DECT_ERR_INVALID_ARG, "dect_pls_edge_weights: bad tau/eps");
    std::lock_guard<std::mutex> lk(g_pls_mu);
    return edges_into(nx, ny, x, tau, eps, w, pls_work(), s);
}

// The image-space work buffers of N pixels in nblk reduction blocks.
static dect_status pls_prepare(PlsWork *W, size_t N, int nblk)
{
    dect_status st;
    if ((st = W->b.ensure(2 * N * 4)) || (st = W->res.ensure(2 * N * 4)) ||
        (st = W->z.ensure(2 * N * 4)) || (st = W->p0.ensure(2 * N * 4)) ||
        (st = W->p1.ensure(2 * N * 4)) || (st = W->q.ensure(2 * N * 4)) ||
        (st = W->minv.ensure(N * 4)) || (st = W->prz0.ensure((size_t)2 * nblk * 8)) ||
        (st = W->prz1.ensure((size_t)2 * nblk * 8)) || (st = W->prr.ensure((size_t)2 * nblk * 8)) ||
        (st = W->pbb.ensure((size_t)2 * nblk * 8)) || (st = W->ppq.ensure((size_t)2 * nblk * 8)) ||
        (st = W->stat.ensure(2 * sizeof(PcgStatus))))
        return st;
    return DECT_OK;
}

// The FP64 vectors of the attenuation-space solve (they replace the FP32
// ones of the same names).
static dect_status pls_prepare_att(PlsWork *W, size_t N)
{
    dect_status st;
    if ((st = W->u64.ensure(2 * N * 8)) || (st = W->res.ensure(2 * N * 8)) ||
        (st = W->z.ensure(2 * N * 8)) || (st = W->p0.ensure(2 * N * 8)) ||
        (st = W->p1.ensure(2 * N * 8)) || (st = W->q.ensure(2 * N * 8)))
        return st;
    return DECT_OK;
}

// The work buffers of a decomposition of N pixels in both modes with the
// edges detected, in the order the calls allocate them (image mode first),
// for a dry run under a SizingScope.
dect_status pls_size_run(size_t N)
{
    const int nblk = (int)((N + 256 * kPix - 1) / (256 * kPix));
    PlsWork W;
    dect_status st;
    if ((st = pls_prepare(&W, N, nblk)) || (st = W.w.ensure(2 * N * 4)) ||
        (st = W.m2.ensure(N * 4)) || (st = W.pmax.ensure((size_t)nblk * 4)) ||
        (st = pls_prepare_att(&W, N)))
        return st;
    return DECT_OK;
}

// The attenuation-space system, from u = D^{-1} x already in u1, u2.
dect_status pls_attenuation(int nx, int ny, const float *xh, const float *xl,
                            const dect_pls_params *P, const float *w, float *u1, float *u2,
                            dect_report *rep, PlsWork *W, int nblk, hipStream_t s)
{
    const size_t N = (size_t)nx * ny;
    dect_status st;
    if ((st = pls_prepare_att(W, N))) return st;
    AttCoef k;
    k.e1h = P->eta_water_high;
    k.e2h = P->eta_bone_high;
    k.e1l = P->eta_water_low;
    k.e2l = P->eta_bone_low;
    k.g11 = k.e1h * k.e1h + k.e1l * k.e1l;
    k.g12 = k.e1h * k.e2h + k.e1l * k.e2l;
    k.g22 = k.e2h * k.e2h + k.e2l * k.e2l;
    const double gamma = P->gamma;
    PcgStatus *stat = (PcgStatus *)W->stat.ptr;
    double *u = (double *)W->u64.ptr, *res = (double *)W->res.ptr, *z = (double *)W->z.ptr;
    double *q = (double *)W->q.ptr;
    double *pbuf[2] = {(double *)W->p0.ptr, (double *)W->p1.ptr};
    double *rzb[2] = {(double *)W->prz0.ptr, (double *)W->prz1.ptr};
    hipLaunchKernelGGL(k_apcg_setup, dim3(nblk), dim3(256), 0, s, xh, xl, (const float *)u1,
                       (const float *)u2, w, gamma, k, u, res, z, pbuf[0], rzb[0],
                       (double *)W->prr.ptr, (double *)W->pbb.ptr, stat, nx, ny);
    DECT_HIP(hipGetLastError());
    int it = 0;
    const int check_every = 16;
    for (; it < P->max_iter; ++it) {
        const double *pold = pbuf[it & 1];
        double *pnew = pbuf[(it + 1) & 1];
        hipLaunchKernelGGL(k_apcg_p, dim3(nblk), dim3(256), 0, s, (const double *)z, pold, pnew,
                           (const double *)rzb[it & 1], (const double *)rzb[(it + 1) & 1],
                           (const double *)W->prr.ptr, (const double *)W->pbb.ptr, stat, it,
                           P->tol, nx, ny, nblk);
        DECT_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_apcg_q, dim3(nblk), dim3(256), 0, s, (const double *)pnew, q, w,
                           gamma, k, (double *)W->ppq.ptr, stat, nx, ny);
        DECT_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_apcg_b, dim3(nblk), dim3(256), 0, s, u, res, z, (const double *)pnew,
                           (const double *)q, w, gamma, k, (const double *)rzb[it & 1],
                           (const double *)W->ppq.ptr, rzb[(it + 1) & 1], (double *)W->prr.ptr,
                           stat, nx, ny, nblk);
        DECT_HIP(hipGetLastError());
        if ((it + 1) % check_every == 0) {
            PcgStatus hs;
            DECT_HIP(hipMemcpyAsync(&hs, stat, sizeof(hs), hipMemcpyDeviceToHost, s));
            DECT_HIP(hipStreamSynchronize(s));
            if (hs.done) {
                ++it;
                break;
            }
        }
    }
    hipLaunchKernelGGL(k_pcg_final, dim3(1), dim3(256), 0, s, (const double *)W->prr.ptr,
                       (const double *)W->pbb.ptr, stat, it, P->tol, nblk);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_apcg_out, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                       (const double *)u, u1, u2, N);
    DECT_HIP(hipGetLastError());
    if (rep) {
        PcgStatus hs;
        DECT_HIP(hipMemcpyAsync(&hs, stat, sizeof(hs), hipMemcpyDeviceToHost, s));
        DECT_HIP(hipStreamSynchronize(s));
        rep->iters = hs.iters;
        rep->pcg_residual = hs.relres;
        rep->objective = 0.0;
        rep->rel_change = 0.0;
        rep->status = hs.done == 3 ? DECT_WARN_MAXITER : DECT_OK;
        if (rep->status == DECT_WARN_MAXITER) {
            set_error("dect_pls_decompose: PCG reached max_iter above tolerance");
            return DECT_WARN_MAXITER;
        }
    }
    return DECT_OK;
}

dect_status pls_decompose(int nx, int ny, const float *xh, const float *xl,
                          const dect_pls_params *P, const float *ew, float *u1, float *u2,
                          dect_report *rep, hipStream_t s)
{
    dect_status st = check_pls_args(nx, ny, xh, xl, P, u1, u2, "dect_pls_decompose");
    if (st) return st;
    std::lock_guard<std::mutex> lk(g_pls_mu);
    PlsWork *W = pls_work();
    const size_t N = (size_t)nx * ny;
    const int nblk = (int)((N + 256 * kPix - 1) / (256 * kPix));
    if ((st = pls_prepare(W, N, nblk))) return st;
    dinv_run(nx, ny, xh, xl, P, u1, u2, (float *)W->b.ptr, s);
    DECT_HIP(hipGetLastError());
    const float *w = ew;
    if (!w) {
        if ((st = W->w.ensure(2 * N * 4))) return st;
        if ((st = edges_into(nx, ny, xl, P->edge_tau, P->edge_eps, (float *)W->w.ptr, W, s)))
            return st;
        w = (const float *)W->w.ptr;
    }
    if (P->mode == DECT_PLS_ATTENUATION)
        return pls_attenuation(nx, ny, xh, xl, P, w, u1, u2, rep, W, nblk, s);
    PlsBufs B;
    B.b = (float *)W->b.ptr;
    B.res = (float *)W->res.ptr;
    B.z = (float *)W->z.ptr;
    B.p0 = (float *)W->p0.ptr;
    B.p1 = (float *)W->p1.ptr;
    B.q = (float *)W->q.ptr;
    B.minv = (float *)W->minv.ptr;
    B.w = nullptr;
    B.m2 = nullptr;
    B.pmax = nullptr;
    B.prz0 = (double *)W->prz0.ptr;
    B.prz1 = (double *)W->prz1.ptr;
    B.prr = (double *)W->prr.ptr;
    B.pbb = (double *)W->pbb.ptr;
    B.ppq = (double *)W->ppq.ptr;
    B.stat = (PcgStatus *)W->stat.ptr;
    return pcg_image_run(nx, ny, P, w, u1, u2, rep, B, s);
}

// ------------------------------------------------ allocation-free form ---
// The work memory of dect_pls_decompose_noalloc: one array per GPU, in the
// code object, sized for kNoAllocMaxPixels pixels.  Host code never passes
// its name to a kernel (on the host the name is not the device address):
// hipGetSymbolAddress gives each device's address once, kept in g_scratch.
constexpr size_t kNoAllocMaxPixels = (size_t)512 * 512;
constexpr size_t kNoAllocBlocks = (kNoAllocMaxPixels + 256 * kPix - 1) / (256 * kPix);
constexpr size_t kScratchBytes =
    16 * 4 * kNoAllocMaxPixels + 10 * 8 * kNoAllocBlocks + 4 * kNoAllocBlocks + (size_t)64 * 1024;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<void *> g_scratch;  // per device id: the array's device address

dect_status scratch_ptr(void **out)
{
    int dev = 0;
    DECT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize((size_t)dev + 1, nullptr);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(DECT_ERR_HIP, std::string("dect_pls_decompose_noalloc: scratch address: ") +
                                          hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return DECT_OK;
}

// Consecutive 256-byte-aligned pieces of one buffer.
struct Carve {
    unsigned char *base;
    size_t off;
    template <class T>
    T *take(size_t n)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = (T *)(base + off);
        off += n * sizeof(T);
        return p;
    }
};

}  // namespace

dect_status pls_decompose_noalloc(int nx, int ny, const float *xh, const float *xl,
                                  const dect_pls_params *P, const float *ew, float *u1,
                                  float *u2, dect_report *rep, hipStream_t s)
{
    dect_status st = check_pls_args(nx, ny, xh, xl, P, u1, u2, "dect_pls_decompose_noalloc");
    if (st) return st;
    if (P->mode != DECT_PLS_IMAGE)
        return fail(DECT_ERR_INVALID_ARG,
                    "dect_pls_decompose_noalloc: image-space mode (DECT_PLS_IMAGE) only");
    const size_t N = (size_t)nx * ny;
    if (N > kNoAllocMaxPixels)
        return fail(DECT_ERR_INVALID_ARG, "dect_pls_decompose_noalloc: at most " +
                                              std::to_string(kNoAllocMaxPixels) +
                                              " pixels, got " + std::to_string(N));
    void *sp = nullptr;
    if ((st = scratch_ptr(&sp))) return st;
    const size_t nblk = (N + 256 * kPix - 1) / (256 * kPix);
    Carve c{(unsigned char *)sp, 0};
    PlsBufs B;
    B.b = c.take<float>(2 * N);
    B.res = c.take<float>(2 * N);
    B.z = c.take<float>(2 * N);
    B.p0 = c.take<float>(2 * N);
    B.p1 = c.take<float>(2 * N);
    B.q = c.take<float>(2 * N);
    B.minv = c.take<float>(N);
    B.w = c.take<float>(2 * N);
    B.m2 = c.take<float>(N);
    B.pmax = c.take<float>(nblk);
    B.prz0 = c.take<double>(2 * nblk);
    B.prz1 = c.take<double>(2 * nblk);
    B.prr = c.take<double>(2 * nblk);
    B.pbb = c.take<double>(2 * nblk);
    B.ppq = c.take<double>(2 * nblk);
    B.stat = c.take<PcgStatus>(2);
    if (c.off > kScratchBytes)
        return fail(DECT_ERR_INVALID_ARG, "dect_pls_decompose_noalloc: scratch too small");
    dinv_run(nx, ny, xh, xl, P, u1, u2, B.b, s);
    DECT_HIP(hipGetLastError());
    const float *w = ew;
    if (!w) {
        if ((st = edges_run(nx, ny, xl, P->edge_tau, P->edge_eps, B.w, B.m2, B.pmax, s)))
            return st;
        w = B.w;
    }
    return pcg_image_run(nx, ny, P, w, u1, u2, rep, B, s);
}

void release_pls_work()
{
    std::lock_guard<std::mutex> lk(g_pls_mu);
    g_pls.clear();
}

}  // namespace dect
