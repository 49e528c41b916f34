// TV-regularised ADM reconstruction (Eq. 10) of both energies on gfx950.
//
// One iteration k, both energies per launch:
//   tv_fused : lambda^k = lambda^{k-1} - xi (grad f^k - z^k)   (Eq. 7, deferred
//              from the previous iteration so grad f^k is computed once),
//              z^{k+1} = shrink(grad f^k - lambda^k / rho, 1/rho) (Eq. 8),
//              G^k = h^k + grad^T(rho (grad f^k - z^{k+1}) - lambda^k) (Eq. 9),
//              with per-block partial sums of TV(f^k), |G|^2, |grad G|^2,
//              |grad f - z|^2 and |f|^2.  G is written straight into the two
//              zero-padded layouts the forward projector reads.
//   fwd      : p = A G^k, |p|^2.
//   scalar   : c^k = |G^k|^2 / (mu |A G^k|^2 + rho |grad G^k|^2).  The BB1
//              step <s,s>/<s,y> of s = -alpha G^k, y = (mu A^T A + rho
//              grad^T grad) s equals c^k, so alpha^{k+1} = c^k and
//              alpha^0 = c^0 (the exact line-search step); logs J^k.
//   update   : f^{k+1} = f^k - alpha^k G^k, r^{k+1} = r^k - alpha^k p (so r
//              stays A f - g without projecting f), |r^{k+1}|^2.
//   adj      : h^{k+1} = mu A^T r^{k+1}.
// Every reduction is a fixed-order tree in FP64: reruns are bitwise equal.
// lambda and z alternate between two buffers (the stencil reads neighbours'
// old values), so a captured graph holds an even/odd pair of iterations.
#include <cmath>
#include <cstring>

#include "common.h"

namespace dect {
namespace {

constexpr int kT = 16;  // tv tile side

struct AdmScalars {
    double alpha;   // step used by the next update
    double c_prev;  // Cauchy step of the previous G
    double rr;      // |r^k|^2 of the current f
    double J;       // last logged objective
    double relchg;  // last relative image change
    double beta;    // Eq. 3 weight of this energy
    int32_t has_prev, stopped, nonfinite_iter, pending;
    int64_t iter;      // iterations completed
    int64_t log_base;  // iteration index of log row 0 for this call
};

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Fixed-order sum over a 256-thread block of NV values; thread t < NV gets
// the t-th total in `out`.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *out)
{
    __shared__ double sh[4][NV];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[wid][i] = v[i];
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        int t = threadIdx.x;
        out[t] = ((sh[0][t] + sh[1][t]) + sh[2][t]) + sh[3][t];
    }
}

// ------------------------------------------------------------- tv_fused ---
// Regions relative to the tile origin (r0, c0): f on rows/cols -2..16 (19),
// w on -1..16 (18), G on -1..15 (17), grad G on the 16x16 tile.
__global__ __launch_bounds__(256) void k_tv_fused(
    const float *__restrict__ f, const float *__restrict__ h, const float *__restrict__ lam_in,
    const float *__restrict__ z_in, float *__restrict__ lam_out, float *__restrict__ z_out,
    float *__restrict__ gpad, float *__restrict__ gpadT, double *__restrict__ partial,
    const AdmScalars *__restrict__ sc, int nx, int ny, float rho, float xi)
{
    const int e = blockIdx.z;
    if (sc[e].stopped) return;
    const bool pending = sc[e].pending != 0;
    __shared__ float sf[19][20];
    __shared__ float swx[18][19], swy[18][19];
    __shared__ float sg[17][18];
    const int r0 = blockIdx.y * kT, c0 = blockIdx.x * kT;
    const size_t N = (size_t)nx * ny;
    const float *fe = f + e * N;
    const float *he = h + e * N;
    const float *lxi = lam_in + (size_t)(2 * e) * N, *lyi = lxi + N;
    const float *zxi = z_in + (size_t)(2 * e) * N, *zyi = zxi + N;
    float *lxo = lam_out + (size_t)(2 * e) * N, *lyo = lxo + N;
    float *zxo = z_out + (size_t)(2 * e) * N, *zyo = zxo + N;
    const float inv_rho = 1.0f / rho;

    for (int i = threadIdx.x; i < 19 * 19; i += 256) {
        int rr = i / 19, cc = i % 19;
        int r = r0 - 2 + rr, c = c0 - 2 + cc;
        sf[rr][cc] = (r >= 0 && r < ny && c >= 0 && c < nx) ? fe[(size_t)r * nx + c] : 0.f;
    }
    __syncthreads();

    double tv = 0.0, pres = 0.0, ff = 0.0;
    for (int i = threadIdx.x; i < 18 * 18; i += 256) {
        int rr = i / 18, cc = i % 18;
        int r = r0 - 1 + rr, c = c0 - 1 + cc;
        float wx = 0.f, wy = 0.f;
        if (r >= 0 && r < ny && c >= 0 && c < nx) {
            size_t o = (size_t)r * nx + c;
            float fc = sf[rr + 1][cc + 1];
            float dx = c >= 1 ? fc - sf[rr + 1][cc] : 0.f;
            float dy = r >= 1 ? fc - sf[rr][cc + 1] : 0.f;
            float lx = lxi[o], ly = lyi[o];
            if (pending) {
                lx -= xi * (dx - zxi[o]);
                ly -= xi * (dy - zyi[o]);
            }
            float vx = dx - lx / rho, vy = dy - ly / rho;
            float n = sqrtf(vx * vx + vy * vy);
            float s = n > inv_rho ? (n - inv_rho) / n : 0.f;
            float zx = s * vx, zy = s * vy;
            wx = rho * (dx - zx) - lx;
            wy = rho * (dy - zy) - ly;
            if (rr >= 1 && rr <= kT && cc >= 1 && cc <= kT) {
                lxo[o] = lx;
                lyo[o] = ly;
                zxo[o] = zx;
                zyo[o] = zy;
                tv += (double)sqrtf(dx * dx + dy * dy);
                double ex = (double)dx - zx, ey = (double)dy - zy;
                pres += ex * ex + ey * ey;
                ff += (double)fc * fc;
            }
        }
        swx[rr][cc] = wx;
        swy[rr][cc] = wy;
    }
    __syncthreads();

    // G = h + grad^T w on rows/cols -1..15
    for (int i = threadIdx.x; i < 17 * 17; i += 256) {
        int rr = i / 17, cc = i % 17;
        int r = r0 - 1 + rr, c = c0 - 1 + cc;
        float gv = 0.f;
        if (r >= 0 && r < ny && c >= 0 && c < nx) {
            float s = he[(size_t)r * nx + c];
            if (c >= 1) s += swx[rr][cc];
            if (c + 1 <= nx - 1) s -= swx[rr][cc + 1];
            if (r >= 1) s += swy[rr][cc];
            if (r + 1 <= ny - 1) s -= swy[rr + 1][cc];
            gv = s;
        }
        sg[rr][cc] = gv;
    }
    __syncthreads();

    double gg = 0.0, gradg = 0.0;
    const int pnx = nx + 2 * kPad, pny = ny + 2 * kPad;
    const size_t poff = (size_t)e * pnx * pny;
    {
        int rr = threadIdx.x / kT, cc = threadIdx.x % kT;
        int r = r0 + rr, c = c0 + cc;
        if (r < ny && c < nx) {
            float gv = sg[rr + 1][cc + 1];
            float gx = c >= 1 ? gv - sg[rr + 1][cc] : 0.f;
            float gy = r >= 1 ? gv - sg[rr][cc + 1] : 0.f;
            gg = (double)gv * gv;
            gradg = (double)gx * gx + (double)gy * gy;
            gpad[poff + (size_t)(r + kPad) * pnx + c + kPad] = gv;
        }
        // transposed write: thread (rr, cc) writes element (cc, rr) of the tile
        int rt = r0 + cc, ct = c0 + rr;
        if (rt < ny && ct < nx) gpadT[poff + (size_t)(ct + kPad) * pny + rt + kPad] = sg[cc + 1][rr + 1];
    }
    double v[5] = {tv, gg, gradg, pres, ff};
    __shared__ double outv[5];
    block_sum<5>(v, outv);
    __syncthreads();
    if (threadIdx.x < 5)
        partial[((size_t)e * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x) * 5 +
                threadIdx.x] = outv[threadIdx.x];
}

// ------------------------------------------------------------- scalar ---
// One block per energy.  nb_tv/nb_fwd: partial counts per energy.
__global__ __launch_bounds__(256) void k_scalar(AdmScalars *__restrict__ sc,
                                                const double *__restrict__ p_tv, int nb_tv,
                                                const double *__restrict__ p_fwd, int nb_fwd,
                                                double *__restrict__ log, int log_rows,
                                                double mu, double rho)
{
    const int e = blockIdx.x;
    AdmScalars &s = sc[e];
    if (s.stopped) return;
    double v[6] = {0, 0, 0, 0, 0, 0};
    const double *pt = p_tv + (size_t)e * nb_tv * 5;
    for (int i = threadIdx.x; i < nb_tv; i += 256)
#pragma unroll
        for (int j = 0; j < 5; ++j) v[j] += pt[(size_t)i * 5 + j];
    const double *pf = p_fwd + (size_t)e * nb_fwd;
    for (int i = threadIdx.x; i < nb_fwd; i += 256) v[5] += pf[i];
    __shared__ double tot[6];
    block_sum<6>(v, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double tvf = tot[0], gg = tot[1], gradg = tot[2], ff = tot[4], pp = tot[5];
    const double den = mu * pp + rho * gradg;
    double c = den > 0.0 ? gg / den : (s.has_prev ? s.c_prev : 0.0);
    double alpha = s.has_prev ? s.c_prev : c;
    const double J = tvf + 0.5 * mu * s.rr;
    const double relchg = ff > 0.0 ? alpha * sqrt(gg) / sqrt(ff) : (gg > 0.0 ? INFINITY : 0.0);
    const int64_t k = s.iter;
    int64_t row = k - s.log_base;
    if (log && row >= 0 && row < log_rows) {
        log[row * 4 + e] = J;
        log[row * 4 + 2 + e] = alpha;
    }
    s.J = J;
    s.alpha = alpha;
    s.c_prev = c;
    s.has_prev = 1;
    s.relchg = relchg;
    if (!isfinite(J) || !isfinite(alpha) || !isfinite(gg) || !isfinite(pp)) {
        s.nonfinite_iter = (int32_t)(k + 1);
        s.stopped = 1;
        s.alpha = 0.0;
    }
}

// ------------------------------------------------------------- update ---
// blocks [0, nbi): f -= alpha G (image); blocks [nbi, nbi+nbs): r -= alpha p
// and per-block |r|^2.
__global__ __launch_bounds__(256) void k_update(float *__restrict__ f,
                                                const float *__restrict__ gpad,
                                                float *__restrict__ r, const float *__restrict__ p,
                                                double *__restrict__ p_rr, AdmScalars *__restrict__ sc,
                                                int nx, int ny, int M, int nbi, int nbs)
{
    const int e = blockIdx.y;
    AdmScalars &s = sc[e];
    if (s.stopped) return;
    const float alpha = (float)s.alpha;
    const size_t N = (size_t)nx * ny;
    if ((int)blockIdx.x < nbi) {
        const int pnx = nx + 2 * kPad, pny = ny + 2 * kPad;
        const float *ge = gpad + (size_t)e * pnx * pny;
        float *fe = f + e * N;
        for (int j = 0; j < 4; ++j) {
            size_t i = ((size_t)blockIdx.x * 4 + j) * 256 + threadIdx.x;
            if (i < N) {
                int rr = (int)(i / nx), cc = (int)(i % nx);
                fe[i] -= alpha * ge[(size_t)(rr + kPad) * pnx + cc + kPad];
            }
        }
        return;
    }
    const int bs = blockIdx.x - nbi;
    float *re = r + (size_t)e * M;
    const float *pe = p + (size_t)e * M;
    double acc[1] = {0.0};
    for (int j = 0; j < 4; ++j) {
        size_t i = ((size_t)bs * 4 + j) * 256 + threadIdx.x;
        if ((int)i < M) {
            float nr = re[i] - alpha * pe[i];
            re[i] = nr;
            acc[0] += (double)nr * nr;
        }
    }
    __shared__ double tot[1];
    block_sum<1>(acc, tot);
    __syncthreads();
    if (threadIdx.x == 0) p_rr[(size_t)e * nbs + bs] = tot[0];
}

// |r|^2 of every energy from the residual partials (fixed order).  After an
// update (step != 0) it also counts the iteration, marks the deferred
// multiplier step as pending and applies the relative-change stop rule.
__global__ __launch_bounds__(256) void k_rr(AdmScalars *__restrict__ sc,
                                            const double *__restrict__ p_rr, int nbs, int step,
                                            double tol)
{
    const int e = blockIdx.x;
    if (step && sc[e].stopped) return;
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < nbs; i += 256) v[0] += p_rr[(size_t)e * nbs + i];
    __shared__ double tot[1];
    block_sum<1>(v, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;
    AdmScalars &s = sc[e];
    s.rr = tot[0];
    if (step) {
        s.pending = 1;
        s.iter += 1;
        if (tol > 0.0 && s.relchg < tol) s.stopped = 1;
    }
}

// ------------------------------------------------------------- set-up ---
// f = beta x0 (or 0), lambda = z = 0 for both parities.
__global__ __launch_bounds__(256) void k_init_image(float *__restrict__ f,
                                                    const float *__restrict__ x0h,
                                                    const float *__restrict__ x0l, float bh,
                                                    float bl, float *__restrict__ lam,
                                                    float *__restrict__ z, size_t N)
{
    const int e = blockIdx.y;
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const float *x0 = e == 0 ? x0h : x0l;
    f[e * N + i] = x0 ? (e == 0 ? bh : bl) * x0[i] : 0.f;
    for (int q = 0; q < 4; ++q) {  // [parity][energy][comp]: zero all of them
        lam[(size_t)q * N * 2 + (size_t)e * N + i] = 0.f;
        z[(size_t)q * N * 2 + (size_t)e * N + i] = 0.f;
    }
}

// r = r - beta m; per-block |r|^2.
__global__ __launch_bounds__(256) void k_init_resid(float *__restrict__ r,
                                                    const float *__restrict__ mh,
                                                    const float *__restrict__ ml, float bh,
                                                    float bl, int M, double *__restrict__ p_rr,
                                                    int nbs)
{
    const int e = blockIdx.y;
    const float *m = e == 0 ? mh : ml;
    const float b = e == 0 ? bh : bl;
    double acc[1] = {0.0};
    for (int j = 0; j < 4; ++j) {
        size_t i = ((size_t)blockIdx.x * 4 + j) * 256 + threadIdx.x;
        if ((int)i < M) {
            float nr = r[(size_t)e * M + i] - b * m[i];
            r[(size_t)e * M + i] = nr;
            acc[0] += (double)nr * nr;
        }
    }
    __shared__ double tot[1];
    block_sum<1>(acc, tot);
    __syncthreads();
    if (threadIdx.x == 0) p_rr[(size_t)e * nbs + blockIdx.x] = tot[0];
}

__global__ void k_init_scalars(AdmScalars *__restrict__ sc, double bh, double bl)
{
    int e = threadIdx.x;
    if (e >= 2) return;
    AdmScalars s;
    memset(&s, 0, sizeof(s));
    s.beta = e == 0 ? bh : bl;
    sc[e] = s;
}

__global__ void k_set_log_base(AdmScalars *__restrict__ sc)
{
    int e = threadIdx.x;
    if (e < 2) sc[e].log_base = sc[e].iter;
}

// TV(f) per block for the final objective.
__global__ __launch_bounds__(256) void k_tv_only(const float *__restrict__ f,
                                                 double *__restrict__ partial, int nx, int ny)
{
    const int e = blockIdx.y;
    const size_t N = (size_t)nx * ny;
    double v[1] = {0.0};
    for (int j = 0; j < 4; ++j) {
        size_t i = ((size_t)blockIdx.x * 4 + j) * 256 + threadIdx.x;
        if (i < N) {
            int r = (int)(i / nx), c = (int)(i % nx);
            float fc = f[e * N + i];
            float dx = c >= 1 ? fc - f[e * N + i - 1] : 0.f;
            float dy = r >= 1 ? fc - f[e * N + i - nx] : 0.f;
            v[0] += (double)sqrtf(dx * dx + dy * dy);
        }
    }
    __shared__ double tot[1];
    block_sum<1>(v, tot);
    __syncthreads();
    if (threadIdx.x == 0) partial[(size_t)e * gridDim.x + blockIdx.x] = tot[0];
}

__global__ __launch_bounds__(256) void k_final_J(AdmScalars *__restrict__ sc,
                                                 const double *__restrict__ p_tv, int nb,
                                                 double *__restrict__ log, int log_rows, double mu)
{
    const int e = blockIdx.x;
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < nb; i += 256) v[0] += p_tv[(size_t)e * nb + i];
    __shared__ double tot[1];
    block_sum<1>(v, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;
    AdmScalars &s = sc[e];
    double J = tot[0] + 0.5 * mu * s.rr;
    int64_t row = s.iter - s.log_base;
    if (log && row >= 0 && row < log_rows) {
        log[row * 4 + e] = J;
        log[row * 4 + 2 + e] = s.alpha;
    }
    s.J = J;
}

// x = f / beta
__global__ __launch_bounds__(256) void k_output(const float *__restrict__ f,
                                                float *__restrict__ xh, float *__restrict__ xl,
                                                float bh, float bl, size_t N)
{
    const int e = blockIdx.y;
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    if (e == 0) xh[i] = f[i] / bh;
    else xl[i] = f[N + i] / bl;
}

}  // namespace
}  // namespace dect

// ------------------------------------------------------------ the state ---
struct dect_adm_state {
    dect::GeomTables *t = nullptr;
    int device = 0;
    bool started = false;
    double mu = 0, rho = 0, xi = 0, bh = 1, bl = 1;
    int nvg = 1, nb_tv = 0, nb_fwd = 0, nbi = 0, nbs = 0, nb_img = 0;
    dect::DevBuf f, h, r, p, lam, z, gpad, gpadT, p_tv, p_fwd, p_rr, adjpart, adjcnt, sc, logbuf,
        p_tvo;
    void *graph_log = nullptr;
    size_t graph_log_bytes = 0;
    double graph_tol = -1.0;
    hipGraphExec_t graph = nullptr;
    hipStream_t cap = nullptr;
    int parity = 0;  // lambda/z buffer holding the current values
    ~dect_adm_state()
    {
        if (graph) (void)hipGraphExecDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace dect {

static dect_status state_alloc(dect_adm_state *S, const dect_geometry *g)
{
    dect_status st = get_tables(g, &S->t);
    if (st != DECT_OK) return st;
    DECT_HIP(hipGetDevice(&S->device));
    const GeomTables &t = *S->t;
    const size_t N = (size_t)g->nx * g->ny, M = (size_t)g->n_views * g->n_bins;
    const size_t P = (size_t)(g->nx + 2 * kPad) * (g->ny + 2 * kPad);
    S->nvg = adj_groups(t, 2);
    S->nb_tv = ((g->nx + kT - 1) / kT) * ((g->ny + kT - 1) / kT);
    S->nb_fwd = fwd_blocks(t);
    S->nbi = (int)((N + 1023) / 1024);
    S->nbs = (int)((M + 1023) / 1024);
    S->nb_img = S->nbi;
    if ((st = S->f.ensure(2 * N * 4)) || (st = S->h.ensure(2 * N * 4)) ||
        (st = S->r.ensure(2 * M * 4)) || (st = S->p.ensure(2 * M * 4)) ||
        (st = S->lam.ensure(8 * N * 4)) || (st = S->z.ensure(8 * N * 4)) ||
        (st = S->gpad.ensure(2 * P * 4, true)) || (st = S->gpadT.ensure(2 * P * 4, true)) ||
        (st = S->p_tv.ensure((size_t)2 * S->nb_tv * 5 * 8)) ||
        (st = S->p_fwd.ensure((size_t)2 * S->nb_fwd * 8)) ||
        (st = S->p_rr.ensure((size_t)2 * S->nbs * 8)) ||
        (st = S->p_tvo.ensure((size_t)2 * S->nbi * 8)) ||
        (st = S->adjpart.ensure(std::max<size_t>(1, adj_partial_floats(t, 2)) * 4)) ||
        (st = S->adjcnt.ensure(adj_counters(t, 2) * sizeof(int), true)) ||
        (st = S->sc.ensure(2 * sizeof(AdmScalars))))
        return st;
    return DECT_OK;
}

// Launch one iteration; `par` selects the lambda/z buffers holding the
// current values.
static dect_status launch_iter(dect_adm_state *S, int par, double tol, hipStream_t s)
{
    const GeomTables &t = *S->t;
    const int nx = t.key.nx, ny = t.key.ny;
    const size_t N = (size_t)nx * ny;
    const int M = t.key.V * t.key.B;
    float *lam = (float *)S->lam.ptr, *z = (float *)S->z.ptr;
    float *lam_in = lam + (size_t)par * 4 * N, *lam_out = lam + (size_t)(1 - par) * 4 * N;
    float *z_in = z + (size_t)par * 4 * N, *z_out = z + (size_t)(1 - par) * 4 * N;
    AdmScalars *sc = (AdmScalars *)S->sc.ptr;
    dim3 gtv((nx + kT - 1) / kT, (ny + kT - 1) / kT, 2);
    hipLaunchKernelGGL(k_tv_fused, gtv, dim3(256), 0, s, (const float *)S->f.ptr,
                       (const float *)S->h.ptr, lam_in, z_in, lam_out, z_out,
                       (float *)S->gpad.ptr, (float *)S->gpadT.ptr, (double *)S->p_tv.ptr, sc,
                       nx, ny, (float)S->rho, (float)S->xi);
    DECT_HIP(hipGetLastError());
    dect_status st = launch_fwd(t, (const float *)S->gpad.ptr, (const float *)S->gpadT.ptr,
                                (float *)S->p.ptr, 2, 1.0f, (double *)S->p_fwd.ptr, s);
    if (st) return st;
    hipLaunchKernelGGL(k_scalar, dim3(2), dim3(256), 0, s, sc, (const double *)S->p_tv.ptr,
                       S->nb_tv, (const double *)S->p_fwd.ptr, S->nb_fwd,
                       (double *)S->logbuf.ptr, (int)(S->logbuf.bytes / 32), S->mu, S->rho);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_update, dim3(S->nbi + S->nbs, 2), dim3(256), 0, s, (float *)S->f.ptr,
                       (const float *)S->gpad.ptr, (float *)S->r.ptr, (const float *)S->p.ptr,
                       (double *)S->p_rr.ptr, sc, nx, ny, M, S->nbi, S->nbs);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_rr, dim3(2), dim3(256), 0, s, sc, (const double *)S->p_rr.ptr, S->nbs, 1,
                       tol);
    DECT_HIP(hipGetLastError());
    return launch_adj(t, (const float *)S->r.ptr, (float *)S->h.ptr, (float *)S->adjpart.ptr,
                      (int *)S->adjcnt.ptr, 2, (float)S->mu, s);
}

static dect_status adm_start(dect_adm_state *S, const dect_geometry *g, const float *mh,
                             const float *ml, const dect_adm_params *P, const float *x0h,
                             const float *x0l, hipStream_t s)
{
    const GeomTables &t = *S->t;
    const size_t N = (size_t)g->nx * g->ny;
    const int M = g->n_views * g->n_bins;
    S->mu = P->mu;
    S->rho = P->rho;
    S->xi = P->xi;
    S->bh = P->beta_high;
    S->bl = P->beta_low;
    S->parity = 0;
    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, s, (AdmScalars *)S->sc.ptr, S->bh,
                       S->bl);
    DECT_HIP(hipGetLastError());
    dim3 gi((unsigned)((N + 255) / 256), 2);
    hipLaunchKernelGGL(k_init_image, gi, dim3(256), 0, s, (float *)S->f.ptr, x0h, x0l,
                       (float)S->bh, (float)S->bl, (float *)S->lam.ptr, (float *)S->z.ptr, N);
    DECT_HIP(hipGetLastError());
    // r = A f - beta m (the padded G buffers serve as f's padded copies here)
    dect_status st = launch_pad(t, (const float *)S->f.ptr, (float *)S->gpad.ptr,
                                (float *)S->gpadT.ptr, 2, s);
    if (st) return st;
    if ((st = launch_fwd(t, (const float *)S->gpad.ptr, (const float *)S->gpadT.ptr,
                         (float *)S->r.ptr, 2, 1.0f, nullptr, s)))
        return st;
    hipLaunchKernelGGL(k_init_resid, dim3(S->nbs, 2), dim3(256), 0, s, (float *)S->r.ptr, mh, ml,
                       (float)S->bh, (float)S->bl, M, (double *)S->p_rr.ptr, S->nbs);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_rr, dim3(2), dim3(256), 0, s, (AdmScalars *)S->sc.ptr,
                       (const double *)S->p_rr.ptr, S->nbs, 0, 0.0);
    DECT_HIP(hipGetLastError());
    if ((st = launch_adj(t, (const float *)S->r.ptr, (float *)S->h.ptr, (float *)S->adjpart.ptr,
                         (int *)S->adjcnt.ptr, 2, (float)S->mu, s)))
        return st;
    S->started = true;
    return DECT_OK;
}

static dect_status build_graph(dect_adm_state *S, double tol)
{
    if (S->graph) {
        (void)hipGraphExecDestroy(S->graph);
        S->graph = nullptr;
    }
    if (!S->cap) DECT_HIP(hipStreamCreateWithFlags(&S->cap, hipStreamNonBlocking));
    DECT_HIP(hipStreamBeginCapture(S->cap, hipStreamCaptureModeThreadLocal));
    dect_status st = launch_iter(S, 0, tol, S->cap);
    if (!st) st = launch_iter(S, 1, tol, S->cap);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(S->cap, &graph);
    if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(DECT_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&S->graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(DECT_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    return DECT_OK;
}

static std::mutex g_adm_mu;
static std::vector<std::unique_ptr<dect_adm_state>> g_tmp_states;

dect_status adm_tv(const dect_geometry *g, const float *mh, const float *ml,
                   const dect_adm_params *P, float *xh, float *xl, dect_adm_state *state,
                   dect_report *rep, hipStream_t s)
{
    if (!P || !mh || !ml || !xh || !xl)
        return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv: null argument");
    if (!(P->mu > 0) || !(P->rho > 0) || !(P->xi >= 0) || !(P->beta_high > 0) ||
        !(P->beta_low > 0) || P->max_iter < 0 || !(P->tol >= 0) || !std::isfinite(P->mu) ||
        !std::isfinite(P->rho) || !std::isfinite(P->xi))
        return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv: invalid parameters");
    dect_status st = validate_geometry(g);
    if (st) return st;
    std::lock_guard<std::mutex> lk(g_adm_mu);
    dect_adm_state *S = state;
    if (!S) {
        // a reusable scratch state per geometry and device
        GeomTables *t = nullptr;
        if ((st = get_tables(g, &t))) return st;
        for (auto &u : g_tmp_states)
            if (u->t == t) S = u.get();
        if (!S) {
            g_tmp_states.push_back(std::make_unique<dect_adm_state>());
            S = g_tmp_states.back().get();
            if ((st = state_alloc(S, g))) {
                g_tmp_states.pop_back();
                return st;
            }
        }
        S->started = false;
    } else {
        GeomTables *t = nullptr;
        if ((st = get_tables(g, &t))) return st;
        if (t != S->t) return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv: state was made for another geometry");
        if (S->started && (S->mu != P->mu || S->rho != P->rho || S->xi != P->xi ||
                           S->bh != P->beta_high || S->bl != P->beta_low))
            return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv: parameters differ from the state's run");
    }
    const size_t N = (size_t)g->nx * g->ny;
    const int K = P->max_iter;
    const size_t log_rows = (size_t)K + 1;
    // the device log keeps at least 4096 rows so that calls of different
    // lengths reuse it (and the captured graph that points at it)
    if ((st = S->logbuf.ensure(std::max<size_t>(log_rows, 4096) * 4 * sizeof(double)))) return st;
    if (!S->started) {
        const bool warm = (P->flags & DECT_WARM_START) != 0;
        if ((st = adm_start(S, g, mh, ml, P, warm ? xh : nullptr, warm ? xl : nullptr, s)))
            return st;
    }
    hipLaunchKernelGGL(k_set_log_base, dim3(1), dim3(64), 0, s, (AdmScalars *)S->sc.ptr);
    DECT_HIP(hipGetLastError());
    // the log buffer and tol are baked into the graph's kernel arguments:
    // rebuild only when they change
    if (K >= 2 && (!S->graph || S->graph_log != S->logbuf.ptr ||
                   S->graph_log_bytes != S->logbuf.bytes || S->graph_tol != P->tol)) {
        if ((st = build_graph(S, P->tol))) return st;
        S->graph_log = S->logbuf.ptr;
        S->graph_log_bytes = S->logbuf.bytes;
        S->graph_tol = P->tol;
    }
    int k = 0;
    if (S->parity == 1 && K > 0) {  // realign so the graph starts on parity 0
        if ((st = launch_iter(S, 1, P->tol, s))) return st;
        S->parity = 0;
        ++k;
    }
    for (; k + 2 <= K; k += 2) DECT_HIP(hipGraphLaunch(S->graph, s));
    if (k < K) {
        if ((st = launch_iter(S, 0, P->tol, s))) return st;
        S->parity = 1;
        ++k;
    }
    // outputs and the final objective
    dim3 go((unsigned)((N + 255) / 256), 2);
    hipLaunchKernelGGL(k_output, go, dim3(256), 0, s, (const float *)S->f.ptr, xh, xl,
                       (float)S->bh, (float)S->bl, N);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_tv_only, dim3(S->nbi, 2), dim3(256), 0, s, (const float *)S->f.ptr,
                       (double *)S->p_tvo.ptr, g->nx, g->ny);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_final_J, dim3(2), dim3(256), 0, s, (AdmScalars *)S->sc.ptr,
                       (const double *)S->p_tvo.ptr, S->nbi, (double *)S->logbuf.ptr,
                       (int)log_rows, S->mu);
    DECT_HIP(hipGetLastError());
    if (rep || P->log) {
        DECT_HIP(hipStreamSynchronize(s));
        AdmScalars hs[2];
        DECT_HIP(hipMemcpy(hs, S->sc.ptr, sizeof(hs), hipMemcpyDeviceToHost));
        if (P->log)
            DECT_HIP(hipMemcpy(P->log, S->logbuf.ptr, log_rows * 4 * sizeof(double),
                               hipMemcpyDeviceToHost));
        dect_status rs = DECT_OK;
        int nf = 0;
        for (int e = 0; e < 2; ++e)
            if (hs[e].nonfinite_iter) nf = nf ? std::min(nf, hs[e].nonfinite_iter) : hs[e].nonfinite_iter;
        if (nf) rs = DECT_ERR_NONFINITE;
        if (rep) {
            rep->iters = (int32_t)std::max(hs[0].iter - hs[0].log_base, hs[1].iter - hs[1].log_base);
            rep->objective = hs[0].J + hs[1].J;
            rep->rel_change = std::max(hs[0].relchg, hs[1].relchg);
            rep->pcg_residual = 0.0;
            rep->status = rs;
        }
        if (rs) return fail(rs, "dect_adm_tv: non-finite value at iteration " + std::to_string(nf));
    }
    return DECT_OK;
}

dect_status adm_state_create(const dect_geometry *g, dect_adm_state **out)
{
    if (!out) return fail(DECT_ERR_INVALID_ARG, "state output pointer is NULL");
    auto S = std::make_unique<dect_adm_state>();
    dect_status st = state_alloc(S.get(), g);
    if (st) return st;
    *out = S.release();
    return DECT_OK;
}

dect_status adm_state_destroy(dect_adm_state *S)
{
    delete S;
    return DECT_OK;
}

void release_adm_states()
{
    std::lock_guard<std::mutex> lk(g_adm_mu);
    g_tmp_states.clear();
}

}  // namespace dect
