// TV-regularised ADM reconstruction (Eq. 10) of both energies on gfx950.
//
// One iteration k, both energies per launch:
//   tv_fused : lambda^k = lambda^{k-1} - xi (grad f^k - z^k)   (Eq. 7, deferred
//              from the previous iteration so grad f^k is computed once),
//              z^{k+1} = shrink(grad f^k - lambda^k / rho, 1/rho) (Eq. 8),
//              G^k = h^k + grad^T(rho (grad f^k - z^{k+1}) - lambda^k) (Eq. 9),
//              with per-block partial sums of TV(f^k), |G|^2, |grad G|^2,
//              |grad f - z|^2, |f|^2, <G^{k-1}, h^k> and <G^k, h^k>.  G is
//              written straight into the two zero-padded layouts the forward
//              projector reads (G^{k-1} is read at each pixel first).
//   fwd      : p = A G^k, |p|^2.
//   scalar   : |r^k|^2 from the previous update's partials; alpha^0 = |G^0|^2
//              / (mu |A G^0|^2 + rho |grad G^0|^2) (the exact line-search
//              step), then the BB1 step <s,s>/<s,y> of s = -alpha G^{k-1}, y
//              = h^k - h^{k-1} + rho grad^T grad s: alpha |G^{k-1}|^2 /
//              (<G^{k-1}, h^{k-1}> - <G^{k-1}, h^k> + alpha rho |grad
//              G^{k-1}|^2), kept when the denominator is not positive; logs
//              J^k, counts the iteration and applies the relative-change stop
//              rule (effective after this update).
//   update   : f^{k+1} = f^k - alpha^k G^k, r^{k+1} = r^k - alpha^k p (so r
//              stays A f - g without projecting f), partials of |r^{k+1}|^2.
//   adj      : h^{k+1} = mu A^T r^{k+1}.
// Every reduction is a fixed-order tree in FP64: reruns are bitwise equal.
// lambda and z alternate between two buffers (the stencil reads neighbours'
// old values), so iterations are captured per starting parity: graphs of 8,
// 2 and 1 iterations for each.
#include <cmath>
#include <cstring>

#include "adm_device.h"
#include "xcd.h"

namespace dect {
namespace {

// ------------------------------------------------------------- kernels ---
// TV stencil: one block per tile of kTX x kTY pixels and energy (tile index
// = energy * tiles per energy + tile row * tile columns + tile column, also
// the slot of its partial sums), taken in XCD order (each XCD a band of tile
// rows, whose halos its blocks share).
template <bool COUPLED>
__global__ __launch_bounds__(256) void k_tv_fused(
    const float *__restrict__ f, const float *__restrict__ hpart, int nvg, float mu,
    const float *__restrict__ lam_in,
    const float *__restrict__ z_in, float *__restrict__ lam_out, float *__restrict__ z_out,
    float *__restrict__ gpad, float *__restrict__ gpadT, double *__restrict__ partial,
    const AdmScalars *__restrict__ sc, int nx, int ny, float rho, float xi, int tiles_x,
    int tiles_y)
{
    const unsigned tpe = (unsigned)(tiles_x * tiles_y);
    const unsigned tile = xcd_order(blockIdx.x, gridDim.x);
    const int e = (int)(tile / tpe), tl = (int)(tile % tpe);
    if (sc[e].stopped || sc[e].stop_next) return;
    const size_t N = (size_t)nx * ny;
    AdmImg m{f + e * N,
             hpart + (size_t)e * 2 * nvg * N,
             lam_in + (2 * e) * N,
             lam_in + (2 * e + 1) * N,
             z_in + (2 * e) * N,
             z_in + (2 * e + 1) * N,
             lam_out + (2 * e) * N,
             lam_out + (2 * e + 1) * N,
             z_out + (2 * e) * N,
             z_out + (2 * e + 1) * N,
             gpad + e,
             gpadT + e,
             f + 2 * N + e * N,
             2 * nvg,
             mu};
    if constexpr (COUPLED) {
        const int o = 1 - e;
        m.f2 = f + o * N;
        m.flo2 = f + 2 * N + o * N;
        m.lxi2 = lam_in + (2 * o) * N;
        m.lyi2 = lam_in + (2 * o + 1) * N;
        m.zxi2 = z_in + (2 * o) * N;
        m.zyi2 = z_in + (2 * o + 1) * N;
        m.pending2 = sc[o].pending != 0;
        m.record_tv = e == 0;
    }
    tv_tile<COUPLED>(tl / tiles_x * kTY, tl % tiles_x * kTX, m, partial + (size_t)tile * kTvParts,
                     sc[e].pending != 0, nx, ny, rho, xi);
}

// One block per energy.  nb_tv/nb_fwd: partial counts per energy.
__global__ __launch_bounds__(256) void k_scalar(AdmScalars *__restrict__ sc,
                                                const double *__restrict__ p_tv, int nb_tv,
                                                const double *__restrict__ p_fwd, int nb_fwd,
                                                double *__restrict__ log, int log_rows,
                                                double mu, double rho, int nonneg,
                                                const double *__restrict__ p_rr, int nbs,
                                                double tol, int step_rule,
                                                const double *__restrict__ p_yy, int nbi)
{
    const int e = blockIdx.x;
    scalar_energy(sc[e], p_tv + (size_t)e * nb_tv * kTvParts, nb_tv, p_fwd + (size_t)e * nb_fwd, nb_fwd,
                  log, log_rows, e, mu, rho, nonneg != 0, nonneg == 0,
                  p_rr + (size_t)e * nbs, nbs, tol, step_rule, p_yy + (size_t)e * nbi, nbi);
}

// ------------------------------------------------ non-negative variant ---
// The projected step (nn_step_chunk), |grad s|^2 and s in both layouts
// (nn_grad_chunk), r += A s (nn_resid_chunk) and the step's scalars
// (nn_rr_energy), one block per chunk and energy.
__global__ __launch_bounds__(256) void k_nn_step(float *__restrict__ f,
                                                 const float *__restrict__ gpad,
                                                 float *__restrict__ gpadT,
                                                 const AdmScalars *__restrict__ sc,
                                                 double *__restrict__ p_ss,
                                                 double *__restrict__ p_ff, int nx, int ny,
                                                 int nbi)
{
    const int e = blockIdx.y;
    if (sc[e].stopped) return;
    const size_t N = (size_t)nx * ny;
    nn_step_chunk(blockIdx.x, e, f + e * N, f + 2 * N + e * N, gpad, gpadT, sc[e].alpha,
                  p_ss + (size_t)e * nbi, p_ff + (size_t)e * nbi, nx, ny);
}

// |grad s|^2 partials (backward differences of Eq. 2) and s copied into the
// normal padded layout, so that the forward projector reads s in both.
__global__ __launch_bounds__(256) void k_nn_grad(float *__restrict__ gpad,
                                                 const float *__restrict__ gpadT,
                                                 const AdmScalars *__restrict__ sc,
                                                 double *__restrict__ p_gs, int nx, int ny,
                                                 int nbi)
{
    const int e = blockIdx.y;
    if (sc[e].stopped) return;
    nn_grad_chunk(blockIdx.x, e, gpad, gpadT, p_gs + (size_t)e * nbi, nx, ny);
}

// (r + rlo) += (p + plo) = A s in FP64; partial |r|^2.
__global__ __launch_bounds__(256) void k_nn_resid(float *__restrict__ r,
                                                  const float *__restrict__ p,
                                                  const AdmScalars *__restrict__ sc,
                                                  double *__restrict__ p_rr, int M, int nbs)
{
    const int e = blockIdx.y;
    if (sc[e].stopped) return;
    const size_t Ms = (size_t)M;
    nn_resid_chunk(blockIdx.x, r + e * Ms, r + 2 * Ms + e * Ms, p + e * Ms, p + 2 * Ms + e * Ms,
                   p_rr + (size_t)e * nbs, M);
}

// |r|^2, <s,s>, <s,y> = mu |A s|^2 + rho |grad s|^2 and |s| / |f| from the
// partials; counts the iteration, marks the deferred multiplier step and
// applies the relative-change stop rule.
__global__ __launch_bounds__(256) void k_nn_rr(AdmScalars *__restrict__ sc,
                                               const double *__restrict__ p_rr, int nbs,
                                               const double *__restrict__ p_ss,
                                               const double *__restrict__ p_ff,
                                               const double *__restrict__ p_gs, int nbi,
                                               const double *__restrict__ p_as, int nb_fwd,
                                               double mu, double rho, double tol)
{
    const int e = blockIdx.x;
    nn_rr_energy(sc[e], p_rr + (size_t)e * nbs, nbs, p_ss + (size_t)e * nbi,
                 p_ff + (size_t)e * nbi, p_gs + (size_t)e * nbi, nbi, p_as + (size_t)e * nb_fwd,
                 nb_fwd, mu, rho, tol);
}

// blocks [0, nbi): f -= alpha G (image); blocks [nbi, nbi+nbs): r -= alpha p
// and per-block |r|^2.  f, r and p hold their low parts after the two
// energies' high parts ([4][N], [4][M]).
__global__ __launch_bounds__(256) void k_update(float *__restrict__ f,
                                                const float *__restrict__ gpad,
                                                float *__restrict__ r, const float *__restrict__ p,
                                                double *__restrict__ p_rr, AdmScalars *__restrict__ sc,
                                                int nx, int ny, int M, int nbi, int nbs)
{
    const int e = blockIdx.y;
    if (sc[e].stopped) return;
    const size_t N = (size_t)nx * ny;
    const size_t Ms = (size_t)M;
    update_chunk(blockIdx.x, f + e * N, f + 2 * N + e * N, gpad + e, r + e * Ms,
                 r + 2 * Ms + e * Ms, p + e * Ms, p + 2 * Ms + e * Ms, p_rr + (size_t)e * nbs,
                 sc[e].alpha, nx, ny, M, nbi);
}

__global__ __launch_bounds__(256) void k_rr(AdmScalars *__restrict__ sc,
                                            const double *__restrict__ p_rr, int nbs, int step,
                                            double tol)
{
    const int e = blockIdx.x;
    rr_energy(sc[e], p_rr + (size_t)e * nbs, nbs, step, tol);
}

// BB2 / adaptive steps: partials of |mu A^T A G + rho grad^T grad G|^2 per
// block of 1024 pixels.
__global__ __launch_bounds__(256) void k_yy(const float *__restrict__ apart, int nplanes,
                                            float mu, const float *__restrict__ gpad, float rho,
                                            const AdmScalars *__restrict__ sc,
                                            double *__restrict__ p_yy, int nx, int ny, int nbi)
{
    const int e = blockIdx.y;
    if (sc[e].stopped) return;
    const size_t N = (size_t)nx * ny;
    yy_chunk(blockIdx.x, e, apart + (size_t)e * nplanes * N, nplanes, mu, gpad, rho,
             p_yy + (size_t)e * nbi, nx, ny);
}

// ------------------------------------------------------------- set-up ---
// f = beta x0 (or 0), lambda = z = 0 for both parities.
__global__ __launch_bounds__(256) void k_init_image(float *__restrict__ f,
                                                    const float *__restrict__ x0h,
                                                    const float *__restrict__ x0l, double bh,
                                                    double bl, float *__restrict__ lam,
                                                    float *__restrict__ z, size_t N)
{
    const int e = blockIdx.y;
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const float *x0 = e == 0 ? x0h : x0l;
    const double d = x0 ? (e == 0 ? bh : bl) * (double)x0[i] : 0.0;
    const float hi = (float)d;
    f[e * N + i] = hi;                                  // f + flo = beta x0
    f[2 * N + e * N + i] = (float)(d - (double)hi);
    for (int q = 0; q < 4; ++q) {  // [parity][energy][comp]: zero all of them
        lam[(size_t)q * N * 2 + (size_t)e * N + i] = 0.f;
        z[(size_t)q * N * 2 + (size_t)e * N + i] = 0.f;
    }
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
// (coupled: the joint TV of both energies in energy 0's partials, none in
// energy 1's)
__global__ __launch_bounds__(256) void k_tv_only(const float *__restrict__ f,
                                                 double *__restrict__ partial, int nx, int ny,
                                                 int coupled)
{
    const int e = blockIdx.y;
    const size_t N = (size_t)nx * ny;
    double v[1] = {0.0};
    const float *fl = f + 2 * N;
    auto grad = [&](int q, size_t i, int r, int c, float &dx, float &dy) {
        float fc = f[q * N + i], lc = fl[q * N + i];
        dx = c >= 1 ? (fc - f[q * N + i - 1]) + (lc - fl[q * N + i - 1]) : 0.f;
        dy = r >= 1 ? (fc - f[q * N + i - nx]) + (lc - fl[q * N + i - nx]) : 0.f;
    };
    for (int j = 0; j < 4; ++j) {
        size_t i = ((size_t)blockIdx.x * 4 + j) * 256 + threadIdx.x;
        if (i < N) {
            int r = (int)(i / nx), c = (int)(i % nx);
            float dx, dy;
            grad(e, i, r, c, dx, dy);
            if (!coupled) {
                v[0] += (double)sqrtf(dx * dx + dy * dy);
            } else if (e == 0) {
                float dx2, dy2;
                grad(1, i, r, c, dx2, dy2);
                const float ta = dx * dx + dy * dy, tb = dx2 * dx2 + dy2 * dy2;
                v[0] += (double)sqrtf(ta + tb);
            }
        }
    }
    __shared__ double tot[1];
    block_sum<1>(v, tot);
    __syncthreads();
    if (threadIdx.x == 0) partial[(size_t)e * gridDim.x + blockIdx.x] = tot[0];
}

// J(f^K): TV from the partials, |r|^2 from the last update's partials (once
// an update has run; else the set-up's value).
__global__ __launch_bounds__(256) void k_final_J(AdmScalars *__restrict__ sc,
                                                 const double *__restrict__ p_tv, int nb,
                                                 const double *__restrict__ p_rr, int nbs,
                                                 double *__restrict__ log, int log_rows, double mu)
{
    const int e = blockIdx.x;
    const bool fresh_rr = sc[e].pending != 0;
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < nb; i += 256) v[0] += p_tv[(size_t)e * nb + i];
    if (fresh_rr)
        for (int i = threadIdx.x; i < nbs; i += 256) v[1] += p_rr[(size_t)e * nbs + i];
    __shared__ double tot[2];
    block_sum<2>(v, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;
    AdmScalars &s = sc[e];
    if (fresh_rr) s.rr = tot[1];
    double J = tot[0] + 0.5 * mu * s.rr;
    int64_t row = s.iter - s.log_base;
    if (log && row >= 0 && row < log_rows) {
        log[row * kLogW + e] = J;
        log[row * kLogW + 2 + e] = s.alpha;
        log[row * kLogW + 4 + e] = 0.0;
        log[row * kLogW + 6 + e] = 0.0;
    }
    s.J = J;
}

// x = (f + flo) / beta
__global__ __launch_bounds__(256) void k_output(const float *__restrict__ f,
                                                float *__restrict__ xh, float *__restrict__ xl,
                                                double bh, double bl, size_t N)
{
    const int e = blockIdx.y;
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const double v = (double)f[e * N + i] + (double)f[2 * N + e * N + i];
    if (e == 0) xh[i] = (float)(v / bh);
    else xl[i] = (float)(v / bl);
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
    dect::DevBuf f, r, p, lam, z, gpad, gpadT, p_tv, p_fwd, p_rr, adjpart, sc, logbuf,
        p_tvo, p_ss, p_ff, p_gs;
    bool nonneg = false;        // the run projects every f-step onto f >= 0
    bool fresh = false;         // no iteration launched since the run's set-up
    bool coupled = false;       // the run couples the TV of the two energies
    int graph_coupled = -1;
    int step_rule = 0;          // 0 BB1, 1 BB2, 2 adaptive
    int graph_step = -1;
    dect::DevBuf apart, p_yy;   // BB2 / adaptive: A^T (A G) partial planes, |y|^2 partials
    int graph_nonneg = -1;
    void *graph_log = nullptr;
    size_t graph_log_bytes = 0;
    double graph_tol = -1.0;
    double graph_mu = -1.0, graph_rho = -1.0, graph_xi = -1.0;
    // captured iterations: [start parity][kGraphIters index]
    hipGraphExec_t graph[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    hipStream_t cap = nullptr;
    int parity = 0;  // lambda/z buffer holding the current values
    void drop_graphs()
    {
        for (auto &gp : graph)
            for (auto &gx : gp)
                if (gx) {
                    (void)hipGraphExecDestroy(gx);
                    gx = nullptr;
                }
    }
    ~dect_adm_state()
    {
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace dect {

// Set-up of a run on raw state pointers: f = beta x0 (or 0), lambda = z = 0,
// r = A f - beta m, h = mu A^T r, scalars reset.
dect_status adm_init(const GeomTables &t, const AdmPtrs &P, int nvg, const float *mh,
                     const float *ml, double mu, double bh, double bl, const float *x0h,
                     const float *x0l, hipStream_t s)
{
    const size_t N = (size_t)t.key.nx * t.key.ny;
    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, s, P.sc, bh, bl);
    DECT_HIP(hipGetLastError());
    dim3 gi((unsigned)((N + 255) / 256), 2);
    hipLaunchKernelGGL(k_init_image, gi, dim3(256), 0, s, P.f, x0h, x0l, bh, bl, P.lam, P.z, N);
    DECT_HIP(hipGetLastError());
    // r + rlo = A f - beta m in FP64 (the padded G buffers serve as f's padded
    // copies here), |r|^2 from the projector's per-block sums
    dect_status st = launch_pad(t, P.f, P.gpad, P.gpadT, 2, s);
    if (st) return st;
    if ((st = launch_fwd(t, P.gpad, P.gpadT, P.r, 2, 1.0f, P.p_fwd, s, mh, ml, bh, bl, P.rlo)))
        return st;
    hipLaunchKernelGGL(k_rr, dim3(2), dim3(256), 0, s, P.sc, (const double *)P.p_fwd, P.nb_fwd,
                       0, 0.0);
    DECT_HIP(hipGetLastError());
    return launch_adj(t, P.r, nullptr, P.adjpart, 2, (float)mu, s, nvg);
}

// Marks the start of a call's log (row 0 = the next iteration).
dect_status adm_mark_log(const AdmPtrs &P, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_log_base, dim3(1), dim3(64), 0, s, P.sc);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

// x = f / beta and the final objective J(f^K) into the scalars and the log.
dect_status adm_finish(const GeomTables &t, const AdmPtrs &P, float *xh, float *xl, double mu,
                       double bh, double bl, hipStream_t s, bool coupled)
{
    const size_t N = (size_t)t.key.nx * t.key.ny;
    dim3 go((unsigned)((N + 255) / 256), 2);
    hipLaunchKernelGGL(k_output, go, dim3(256), 0, s, (const float *)P.f, xh, xl, bh, bl, N);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_tv_only, dim3(P.nbi, 2), dim3(256), 0, s, (const float *)P.f, P.p_tvo,
                       t.key.nx, t.key.ny, coupled ? 1 : 0);
    DECT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_final_J, dim3(2), dim3(256), 0, s, P.sc, (const double *)P.p_tvo, P.nbi,
                       (const double *)P.p_rr, P.nbs, P.log, P.log_rows, mu);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

static AdmPtrs ptrs_of(dect_adm_state *S)
{
    AdmPtrs P;
    P.f = (float *)S->f.ptr;
    P.flo = P.f + 2 * (size_t)S->t->key.nx * S->t->key.ny;
    const size_t M = (size_t)S->t->key.V * S->t->key.B;
    P.r = (float *)S->r.ptr;
    P.rlo = P.r + 2 * M;
    P.p = (float *)S->p.ptr;
    P.plo = P.p + 2 * M;
    P.lam = (float *)S->lam.ptr;
    P.z = (float *)S->z.ptr;
    P.gpad = (float *)S->gpad.ptr;
    P.gpadT = (float *)S->gpadT.ptr;
    P.adjpart = (float *)S->adjpart.ptr;
    P.p_tv = (double *)S->p_tv.ptr;
    P.p_fwd = (double *)S->p_fwd.ptr;
    P.p_rr = (double *)S->p_rr.ptr;
    P.p_tvo = (double *)S->p_tvo.ptr;
    P.p_ss = (double *)S->p_ss.ptr;
    P.p_ff = (double *)S->p_ff.ptr;
    P.p_gs = (double *)S->p_gs.ptr;
    P.log = (double *)S->logbuf.ptr;
    P.log_rows = (int)(S->logbuf.bytes / (kLogW * sizeof(double)));
    P.sc = (AdmScalars *)S->sc.ptr;
    P.nb_tv = S->nb_tv;
    P.nb_fwd = S->nb_fwd;
    P.nbi = S->nbi;
    P.nbs = S->nbs;
    return P;
}

static dect_status state_alloc(dect_adm_state *S, const dect_geometry *g)
{
    dect_status st = get_tables(g, &S->t);
    if (st != DECT_OK) return st;
    DECT_HIP(hipGetDevice(&S->device));
    const GeomTables &t = *S->t;
    const size_t N = (size_t)g->nx * g->ny, M = (size_t)g->n_views * g->n_bins;
    const size_t P = (size_t)(g->nx + 2 * kPad) * (g->ny + 2 * kPad);
    S->nvg = adj_groups(t, 2);
    S->nb_tv = ((g->nx + kTX - 1) / kTX) * ((g->ny + kTY - 1) / kTY);
    S->nb_fwd = fwd_blocks(t);
    S->nbi = (int)((N + 1023) / 1024);
    S->nbs = (int)((M + 1023) / 1024);
    S->nb_img = S->nbi;
    if ((st = S->f.ensure(4 * N * 4)) ||
        (st = S->r.ensure(4 * M * 4)) || (st = S->p.ensure(4 * M * 4)) ||
        (st = S->lam.ensure(8 * N * 4)) || (st = S->z.ensure(8 * N * 4)) ||
        (st = S->gpad.ensure(2 * P * 4, true)) || (st = S->gpadT.ensure(2 * P * 4, true)) ||
        (st = S->p_tv.ensure((size_t)2 * S->nb_tv * kTvParts * 8)) ||
        (st = S->p_fwd.ensure((size_t)2 * S->nb_fwd * 8)) ||
        (st = S->p_rr.ensure((size_t)2 * S->nbs * 8)) ||
        (st = S->p_tvo.ensure((size_t)2 * S->nbi * 8)) ||
        (st = S->p_ss.ensure((size_t)2 * S->nbi * 8)) ||
        (st = S->p_ff.ensure((size_t)2 * S->nbi * 8)) ||
        (st = S->p_gs.ensure((size_t)2 * S->nbi * 8)) ||
        (st = S->adjpart.ensure(std::max<size_t>(1, adj_partial_floats(t, 2)) * 4)) ||
        (st = S->sc.ensure(2 * sizeof(AdmScalars))))
        return st;
    return DECT_OK;
}

// Launch one iteration; `par` selects the lambda/z buffers holding the
// current values.
static dect_status launch_iter(dect_adm_state *S, int par, double tol, hipStream_t s,
                               bool first = false)
{
    const GeomTables &t = *S->t;
    const int nx = t.key.nx, ny = t.key.ny;
    const size_t N = (size_t)nx * ny;
    const int M = t.key.V * t.key.B;
    float *lam = (float *)S->lam.ptr, *z = (float *)S->z.ptr;
    float *lam_in = lam + (size_t)par * 4 * N, *lam_out = lam + (size_t)(1 - par) * 4 * N;
    float *z_in = z + (size_t)par * 4 * N, *z_out = z + (size_t)(1 - par) * 4 * N;
    AdmScalars *sc = (AdmScalars *)S->sc.ptr;
    const int tiles_x = (nx + kTX - 1) / kTX, tiles_y = (ny + kTY - 1) / kTY;
    DECT_TRACE("adm iteration");
    hipLaunchKernelGGL(S->coupled ? k_tv_fused<true> : k_tv_fused<false>,
                       dim3(2 * tiles_x * tiles_y), dim3(256), 0, s, (const float *)S->f.ptr,
                       (const float *)S->adjpart.ptr, S->nvg, (float)S->mu, lam_in, z_in, lam_out,
                       z_out, (float *)S->gpad.ptr, (float *)S->gpadT.ptr, (double *)S->p_tv.ptr,
                       sc, nx, ny, (float)S->rho, (float)S->xi, tiles_x, tiles_y);
    DECT_HIP(hipGetLastError());
    float *p = (float *)S->p.ptr;
    dect_status st = DECT_OK;
    // A G: the step and the residual update of the plain iteration; with the
    // projection only the first (Cauchy) step needs it
    if (!S->nonneg || first) {
        st = launch_fwd(t, (const float *)S->gpad.ptr, (const float *)S->gpadT.ptr, p, 2, 1.0f,
                        (double *)S->p_fwd.ptr, s, nullptr, nullptr, 0.0, 0.0,
                        p + 2 * (size_t)M);
        if (st) return st;
    }
    hipLaunchKernelGGL(k_scalar, dim3(2), dim3(256), 0, s, sc, (const double *)S->p_tv.ptr,
                       S->nb_tv, (const double *)S->p_fwd.ptr, S->nb_fwd,
                       (double *)S->logbuf.ptr, (int)(S->logbuf.bytes / (kLogW * sizeof(double))),
                       S->mu, S->rho,
                       S->nonneg ? 1 : 0, (const double *)S->p_rr.ptr, S->nbs, tol,
                       S->step_rule, (const double *)S->p_yy.ptr, S->nbi);
    DECT_HIP(hipGetLastError());
    if (S->nonneg) {
        // projected step s, |grad s|^2, p = A s, r += p, then the step's sums
        hipLaunchKernelGGL(k_nn_step, dim3(S->nbi, 2), dim3(256), 0, s, (float *)S->f.ptr,
                           (const float *)S->gpad.ptr, (float *)S->gpadT.ptr,
                           (const AdmScalars *)sc, (double *)S->p_ss.ptr, (double *)S->p_ff.ptr,
                           nx, ny, S->nbi);
        DECT_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_nn_grad, dim3(S->nbi, 2), dim3(256), 0, s, (float *)S->gpad.ptr,
                           (const float *)S->gpadT.ptr, (const AdmScalars *)sc,
                           (double *)S->p_gs.ptr, nx, ny, S->nbi);
        DECT_HIP(hipGetLastError());
        if ((st = launch_fwd(t, (const float *)S->gpad.ptr, (const float *)S->gpadT.ptr, p, 2,
                             1.0f, (double *)S->p_fwd.ptr, s, nullptr, nullptr, 0.0, 0.0,
                             p + 2 * (size_t)M)))
            return st;
        hipLaunchKernelGGL(k_nn_resid, dim3(S->nbs, 2), dim3(256), 0, s, (float *)S->r.ptr,
                           (const float *)p, (const AdmScalars *)sc, (double *)S->p_rr.ptr, M,
                           S->nbs);
        DECT_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_nn_rr, dim3(2), dim3(256), 0, s, sc, (const double *)S->p_rr.ptr,
                           S->nbs, (const double *)S->p_ss.ptr, (const double *)S->p_ff.ptr,
                           (const double *)S->p_gs.ptr, S->nbi, (const double *)S->p_fwd.ptr,
                           S->nb_fwd, S->mu, S->rho, tol);
        DECT_HIP(hipGetLastError());
        return launch_adj(t, (const float *)S->r.ptr, nullptr, (float *)S->adjpart.ptr, 2,
                          (float)S->mu, s, S->nvg);
    }
    hipLaunchKernelGGL(k_update, dim3(S->nbi + S->nbs, 2), dim3(256), 0, s, (float *)S->f.ptr,
                       (const float *)S->gpad.ptr, (float *)S->r.ptr, (const float *)S->p.ptr,
                       (double *)S->p_rr.ptr, sc, nx, ny, M, S->nbi, S->nbs);
    DECT_HIP(hipGetLastError());
    // |r|^2 of this update is summed by the next iteration's scalar kernel
    if (S->step_rule) {  // |mu A^T A G + rho grad^T grad G|^2 for the next step
        if ((st = launch_adj(t, (const float *)p, nullptr, (float *)S->apart.ptr, 2, 1.0f, s,
                             S->nvg)))
            return st;
        hipLaunchKernelGGL(k_yy, dim3(S->nbi, 2), dim3(256), 0, s, (const float *)S->apart.ptr,
                           2 * S->nvg, (float)S->mu, (const float *)S->gpad.ptr, (float)S->rho,
                           (const AdmScalars *)sc, (double *)S->p_yy.ptr, nx, ny, S->nbi);
        DECT_HIP(hipGetLastError());
    }
    return launch_adj(t, (const float *)S->r.ptr, nullptr, (float *)S->adjpart.ptr, 2,
                      (float)S->mu, s, S->nvg);
}

static dect_status adm_start(dect_adm_state *S, const dect_adm_params *P, const float *mh,
                             const float *ml, const float *x0h, const float *x0l, hipStream_t s)
{
    S->mu = P->mu;
    S->rho = P->rho;
    S->xi = P->xi;
    S->bh = P->beta_high;
    S->bl = P->beta_low;
    S->nonneg = (P->flags & DECT_NONNEG) != 0;
    S->coupled = (P->flags & DECT_COUPLED_TV) != 0;
    S->step_rule = (P->flags & DECT_STEP_BB2) ? 1 : (P->flags & DECT_STEP_ABB) ? 2 : 0;
    if (S->step_rule) {
        dect_status st = DECT_OK;
        if ((st = S->apart.ensure(std::max<size_t>(1, adj_partial_floats(*S->t, 2, S->nvg)) * 4)) ||
            (st = S->p_yy.ensure((size_t)2 * S->nbi * 8)))
            return st;
    }
    S->fresh = true;
    S->parity = 0;
    dect_status st =
        adm_init(*S->t, ptrs_of(S), S->nvg, mh, ml, S->mu, S->bh, S->bl, x0h, x0l, s);
    if (st) return st;
    S->started = true;
    return DECT_OK;
}

// Iteration counts of the captured graphs (each replay of a longer graph
// saves the gaps between replays of shorter ones).
static constexpr int kGraphIters[3] = {1, 2, 8};

// The graph of kGraphIters[gi] iterations starting on lambda/z parity `par`.
static dect_status build_graph(dect_adm_state *S, double tol, int par, int gi)
{
    hipGraphExec_t &out = S->graph[par][gi];
    if (out) {
        (void)hipGraphExecDestroy(out);
        out = nullptr;
    }
    if (!S->cap) DECT_HIP(hipStreamCreateWithFlags(&S->cap, hipStreamNonBlocking));
    DECT_HIP(hipStreamBeginCapture(S->cap, hipStreamCaptureModeThreadLocal));
    dect_status st = DECT_OK;
    for (int i = 0; i < kGraphIters[gi] && !st; ++i) st = launch_iter(S, par ^ (i & 1), tol, S->cap);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(S->cap, &graph);
    if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(DECT_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(DECT_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    return DECT_OK;
}

static std::mutex g_adm_mu;
// rows the device log keeps at least (calls of different lengths share it)
static constexpr size_t kLogRowsMin = 4096;
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
    if ((P->flags & DECT_COUPLED_TV) && P->tol > 0.0)
        return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv: coupled TV runs a fixed iteration count (tol 0)");
    if ((P->flags & DECT_STEP_BB2) && (P->flags & DECT_STEP_ABB))
        return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv: DECT_STEP_BB2 and DECT_STEP_ABB exclude each other");
    if ((P->flags & (DECT_STEP_BB2 | DECT_STEP_ABB)) && (P->flags & DECT_NONNEG))
        return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv: the BB2 / adaptive steps have no non-negative variant");
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
                           S->bh != P->beta_high || S->bl != P->beta_low ||
                           S->nonneg != ((P->flags & DECT_NONNEG) != 0) ||
                           S->coupled != ((P->flags & DECT_COUPLED_TV) != 0) ||
                           S->step_rule != ((P->flags & DECT_STEP_BB2) ? 1
                                            : (P->flags & DECT_STEP_ABB) ? 2 : 0)))
            return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv: parameters differ from the state's run");
    }
    const int K = P->max_iter;
    const size_t log_rows = (size_t)K + 1;
    // the device log keeps at least 4096 rows so that calls of different
    // lengths reuse it (and the captured graph that points at it)
    if ((st = S->logbuf.ensure(std::max<size_t>(log_rows, kLogRowsMin) * kLogW * sizeof(double))))
        return st;
    if (!S->started) {
        DECT_TRACE("adm set-up");
        const bool warm = (P->flags & DECT_WARM_START) != 0;
        if ((st = adm_start(S, P, mh, ml, warm ? xh : nullptr, warm ? xl : nullptr, s))) return st;
    }
    if ((st = adm_mark_log(ptrs_of(S), s))) return st;
    // the log buffer, tol, the variant and (mu, rho, xi) are baked into the
    // graphs' kernel arguments: drop them when these change (each is captured
    // again when first needed)
    if (S->graph_log != S->logbuf.ptr || S->graph_log_bytes != S->logbuf.bytes ||
        S->graph_tol != P->tol || S->graph_nonneg != (int)S->nonneg ||
        S->graph_coupled != (int)S->coupled || S->graph_step != S->step_rule ||
        S->graph_mu != S->mu || S->graph_rho != S->rho || S->graph_xi != S->xi) {
        S->drop_graphs();
        S->graph_mu = S->mu;
        S->graph_rho = S->rho;
        S->graph_xi = S->xi;
        S->graph_log = S->logbuf.ptr;
        S->graph_log_bytes = S->logbuf.bytes;
        S->graph_tol = P->tol;
        S->graph_nonneg = (int)S->nonneg;
        S->graph_coupled = (int)S->coupled;
        S->graph_step = S->step_rule;
    }
    int k = 0;
    if (S->fresh && S->nonneg && K > 0) {  // the first projected step starts from A G
        if ((st = launch_iter(S, S->parity, P->tol, s, true))) return st;
        S->parity ^= 1;
        ++k;
    }
    if (k > 0 || K > 0) S->fresh = false;
    // runs of 8, then pairs, then a single iteration, each replayed from a
    // graph captured for the current parity.  A call of two or more
    // iterations captures all six shapes at once, so that later calls (a
    // resumed state lands on either parity) replay without capturing; a call
    // of one iteration captures none.
    if (K - k >= 2 && !S->graph[0][1]) {
        DECT_TRACE("adm graph capture");
        for (int par = 0; par < 2; ++par)
            for (int gi = 0; gi < 3; ++gi)
                if ((st = build_graph(S, P->tol, par, gi))) return st;
    }
    if (k + 2 <= K) {
        DECT_TRACE("adm iterations (graph)");
        for (int gi = 2; gi >= 1; --gi) {
            const int n = kGraphIters[gi];  // even: the parity is unchanged
            for (; k + n <= K; k += n) DECT_HIP(hipGraphLaunch(S->graph[S->parity][gi], s));
        }
    }
    if (k < K) {
        if (S->graph[S->parity][0]) DECT_HIP(hipGraphLaunch(S->graph[S->parity][0], s));
        else if ((st = launch_iter(S, S->parity, P->tol, s))) return st;
        S->parity ^= 1;
        ++k;
    }
    // outputs and the final objective
    {
        DECT_TRACE("adm finish");
        if ((st = adm_finish(*S->t, ptrs_of(S), xh, xl, S->mu, S->bh, S->bl, s, S->coupled)))
            return st;
    }
    if (rep || P->log || P->log_aux) {
        DECT_HIP(hipStreamSynchronize(s));
        AdmScalars hs[2];
        DECT_HIP(hipMemcpy(hs, S->sc.ptr, sizeof(hs), hipMemcpyDeviceToHost));
        if (P->log || P->log_aux) {
            std::vector<double> h(log_rows * kLogW);
            DECT_HIP(hipMemcpy(h.data(), S->logbuf.ptr, h.size() * sizeof(double),
                               hipMemcpyDeviceToHost));
            for (size_t r = 0; r < log_rows; ++r)
                for (int c = 0; c < 4; ++c) {
                    if (P->log) P->log[r * 4 + c] = h[r * kLogW + c];
                    if (P->log_aux) P->log_aux[r * 4 + c] = h[r * kLogW + 4 + c];
                }
        }
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

// The buffers one ADM run without a caller state allocates (the state, a log
// of kLogRowsMin rows, the BB2 / adaptive-step extras), for a dry run under a
// SizingScope.
dect_status adm_size_run(const dect_geometry *g)
{
    auto S = std::make_unique<dect_adm_state>();
    dect_status st = state_alloc(S.get(), g);
    if (st) return st;
    if ((st = S->logbuf.ensure(kLogRowsMin * kLogW * sizeof(double))) ||
        (st = S->apart.ensure(std::max<size_t>(1, adj_partial_floats(*S->t, 2, S->nvg)) * 4)) ||
        (st = S->p_yy.ensure((size_t)2 * S->nbi * 8)))
        return st;
    return DECT_OK;
}

dect_status adm_state_reset(dect_adm_state *S)
{
    if (!S) return fail(DECT_ERR_INVALID_ARG, "dect_adm_state_reset: state is NULL");
    std::lock_guard<std::mutex> lk(g_adm_mu);
    S->started = false;
    return DECT_OK;
}

void release_adm_states()
{
    std::lock_guard<std::mutex> lk(g_adm_mu);
    g_tmp_states.clear();
}

}  // namespace dect
