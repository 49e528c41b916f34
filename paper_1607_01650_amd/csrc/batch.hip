// Batched ADM-TV: many slices of uneven size and view count, both energies,
// advanced together.  Each phase of an iteration (tv stencil, forward
// projection, step, update, residual norm, back-projection) is ONE
// launch over a work list that spans every slice (and energy,
// for the image-domain phases; a projector item carries both energies of its
// slice); a captured hipGraph replays an even/odd pair of iterations.  Items are
// sorted by estimated cost (longest first), one block per item (or, as a
// tuner candidate, handed round-robin to a persistent grid); the adjoint's view-group depth (how many blocks share
// one output tile) is chosen per batch by a timing autotuner.  Slices with
// the coupled TV, and Siddon slices, get lists of their own in the phases
// that differ (the stencil; the projectors), each one more launch;
// the projected slices (DECT_NONNEG) replace the update by the projected
// step, a forward projection of it and its residual update, and the BB2 /
// adaptive slices add a back-projection of A G and the |y|^2 partials, each
// phase over the slices that have it.
#include <algorithm>
#include <array>
#include <cstring>
#include <mutex>
#include <numeric>

#include "adm_device.h"
#include "proj_device.h"

namespace dect {

struct SliceDev {
    int nx, ny, V, B, nbundle, nvg, M;
    const RayFwd *fwd;
    const float *len;
    const Bundle *bundles;
    const BinRange *bins;
    const LaneRange *lanes;
    const SidW *sid;  // Siddon weight terms (null: Joseph)
    int coupled;      // the TV couples the two energies
    int nonneg;       // every f-step projected onto f >= 0
    int step_rule;    // 0 BB1, 1 BB2, 2 adaptive
    float *apart;     // BB2 / adaptive: [2][2 nvg] partial planes of A^T (A G)
    double *p_yy;     // BB2 / adaptive: [2][nbi] partials of |y|^2
    float rho, xi, muf;
    double mu, rhod, tol;
    AdmPtrs P;
};

namespace {

__device__ __forceinline__ AdmImg img_of(const SliceDev &d, int e, int par)
{
    const size_t N = (size_t)d.nx * d.ny;
    const float *lin = d.P.lam + (size_t)par * 4 * N, *zin = d.P.z + (size_t)par * 4 * N;
    float *lout = d.P.lam + (size_t)(1 - par) * 4 * N, *zout = d.P.z + (size_t)(1 - par) * 4 * N;
    return AdmImg{d.P.f + e * N,
                  d.P.adjpart + (size_t)e * 2 * d.nvg * N,
                  lin + (2 * e) * N,
                  lin + (2 * e + 1) * N,
                  zin + (2 * e) * N,
                  zin + (2 * e + 1) * N,
                  lout + (2 * e) * N,
                  lout + (2 * e + 1) * N,
                  zout + (2 * e) * N,
                  zout + (2 * e + 1) * N,
                  d.P.gpad + e,
                  d.P.gpadT + e,
                  d.P.flo + e * N,
                  2 * d.nvg,
                  d.muf};
}

// item = (slice, energy, tile row, tile column); COUPLED: slices whose TV
// couples the energies (the tile also reads the other energy's state)
template <bool COUPLED>
__global__ __launch_bounds__(256) void kb_tv(const SliceDev *__restrict__ S,
                                             const int4 *__restrict__ items, int n, int par)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        const SliceDev &d = S[w.x];
        const int e = w.y;
        if (!d.P.sc[e].stopped && !d.P.sc[e].stop_next) {
            const int gx = (d.nx + kTX - 1) / kTX, gy = (d.ny + kTY - 1) / kTY;
            const size_t blk = (size_t)e * gx * gy + (size_t)w.z * gx + w.w;
            AdmImg m = img_of(d, e, par);
            if constexpr (COUPLED) {
                const size_t N = (size_t)d.nx * d.ny;
                const int o = 1 - e;
                const float *lin = d.P.lam + (size_t)par * 4 * N, *zin = d.P.z + (size_t)par * 4 * N;
                m.f2 = d.P.f + o * N;
                m.flo2 = d.P.flo + o * N;
                m.lxi2 = lin + (2 * o) * N;
                m.lyi2 = lin + (2 * o + 1) * N;
                m.zxi2 = zin + (2 * o) * N;
                m.zyi2 = zin + (2 * o + 1) * N;
                m.pending2 = d.P.sc[o].pending != 0;
                m.record_tv = e == 0;
            }
            tv_tile<COUPLED>(w.z * kTY, w.w * kTX, m, d.P.p_tv + blk * kTvParts,
                             d.P.sc[e].pending != 0, d.nx, d.ny, d.rho, d.xi);
        }
        __syncthreads();
    }
}

// item = (slice, (view, bundle) block): both energies; SID: Siddon slices
template <bool SID>
__global__ __launch_bounds__(kFwdThreads) void kb_fwd(const SliceDev *__restrict__ S,
                                                      const int4 *__restrict__ items, int n)
{
    __shared__ FwdShared sh;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        const SliceDev &d = S[w.x];
        const int blk = w.y;
        if (!(d.P.sc[0].stopped && d.P.sc[1].stopped)) {
            FwdOut o;
            for (int e = 0; e < 2; ++e) {
                o.sino[e] = d.P.p + (size_t)e * d.M;
                o.lo[e] = d.P.plo + (size_t)e * d.M;
                o.sub[e] = nullptr;
                o.sub_scale[e] = 0.0;
            }
            double res[2];
            fwd_block<SID>(sh, d.P.gpad, d.P.gpadT, d.fwd, d.len, d.sid, d.bundles, o, d.nx,
                             d.ny, d.V, d.B, d.nbundle, blk, 1.0f, res);
            if (threadIdx.x < 64) {  // the values live in wavefront 0
                const double t0 = lane_sum(res[0] * res[0]);
                const double t1 = lane_sum(res[1] * res[1]);
                if (threadIdx.x == 0) {
                    d.P.p_fwd[blk] = t0;
                    d.P.p_fwd[(size_t)d.P.nb_fwd + blk] = t1;
                }
            }
        }
        __syncthreads();
    }
}

// item = (slice, energy)
__global__ __launch_bounds__(256) void kb_scalar(const SliceDev *__restrict__ S,
                                                 const int4 *__restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        const SliceDev &d = S[w.x];
        const int e = w.y;
        scalar_energy(d.P.sc[e], d.P.p_tv + (size_t)e * d.P.nb_tv * kTvParts, d.P.nb_tv,
                      d.P.p_fwd + (size_t)e * d.P.nb_fwd, d.P.nb_fwd, d.P.log, d.P.log_rows, e,
                      d.mu, d.rhod, d.nonneg != 0, d.nonneg == 0,
                      d.P.p_rr + (size_t)e * d.P.nbs, d.P.nbs, d.tol, d.step_rule,
                      d.p_yy ? d.p_yy + (size_t)e * d.P.nbi : nullptr, d.P.nbi);
    }
}

// item = (slice, energy, chunk)
__global__ __launch_bounds__(256) void kb_update(const SliceDev *__restrict__ S,
                                                 const int4 *__restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        const SliceDev &d = S[w.x];
        const int e = w.y;
        if (!d.P.sc[e].stopped) {
            const size_t N = (size_t)d.nx * d.ny;
            update_chunk(w.z, d.P.f + e * N, d.P.flo + e * N, d.P.gpad + e,
                         d.P.r + (size_t)e * d.M, d.P.rlo + (size_t)e * d.M,
                         d.P.p + (size_t)e * d.M, d.P.plo + (size_t)e * d.M,
                         d.P.p_rr + (size_t)e * d.P.nbs, d.P.sc[e].alpha, d.nx, d.ny, d.M,
                         d.P.nbi);
        }
        __syncthreads();
    }
}

// Projected step (DECT_NONNEG): item = (slice, energy, image chunk).
__global__ __launch_bounds__(256) void kb_nn_step(const SliceDev *__restrict__ S,
                                                  const int4 *__restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        const SliceDev &d = S[w.x];
        const int e = w.y;
        if (!d.P.sc[e].stopped) {
            const size_t N = (size_t)d.nx * d.ny;
            nn_step_chunk(w.z, e, d.P.f + e * N, d.P.flo + e * N, d.P.gpad, d.P.gpadT,
                          d.P.sc[e].alpha, d.P.p_ss + (size_t)e * d.P.nbi,
                          d.P.p_ff + (size_t)e * d.P.nbi, d.nx, d.ny);
        }
        __syncthreads();
    }
}

// |grad s|^2 and s into both padded layouts: item = (slice, energy, image chunk).
__global__ __launch_bounds__(256) void kb_nn_grad(const SliceDev *__restrict__ S,
                                                  const int4 *__restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        const SliceDev &d = S[w.x];
        const int e = w.y;
        if (!d.P.sc[e].stopped)
            nn_grad_chunk(w.z, e, d.P.gpad, d.P.gpadT, d.P.p_gs + (size_t)e * d.P.nbi, d.nx,
                          d.ny);
        __syncthreads();
    }
}

// r += A s: item = (slice, energy, sinogram chunk).
__global__ __launch_bounds__(256) void kb_nn_resid(const SliceDev *__restrict__ S,
                                                   const int4 *__restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        const SliceDev &d = S[w.x];
        const int e = w.y;
        if (!d.P.sc[e].stopped) {
            const size_t M = (size_t)d.M;
            nn_resid_chunk(w.z, d.P.r + e * M, d.P.rlo + e * M, d.P.p + e * M, d.P.plo + e * M,
                           d.P.p_rr + (size_t)e * d.P.nbs, d.M);
        }
        __syncthreads();
    }
}

// The projected step's scalars: item = (slice, energy).
__global__ __launch_bounds__(256) void kb_nn_rr(const SliceDev *__restrict__ S,
                                                const int4 *__restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        const SliceDev &d = S[w.x];
        const int e = w.y;
        nn_rr_energy(d.P.sc[e], d.P.p_rr + (size_t)e * d.P.nbs, d.P.nbs,
                     d.P.p_ss + (size_t)e * d.P.nbi, d.P.p_ff + (size_t)e * d.P.nbi,
                     d.P.p_gs + (size_t)e * d.P.nbi, d.P.nbi, d.P.p_fwd + (size_t)e * d.P.nb_fwd,
                     d.P.nb_fwd, d.mu, d.rhod, d.tol);
    }
}

// |y|^2 partials of the BB2 / adaptive steps: item = (slice, energy, image chunk).
__global__ __launch_bounds__(256) void kb_yy(const SliceDev *__restrict__ S,
                                             const int4 *__restrict__ items, int n)
{
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        const SliceDev &d = S[w.x];
        const int e = w.y;
        if (!d.P.sc[e].stopped) {
            const size_t N = (size_t)d.nx * d.ny;
            yy_chunk(w.z, e, d.apart + (size_t)e * 2 * d.nvg * N, 2 * d.nvg, d.muf, d.P.gpad,
                     d.rho, d.p_yy + (size_t)e * d.P.nbi, d.nx, d.ny);
        }
        __syncthreads();
    }
}

// item = (slice, strip of either ray class, view group, source): both
// energies; SID: Siddon slices.  source 0: r into the partial planes of
// mu A^T r; 1 (BB2 / adaptive): p = A G into those of A^T A G.
template <bool SID>
__global__ __launch_bounds__(kAdjThreads) void kb_adj(const SliceDev *__restrict__ S,
                                              const int4 *__restrict__ items, int n)
{
    __shared__ AdjShared<2> sh;
    __shared__ AdjStage stage;
    __shared__ SidW sid_stage[SID ? kStageSlots : 1];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int4 w = items[it];
        const SliceDev &d = S[w.x];
        const int strip = w.y, g = w.z;
        const size_t plane = (size_t)d.nx * d.ny;
        const int cls = strip < adj_strips_x(d.nx, d.ny) ? 0 : 1;
        if (!(d.P.sc[0].stopped && d.P.sc[1].stopped)) {
            const float *src = w.w ? d.P.p : d.P.r;
            float *dst = w.w ? d.apart : d.P.adjpart;
            const float *s[2] = {src, src + d.M};
            float *p[2];
            for (int e = 0; e < 2; ++e)
                p[e] = dst + ((size_t)e * 2 * d.nvg + (size_t)cls * d.nvg + g) * plane;
            adj_block<2, SID>(sh, s, d.fwd, d.len, d.sid, d.bins, d.lanes, d.nx, d.ny, d.V,
                              d.B, strip, g, d.nvg, p, stage, SID ? sid_stage : nullptr);
        }
        __syncthreads();
    }
}

}  // namespace
}  // namespace dect

struct dect_batch {
    int n = 0;
    std::vector<dect::GeomTables *> t;
    std::vector<dect_adm_params> prm;
    std::vector<dect::SliceDev> host;
    std::vector<size_t> off;  // arena offsets per slice
    // a work list of one phase: items, count, grid
    struct WList {
        dect::DevBuf buf;
        int n = 0, g = 0;
    };
    // the stencil's lists split by coupled TV, the projectors' by model;
    // fwdn: A G (first iteration) and A s of the projected slices; adjp: A^T
    // A G of the BB2 / adaptive slices
    dect::DevBuf arena, slices;
    WList tv[2], fwd[2], fwdn[2], se, upd, nnc, nnr, nne, adjp[2], yyc, adj[2];
    bool any_nonneg = false;
    int nvg_max = 16, group_choice = 0;  // 0: per-slice heuristic, else fixed
    // autotuned shape: the adjoint view-group depth per slice (0: as
    // group_choice) and the grids of the adjoint and forward phases (0: one
    // block per work item; k: a persistent grid of k blocks per CU)
    std::vector<int> slice_groups;
    int adj_per_cu = 0, fwd_per_cu = 0;
    bool tuned_from_cache = false;
    hipGraphExec_t graph = nullptr;
    hipStream_t cap = nullptr;
    ~dect_batch()
    {
        if (graph) (void)hipGraphExecDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace dect {
namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int heuristic_groups(const GeomTables &t) { return adj_groups(t, 2); }

// Work lists and persistent grid sizes for the current view-group choice.
dect_status build_work(dect_batch *b)
{
    std::vector<std::pair<double, int4>> tv[2], fwd[2], fwdn[2], se, upd, nnc, nnr, nne, adjp[2],
        yyc, adj[2];
    b->any_nonneg = false;
    for (int s = 0; s < b->n; ++s) {
        SliceDev &d = b->host[s];
        const GeomTables &t = *b->t[s];
        // the built-in choice equals the single-slice path's (bitwise equal
        // results); a tuned choice is capped by the views per group
        const int want = (s < (int)b->slice_groups.size() && b->slice_groups[s])
                             ? b->slice_groups[s] : b->group_choice;
        int nvg = want ? std::min(want, std::max(1, d.V / 8)) : heuristic_groups(t);
        d.nvg = nvg;
        const int gx = (d.nx + kTX - 1) / kTX, gy = (d.ny + kTY - 1) / kTY;
        const int nstrips = adj_strips(d.nx, d.ny);
        const int c = d.coupled ? 1 : 0, m = d.sid ? 1 : 0;
        b->any_nonneg = b->any_nonneg || d.nonneg;
        for (int e = 0; e < 2; ++e) {
            for (int ty = 0; ty < gy; ++ty)
                for (int tx = 0; tx < gx; ++tx) tv[c].push_back({1.0, make_int4(s, e, ty, tx)});
            se.push_back({1.0, make_int4(s, e, 0, 0)});
            if (d.nonneg) {
                for (int k = 0; k < d.P.nbi; ++k) nnc.push_back({1.0, make_int4(s, e, k, 0)});
                for (int k = 0; k < d.P.nbs; ++k) nnr.push_back({1.0, make_int4(s, e, k, 0)});
                nne.push_back({1.0, make_int4(s, e, 0, 0)});
            } else {
                for (int k = 0; k < d.P.nbi + d.P.nbs; ++k)
                    upd.push_back({1.0, make_int4(s, e, k, 0)});
            }
            if (d.step_rule)
                for (int k = 0; k < d.P.nbi; ++k) yyc.push_back({1.0, make_int4(s, e, k, 0)});
        }
        // the projectors carry both energies per item
        for (int k = 0; k < d.P.nb_fwd; ++k)
            (d.nonneg ? fwdn : fwd)[m].push_back({(double)std::max(d.nx, d.ny),
                                                  make_int4(s, k, 0, 0)});
        for (int strip = 0; strip < nstrips; ++strip)
            for (int g = 0; g < nvg; ++g) {
                adj[m].push_back({(double)d.V / nvg, make_int4(s, strip, g, 0)});
                if (d.step_rule) adjp[m].push_back({(double)d.V / nvg, make_int4(s, strip, g, 1)});
            }
    }
    auto upload = [&](std::vector<std::pair<double, int4>> &v, dect_batch::WList &w) {
        std::stable_sort(v.begin(), v.end(),
                         [](const auto &a, const auto &c) { return a.first > c.first; });
        std::vector<int4> flat(v.size());
        for (size_t i = 0; i < v.size(); ++i) flat[i] = v[i].second;
        w.n = (int)flat.size();
        dect_status st = w.buf.ensure(std::max<size_t>(1, flat.size()) * sizeof(int4));
        if (st) return st;
        DECT_HIP(hipMemcpy(w.buf.ptr, flat.data(), flat.size() * sizeof(int4), hipMemcpyHostToDevice));
        return DECT_OK;
    };
    dect_status st;
    for (int k = 0; k < 2; ++k)
        if ((st = upload(tv[k], b->tv[k])) || (st = upload(fwd[k], b->fwd[k])) ||
            (st = upload(fwdn[k], b->fwdn[k])) || (st = upload(adj[k], b->adj[k])) ||
            (st = upload(adjp[k], b->adjp[k])))
            return st;
    if ((st = upload(se, b->se)) || (st = upload(upd, b->upd)) || (st = upload(nnc, b->nnc)) ||
        (st = upload(nnr, b->nnr)) || (st = upload(nne, b->nne)) || (st = upload(yyc, b->yyc)))
        return st;
    DECT_HIP(hipMemcpy(b->slices.ptr, b->host.data(), b->host.size() * sizeof(SliceDev),
                       hipMemcpyHostToDevice));
    int dev = 0, cus = 0;
    DECT_HIP(hipGetDevice(&dev));
    DECT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // cap 0: one block per item (the hardware starts a block as soon as one
    // ends, measured 12% faster over the 64-slice batch than a resident grid
    // whose blocks walk the list); cap k > 0: a persistent grid of at most k
    // blocks per CU (a tuner candidate)
    auto grid = [&](const void *fn, int items, int threads = 256, int cap = 0) {
        if (cap <= 0) return std::max(1, items);
        int per = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, 0) != hipSuccess ||
            per < 1)
            per = 1;
        per = std::min(per, cap);
        return std::max(1, std::min(items, per * cus));
    };
    b->tv[0].g = grid((const void *)kb_tv<false>, b->tv[0].n);
    b->tv[1].g = grid((const void *)kb_tv<true>, b->tv[1].n);
    for (int k = 0; k < 2; ++k) {
        const void *kf = k ? (const void *)kb_fwd<true> : (const void *)kb_fwd<false>;
        const void *ka = k ? (const void *)kb_adj<true> : (const void *)kb_adj<false>;
        b->fwd[k].g = grid(kf, b->fwd[k].n, kFwdThreads, b->fwd_per_cu);
        b->fwdn[k].g = grid(kf, b->fwdn[k].n, kFwdThreads, b->fwd_per_cu);
        b->adj[k].g = grid(ka, b->adj[k].n, kAdjThreads, b->adj_per_cu);
        b->adjp[k].g = grid(ka, b->adjp[k].n, kAdjThreads, b->adj_per_cu);
    }
    b->se.g = std::max(1, b->se.n);
    b->nne.g = std::max(1, b->nne.n);
    b->upd.g = grid((const void *)kb_update, b->upd.n);
    b->nnc.g = grid((const void *)kb_nn_step, b->nnc.n);
    b->nnr.g = grid((const void *)kb_nn_resid, b->nnr.n);
    b->yyc.g = grid((const void *)kb_yy, b->yyc.n);
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    return DECT_OK;
}

// One iteration of every slice; `first`: the projected slices' first step
// also needs A G (the exact line search along -G).
dect_status launch_batch_iter(dect_batch *b, int par, hipStream_t s, bool first = false)
{
    const SliceDev *S = (const SliceDev *)b->slices.ptr;
    using Kern = void (*)(const SliceDev *, const int4 *, int);
    auto go = [&](Kern fn, const dect_batch::WList &w, int threads) {
        if (w.n)
            hipLaunchKernelGGL(fn, dim3(w.g), dim3(threads), 0, s, S, (const int4 *)w.buf.ptr, w.n);
    };
    // each phase: one launch per non-empty list
    if (b->tv[0].n)
        hipLaunchKernelGGL(kb_tv<false>, dim3(b->tv[0].g), dim3(256), 0, s, S,
                           (const int4 *)b->tv[0].buf.ptr, b->tv[0].n, par);
    if (b->tv[1].n)
        hipLaunchKernelGGL(kb_tv<true>, dim3(b->tv[1].g), dim3(256), 0, s, S,
                           (const int4 *)b->tv[1].buf.ptr, b->tv[1].n, par);
    go(kb_fwd<false>, b->fwd[0], kFwdThreads);
    go(kb_fwd<true>, b->fwd[1], kFwdThreads);
    if (first) {
        go(kb_fwd<false>, b->fwdn[0], kFwdThreads);
        go(kb_fwd<true>, b->fwdn[1], kFwdThreads);
    }
    go(kb_scalar, b->se, 256);
    go(kb_update, b->upd, 256);
    // the projected slices: the step, s in both layouts, r += A s, scalars
    go(kb_nn_step, b->nnc, 256);
    go(kb_nn_grad, b->nnc, 256);
    go(kb_fwd<false>, b->fwdn[0], kFwdThreads);
    go(kb_fwd<true>, b->fwdn[1], kFwdThreads);
    go(kb_nn_resid, b->nnr, 256);
    go(kb_nn_rr, b->nne, 256);
    // the BB2 / adaptive slices: A^T A G and |y|^2 for the next step
    go(kb_adj<false>, b->adjp[0], kAdjThreads);
    go(kb_adj<true>, b->adjp[1], kAdjThreads);
    go(kb_yy, b->yyc, 256);
    go(kb_adj<false>, b->adj[0], kAdjThreads);
    go(kb_adj<true>, b->adj[1], kAdjThreads);
    DECT_HIP(hipGetLastError());
    return DECT_OK;
}

// The graph of an even/odd iteration pair (rebuilt when the work lists change).
dect_status batch_graph(dect_batch *b)
{
    if (b->graph) return DECT_OK;
    if (!b->cap) DECT_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    DECT_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    dect_status st = launch_batch_iter(b, 0, b->cap);
    if (!st) st = launch_batch_iter(b, 1, b->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(DECT_ERR_HIP, std::string("batch capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(DECT_ERR_HIP, std::string("batch instantiate: ") + hipGetErrorString(e));
    return DECT_OK;
}

// Start every slice (f = 0) and run `iters` iterations (even/odd pairs from
// the graph, an odd last one launched directly).
dect_status batch_run(dect_batch *b, const float *const *mh, const float *const *ml, int iters,
                      hipStream_t s)
{
    dect_status st;
    for (int i = 0; i < b->n; ++i) {
        const dect_adm_params &p = b->prm[i];
        if ((st = adm_init(*b->t[i], b->host[i].P, b->host[i].nvg, mh[i], ml[i], p.mu,
                           p.beta_high, p.beta_low, nullptr, nullptr, s)))
            return st;
        if ((st = adm_mark_log(b->host[i].P, s))) return st;
    }
    if ((st = batch_graph(b))) return st;
    int k = 0;
    if (b->any_nonneg && iters > 0) {  // the projected slices' first step starts from A G
        if ((st = launch_batch_iter(b, 0, s, true))) return st;
        if (iters > 1 && (st = launch_batch_iter(b, 1, s))) return st;
        k = std::min(iters, 2);
    }
    for (; k + 2 <= iters; k += 2) DECT_HIP(hipGraphLaunch(b->graph, s));
    if (k < iters && (st = launch_batch_iter(b, 0, s))) return st;
    return DECT_OK;
}

}  // namespace

dect_status batch_create(const dect_geometry *geoms, const dect_adm_params *prm, int n,
                         dect_batch **out)
{
    if (!geoms || !prm || !out || n <= 0)
        return fail(DECT_ERR_INVALID_ARG, "dect_batch_create: bad arguments");
    auto b = std::make_unique<dect_batch>();
    b->n = n;
    b->t.resize(n);
    b->prm.assign(prm, prm + n);
    b->host.resize(n);
    b->off.resize(n + 1);
    dect_status st;
    size_t total = 0;
    struct Sizes { size_t N, M, Pp, nb_tv, nb_fwd, nbi, nbs, part; };
    std::vector<Sizes> sz(n);
    for (int i = 0; i < n; ++i) {
        const dect_adm_params &p = prm[i];
        if (!(p.mu > 0) || !(p.rho > 0) || !(p.xi >= 0) || !(p.beta_high > 0) || !(p.beta_low > 0))
            return fail(DECT_ERR_INVALID_ARG, "dect_batch_create: invalid ADM parameters");
        if ((p.flags & DECT_STEP_BB2) && (p.flags & DECT_STEP_ABB))
            return fail(DECT_ERR_INVALID_ARG, "DECT_STEP_BB2 and DECT_STEP_ABB exclude each other");
        if ((p.flags & (DECT_STEP_BB2 | DECT_STEP_ABB)) && (p.flags & DECT_NONNEG))
            return fail(DECT_ERR_INVALID_ARG,
                        "the BB2 / adaptive steps have no non-negative variant");
        if ((p.flags & DECT_COUPLED_TV) && p.tol != 0.0)
            return fail(DECT_ERR_INVALID_ARG,
                        "batched ADM: coupled TV runs a fixed iteration count (tol 0)");
        if ((st = get_tables(&geoms[i], &b->t[i]))) return st;
        const GeomTables &t = *b->t[i];
        Sizes &z = sz[i];
        z.N = (size_t)t.key.nx * t.key.ny;
        z.M = (size_t)t.key.V * t.key.B;
        z.Pp = (size_t)(t.key.nx + 2 * kPad) * (t.key.ny + 2 * kPad);
        z.nb_tv = (size_t)((t.key.nx + kTX - 1) / kTX) * ((t.key.ny + kTY - 1) / kTY);
        z.nb_fwd = (size_t)fwd_blocks(t);
        z.nbi = (z.N + 1023) / 1024;
        z.nbs = (z.M + 1023) / 1024;
        z.part = adj_partial_floats(t, 2, std::max(b->nvg_max, adj_groups(t, 2)));
        size_t bytes = 0;
        bytes += align256(4 * z.N * 4);             // f (+ flo)
        bytes += align256(4 * z.M * 4) * 2;         // r (+ rlo), p (+ plo)
        bytes += align256(8 * z.N * 4) * 2;         // lam, z
        bytes += align256(2 * z.Pp * 4) * 2;        // gpad, gpadT
        bytes += align256(z.part * 4);
        bytes += align256(2 * z.nb_tv * kTvParts * 8) + align256(2 * z.nb_fwd * 8) +
                 align256(2 * z.nbs * 8) + align256(2 * z.nbi * 8);
        bytes += align256(2 * sizeof(AdmScalars));
        if (p.flags & DECT_NONNEG) bytes += 3 * align256(2 * z.nbi * 8);  // <s,s>, |f|^2, |grad s|^2
        if (p.flags & (DECT_STEP_BB2 | DECT_STEP_ABB))
            bytes += align256(z.part * 4) + align256(2 * z.nbi * 8);     // A^T A G planes, |y|^2
        b->off[i] = total;
        total += bytes;
    }
    b->off[n] = total;
    if ((st = b->arena.ensure(total, true))) return st;  // zero: pad borders
    if ((st = b->slices.ensure(n * sizeof(SliceDev)))) return st;
    for (int i = 0; i < n; ++i) {
        const GeomTables &t = *b->t[i];
        const Sizes &z = sz[i];
        char *base = (char *)b->arena.ptr + b->off[i];
        auto take = [&](size_t bytes) {
            char *p = base;
            base += align256(bytes);
            return (void *)p;
        };
        SliceDev &d = b->host[i];
        std::memset(&d, 0, sizeof(d));
        d.P.f = (float *)take(4 * z.N * 4);
        d.P.flo = d.P.f + 2 * z.N;
        d.P.r = (float *)take(4 * z.M * 4);
        d.P.rlo = d.P.r + 2 * z.M;
        d.P.p = (float *)take(4 * z.M * 4);
        d.P.plo = d.P.p + 2 * z.M;
        d.P.lam = (float *)take(8 * z.N * 4);
        d.P.z = (float *)take(8 * z.N * 4);
        d.P.gpad = (float *)take(2 * z.Pp * 4);
        d.P.gpadT = (float *)take(2 * z.Pp * 4);
        d.P.adjpart = (float *)take(z.part * 4);
        d.P.p_tv = (double *)take(2 * z.nb_tv * kTvParts * 8);
        d.P.p_fwd = (double *)take(2 * z.nb_fwd * 8);
        d.P.p_rr = (double *)take(2 * z.nbs * 8);
        d.P.p_tvo = (double *)take(2 * z.nbi * 8);
        d.P.sc = (AdmScalars *)take(2 * sizeof(AdmScalars));
        d.nonneg = (prm[i].flags & DECT_NONNEG) ? 1 : 0;
        d.step_rule = (prm[i].flags & DECT_STEP_BB2) ? 1 : (prm[i].flags & DECT_STEP_ABB) ? 2 : 0;
        if (d.nonneg) {
            d.P.p_ss = (double *)take(2 * z.nbi * 8);
            d.P.p_ff = (double *)take(2 * z.nbi * 8);
            d.P.p_gs = (double *)take(2 * z.nbi * 8);
        }
        if (d.step_rule) {
            d.apart = (float *)take(z.part * 4);
            d.p_yy = (double *)take(2 * z.nbi * 8);
        }
        d.P.log = nullptr;
        d.P.log_rows = 0;
        d.P.nb_tv = (int)z.nb_tv;
        d.P.nb_fwd = (int)z.nb_fwd;
        d.P.nbi = (int)z.nbi;
        d.P.nbs = (int)z.nbs;
        d.nx = t.key.nx;
        d.ny = t.key.ny;
        d.V = t.key.V;
        d.B = t.key.B;
        d.M = (int)z.M;
        d.nbundle = t.nbundle;
        d.fwd = t.fwd;
        d.len = t.len;
        d.bundles = t.bundles;
        d.bins = t.adj_bins;
        d.lanes = t.adj_lanes;
        d.sid = t.sid;
        d.coupled = (prm[i].flags & DECT_COUPLED_TV) ? 1 : 0;
        d.rho = (float)prm[i].rho;
        d.xi = (float)prm[i].xi;
        d.muf = (float)prm[i].mu;
        d.mu = prm[i].mu;
        d.rhod = prm[i].rho;
        d.tol = prm[i].tol;
    }
    if ((st = build_work(b.get()))) return st;
    *out = b.release();
    return DECT_OK;
}

dect_status batch_destroy(dect_batch *b)
{
    delete b;
    return DECT_OK;
}

dect_status adm_tv_batched(dect_batch *b, const float *const *mh, const float *const *ml,
                           float *const *xh, float *const *xl, int iters, double *objective,
                           hipStream_t s)
{
    if (!b || !mh || !ml || !xh || !xl || iters < 0)
        return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv_batched: bad arguments");
    for (int i = 0; i < b->n; ++i)
        if (!mh[i] || !ml[i] || !xh[i] || !xl[i])
            return fail(DECT_ERR_INVALID_ARG, "dect_adm_tv_batched: null slice buffer");
    dect_status st = batch_run(b, mh, ml, iters, s);
    if (st) return st;
    for (int i = 0; i < b->n; ++i) {
        const dect_adm_params &p = b->prm[i];
        if ((st = adm_finish(*b->t[i], b->host[i].P, xh[i], xl[i], p.mu, p.beta_high, p.beta_low, s,
                             b->host[i].coupled != 0)))
            return st;
    }
    if (objective) {
        DECT_HIP(hipStreamSynchronize(s));
        int nf = 0;
        for (int i = 0; i < b->n; ++i) {
            AdmScalars hs[2];
            DECT_HIP(hipMemcpy(hs, b->host[i].P.sc, sizeof(hs), hipMemcpyDeviceToHost));
            objective[i] = hs[0].J + hs[1].J;
            if (hs[0].nonfinite_iter || hs[1].nonfinite_iter) nf = i + 1;
        }
        if (nf) return fail(DECT_ERR_NONFINITE, "dect_adm_tv_batched: non-finite value in slice " +
                                                    std::to_string(nf - 1));
    }
    return DECT_OK;
}

// Tuned shapes, kept for the process: a batch of the same slice shapes (the
// multiset of image size, views and bins) reuses them without timing.
struct TunedShape {
    std::vector<std::array<int, 8>> shapes;  // sorted (nx, ny, V, B, model, variants) per slice
    std::vector<int> groups;                 // per sorted slice
    int adj_per_cu = 0, fwd_per_cu = 0;
    double ms = 0.0;
};
static std::mutex g_tune_mu;
static std::vector<TunedShape> g_tuned;

static std::vector<int> shape_order(const dect_batch *b, std::vector<std::array<int, 8>> &shapes)
{
    std::vector<int> order(b->n);
    std::iota(order.begin(), order.end(), 0);
    auto key = [&](int i) {
        const SliceDev &d = b->host[i];
        return std::array<int, 8>{d.nx, d.ny, d.V, d.B, d.sid ? 1 : 0, d.coupled, d.nonneg,
                                  d.step_rule};
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return key(a) < key(c); });
    shapes.resize(b->n);
    for (int k = 0; k < b->n; ++k) shapes[k] = key(order[k]);
    return order;
}

// Time `iters` iterations of the current shape (after a 2-iteration warm-up
// that also captures the graph).
static dect_status time_shape(dect_batch *b, const float *const *mh, const float *const *ml,
                              int iters, hipStream_t s, hipEvent_t e0, hipEvent_t e1, double *ms)
{
    dect_status st;
    if ((st = build_work(b)) || (st = batch_run(b, mh, ml, 2, s))) return st;
    DECT_HIP(hipStreamSynchronize(s));
    DECT_HIP(hipEventRecord(e0, s));
    if ((st = batch_run(b, mh, ml, iters, s))) return st;
    DECT_HIP(hipEventRecord(e1, s));
    DECT_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    DECT_HIP(hipEventElapsedTime(&t, e0, e1));
    *ms = t;
    return DECT_OK;
}

// Coordinate descent over the batch's shape: for each class of equal slices
// (image size and views; the costliest class first) the adjoint view-group
// depth 1, 2, 4, 8 or 16 (how many blocks share one output strip, i.e. how
// many views each adjoint tile walks), then the adjoint and forward grids
// (one block per work item, or a persistent grid of 1 or 2 blocks per CU).  Each
// candidate is timed over `iters` iterations on the given data; the fastest
// is kept and remembered for batches of the same slice shapes.
dect_status batch_tune(dect_batch *b, const float *const *mh, const float *const *ml, int iters,
                       int32_t *chosen, double *ms_per_iter, hipStream_t s)
{
    if (!b || !mh || !ml || iters < 2)
        return fail(DECT_ERR_INVALID_ARG, "dect_batch_tune: bad arguments");
    std::vector<std::array<int, 8>> shapes;
    const std::vector<int> order = shape_order(b, shapes);
    // the slice of the costliest class reports its depth in *chosen
    int big = 0;
    double big_w = -1.0;
    for (int i = 0; i < b->n; ++i) {
        const SliceDev &d = b->host[i];
        const double w = (double)d.V * std::max(d.nx, d.ny) * std::max(d.nx, d.ny);
        if (w > big_w) {
            big_w = w;
            big = i;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const TunedShape &c : g_tuned)
            if (c.shapes == shapes) {
                b->slice_groups.assign(b->n, 0);
                for (int k = 0; k < b->n; ++k) b->slice_groups[order[k]] = c.groups[k];
                b->adj_per_cu = c.adj_per_cu;
                b->fwd_per_cu = c.fwd_per_cu;
                b->tuned_from_cache = true;
                dect_status st = build_work(b);
                if (st) return st;
                if (chosen) *chosen = b->slice_groups[big];
                if (ms_per_iter) *ms_per_iter = c.ms / iters;
                return DECT_OK;
            }
    }
    // classes of equal (nx, ny, V), costliest first
    std::vector<std::pair<double, std::vector<int>>> classes;
    for (int i = 0; i < b->n; ++i) {
        const SliceDev &d = b->host[i];
        bool found = false;
        for (auto &c : classes) {
            const SliceDev &o = b->host[c.second[0]];
            if (o.nx == d.nx && o.ny == d.ny && o.V == d.V) {
                c.second.push_back(i);
                c.first += (double)d.V * d.nx * d.ny;
                found = true;
                break;
            }
        }
        if (!found) classes.push_back({(double)d.V * d.nx * d.ny, {i}});
    }
    std::stable_sort(classes.begin(), classes.end(),
                     [](const auto &a, const auto &c) { return a.first > c.first; });
    hipEvent_t e0, e1;
    DECT_HIP(hipEventCreate(&e0));
    DECT_HIP(hipEventCreate(&e1));
    dect_status st = DECT_OK;
    b->slice_groups.assign(b->n, 0);
    b->adj_per_cu = 0;
    b->fwd_per_cu = 0;
    double best = 0.0;
    for (int i = 0; i < b->n; ++i) b->slice_groups[i] = adj_groups(*b->t[i], 2);
    st = time_shape(b, mh, ml, iters, s, e0, e1, &best);
    for (size_t c = 0; c < classes.size() && !st; ++c) {
        const std::vector<int> &mem = classes[c].second;
        const int keep = b->slice_groups[mem[0]];
        int best_g = keep;
        for (int g : {1, 2, 4, 8, 16}) {
            if (g == keep || g > std::max(1, b->host[mem[0]].V / 8)) continue;
            for (int i : mem) b->slice_groups[i] = g;
            double ms = 0.0;
            if ((st = time_shape(b, mh, ml, iters, s, e0, e1, &ms))) break;
            if (ms < best) {
                best = ms;
                best_g = g;
            }
        }
        for (int i : mem) b->slice_groups[i] = best_g;
    }
    for (int which = 0; which < 2 && !st; ++which) {
        int &knob = which == 0 ? b->adj_per_cu : b->fwd_per_cu;
        int best_k = knob;
        for (int k : {1, 2}) {
            knob = k;
            double ms = 0.0;
            if ((st = time_shape(b, mh, ml, iters, s, e0, e1, &ms))) break;
            if (ms < best) {
                best = ms;
                best_k = k;
            }
        }
        knob = best_k;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    b->tuned_from_cache = false;
    if ((st = build_work(b))) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        TunedShape c;
        c.shapes = shapes;
        c.groups.resize(b->n);
        for (int k = 0; k < b->n; ++k) c.groups[k] = b->slice_groups[order[k]];
        c.adj_per_cu = b->adj_per_cu;
        c.fwd_per_cu = b->fwd_per_cu;
        c.ms = best;
        g_tuned.push_back(std::move(c));
    }
    if (chosen) *chosen = b->slice_groups[big];
    if (ms_per_iter) *ms_per_iter = best / iters;
    return DECT_OK;
}

dect_status batch_shape(const dect_batch *b, int32_t *groups, int32_t *adj_per_cu,
                        int32_t *fwd_per_cu, int32_t *from_cache)
{
    if (!b) return fail(DECT_ERR_INVALID_ARG, "dect_batch_shape: batch is NULL");
    if (groups)
        for (int i = 0; i < b->n; ++i) groups[i] = b->host[i].nvg;
    if (adj_per_cu) *adj_per_cu = b->adj_per_cu;
    if (fwd_per_cu) *fwd_per_cu = b->fwd_per_cu;
    if (from_cache) *from_cache = b->tuned_from_cache ? 1 : 0;
    return DECT_OK;
}

dect_status batch_set_groups(dect_batch *b, int groups)
{
    if (!b || groups < 0 || groups > b->nvg_max)
        return fail(DECT_ERR_INVALID_ARG, "dect_batch_set_groups: 0 (heuristic) .. 16");
    b->group_choice = groups;
    b->slice_groups.clear();
    b->adj_per_cu = 0;
    b->fwd_per_cu = 0;
    b->tuned_from_cache = false;
    return build_work(b);
}

}  // namespace dect
