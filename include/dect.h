/*
 * dect.h -- C ABI of libdect, the MI355X (gfx950) library for the hot path of
 * dual-energy CT reconstruction and decomposition after Li et al.,
 * "Efficient Image Reconstruction and Practical Decomposition for
 * Dual-energy Computed Tomography" (arXiv 1607.01650).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Image: float32, row-major [ny][nx] (column index fastest).  Pixel (r, c)
 *   has its centre at x = (c - (nx-1)/2) * pixel_mm, y = (r - (ny-1)/2) *
 *   pixel_mm: the image is centred on the isocentre.
 * Views: theta_v = 2*pi*v/n_views (counter-clockwise from +x) unless
 *   angles_rad is given.  Source at sod_mm * (cos, sin)(theta).  Flat
 *   detector line centred at -(sdd_mm - sod_mm) * (cos, sin)(theta) with axis
 *   (-sin, cos)(theta); bin b is centred at u = (b - (n_bins-1)/2) * bin_mm +
 *   det_offset_mm.  This is the central slice of the paper's cone-beam
 *   scanner (Sec. 2.1, Fig. 1; Sec. 3).
 * Sinogram: float32, row-major [n_views][n_bins].
 * Batched arrays are stacked contiguously: item i starts at i * (ny*nx) or
 *   i * (n_views*n_bins) elements.
 * Memory: every d_* pointer is device memory owned by the caller, on the
 *   current HIP device; the library never frees it.  The library owns its
 *   cached geometry tables and scratch workspaces (per device, per geometry),
 *   released by dect_release_caches() or at process exit.
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *   asynchronous on it unless a host-side report/log is requested, in which
 *   case the call synchronises the stream before returning.
 * Errors: every call returns a dect_status; arguments and geometry are
 *   validated on the host before any launch and nothing is launched on
 *   error.  dect_last_error() gives a message for the calling thread.
 *   Calls are thread-safe with respect to the caches; concurrent calls that
 *   share output buffers race like any other kernels.
 */
#ifndef DECT_H
#define DECT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DECT_OK = 0,
    DECT_ERR_INVALID_ARG = 1, /* null pointer, non-positive size, bad parameter */
    DECT_ERR_GEOMETRY = 2,    /* source inside the image, SDD <= SOD, fan >= 90 deg */
    DECT_ERR_HIP = 3,         /* a HIP runtime call failed */
    DECT_ERR_NONFINITE = 4,   /* a reduction produced NaN/Inf (report.iters says when) */
    DECT_WARN_MAXITER = 5     /* PCG stopped at max_iter above tolerance */
} dect_status;

/* Ray model of the system matrix A (Eq. 1).
 * DECT_JOSEPH: each ray steps along the image axis it is more aligned with
 *   and interpolates linearly between the two nearest pixel centres of every
 *   line it crosses; samples are scaled by the path length per line.
 * DECT_SIDDON: A[ray, pixel] is the exact length of the source-to-bin-centre
 *   segment inside the pixel square (the model Sec. 2.1 names).  Along a
 *   line of the driving axis the ray crosses at most two adjacent pixels, so
 *   it is evaluated as two taps per line like Joseph, with the path length
 *   per line split at the pixel boundary (the boundary's position is rounded
 *   to 2^-32 pixel). */
enum { DECT_JOSEPH = 0, DECT_SIDDON = 1 };

/* 2-D fan-beam geometry with a flat detector line (Sec. 2.1 and Sec. 3:
 * SOD, SDD, views and detector bins define the system matrix A of Eq. 1). */
typedef struct {
    int32_t nx, ny;           /* image size in pixels */
    double pixel_mm;          /* square pixel side */
    int32_t n_views;          /* number of projection views */
    const double *angles_rad; /* host array [n_views] or NULL for 2*pi*v/n_views */
    int32_t n_bins;           /* detector bins per view */
    double bin_mm;            /* bin pitch on the detector line */
    double det_offset_mm;     /* shift of the detector centre along its axis */
    double sod_mm;            /* source to isocentre */
    double sdd_mm;            /* source to detector */
    int32_t model;            /* DECT_JOSEPH or DECT_SIDDON (else DECT_ERR_INVALID_ARG) */
} dect_geometry;

/* ADM-TV parameters (Eqs. 3-10 and Sec. 2.4). */
enum {
    DECT_WARM_START = 1, /* start from d_x_* instead of zero images */
    DECT_NONNEG = 2,     /* project every f-step onto f >= 0 (attenuation maps are
                            non-negative); the BB1 step is then taken from the
                            projected step s: <s,s> / (mu |A s|^2 + rho |grad s|^2),
                            kept when the denominator is not positive.  The
                            step's own projection A s replaces A G after the
                            first iteration. */
    DECT_COUPLED_TV = 4, /* the TV norm of Eq. 2 over the 4-vector (on volumes the
                            6-vector) of both energies' gradients (one joint
                            z-step; each energy keeps its own f-step and BB
                            step); log column J_high then holds the
                            joint TV and J_low none, so the two sum to the
                            objective.  Needs tol = 0 (fixed iteration count). */
    DECT_STEP_BB2 = 8,   /* BB2 step <s,y>/<y,y> instead of BB1 <s,s>/<s,y> (Eq. 9
                            names a BB step without its variant); one more back-projection per
                            iteration (A^T A G for |y|^2) */
    DECT_STEP_ABB = 16   /* adaptive: BB2 where BB2/BB1 < 1/2, else BB1; same cost.
                            Neither step flag combines with DECT_NONNEG. */
};
typedef struct {
    double mu;        /* data-fidelity weight of Eq. 4 */
    double rho;       /* augmented-Lagrangian penalty of Eq. 6 */
    double xi;        /* multiplier step of Eq. 7 */
    double beta_high; /* noise-balancing scalar beta_1 of Eq. 3 (high energy) */
    double beta_low;  /* beta_2 (low energy) */
    int32_t max_iter; /* iterations to run (>= 0) */
    double tol;       /* stop once |f^{k+1}-f^k| / |f^k| < tol for both
                         energies (0 = run max_iter iterations) */
    int32_t flags;    /* DECT_WARM_START, DECT_NONNEG, DECT_COUPLED_TV, DECT_STEP_BB2 or
                         DECT_STEP_ABB */
    double *log;      /* host [max_iter+1][4] or NULL: per energy-pair row
                         {J_high(f^k), J_low(f^k), alpha_high^k, alpha_low^k};
                         filling it synchronises the stream */
    double *log_aux;  /* host [max_iter+1][4] or NULL: per row {|grad f - z|_high,
                         |grad f - z|_low, |G|_high, |G|_low} of the iteration's
                         z-step and f-gradient (Eqs. 8-9), before its step; the
                         final row holds zeros.  Filling it synchronises the
                         stream.  (The batched call takes neither log.) */
} dect_adm_params;

/* PLS decomposition parameters (Eqs. 11-15, Sec. 2.4, Sec. 3). */
typedef struct {
    double eta_water_high, eta_bone_high; /* eta_1H, eta_2H of Eq. 12 (1/mm) */
    double eta_water_low, eta_bone_low;   /* eta_1L, eta_2L */
    double gamma;                         /* smoothing weight of Eq. 13 */
    double edge_eps;                      /* e_ik for pairs touching an edge pixel */
    double edge_tau;                      /* edge if |Prewitt| > tau * max |Prewitt| */
    int32_t max_iter;                     /* PCG iteration cap (paper: 500) */
    double tol;                           /* PCG stop: |res| <= tol * |rhs| */
    int32_t mode;                         /* DECT_PLS_IMAGE or DECT_PLS_ATTENUATION */
} dect_pls_params;

/* PLS objective.  DECT_PLS_IMAGE: Eqs. 13 and 15 as printed, |u - D^{-1} x|^2
 * + gamma R(u), i.e. (I + gamma L) u_m = (D^{-1} x)_m per material.
 * DECT_PLS_ATTENUATION: |x - D u|^2 + gamma R(u) (the data term in the
 * measured attenuation space, for which the gamma range of Sec. 2.4 is
 * scaled), i.e. (D^T D (x) I + gamma I (x) L) u = D^T x with both materials
 * coupled per pixel; solved by block-Jacobi CG in FP64 (D^T D is
 * ill-conditioned), joint tolerance over both materials. */
enum { DECT_PLS_IMAGE = 0, DECT_PLS_ATTENUATION = 1 };

typedef struct {
    int32_t iters;       /* ADM iterations run, or the larger PCG count */
    double objective;    /* ADM: J of Eq. 4 summed over both energies at exit */
    double rel_change;   /* ADM: last max relative image change */
    double pcg_residual; /* PLS: max final relative residual of the materials */
    int32_t status;      /* dect_status of the run */
} dect_report;

/* Opaque resumable ADM state: f, lambda, z, h, r and the step for both
 * energies of one geometry.  Running K1 then K2 iterations through a state
 * gives bitwise the same images as K1 + K2 iterations in one call. */
typedef struct dect_adm_state dect_adm_state;

/*
 * Forward projection d_sino = A d_img (Eq. 1; Sec. 2.4's forward projector),
 * with A the ray model geom->model selects (Joseph or Siddon, see above).
 * batch images [batch][ny][nx] -> [batch][n_views][n_bins].
 */
dect_status dect_project(const dect_geometry *geom, const float *d_img, float *d_sino,
                         int32_t batch, void *stream);

/*
 * Back-projection d_img = A^T d_sino: the exact transpose of dect_project's
 * matrix (the W^T of the gradient G_f after Eq. 9), evaluated in gather form:
 * every output pixel sums over the rays that touch it, with the same
 * interpolation weights as the forward pass, bit for bit; no atomics.
 */
dect_status dect_backproject(const dect_geometry *geom, const float *d_sino, float *d_img,
                             int32_t batch, void *stream);

/*
 * Fan-beam filtered back-projection d_img = FBP(d_sino): the analytic
 * reconstruction the paper compares with (Sec. 3, FBP rows of its tables),
 * usable as the start image of dect_adm_tv (DECT_WARM_START).  Textbook form
 * for an equally spaced flat detector over a full turn: each view is
 * weighted by R / sqrt(R^2 + s^2) (s the bin position scaled to the
 * isocentre, R = SOD), convolved with the band-limited ramp kernel and
 * halved, then back-projected pixel by pixel with linear interpolation and
 * the weight R^2 / (R - p . e_s)^2 (e_s towards the source), times 2 pi / V.
 * Independent of geom->model.  batch sinograms [batch][n_views][n_bins] ->
 * images [batch][ny][nx].  DECT_ERR_INVALID_ARG when geom->angles_rad is not
 * NULL (the views must be the equally spaced full turn) or n_bins > 6144.
 * Uses a library-owned workspace per (device, stream).
 */
dect_status dect_fbp(const dect_geometry *geom, const float *d_sino, float *d_img, int32_t batch,
                     void *stream);

/*
 * TV-regularised ADM reconstruction of both energies (Eq. 10): the stacked
 * system of Eq. 3 with f = (beta_1 x_h; beta_2 x_l), g = (beta_1 m_h;
 * beta_2 m_l), minimising |grad f| + mu/2 |W f - g|^2 (Eq. 4) by the
 * z-shrinkage (Eq. 8), one gradient step on f with a Barzilai-Borwein step
 * (Eq. 9) and the multiplier step (Eq. 7).  TV is applied to each energy
 * image separately.
 * d_m_high/d_m_low: measured sinograms [n_views][n_bins].
 * d_x_high/d_x_low: [ny][nx] outputs (x = f / beta); inputs too when
 *   flags has DECT_WARM_START.
 * state: NULL, or a state from dect_adm_state_create for this geometry;
 *   an empty state starts a run, a used one continues it (x inputs ignored).
 * rep: NULL, or filled after synchronising the stream.
 * Non-finite values: the iteration records the first iteration at which a
 *   sum turned non-finite in a device flag.  The flag is read, and
 *   DECT_ERR_NONFINITE returned, only by a call that synchronises (rep or
 *   params->log not NULL); a call with neither returns DECT_OK without
 *   looking, and the next synchronising call on the same state reports it.
 */
dect_status dect_adm_tv(const dect_geometry *geom, const float *d_m_high, const float *d_m_low,
                        const dect_adm_params *params, float *d_x_high, float *d_x_low,
                        dect_adm_state *state, dect_report *rep, void *stream);

dect_status dect_adm_state_create(const dect_geometry *geom, dect_adm_state **out);
dect_status dect_adm_state_destroy(dect_adm_state *state);

/*
 * Empty a state, so that the next dect_adm_tv call on it starts a new run
 * (from zero, or from its x inputs with DECT_WARM_START).  The state keeps its
 * buffers and captured iteration graphs.  Asynchronous work already queued on
 * the state must be on the stream the next call uses.  DECT_ERR_INVALID_ARG
 * for a NULL state.
 */
dect_status dect_adm_state_reset(dect_adm_state *state);

/*
 * Image-domain decomposition by penalised least squares (Eqs. 11-15): the
 * direct decomposition b = D^{-1} x per pixel (Eq. 12), then per material
 * (I + gamma L) u = b, the normal equations of Eq. 13 with the edge-weighted
 * quadratic smoothness of Eq. 14 (grad R = 2 L, Eq. 15), solved by
 * Jacobi-preconditioned CG from u = b.
 * d_edge_w: NULL to detect edges on d_x_low (Prewitt, see
 *   dect_pls_edge_weights), or a [2][ny][nx] map (right pairs, down pairs).
 * d_u_water/d_u_bone: [ny][nx] outputs (unitless material fractions).
 * rep: NULL or filled after synchronising (iterations, final residual).
 */
dect_status dect_pls_decompose(int32_t nx, int32_t ny, const float *d_x_high,
                               const float *d_x_low, const dect_pls_params *params,
                               const float *d_edge_w, float *d_u_water, float *d_u_bone,
                               dect_report *rep, void *stream);

/*
 * dect_pls_decompose for callers that cannot allocate device memory (code
 * under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, results (bit for bit) and errors, and no
 * allocation of any kind.  Limits: mode DECT_PLS_IMAGE only and
 * nx * ny <= 262144 pixels (512 x 512); DECT_ERR_INVALID_ARG otherwise.
 * Its work memory is one library-owned array per GPU (about 17 MB, in the
 * library's code object), held until the process ends.  All calls on one GPU
 * share that array, so calls that overlap on one GPU (other streams or
 * threads) race: the caller serialises them.  Every call writes the parts of
 * the array it reads before reading them, so nothing needs clearing between
 * calls.
 */
dect_status dect_pls_decompose_noalloc(int32_t nx, int32_t ny, const float *d_x_high,
                                       const float *d_x_low, const dect_pls_params *params,
                                       const float *d_edge_w, float *d_u_water, float *d_u_bone,
                                       dect_report *rep, void *stream);

/*
 * Edge weights e_ik of Eq. 14 from a Prewitt edge map of d_x (Sec. 2.3:
 * small at edges, one elsewhere): m2 = fmaf(gx, gx, gy*gy) with gx, gy the
 * Prewitt responses (replicated borders), edge where m2 > fp32(tau^2) *
 * max m2.  d_w[0][r][c] couples (r,c)-(r,c+1), d_w[1][r][c] couples
 * (r,c)-(r+1,c): eps if either pixel is an edge, 1 otherwise, 0 for pairs
 * leaving the image.  d_w is [2][ny][nx] float32.
 */
dect_status dect_pls_edge_weights(int32_t nx, int32_t ny, const float *d_x, double tau,
                                  double eps, float *d_w, void *stream);

/*
 * Batched ADM-TV (Eq. 10 for many slices at once): slices of uneven image
 * size, view count and parameters, both energies each, advanced together;
 * every phase of an iteration is one launch over a work list that
 * spans all slices, replayed from a hipGraph.  Starts from zero images.
 * geoms/params: host arrays [n] (params[i].max_iter and DECT_WARM_START are ignored);
 *   each slice takes either projector model and the flags of dect_adm_tv
 *   with the same restrictions (DECT_COUPLED_TV with tol 0; DECT_STEP_BB2 /
 *   DECT_STEP_ABB neither together nor with DECT_NONNEG; else
 *   DECT_ERR_INVALID_ARG); every slice's result is bit for bit its
 *   dect_adm_tv run with the same view grouping.
 * d_m_high, d_m_low, d_x_high, d_x_low: host arrays [n] of device pointers
 *   to slice i's sinograms [V_i][B_i] and output images [ny_i][nx_i].
 * objective: NULL or host [n], filled after synchronising the stream with
 *   J(f^K) of Eq. 4 summed over both energies.
 * dect_batch_tune chooses the batch's launch shape by timing `iters`
 * iterations per candidate on the given data (coordinate descent): for each
 * class of equal slices (image size and view count, costliest first) the
 * adjoint view-group depth 1, 2, 4, 8 or 16 (blocks sharing one output
 * strip, i.e. views per adjoint tile), then the adjoint and forward grids
 * (one block per work item, or a persistent grid of 1 or 2 blocks per CU).
 * The choice is remembered for the process: a batch with the same multiset
 * of slice shapes (nx, ny, n_views, n_bins, model, variant flags) takes it
 * without timing.  *chosen_groups receives the depth of the costliest slice,
 * *ms_per_iter the tuned time per iteration.  dect_batch_set_groups fixes
 * one depth for every slice (0 = built-in heuristic) and drops the tuned
 * shape; dect_batch_shape reports the depth per slice (host array [n]), the
 * grids (0 = one block per work item, k = k blocks per CU) and whether the
 * last tune came from the process cache.
 */
typedef struct dect_batch dect_batch;
dect_status dect_batch_create(const dect_geometry *geoms, const dect_adm_params *params,
                              int32_t n, dect_batch **out);
dect_status dect_batch_destroy(dect_batch *batch);
dect_status dect_adm_tv_batched(dect_batch *batch, const float *const *d_m_high,
                                const float *const *d_m_low, float *const *d_x_high,
                                float *const *d_x_low, int32_t iters, double *objective,
                                void *stream);
dect_status dect_batch_tune(dect_batch *batch, const float *const *d_m_high,
                            const float *const *d_m_low, int32_t iters, int32_t *chosen_groups,
                            double *ms_per_iter, void *stream);
dect_status dect_batch_set_groups(dect_batch *batch, int32_t groups);
dect_status dect_batch_shape(const dect_batch *batch, int32_t *groups_per_slice,
                             int32_t *adj_blocks_per_cu, int32_t *fwd_blocks_per_cu,
                             int32_t *from_cache);

/*
 * 3-D circular cone beam with a flat panel (the scanner of Sec. 3, of which
 * dect_geometry is the central plane z = 0).  Source at SOD (cos t, sin t,
 * 0); panel centred at -(SDD - SOD)(cos t, sin t, 0), bin b of row j at
 * u_b = (b - (n_bins-1)/2) bin_mm + det_offset_mm along (-sin t, cos t, 0)
 * and v_j = (j - (n_rows-1)/2) row_mm along z.  Volume [nz][ny][nx] of cubic
 * voxels of side voxel_mm centred on the isocentre; projections
 * [n_views][n_rows][n_bins].  angles_rad: NULL for 2 pi v / n_views, else
 * n_views host values.  Checked: sizes positive (nx, ny, nz <= 4096, bins and
 * rows <= 16384, views <= 65536), the orbit outside the volume, SDD > SOD,
 * fan angle below 90 degrees and cone half-angle below atan(1/2) (so the
 * height never drives a ray).
 */
typedef struct {
    int32_t nx, ny, nz;
    double voxel_mm;
    int32_t n_views;
    const double *angles_rad;
    int32_t n_bins, n_rows;
    double bin_mm, row_mm, det_offset_mm, sod_mm, sdd_mm;
} dect_cone_geometry;

/*
 * Cone-beam forward projection d_proj = A3 d_vol: Joseph's model (Sec. 2.4's
 * projector) carried to 3-D -- each ray steps along the in-plane axis it is
 * more aligned with and, on every plane of that axis, interpolates
 * bilinearly between the four nearest voxel centres (other in-plane axis and
 * height), scaled by the path length per plane; outside the volume is zero.
 * Device buffers: d_vol [nz][ny][nx], d_proj [n_views][n_rows][n_bins]
 * (caller-owned, not aliased).  Uses a library-owned workspace per (device,
 * stream) holding two padded copies of the volume.  Asynchronous on
 * `stream` except when the view table changes (then the stream is
 * synchronised once).
 */
dect_status dect_cone_project(const dect_cone_geometry *geom, const float *d_vol, float *d_proj,
                              void *stream);

/*
 * Cone-beam back-projection d_vol = A3^T d_proj: the transpose of
 * dect_cone_project's matrix in gather form -- every voxel sums over the
 * rays that reach it, with the forward pass's in-plane interpolation weight
 * (the same 32.32 coordinate) and its height weight evaluated in FP64; no
 * atomics, so repeated calls agree bit for bit.  d_vol is overwritten.
 * Uses the workspace of dect_cone_project plus a scaled copy of d_proj.
 */
dect_status dect_cone_backproject(const dect_cone_geometry *geom, const float *d_proj,
                                  float *d_vol, void *stream);

/*
 * ADM-TV of both energies on a volume (Eq. 10 with the TV of Eq. 2 taken
 * over backward differences along x, y and z -- the six-neighbour form --
 * and the isotropic shrinkage of Eq. 8 on the 3-vector), with A the
 * cone-beam pair above.  d_m_* [n_views][n_rows][n_bins] device, d_x_*
 * [nz][ny][nx] device outputs (x = f / beta), and with DECT_WARM_START
 * also the start images (f = beta x; they may be the same buffers).  params
 * as for dect_adm_tv, flags DECT_WARM_START, DECT_NONNEG (each step
 * projected onto f >= 0, the BB step from the projected step; the residual
 * follows A s of that step, so A G is formed for the first step only),
 * DECT_STEP_BB2 or DECT_STEP_ABB (which here combine with DECT_NONNEG),
 * DECT_COUPLED_TV (the shrinkage of Eq. 8 on the 6-vector of both energies'
 * gradients; BB1 step and tol = 0 only, else DECT_ERR_INVALID_ARG; J_high
 * then holds the joint TV and J_low none).  tol must be finite and >= 0.  tol > 0: each energy stops after the first iteration whose
 * relative change |f^{k+1}-f^k| / |f^k| is below tol, the other running on
 * until it stops too or max_iter is reached (the host reads both relative
 * changes after every iteration, one stream synchronisation each).
 * params->log, when not NULL, receives the [max_iter+1][4] rows {J_high,
 * J_low, alpha_high, alpha_low}; an energy's rows after its last iteration
 * hold zeros.  rep->iters is the larger of the two iteration counts.
 * The two energies advance together (each with its own step), every
 * projector call walking both volumes at once.  The iterate and the
 * residual A f - beta m are pairs of FP32 values updated in FP64 (the
 * residual by the recurrence r -= alpha A G), the rest of the state FP32,
 * reductions FP64.  Its work buffers (per energy 15 volume-sized arrays
 * and 4 projection sets) are library-owned per device and kept between calls;
 * the call synchronises the stream before returning.
 * DECT_ERR_NONFINITE when a logged objective or step is not finite.
 */
dect_status dect_adm_tv3(const dect_cone_geometry *geom, const float *d_m_high,
                         const float *d_m_low, const dect_adm_params *params, float *d_x_high,
                         float *d_x_low, dect_report *rep, void *stream);

/*
 * PLS decomposition of volumes (Eqs. 11-15 with R of Eq. 14 over the six
 * face neighbours), L the six-neighbour Laplacian with pair weights from
 * d_edge_w.  DECT_PLS_IMAGE: u = D^{-1} x per voxel (Eq. 12), then (I +
 * gamma L) u_m = (D^{-1} x)_m per material by Jacobi-PCG from u = D^{-1} x
 * (FP32 vectors, FP64 dot products).  DECT_PLS_ATTENUATION: the coupled
 * system (D^T D (x) I + gamma I (x) L) u = D^T x of |x - D u|^2 + gamma R(u),
 * block-Jacobi CG from D^{-1} x with one tolerance over both materials, in
 * FP64.  Device buffers d_x_* [nz][ny][nx] in, d_u_water / d_u_bone
 * [nz][ny][nx] out.
 * d_edge_w: NULL to detect edges on d_x_low (dect_pls_edge_weights3), or a
 *   [3][nz][ny][nx] map of pair weights (x, y and z pairs as there).
 * params as for dect_pls_decompose; stops when |res| <= tol |b| or after
 * max_iter iterations (per material in image mode).  Work buffers (about 10
 * FP32 volumes in image mode, 10 FP64 ones in the attenuation mode) are
 * library-owned per device and kept between calls; the call synchronises the
 * stream.  rep: iters (the larger of the two materials) and pcg_residual;
 * DECT_WARN_MAXITER (also returned) when max_iter stopped a solve above its
 * tolerance, the outputs then holding the last iterate.
 */
dect_status dect_pls_decompose3(int32_t nx, int32_t ny, int32_t nz, const float *d_x_high,
                                const float *d_x_low, const dect_pls_params *params,
                                const float *d_edge_w, float *d_u_water, float *d_u_bone,
                                dect_report *rep, void *stream);

/*
 * Pair weights e_ik of Eq. 14 over the six face neighbours from the 3-D
 * Prewitt edge map of d_x (per axis, the 3 x 3 face sum at +1 minus the one
 * at -1, borders replicated): an edge where the squared magnitude exceeds
 * tau^2 times the largest (evaluated in FP32 as
 * fmaf(gx, gx, fmaf(gy, gy, gz*gz)) against fp32(tau^2) * max).  d_w[0]
 * couples i and i + 1 (x), d_w[1] i and i + nx (y), d_w[2] i and i + nx ny
 * (z): eps if either voxel is an edge, 1 otherwise, 0 for pairs leaving the
 * volume.  d_x [nz][ny][nx], d_w [3][nz][ny][nx] float32, both device
 * memory of the caller.  DECT_ERR_INVALID_ARG for bad sizes, tau or eps.
 */
dect_status dect_pls_edge_weights3(int32_t nx, int32_t ny, int32_t nz, const float *d_x,
                                   double tau, double eps, float *d_w, void *stream);

/*
 * Unrolled ADM-TV (the reconstruction procedure of Eq. 10 with a given step
 * alpha_k in place of the BB step, and learnable (mu_k, rho_k, xi_k,
 * alpha_k)), the differentiable path of the learned parameters.  A step
 * runs as: p = A f (dect_project), r = p - g (dect_unrolled_residual),
 * hb = A^T r (dect_backproject), then dect_unrolled_step.  Their
 * vector-Jacobian products are dect_backproject, identity, dect_project and
 * dect_unrolled_step_backward.
 *
 * dect_unrolled_residual: d_r[i] = d_p[i] - d_g[i] for i < n, device
 * buffers of n float32 (d_r may equal d_p).  DECT_ERR_INVALID_ARG for n < 0
 * or a NULL buffer with n > 0.
 */
dect_status dect_unrolled_residual(int64_t n, const float *d_p, const float *d_g, float *d_r,
                                   void *stream);

/*
 * One unrolled step for `batch` images [batch][ny][nx] (float32, device):
 *   z       = shrink(grad f - lambda / rho, 1 / rho)                   (Eq. 8)
 *   G       = mu hb + grad^T (rho (grad f - z) - lambda)               (Eq. 9)
 *   f_out   = f - alpha G
 *   lam_out = lambda - xi (grad f_out - z)                             (Eq. 7)
 * grad: the backward differences of Eq. 2 (x along a row, y down the
 * columns; zero on the first column and row), grad^T its exact adjoint;
 * shrink(v, t) = max(|v| - t, 0) v / |v| with |v| evaluated as sqrt(max(
 * |v|^2, 1e-30)).  lambda = (d_lx, d_ly); d_hb = A^T (A f - g) of each
 * image; d_params: device float32 [4] = (mu, rho, xi, alpha), read on the
 * device (no host synchronisation).  Outputs must not overlap the inputs or
 * each other (DECT_ERR_INVALID_ARG); bad sizes give DECT_ERR_INVALID_ARG.
 * Asynchronous on `stream`; no allocation.
 */
dect_status dect_unrolled_step(int32_t nx, int32_t ny, int32_t batch, const float *d_f,
                               const float *d_lx, const float *d_ly, const float *d_hb,
                               const float *d_params, float *d_f_out, float *d_lx_out,
                               float *d_ly_out, void *stream);

/*
 * The vector-Jacobian product of dect_unrolled_step at (d_f, d_lx, d_ly,
 * d_hb, d_params) for the cotangents d_gf_out, d_glx_out, d_gly_out of its
 * three outputs: d_gf, d_glx, d_gly, d_ghb receive the cotangents of f,
 * lambda and hb ([batch][ny][nx] float32, device) and d_gparams (device
 * float32 [4]) those of (mu, rho, xi, alpha), each the FP64 sum of per-block
 * partial sums in a fixed order (bitwise reproducible).  The shrinkage is
 * differentiated where |v| > 1/rho and has zero derivative elsewhere.
 * Outputs must not overlap the inputs or each other.  Work memory (six
 * images of the batch) is library-owned per device and kept between calls
 * (or drawn from the workspace of dect_set_workspace).
 */
dect_status dect_unrolled_step_backward(int32_t nx, int32_t ny, int32_t batch, const float *d_f,
                                        const float *d_lx, const float *d_ly, const float *d_hb,
                                        const float *d_params, const float *d_gf_out,
                                        const float *d_glx_out, const float *d_gly_out,
                                        float *d_gf, float *d_glx, float *d_gly, float *d_ghb,
                                        float *d_gparams, void *stream);

/* Number of Joseph samples (ray, line) with the crossing inside (-1, n)
 * for a geometry: the unit of projector work. */
dect_status dect_count_samples(const dect_geometry *geom, int64_t *out);

/* Free every library-owned device buffer: cached geometry tables, work
 * buffers and the ADM states the library made for calls without one (states
 * and batches that callers created stay).  Waits for the device first. */
dect_status dect_release_caches(void);

/*
 * Caller-provided device memory for the library's own buffers (the
 * library owns its tables and work buffers unless the caller hands it a
 * region).  After dect_set_workspace(d_ptr, bytes) every device
 * allocation the library makes on the current device (geometry tables, work
 * buffers, ADM states and batches created from then on) is a consecutive
 * 256-byte-aligned piece of [d_ptr, d_ptr + bytes) instead of a hipMalloc;
 * pieces are never reused or returned one by one.  A call that needs more
 * than is left fails with DECT_ERR_INVALID_ARG before launching anything.
 * The call waits for the device and first releases every buffer the library
 * holds on this device (as dect_release_caches), so the next calls rebuild
 * theirs inside the workspace.  d_ptr NULL with bytes 0 returns to hipMalloc.
 * The caller keeps the memory alive and untouched until it replaces or
 * clears the workspace, and destroys states and batches created while it was
 * set before doing so.  d_ptr must be 256-byte aligned (DECT_ERR_INVALID_ARG
 * otherwise).
 */
dect_status dect_set_workspace(void *d_ptr, size_t bytes);

/* Bytes of the current device's caller workspace in use (0 without one). */
dect_status dect_workspace_used(size_t *bytes);

/*
 * Bytes the 2-D calls need on geom when the library holds nothing yet: its
 * geometry tables, one dect_adm_tv run without a caller state (any step
 * rule), dect_project / dect_backproject / dect_fbp on up to `batch` items
 * on one stream, and dect_pls_decompose at the geometry's image size in
 * either mode with edges detected.  Computed by a dry run of those
 * allocations that builds the tables on the host and touches no device
 * memory.  Later calls with larger batches, other streams or other
 * geometries need more.  DECT_ERR_INVALID_ARG for batch <= 0 or bytes NULL;
 * geometry errors as dect_project.
 */
dect_status dect_workspace_size(const dect_geometry *geom, int32_t batch, size_t *bytes);

/* Message of the last failure on the calling thread ("" if none). */
const char *dect_last_error(void);

/* Library version string. */
const char *dect_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DECT_H */
