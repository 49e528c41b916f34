// extern "C" entry points of libdect (declared in include/dect.h).
#include "common.h"
#include "volume.h"

namespace dect {
const char *last_error();
dect_status adm_tv(const dect_geometry *g, const float *mh, const float *ml,
                   const dect_adm_params *P, float *xh, float *xl, dect_adm_state *state,
                   dect_report *rep, hipStream_t s);
dect_status adm_state_create(const dect_geometry *g, dect_adm_state **out);
dect_status adm_state_destroy(dect_adm_state *S);
dect_status adm_state_reset(dect_adm_state *S);
dect_status pls_decompose(int nx, int ny, const float *xh, const float *xl,
                          const dect_pls_params *P, const float *ew, float *u1, float *u2,
                          dect_report *rep, hipStream_t s);
dect_status pls_edge_weights(int nx, int ny, const float *x, double tau, double eps, float *w,
                             hipStream_t s);
dect_status pls_decompose_noalloc(int nx, int ny, const float *xh, const float *xl,
                                  const dect_pls_params *P, const float *ew, float *u1,
                                  float *u2, dect_report *rep, hipStream_t s);
dect_status batch_create(const dect_geometry *geoms, const dect_adm_params *prm, int n,
                         dect_batch **out);
dect_status batch_destroy(dect_batch *b);
dect_status adm_tv_batched(dect_batch *b, const float *const *mh, const float *const *ml,
                           float *const *xh, float *const *xl, int iters, double *objective,
                           hipStream_t s);
dect_status batch_tune(dect_batch *b, const float *const *mh, const float *const *ml, int iters,
                       int32_t *chosen, double *ms_per_iter, hipStream_t s);
dect_status batch_set_groups(dect_batch *b, int groups);
dect_status batch_shape(const dect_batch *b, int32_t *groups, int32_t *adj_per_cu,
                        int32_t *fwd_per_cu, int32_t *from_cache);
dect_status unrolled_residual(int64_t n, const float *p, const float *g, float *r, hipStream_t s);
dect_status unrolled_step(int nx, int ny, int batch, const float *f, const float *lx,
                          const float *ly, const float *hb, const float *prm, float *fo,
                          float *lxo, float *lyo, hipStream_t s);
dect_status unrolled_step_backward(int nx, int ny, int batch, const float *f, const float *lx,
                                   const float *ly, const float *hb, const float *prm,
                                   const float *gfo, const float *glxo, const float *glyo,
                                   float *gf, float *glx, float *gly, float *ghb, float *gprm,
                                   hipStream_t s);

// Bytes the 2-D calls allocate on geom when nothing is held yet: a dry run
// of their allocations (tables, one ADM run without a caller state, the
// projector pair and FBP for `batch` items on one stream, PLS in both modes),
// counted by a SizingScope and never touching device memory.
dect_status workspace_size(const dect_geometry *g, int batch, size_t *bytes)
{
    if (!bytes) return fail(DECT_ERR_INVALID_ARG, "dect_workspace_size: bytes is NULL");
    if (batch <= 0) return fail(DECT_ERR_INVALID_ARG, "dect_workspace_size: batch must be positive");
    dect_status st = validate_geometry(g);
    if (st) return st;
    SizingScope sc;
    if ((st = adm_size_run(g)) || (st = proj_size_run(g, batch)) ||
        (st = fbp_size_run(g, batch)) || (st = pls_size_run((size_t)g->nx * g->ny)))
        return st;
    *bytes = sc.bytes;
    return DECT_OK;
}

void release_device_buffers()
{
    release_adm_states();
    release_proj_work();
    release_fbp_work();
    release_pls_work();
    release_pls3_work();
    release_cone_work();
    release_adm3_work();
    release_unrolled_work();
    release_tables();
}
}  // namespace dect

extern "C" {

dect_status dect_batch_create(const dect_geometry *geoms, const dect_adm_params *params,
                              int32_t n, dect_batch **out)
{
    dect::set_error("");
    return dect::batch_create(geoms, params, n, out);
}

dect_status dect_batch_destroy(dect_batch *batch) { return dect::batch_destroy(batch); }

dect_status dect_adm_tv_batched(dect_batch *batch, const float *const *d_m_high,
                                const float *const *d_m_low, float *const *d_x_high,
                                float *const *d_x_low, int32_t iters, double *objective,
                                void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_adm_tv_batched");
    return dect::adm_tv_batched(batch, d_m_high, d_m_low, d_x_high, d_x_low, iters, objective,
                                (hipStream_t)stream);
}

dect_status dect_batch_tune(dect_batch *batch, const float *const *d_m_high,
                            const float *const *d_m_low, int32_t iters, int32_t *chosen_groups,
                            double *ms_per_iter, void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_batch_tune");
    return dect::batch_tune(batch, d_m_high, d_m_low, iters, chosen_groups, ms_per_iter,
                            (hipStream_t)stream);
}

dect_status dect_batch_set_groups(dect_batch *batch, int32_t groups)
{
    dect::set_error("");
    return dect::batch_set_groups(batch, groups);
}

dect_status dect_batch_shape(const dect_batch *batch, int32_t *groups_per_slice,
                             int32_t *adj_blocks_per_cu, int32_t *fwd_blocks_per_cu,
                             int32_t *from_cache)
{
    dect::set_error("");
    return dect::batch_shape(batch, groups_per_slice, adj_blocks_per_cu, fwd_blocks_per_cu,
                             from_cache);
}

dect_status dect_project(const dect_geometry *geom, const float *d_img, float *d_sino,
                         int32_t batch, void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_project");
    return dect::project(geom, d_img, d_sino, batch, (hipStream_t)stream);
}

dect_status dect_backproject(const dect_geometry *geom, const float *d_sino, float *d_img,
                             int32_t batch, void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_backproject");
    return dect::backproject(geom, d_sino, d_img, batch, (hipStream_t)stream);
}

dect_status dect_fbp(const dect_geometry *geom, const float *d_sino, float *d_img, int32_t batch,
                     void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_fbp");
    return dect::fbp(geom, d_sino, d_img, batch, (hipStream_t)stream);
}

dect_status dect_cone_project(const dect_cone_geometry *geom, const float *d_vol, float *d_proj,
                              void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_cone_project");
    return dect::cone_project(geom, d_vol, d_proj, (hipStream_t)stream);
}

dect_status dect_cone_backproject(const dect_cone_geometry *geom, const float *d_proj,
                                  float *d_vol, void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_cone_backproject");
    return dect::cone_backproject(geom, d_proj, d_vol, (hipStream_t)stream);
}

dect_status dect_adm_tv3(const dect_cone_geometry *geom, const float *d_m_high,
                         const float *d_m_low, const dect_adm_params *params, float *d_x_high,
                         float *d_x_low, dect_report *rep, void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_adm_tv3");
    return dect::adm_tv3(geom, d_m_high, d_m_low, params, d_x_high, d_x_low, rep,
                         (hipStream_t)stream);
}

dect_status dect_pls_decompose3(int32_t nx, int32_t ny, int32_t nz, const float *d_x_high,
                                const float *d_x_low, const dect_pls_params *params,
                                const float *d_edge_w, float *d_u_water, float *d_u_bone,
                                dect_report *rep, void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_pls_decompose3");
    return dect::pls_decompose3(nx, ny, nz, d_x_high, d_x_low, params, d_edge_w, d_u_water,
                                d_u_bone, rep, (hipStream_t)stream);
}

dect_status dect_pls_edge_weights3(int32_t nx, int32_t ny, int32_t nz, const float *d_x,
                                   double tau, double eps, float *d_w, void *stream)
{
    dect::set_error("");
    return dect::pls_edge_weights3(nx, ny, nz, d_x, tau, eps, d_w, (hipStream_t)stream);
}

dect_status dect_adm_tv(const dect_geometry *geom, const float *d_m_high, const float *d_m_low,
                        const dect_adm_params *params, float *d_x_high, float *d_x_low,
                        dect_adm_state *state, dect_report *rep, void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_adm_tv");
    return dect::adm_tv(geom, d_m_high, d_m_low, params, d_x_high, d_x_low, state, rep,
                        (hipStream_t)stream);
}

dect_status dect_adm_state_create(const dect_geometry *geom, dect_adm_state **out)
{
    dect::set_error("");
    return dect::adm_state_create(geom, out);
}

dect_status dect_adm_state_destroy(dect_adm_state *state)
{
    return dect::adm_state_destroy(state);
}

dect_status dect_adm_state_reset(dect_adm_state *state)
{
    return dect::adm_state_reset(state);
}

dect_status dect_pls_decompose(int32_t nx, int32_t ny, const float *d_x_high,
                               const float *d_x_low, const dect_pls_params *params,
                               const float *d_edge_w, float *d_u_water, float *d_u_bone,
                               dect_report *rep, void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_pls_decompose");
    return dect::pls_decompose(nx, ny, d_x_high, d_x_low, params, d_edge_w, d_u_water, d_u_bone,
                               rep, (hipStream_t)stream);
}

dect_status dect_pls_decompose_noalloc(int32_t nx, int32_t ny, const float *d_x_high,
                                       const float *d_x_low, const dect_pls_params *params,
                                       const float *d_edge_w, float *d_u_water, float *d_u_bone,
                                       dect_report *rep, void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_pls_decompose_noalloc");
    return dect::pls_decompose_noalloc(nx, ny, d_x_high, d_x_low, params, d_edge_w, d_u_water,
                                       d_u_bone, rep, (hipStream_t)stream);
}

dect_status dect_pls_edge_weights(int32_t nx, int32_t ny, const float *d_x, double tau,
                                  double eps, float *d_w, void *stream)
{
    dect::set_error("");
    return dect::pls_edge_weights(nx, ny, d_x, tau, eps, d_w, (hipStream_t)stream);
}

dect_status dect_count_samples(const dect_geometry *geom, int64_t *out)
{
    dect::set_error("");
    if (!out) return dect::fail(DECT_ERR_INVALID_ARG, "dect_count_samples: out is NULL");
    dect::GeomTables *t = nullptr;
    dect_status st = dect::get_tables(geom, &t);
    if (st != DECT_OK) return st;
    *out = t->samples;
    return DECT_OK;
}

dect_status dect_release_caches(void)
{
    (void)hipDeviceSynchronize();
    dect::release_device_buffers();
    return DECT_OK;
}

dect_status dect_set_workspace(void *d_ptr, size_t bytes)
{
    dect::set_error("");
    return dect::set_workspace(d_ptr, bytes);
}

dect_status dect_workspace_used(size_t *bytes)
{
    dect::set_error("");
    return dect::workspace_used(bytes);
}

dect_status dect_workspace_size(const dect_geometry *geom, int32_t batch, size_t *bytes)
{
    dect::set_error("");
    return dect::workspace_size(geom, batch, bytes);
}

dect_status dect_unrolled_residual(int64_t n, const float *d_p, const float *d_g, float *d_r,
                                   void *stream)
{
    dect::set_error("");
    return dect::unrolled_residual(n, d_p, d_g, d_r, (hipStream_t)stream);
}

dect_status dect_unrolled_step(int32_t nx, int32_t ny, int32_t batch, const float *d_f,
                               const float *d_lx, const float *d_ly, const float *d_hb,
                               const float *d_params, float *d_f_out, float *d_lx_out,
                               float *d_ly_out, void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_unrolled_step");
    return dect::unrolled_step(nx, ny, batch, d_f, d_lx, d_ly, d_hb, d_params, d_f_out, d_lx_out,
                               d_ly_out, (hipStream_t)stream);
}

dect_status dect_unrolled_step_backward(int32_t nx, int32_t ny, int32_t batch, const float *d_f,
                                        const float *d_lx, const float *d_ly, const float *d_hb,
                                        const float *d_params, const float *d_gf_out,
                                        const float *d_glx_out, const float *d_gly_out,
                                        float *d_gf, float *d_glx, float *d_gly, float *d_ghb,
                                        float *d_gparams, void *stream)
{
    dect::set_error("");
    DECT_TRACE("dect_unrolled_step_backward");
    return dect::unrolled_step_backward(nx, ny, batch, d_f, d_lx, d_ly, d_hb, d_params, d_gf_out,
                                        d_glx_out, d_gly_out, d_gf, d_glx, d_gly, d_ghb,
                                        d_gparams, (hipStream_t)stream);
}

const char *dect_last_error(void) { return dect::last_error(); }

const char *dect_version(void) { return "libdect 0.1 (gfx950)"; }

}  // extern "C"
