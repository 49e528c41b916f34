// Internal declarations of the volume solvers (3-D ADM-TV and 3-D PLS).
#pragma once

#include "common.h"

namespace dect {

// The cone-beam pair on two volumes sharing one geometry (both walked
// together, interleaved; each result equal to the single-volume call's).
dect_status cone_project2(const dect_cone_geometry *g, const float *const vol[2],
                          float *const proj[2], hipStream_t s);
// cone_project2 that also writes lo[e] = (FP64 ray sum) - proj[e] rounded to
// FP32, so that proj + lo is the ray sum to about 2^-48 relative.
dect_status cone_project2_lo(const dect_cone_geometry *g, const float *const vol[2],
                             float *const proj[2], float *const lo[2], hipStream_t s);
dect_status cone_backproject2(const dect_cone_geometry *g, const float *const proj[2],
                              float *const vol[2], hipStream_t s);

dect_status adm_tv3(const dect_cone_geometry *g, const float *m_high, const float *m_low,
                    const dect_adm_params *p, float *x_high, float *x_low, dect_report *rep,
                    hipStream_t s);
dect_status pls_decompose3(int nx, int ny, int nz, const float *xh, const float *xl,
                           const dect_pls_params *p, const float *ew, float *u1, float *u2,
                           dect_report *rep, hipStream_t s);
dect_status pls_edge_weights3(int nx, int ny, int nz, const float *x, double tau, double eps,
                              float *w, hipStream_t s);
void release_pls3_work();

}  // namespace dect
