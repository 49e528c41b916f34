// Internal declarations of the volume solvers (3-D ADM-TV and 3-D PLS).
#pragma once

#include "common.h"

namespace dect {

dect_status adm_tv3(const dect_cone_geometry *g, const float *m_high, const float *m_low,
                    const dect_adm_params *p, float *x_high, float *x_low, dect_report *rep,
                    hipStream_t s);
dect_status pls_decompose3(int nx, int ny, int nz, const float *xh, const float *xl,
                           const dect_pls_params *p, float *u1, float *u2, dect_report *rep,
                           hipStream_t s);

}  // namespace dect
