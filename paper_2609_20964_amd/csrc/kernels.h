// Kernel declarations shared between the HIP translation units (internal).
#pragma once

#include "common.h"

namespace wg {

// Grid geometry handed to point- and query-side kernels.
struct GridF {
    Dims d;
    double lo[3];
    double h;
};

// ---- splat.hip -------------------------------------------------------------
__global__ void k_splat_div(const float *xyz, const float *nrm, int npts, GridF g, float *b, int32_t *keys,
                            float *xyz_c, float *nrm_c, int *err);
__global__ void k_iso_partial(const float *xyz, int npts, GridF g, const double *chi, double *partials);
__global__ void k_iso_finalize(const double *partials, int nb, int npts, double *out);
__global__ void k_iso_T(const float *xyz, int npts, GridF g, const double *g_c, float *g_chi);
__global__ void k_splat_T(const float *xyz, const float *nrm, const int32_t *keys, int npts, GridF g,
                          const double *lam, const double *chi, const double *g_c, float *gxyz, float *gnrm);

}  // namespace wg
