// Launchers of the directional TV prior (defined in lm_dtv.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "lm_device.hpp"

namespace lmk {

// xi = grad v / sqrt(|grad v|^2 + eta^2) of the row-major prior image v,
// written in layout L (ncomp components of ne elements; padding untouched).
int launch_dtv_field(const int n[3], const Layout &L, int ncomp, long long ne, const float *v, float eta, float *xi,
                     hipStream_t st);

// Prior update of LM-SPDHG with K = D grad, D = I - xi xi^T, in two passes
// (the plan uses it for one-slice images; 3D images take launch_tv_fused
// with xi):
// w_out = proj_beta(w + Sp D grad x), dz = grad^T D (w_out - w) (pd holds
// D (w_out - w), ncomp components), z += dz, zbar = z + dz inv_p, and
// fuse ? x = max(0, x - T zbar) in place : store zbar.  All in layout L.
int launch_dtv_prior(const int n[3], const Layout &L, int ncomp, long long ne, float *x, const float *w,
                     float *w_out, const float *xi, float *pd, float *z, const float *T, float *zbar, float Sp,
                     float beta, float inv_p, bool fuse, hipStream_t st);

}  // namespace lmk
