// Launchers of the image-space kernels (defined in lm_image.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "lm_device.hpp"

namespace lmk {

// x <- max(0, x - T zbar)
int launch_primal(float *x, const float *T, const float *zbar, long long nv, hipStream_t st);

// z += dz; zbar = z + dz * inv_p; fuse ? x <- max(0, x - T zbar) : store zbar; dz = 0
int launch_dual_image(float *z, float *dz, float *x, const float *T, float *zbar, float inv_p, bool fuse,
                      long long nv, hipStream_t st);

// Images of the prior update use layout L (padding skipped).
// The whole prior update in one pass: w_out = proj_beta(w + Sp K x),
// dz = K^T(w_out - w), z += dz, zbar = z + dz inv_p, fuse ? x_out = max(0,
// x - T zbar) : store zbar.  x and w are only read (x_out, w_out separate).
// K = grad (TV), or with xi != NULL K = D grad with D = I - xi xi^T per
// voxel (DTV; xi: 3 components in layout L), which needs prior_march_ok.
int launch_tv_fused(const int n[3], const Layout &L, int ncomp, const float *x, const float *w, const float *xi,
                    float *w_out, float *z, float *x_out, const float *T, float *zbar, float Sp, float beta,
                    float inv_p, bool fuse, hipStream_t st);
// Layouts whose prior update runs as one pass marching along z (4x4x4
// bricks, 3 components).
bool prior_march_ok(const Layout &L, int ncomp);

// Conversions between the caller's row-major images (ncomp components of
// n[0] n[1] n[2] elements) and layout L (ncomp components of layout_size(L)).
int launch_to_layout(const int n[3], const Layout &L, int ncomp, const float *src, float *dst, hipStream_t st);
int launch_from_layout(const int n[3], const Layout &L, int ncomp, const float *src, float *dst, hipStream_t st);

int launch_grad(const int n[3], const float *x, float *gx, hipStream_t st);
int launch_div(const int n[3], const float *w, float *out, hipStream_t st);

}  // namespace lmk
