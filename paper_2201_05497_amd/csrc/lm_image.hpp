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
// wn = proj_beta(w + Sp K x); ncomp = 3 for a 3D image, 2 when nz == 1.
int launch_tv_dual(const int n[3], const Layout &L, int ncomp, const float *x, const float *w, float *wn, float Sp,
                   float beta, hipStream_t st);
// dz = K^T(wn - w); z += dz; zbar = z + dz inv_p; fuse ? x update : store zbar.
int launch_tv_adjoint(const int n[3], const Layout &L, int ncomp, const float *w, const float *wn, float *z,
                      float *x, const float *T, float *zbar, float inv_p, bool fuse, hipStream_t st);

// Conversions between the caller's row-major images (ncomp components of
// n[0] n[1] n[2] elements) and layout L (ncomp components of layout_size(L)).
int launch_to_layout(const int n[3], const Layout &L, int ncomp, const float *src, float *dst, hipStream_t st);
int launch_from_layout(const int n[3], const Layout &L, int ncomp, const float *src, float *dst, hipStream_t st);

int launch_grad(const int n[3], const float *x, float *gx, hipStream_t st);
int launch_div(const int n[3], const float *w, float *out, hipStream_t st);

}  // namespace lmk
