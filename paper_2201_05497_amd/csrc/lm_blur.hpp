// Image-space resolution model of the forward model (defined in
// lm_blur.hip): a separable Gaussian convolution B, so that P = G B.
#pragma once

#include <hip/hip_runtime.h>

#include "lm_device.hpp"

namespace lmk {

constexpr int kMaxBlurRadius = 16;  // taps per axis: 2 r + 1 <= 33

struct BlurAxis {
  int r;                              // radius in voxels (0: axis left alone)
  float w[2 * kMaxBlurRadius + 1];    // taps w[t + r], t = -r..r, sum 1
};
struct Blur {
  BlurAxis ax[3];  // x, y, z
  bool on;
};

// Taps for a Gaussian of FWHM fwhm[a] voxels along each axis, truncated at
// ceil(3 sigma) and normalised to sum 1; fwhm 0 leaves an axis alone.
// LM_EINVAL for a negative FWHM or one whose radius exceeds kMaxBlurRadius.
int make_blur(const double fwhm[3], Blur *b);

// out = B in for images in layout L (ne elements; padding neither read nor
// written); t1, t2 are temporaries of ne elements.
int launch_blur(const int n[3], const Layout &L, long long ne, const Blur &b, const float *in, float *out, float *t1,
                float *t2, hipStream_t st);

// The z step of Algorithm 2 after a data update under the resolution
// model: dzb = B dz, z += dzb, zbar = z + dzb inv_p, fuse ? x = max(0, x -
// T zbar) (in place) : store zbar, and dz = 0.  The last blur pass carries
// the z step; t1, t2 are temporaries of ne elements.
int launch_blur_dual_image(const int n[3], const Layout &L, long long ne, const Blur &b, float *dz, float *t1,
                           float *t2, float *z, float *x, const float *T, float *zbar, float inv_p, bool fuse,
                           hipStream_t st);

}  // namespace lmk
