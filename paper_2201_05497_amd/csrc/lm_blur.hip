// Image-space resolution model (Section 1: the forward model includes
// limited spatial resolution): P = G B with B a separable Gaussian
// convolution, zero outside the image, so that B is symmetric and the back
// projection applies the same B after G^T.  One pass per blurred axis over
// the plan's bricked images; each voxel reads 2 r + 1 neighbours along the
// axis (L2 hits, all loads in flight at once) and writes one value.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lm_blur.hpp"
#include "lm_host.hpp"
#include "lm_layout32.hpp"

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// The blur along one axis at the voxel of layout position p with
// coordinate c0 along that axis (n voxels): the sum over t = -R..R, in that
// order, of w[t + R] x(c0 + t), taps outside the image skipped.  The 2R + 1
// loads (at clamped, always valid positions) are all issued before the
// first product, so a wavefront waits for memory once per voxel, not once
// per tap.
template <int R>
__device__ __forceinline__ float blur_at(const float *__restrict__ in, const lmk::AxisTerm &ta, unsigned p, int c0,
                                         int n, const lmk::BlurAxis &taps) {
  const int base = (int)p - lmk::axis_index(ta, c0);
  float v[2 * R + 1];
#pragma unroll
  for (int t = -R; t <= R; ++t) v[t + R] = in[base + lmk::axis_index(ta, min(max(c0 + t, 0), n - 1))];
  float acc = 0.0f;
#pragma unroll
  for (int t = -R; t <= R; ++t)
    if (c0 + t >= 0 && c0 + t < n) acc = fmaf(taps.w[t + R], v[t + R], acc);
  return acc;
}

// out = blur of `in` along `axis` with radius R (= taps.r).
template <int R>
__global__ __launch_bounds__(kBlock) void k_blur_axis(const float *__restrict__ in, float *__restrict__ out,
                                                      lmk::Layout L, int nx, int ny, int nz, long long ne, int axis,
                                                      lmk::BlurAxis taps) {
  const unsigned p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= ne) return;
  int c[3];
  lmk::vpos32(L, p, c[0], c[1], c[2]);
  if (c[0] >= nx || c[1] >= ny || c[2] >= nz) return;  // padding
  const int n = axis == 0 ? nx : axis == 1 ? ny : nz;
  out[p] = blur_at<R>(in, lmk::axis_term(L, axis), p, c[axis], n, taps);
}

// The last blur pass of a data update's back projection fused with the z
// step: d = (blur along `axis` of src)_p, z += d, zbar = z + d inv_p,
// fuse ? x = max(0, x - T zbar) : store zbar, and dz = 0 for the next
// update's atomics (dz is not read by this pass: src is a temporary).
template <int R>
__global__ __launch_bounds__(kBlock) void k_blur_axis_dual(const float *__restrict__ src, float *__restrict__ dz,
                                                           float *__restrict__ z, float *__restrict__ x,
                                                           const float *__restrict__ T, float *__restrict__ zbar,
                                                           float inv_p, int fuse, lmk::Layout L, int nx, int ny,
                                                           int nz, long long ne, int axis, lmk::BlurAxis taps) {
  const unsigned p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= ne) return;
  int c[3];
  lmk::vpos32(L, p, c[0], c[1], c[2]);
  if (c[0] >= nx || c[1] >= ny || c[2] >= nz) return;  // padding (stays zero)
  const int n = axis == 0 ? nx : axis == 1 ? ny : nz;
  const float d = blur_at<R>(src, lmk::axis_term(L, axis), p, c[axis], n, taps);
  const float zn = z[p] + d;
  const float zb = fmaf(d, inv_p, zn);
  z[p] = zn;
  if (fuse)
    x[p] = fmaxf(0.0f, fmaf(-T[p], zb, x[p]));
  else
    zbar[p] = zb;
  dz[p] = 0.0f;
}

// The kernels of radius taps.r (0..kMaxBlurRadius).
#define LM_BLUR_RADII(M) \
  M(0) M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16)
static_assert(lmk::kMaxBlurRadius == 16, "one kernel per radius up to kMaxBlurRadius");

int launch_axis(const float *in, float *out, const lmk::Layout &L, const int n[3], long long ne, int axis,
                const lmk::BlurAxis &taps, hipStream_t st) {
  switch (taps.r) {
#define LM_CASE(R_)                                                                                              \
  case R_:                                                                                                       \
    hipLaunchKernelGGL((k_blur_axis<R_>), dim3(grid_for(ne)), dim3(kBlock), 0, st, in, out, L, n[0], n[1], n[2], \
                       ne, axis, taps);                                                                          \
    break;
    LM_BLUR_RADII(LM_CASE)
#undef LM_CASE
    default:
      lmh::set_error("blur radius %d outside 0..%d", taps.r, lmk::kMaxBlurRadius);
      return LM_EINVAL;
  }
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_axis_dual(const float *src, float *dz, float *z, float *x, const float *T, float *zbar, float inv_p,
                     bool fuse, const lmk::Layout &L, const int n[3], long long ne, int axis,
                     const lmk::BlurAxis &taps, hipStream_t st) {
  switch (taps.r) {
#define LM_CASE(R_)                                                                                              \
  case R_:                                                                                                       \
    hipLaunchKernelGGL((k_blur_axis_dual<R_>), dim3(grid_for(ne)), dim3(kBlock), 0, st, src, dz, z, x, T, zbar,  \
                       inv_p, fuse ? 1 : 0, L, n[0], n[1], n[2], ne, axis, taps);                                \
    break;
    LM_BLUR_RADII(LM_CASE)
#undef LM_CASE
    default:
      lmh::set_error("blur radius %d outside 0..%d", taps.r, lmk::kMaxBlurRadius);
      return LM_EINVAL;
  }
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

}  // namespace

namespace lmk {

int make_blur(const double fwhm[3], Blur *b) {
  b->on = false;
  for (int a = 0; a < 3; ++a) {
    BlurAxis &ax = b->ax[a];
    ax.r = 0;
    for (float &w : ax.w) w = 0.0f;
    const double f = fwhm[a];
    LM_REQUIRE(f >= 0.0 && std::isfinite(f), LM_EINVAL, "FWHM along axis %d must be finite and >= 0", a);
    if (f == 0.0) continue;
    const double sig = f / (2.0 * std::sqrt(2.0 * std::log(2.0)));
    const int r = (int)std::ceil(3.0 * sig);
    LM_REQUIRE(r <= kMaxBlurRadius, LM_EINVAL, "FWHM %.3g voxels along axis %d exceeds the largest supported (%d taps)",
               f, a, 2 * kMaxBlurRadius + 1);
    double w[2 * kMaxBlurRadius + 1], sum = 0.0;
    for (int t = -r; t <= r; ++t) sum += (w[t + r] = std::exp(-(double)t * t / (2.0 * sig * sig)));
    for (int t = -r; t <= r; ++t) ax.w[t + r] = (float)(w[t + r] / sum);
    ax.r = r;
    b->on = true;
  }
  return LM_OK;
}

int launch_blur(const int n[3], const Layout &L, long long ne, const Blur &b, const float *in, float *out, float *t1,
                float *t2, hipStream_t st) {
  int axes[3], na = 0;
  for (int a = 0; a < 3; ++a)
    if (b.ax[a].r > 0) axes[na++] = a;
  if (na == 0) {
    LM_TRY_HIP(hipMemcpyAsync(out, in, (size_t)ne * sizeof(float), hipMemcpyDeviceToDevice, st));
    return LM_OK;
  }
  const float *src = in;
  for (int k = 0; k < na; ++k) {
    float *dst = k + 1 == na ? out : (k % 2 == 0 ? t1 : t2);
    if (int rc = launch_axis(src, dst, L, n, ne, axes[k], b.ax[axes[k]], st)) return rc;
    src = dst;
  }
  return LM_OK;
}

int launch_blur_dual_image(const int n[3], const Layout &L, long long ne, const Blur &b, float *dz, float *t1,
                           float *t2, float *z, float *x, const float *T, float *zbar, float inv_p, bool fuse,
                           hipStream_t st) {
  int axes[3], na = 0;
  for (int a = 0; a < 3; ++a)
    if (b.ax[a].r > 0) axes[na++] = a;
  LM_REQUIRE(na > 0, LM_EINVAL, "no blurred axis");
  // all passes but the last; with one blurred axis that pass goes to t1
  // and the fused pass applies the identity (it must not read dz)
  const float *src = dz;
  const int plain = na == 1 ? 1 : na - 1;
  for (int k = 0; k < plain; ++k) {
    float *dst = k % 2 == 0 ? t1 : t2;
    if (int rc = launch_axis(src, dst, L, n, ne, axes[k], b.ax[axes[k]], st)) return rc;
    src = dst;
  }
  BlurAxis last{};
  int axis = 0;
  if (na == 1) {
    last.r = 0;
    last.w[0] = 1.0f;
  } else {
    axis = axes[na - 1];
    last = b.ax[axis];
  }
  return launch_axis_dual(src, dz, z, x, T, zbar, inv_p, fuse, L, n, ne, axis, last, st);
}

}  // namespace lmk
