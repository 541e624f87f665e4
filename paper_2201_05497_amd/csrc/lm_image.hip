// Image-space kernels of LM-SPDHG on gfx950: the primal step with the
// non-negativity prox, the z / zbar updates, the TV dual update with its
// adjoint stencil, and the tv_grad / tv_div entry points.
//
// All of these stream whole images and are bound by memory bandwidth; each
// thread handles one voxel, loads are coalesced along x (the fastest axis)
// and every pass that can be fused with the next primal step is.
#include <hip/hip_runtime.h>

#include "lm_host.hpp"
#include "lm_image.hpp"

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Primal step of Algorithm 2: x <- max(0, x - T zbar).
__global__ __launch_bounds__(kBlock) void k_primal(float *__restrict__ x, const float *__restrict__ T,
                                                   const float *__restrict__ zbar, long long nv) {
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v < nv) x[v] = fmaxf(0.0f, fmaf(-T[v], zbar[v], x[v]));
}

// The z / zbar step of Algorithm 2 after a data update, fused with the
// primal step of the next update when `fuse` is set:
//   z += dz;  zbar = z + dz / p;  (fuse ? x = max(0, x - T zbar) : store zbar);
//   dz = 0 (ready for the next subset's atomics).
__global__ __launch_bounds__(kBlock) void k_dual_image(float *__restrict__ z, float *__restrict__ dz,
                                                       float *__restrict__ x, const float *__restrict__ T,
                                                       float *__restrict__ zbar, float inv_p, int fuse,
                                                       long long nv) {
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nv) return;
  const float d = dz[v];
  const float zn = z[v] + d;
  const float zb = fmaf(d, inv_p, zn);
  z[v] = zn;
  dz[v] = 0.0f;
  if (fuse)
    x[v] = fmaxf(0.0f, fmaf(-T[v], zb, x[v]));
  else
    zbar[v] = zb;
}

// Prior update, part 1 (the dual prior step of Algorithm 2, R = ||.||_{2,1}):
//   v = w + S_prior K x;  w_new = v / max(1, |v| / beta)  (pointwise norm).
// Images use layout L (ne elements, padding skipped); w and w_new hold ncomp
// components of ne elements each (ncomp = 2 for a single-slice image, whose
// z-component is identically zero).
__global__ __launch_bounds__(kBlock) void k_tv_dual(const float *__restrict__ x, const float *__restrict__ w,
                                                    float *__restrict__ wn, lmk::Layout L, int nx, int ny, int nz,
                                                    long long ne, int ncomp, float Sp, float beta) {
  const long long p = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (p >= ne) return;
  int i, j, k;
  lmk::vpos(L, p, i, j, k);
  if (i >= nx || j >= ny || k >= nz) return;
  const float xv = x[p];
  const float gx = (i < nx - 1) ? x[lmk::vidx(L, i + 1, j, k)] - xv : 0.0f;
  const float gy = (j < ny - 1) ? x[lmk::vidx(L, i, j + 1, k)] - xv : 0.0f;
  const float gz = (ncomp == 3 && k < nz - 1) ? x[lmk::vidx(L, i, j, k + 1)] - xv : 0.0f;
  const float v0 = fmaf(Sp, gx, w[p]);
  const float v1 = fmaf(Sp, gy, w[ne + p]);
  const float v2 = (ncomp == 3) ? fmaf(Sp, gz, w[2 * ne + p]) : 0.0f;
  const float nrm = sqrtf(fmaf(v0, v0, fmaf(v1, v1, v2 * v2)));
  const float sc = 1.0f / fmaxf(1.0f, nrm / beta);
  wn[p] = v0 * sc;
  wn[ne + p] = v1 * sc;
  if (ncomp == 3) wn[2 * ne + p] = v2 * sc;
}

// Prior update, part 2 (the back-projection through K^T and the z / zbar
// step of Algorithm 2, fused with the next primal step when `fuse` is set):
//   dz = K^T (w_new - w);  z += dz;  zbar = z + dz / p;  x or zbar as above.
__global__ __launch_bounds__(kBlock) void k_tv_adjoint(const float *__restrict__ w,
                                                       const float *__restrict__ wn, float *__restrict__ z,
                                                       float *__restrict__ x, const float *__restrict__ T,
                                                       float *__restrict__ zbar, lmk::Layout L, int nx, int ny,
                                                       int nz, long long ne, int ncomp, float inv_p, int fuse) {
  const long long p = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (p >= ne) return;
  int i, j, k;
  lmk::vpos(L, p, i, j, k);
  if (i >= nx || j >= ny || k >= nz) return;
  float d = 0.0f;
  if (i < nx - 1) d -= wn[p] - w[p];
  if (i > 0) {
    const int q = lmk::vidx(L, i - 1, j, k);
    d += wn[q] - w[q];
  }
  if (j < ny - 1) d -= wn[ne + p] - w[ne + p];
  if (j > 0) {
    const long long q = ne + lmk::vidx(L, i, j - 1, k);
    d += wn[q] - w[q];
  }
  if (ncomp == 3) {
    if (k < nz - 1) d -= wn[2 * ne + p] - w[2 * ne + p];
    if (k > 0) {
      const long long q = 2 * ne + lmk::vidx(L, i, j, k - 1);
      d += wn[q] - w[q];
    }
  }
  const float zn = z[p] + d;
  const float zb = fmaf(d, inv_p, zn);
  z[p] = zn;
  if (fuse)
    x[p] = fmaxf(0.0f, fmaf(-T[p], zb, x[p]));
  else
    zbar[p] = zb;
}

// Row-major image (caller layout) -> layout L, ncomp components; padding is
// left untouched (zero).
__global__ __launch_bounds__(kBlock) void k_to_layout(const float *__restrict__ src, float *__restrict__ dst,
                                                      lmk::Layout L, int nx, int ny, int nz, long long ne,
                                                      int ncomp) {
  const long long nv = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nv) return;
  const int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((long long)nx * ny));
  const int q = lmk::vidx(L, i, j, k);
  for (int c = 0; c < ncomp; ++c) dst[c * ne + q] = src[c * nv + v];
}

// Layout L -> row-major image, ncomp components.
__global__ __launch_bounds__(kBlock) void k_from_layout(const float *__restrict__ src, float *__restrict__ dst,
                                                        lmk::Layout L, int nx, int ny, int nz, long long ne,
                                                        int ncomp) {
  const long long nv = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nv) return;
  const int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((long long)nx * ny));
  const int q = lmk::vidx(L, i, j, k);
  for (int c = 0; c < ncomp; ++c) dst[c * nv + v] = src[c * ne + q];
}

// gx = K x (three components).
__global__ __launch_bounds__(kBlock) void k_grad(const float *__restrict__ x, float *__restrict__ gx, int nx,
                                                 int ny, int nz) {
  const long long nv = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nv) return;
  const int i = (int)(v % nx);
  const int j = (int)((v / nx) % ny);
  const int k = (int)(v / ((long long)nx * ny));
  const float xv = x[v];
  gx[v] = (i < nx - 1) ? x[v + 1] - xv : 0.0f;
  gx[nv + v] = (j < ny - 1) ? x[v + nx] - xv : 0.0f;
  gx[2 * nv + v] = (k < nz - 1) ? x[v + (long long)nx * ny] - xv : 0.0f;
}

// out = -K^T w (the divergence).
__global__ __launch_bounds__(kBlock) void k_div(const float *__restrict__ w, float *__restrict__ out, int nx,
                                                int ny, int nz) {
  const long long nv = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nv) return;
  const int i = (int)(v % nx);
  const int j = (int)((v / nx) % ny);
  const int k = (int)(v / ((long long)nx * ny));
  const long long sxy = (long long)nx * ny;
  float d = 0.0f;
  if (i < nx - 1) d += w[v];
  if (i > 0) d -= w[v - 1];
  if (j < ny - 1) d += w[nv + v];
  if (j > 0) d -= w[nv + v - nx];
  if (k < nz - 1) d += w[2 * nv + v];
  if (k > 0) d -= w[2 * nv + v - sxy];
  out[v] = d;
}

}  // namespace

namespace lmk {

using lmk::Layout;

int launch_primal(float *x, const float *T, const float *zbar, long long nv, hipStream_t st) {
  hipLaunchKernelGGL(k_primal, dim3(grid_for(nv)), dim3(kBlock), 0, st, x, T, zbar, nv);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_dual_image(float *z, float *dz, float *x, const float *T, float *zbar, float inv_p, bool fuse,
                      long long nv, hipStream_t st) {
  hipLaunchKernelGGL(k_dual_image, dim3(grid_for(nv)), dim3(kBlock), 0, st, z, dz, x, T, zbar, inv_p,
                     fuse ? 1 : 0, nv);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_tv_dual(const int n[3], const Layout &L, int ncomp, const float *x, const float *w, float *wn, float Sp,
                   float beta, hipStream_t st) {
  const long long ne = layout_size(L);
  hipLaunchKernelGGL(k_tv_dual, dim3(grid_for(ne)), dim3(kBlock), 0, st, x, w, wn, L, n[0], n[1], n[2], ne, ncomp,
                     Sp, beta);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_tv_adjoint(const int n[3], const Layout &L, int ncomp, const float *w, const float *wn, float *z,
                      float *x, const float *T, float *zbar, float inv_p, bool fuse, hipStream_t st) {
  const long long ne = layout_size(L);
  hipLaunchKernelGGL(k_tv_adjoint, dim3(grid_for(ne)), dim3(kBlock), 0, st, w, wn, z, x, T, zbar, L, n[0], n[1],
                     n[2], ne, ncomp, inv_p, fuse ? 1 : 0);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_to_layout(const int n[3], const Layout &L, int ncomp, const float *src, float *dst, hipStream_t st) {
  const long long nv = (long long)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_to_layout, dim3(grid_for(nv)), dim3(kBlock), 0, st, src, dst, L, n[0], n[1], n[2],
                     layout_size(L), ncomp);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_from_layout(const int n[3], const Layout &L, int ncomp, const float *src, float *dst, hipStream_t st) {
  const long long nv = (long long)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_from_layout, dim3(grid_for(nv)), dim3(kBlock), 0, st, src, dst, L, n[0], n[1], n[2],
                     layout_size(L), ncomp);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_grad(const int n[3], const float *x, float *gx, hipStream_t st) {
  const long long nv = (long long)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_grad, dim3(grid_for(nv)), dim3(kBlock), 0, st, x, gx, n[0], n[1], n[2]);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_div(const int n[3], const float *w, float *out, hipStream_t st) {
  const long long nv = (long long)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_div, dim3(grid_for(nv)), dim3(kBlock), 0, st, w, out, n[0], n[1], n[2]);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

}  // namespace lmk

extern "C" {

static int check_dims(const int32_t n[3]) {
  LM_REQUIRE(n != nullptr, LM_EINVAL, "NULL size");
  for (int a = 0; a < 3; ++a)
    LM_REQUIRE(n[a] >= 1 && n[a] <= (1 << 20), LM_EINVAL, "image size n[%d]=%d invalid", a, n[a]);
  LM_REQUIRE((long long)n[0] * n[1] * n[2] < (1LL << 40), LM_EINVAL, "image too large");
  return LM_OK;
}

int tv_grad(const int32_t n[3], const float *x, float *gx, void *stream) {
  lmh::clear_error();
  if (int rc = check_dims(n)) return rc;
  LM_REQUIRE(x && gx, LM_EINVAL, "NULL array");
  const int nn[3] = {n[0], n[1], n[2]};
  return lmk::launch_grad(nn, x, gx, lmh::as_stream(stream));
}

int tv_div(const int32_t n[3], const float *w, float *out, void *stream) {
  lmh::clear_error();
  if (int rc = check_dims(n)) return rc;
  LM_REQUIRE(w && out, LM_EINVAL, "NULL array");
  const int nn[3] = {n[0], n[1], n[2]};
  return lmk::launch_div(nn, w, out, lmh::as_stream(stream));
}

}  // extern "C"
