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
// w and w_new hold ncomp components of nv voxels each (ncomp = 2 for a 2D
// image, whose z-component is identically zero).
__global__ __launch_bounds__(kBlock) void k_tv_dual(const float *__restrict__ x, const float *__restrict__ w,
                                                    float *__restrict__ wn, int nx, int ny, int nz,
                                                    int ncomp, float Sp, float beta) {
  const long long nv = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nv) return;
  const int i = (int)(v % nx);
  const int j = (int)((v / nx) % ny);
  const int k = (int)(v / ((long long)nx * ny));
  const float xv = x[v];
  const float gx = (i < nx - 1) ? x[v + 1] - xv : 0.0f;
  const float gy = (j < ny - 1) ? x[v + nx] - xv : 0.0f;
  const float gz = (ncomp == 3 && k < nz - 1) ? x[v + (long long)nx * ny] - xv : 0.0f;
  const float v0 = fmaf(Sp, gx, w[v]);
  const float v1 = fmaf(Sp, gy, w[nv + v]);
  const float v2 = (ncomp == 3) ? fmaf(Sp, gz, w[2 * nv + v]) : 0.0f;
  const float nrm = sqrtf(fmaf(v0, v0, fmaf(v1, v1, v2 * v2)));
  const float sc = 1.0f / fmaxf(1.0f, nrm / beta);
  wn[v] = v0 * sc;
  wn[nv + v] = v1 * sc;
  if (ncomp == 3) wn[2 * nv + v] = v2 * sc;
}

// Prior update, part 2 (the back-projection through K^T and the z / zbar
// step of Algorithm 2, fused with the next primal step when `fuse` is set):
//   dz = K^T (w_new - w);  z += dz;  zbar = z + dz / p;  x or zbar as above.
__global__ __launch_bounds__(kBlock) void k_tv_adjoint(const float *__restrict__ w,
                                                       const float *__restrict__ wn, float *__restrict__ z,
                                                       float *__restrict__ x, const float *__restrict__ T,
                                                       float *__restrict__ zbar, int nx, int ny, int nz,
                                                       int ncomp, float inv_p, int fuse) {
  const long long nv = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nv) return;
  const int i = (int)(v % nx);
  const int j = (int)((v / nx) % ny);
  const int k = (int)(v / ((long long)nx * ny));
  const long long sxy = (long long)nx * ny;
  float d = 0.0f;
  if (i < nx - 1) d -= wn[v] - w[v];
  if (i > 0) d += wn[v - 1] - w[v - 1];
  if (j < ny - 1) d -= wn[nv + v] - w[nv + v];
  if (j > 0) d += wn[nv + v - nx] - w[nv + v - nx];
  if (ncomp == 3) {
    if (k < nz - 1) d -= wn[2 * nv + v] - w[2 * nv + v];
    if (k > 0) d += wn[2 * nv + v - sxy] - w[2 * nv + v - sxy];
  }
  const float zn = z[v] + d;
  const float zb = fmaf(d, inv_p, zn);
  z[v] = zn;
  if (fuse)
    x[v] = fmaxf(0.0f, fmaf(-T[v], zb, x[v]));
  else
    zbar[v] = zb;
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

int launch_tv_dual(const int n[3], int ncomp, const float *x, const float *w, float *wn, float Sp, float beta,
                   hipStream_t st) {
  const long long nv = (long long)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_tv_dual, dim3(grid_for(nv)), dim3(kBlock), 0, st, x, w, wn, n[0], n[1], n[2], ncomp,
                     Sp, beta);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_tv_adjoint(const int n[3], int ncomp, const float *w, const float *wn, float *z, float *x,
                      const float *T, float *zbar, float inv_p, bool fuse, hipStream_t st) {
  const long long nv = (long long)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_tv_adjoint, dim3(grid_for(nv)), dim3(kBlock), 0, st, w, wn, z, x, T, zbar, n[0],
                     n[1], n[2], ncomp, inv_p, fuse ? 1 : 0);
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
