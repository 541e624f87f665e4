// Directional TV prior of LM-SPDHG (Section 3, DTV; Ehrhardt & Betcke,
// SIAM J. Imaging Sci. 9, 2016): K = D grad with D_j = I - xi_j xi_j^T,
// where xi = grad v / sqrt(|grad v|^2 + eta^2) is the normalised gradient of
// a structural prior image v.  D removes from each voxel's finite-difference
// vector its component along xi; it is symmetric with |D_j| <= 1, so the
// step sizes computed with ||grad|| stay valid.
//
// In 3D the prior update is the TV pass marching along z with xi read next
// to w (k_tv_march in lm_image.hip).  On one slice it is two passes over
// the plan's bricked images: the dual step (forward differences of x at the
// voxel, D, the projection onto the beta-ball) storing D (w_out - w), then
// its adjoint stencil fused with the z / zbar step and the next primal
// step.  The first pass reads x, w, xi and writes w_out and D (w_out - w)
// (ncomp components each); the second reads the latter back with z, T and
// x and writes z and x (or zbar): bound by HBM bandwidth.
#include <hip/hip_runtime.h>

#include "lm_dtv.hpp"
#include "lm_host.hpp"
#include "lm_layout32.hpp"

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__global__ __launch_bounds__(kBlock) void k_dtv_field(const float *__restrict__ v, float *__restrict__ xi,
                                                      lmk::Layout L, int nx, int ny, int nz, long long ne, int ncomp,
                                                      float eta) {
  const long long nxy = (long long)nx * ny, nv = nxy * nz;
  const long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (r >= nv) return;
  const int i = (int)(r % nx), j = (int)((r / nx) % ny), k = (int)(r / nxy);
  const float c = v[r];
  const float gx = i + 1 < nx ? v[r + 1] - c : 0.0f;
  const float gy = j + 1 < ny ? v[r + nx] - c : 0.0f;
  const float gz = k + 1 < nz ? v[r + nxy] - c : 0.0f;
  const float s = 1.0f / sqrtf(gx * gx + gy * gy + gz * gz + eta * eta);
  const int q = lmk::vidx(L, i, j, k);
  xi[q] = gx * s;
  xi[ne + q] = gy * s;
  if (ncomp == 3) xi[2 * ne + q] = gz * s;
}

// Dual step at each voxel: a = D grad x, w_out = w + Sp a projected onto the
// ball of radius beta, pd = D (w_out - w).
__global__ __launch_bounds__(kBlock) void k_dtv_dual(const float *__restrict__ x, const float *__restrict__ w,
                                                     float *__restrict__ w_out, const float *__restrict__ xi,
                                                     float *__restrict__ pd, lmk::Layout L, int nx, int ny, int nz,
                                                     long long ne, int ncomp, float Sp, float beta) {
  const unsigned p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= ne) return;
  int i, j, k;
  lmk::vpos32(L, p, i, j, k);
  if (i >= nx || j >= ny || k >= nz) return;  // padding
  const float c = x[p];
  float g[3], e[3], wv[3];
  g[0] = i + 1 < nx ? x[lmk::vidx(L, i + 1, j, k)] - c : 0.0f;
  g[1] = j + 1 < ny ? x[lmk::vidx(L, i, j + 1, k)] - c : 0.0f;
  g[2] = ncomp == 3 && k + 1 < nz ? x[lmk::vidx(L, i, j, k + 1)] - c : 0.0f;
  float eg = 0.0f;
  for (int a = 0; a < 3; ++a) {
    e[a] = a < ncomp ? xi[a * ne + p] : 0.0f;
    wv[a] = a < ncomp ? w[a * ne + p] : 0.0f;
    eg = fmaf(e[a], g[a], eg);
  }
  float v[3], nrm2 = 0.0f;
  for (int a = 0; a < 3; ++a) {
    v[a] = fmaf(Sp, fmaf(-e[a], eg, g[a]), wv[a]);
    nrm2 = fmaf(v[a], v[a], nrm2);
  }
  const float sc = 1.0f / fmaxf(1.0f, sqrtf(nrm2) / beta);
  float d[3], ed = 0.0f;
  for (int a = 0; a < 3; ++a) {
    v[a] *= sc;
    d[a] = v[a] - wv[a];
    ed = fmaf(e[a], d[a], ed);
  }
  for (int a = 0; a < ncomp; ++a) {
    w_out[a * ne + p] = v[a];
    pd[a * ne + p] = fmaf(-e[a], ed, d[a]);
  }
}

// dz = grad^T pd (the sum over axes of pd_a at the lower neighbour, if
// any, minus pd_a at the voxel, unless it is in the last layer), then
//   z += dz;  zbar = z + dz / p;  (fuse ? x = max(0, x - T zbar) : store zbar).
// x is read and written at the thread's own voxel only.  Padding positions
// are left alone (they stay zero).
__global__ __launch_bounds__(kBlock) void k_dtv_adjoint_image(const float *__restrict__ pd, float *__restrict__ z,
                                                              float *__restrict__ x, const float *__restrict__ T,
                                                              float *__restrict__ zbar, float inv_p, int fuse,
                                                              lmk::Layout L, int nx, int ny, int nz, long long ne,
                                                              int ncomp) {
  const unsigned p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= ne) return;
  int i, j, k;
  lmk::vpos32(L, p, i, j, k);
  if (i >= nx || j >= ny || k >= nz) return;
  float s = 0.0f;
  if (i > 0) s += pd[lmk::vidx(L, i - 1, j, k)];
  if (i + 1 < nx) s -= pd[p];
  if (j > 0) s += pd[ne + lmk::vidx(L, i, j - 1, k)];
  if (j + 1 < ny) s -= pd[ne + p];
  if (ncomp == 3) {
    if (k > 0) s += pd[2 * ne + lmk::vidx(L, i, j, k - 1)];
    if (k + 1 < nz) s -= pd[2 * ne + p];
  }
  const float zn = z[p] + s;
  const float zb = fmaf(s, inv_p, zn);
  z[p] = zn;
  if (fuse)
    x[p] = fmaxf(0.0f, fmaf(-T[p], zb, x[p]));
  else
    zbar[p] = zb;
}

}  // namespace

namespace lmk {

int launch_dtv_field(const int n[3], const Layout &L, int ncomp, long long ne, const float *v, float eta, float *xi,
                     hipStream_t st) {
  const long long nv = lmh::nvox_of(n);
  hipLaunchKernelGGL(k_dtv_field, dim3(grid_for(nv)), dim3(kBlock), 0, st, v, xi, L, n[0], n[1], n[2], ne, ncomp,
                     eta);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_dtv_prior(const int n[3], const Layout &L, int ncomp, long long ne, float *x, const float *w,
                     float *w_out, const float *xi, float *pd, float *z, const float *T, float *zbar, float Sp,
                     float beta, float inv_p, bool fuse, hipStream_t st) {
  hipLaunchKernelGGL(k_dtv_dual, dim3(grid_for(ne)), dim3(kBlock), 0, st, x, w, w_out, xi, pd, L, n[0], n[1], n[2],
                     ne, ncomp, Sp, beta);
  LM_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_dtv_adjoint_image, dim3(grid_for(ne)), dim3(kBlock), 0, st, pd, z, x, T, zbar, inv_p,
                     fuse ? 1 : 0, L, n[0], n[1], n[2], ne, ncomp);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

}  // namespace lmk
