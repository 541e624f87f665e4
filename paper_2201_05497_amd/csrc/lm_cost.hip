// The objective of the paper's problem (Eq. 1) in listmode form, for
// monitoring a reconstruction (relative cost and convergence studies):
//
//   c(x) = <g, x> - sum_e log((P^LM x)_e + s_e) + beta ||K x||_{2,1},
//
// with g = P^T 1.  Over all sinogram bins i, sum_i (Px)_i = <P^T 1, x>, and
// the bins with counts contribute d_i log (Px + s)_i, which the event list
// gives as one term per event (an event of a bin counted d_i times appears
// d_i times).  The constant sum_i s_i over all bins is left out: it cancels
// in relative costs.  The forward projection runs in the projector kernels
// (float32); the three sums are accumulated in double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "lm_device.hpp"
#include "lm_host.hpp"
#include "lm_image.hpp"

namespace {

constexpr int kBlock = 256;
constexpr int kMaxPartials = 2048;

__device__ __forceinline__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// partial[b] = sum over the block's events of log(q_e + s_e)
__global__ __launch_bounds__(kBlock) void k_log_partials(const float *q, const float *s, long long n,
                                                         double *partial) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < n; e += (long long)gridDim.x * kBlock)
    acc += log((double)q[e] + (double)s[e]);
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// pg[b] = sum g x, ptv[b] = sum over voxels of |K x|_2 (forward differences,
// zero in the last layer of each axis) over the block's voxels of the
// row-major images
__global__ __launch_bounds__(kBlock) void k_image_partials(const float *x, const float *g, int nx, int ny, int nz,
                                                           double *pg, double *ptv) {
  __shared__ double red[kBlock];
  const long long nv = (long long)nx * ny * nz;
  double ag = 0.0, atv = 0.0;
  for (long long v = (long long)blockIdx.x * kBlock + threadIdx.x; v < nv; v += (long long)gridDim.x * kBlock) {
    const int i = (int)(v % nx);
    const int j = (int)((v / nx) % ny);
    const int k = (int)(v / ((long long)nx * ny));
    const double xv = x[v];
    ag += (double)g[v] * xv;
    const double dx = i + 1 < nx ? (double)x[v + 1] - xv : 0.0;
    const double dy = j + 1 < ny ? (double)x[v + nx] - xv : 0.0;
    const double dz = k + 1 < nz ? (double)x[v + (long long)nx * ny] - xv : 0.0;
    atv += sqrt(dx * dx + dy * dy + dz * dz);
  }
  const double tg = block_sum(ag, red);
  const double tt = block_sum(atv, red);
  if (threadIdx.x == 0) {
    pg[blockIdx.x] = tg;
    ptv[blockIdx.x] = tt;
  }
}

// out[t] = sum of the nb[t] partials of term t (one block)
__global__ __launch_bounds__(kBlock) void k_sum_terms(const double *partials, int nb_log, int nb_img, double *out) {
  __shared__ double red[kBlock];
  const double *pl = partials, *pg = partials + kMaxPartials, *pt = partials + 2 * kMaxPartials;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nb_log; i += kBlock) a += pl[i];
  for (int i = threadIdx.x; i < nb_img; i += kBlock) {
    b += pg[i];
    c += pt[i];
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  c = block_sum(c, red);
  if (threadIdx.x == 0) {
    out[0] = b;  // <g, x>
    out[1] = a;  // sum_e log((P x)_e + s_e)
    out[2] = c;  // ||K x||_{2,1}
  }
}

}  // namespace

extern "C" {

int lm_cost(const lm_geom *G, const float *x, const int16_t *ev, const float *s, int64_t n, const float *g,
            double beta, double *cost, double *terms, void *stream) {
  lmh::clear_error();
  lmk::GeomDev gd;
  if (int rc = lmh::make_geom(G, &gd)) return rc;
  LM_REQUIRE(n >= 0, LM_EINVAL, "negative event count");
  LM_REQUIRE(x && g && (n == 0 || (ev && s)), LM_EINVAL, "NULL array");
  LM_REQUIRE(cost || terms, LM_EINVAL, "no output");
  LM_REQUIRE(beta >= 0.0 && std::isfinite(beta), LM_EINVAL, "beta must be finite and >= 0");
  hipStream_t st = lmh::as_stream(stream);
  const long long nv = lmh::nvox_of(gd.n);
  float *q = nullptr;
  double *part = nullptr, *out = nullptr;
  auto release = [&]() {  // release errors are not reported
    if (q) (void)hipFreeAsync(q, st);
    if (part) (void)hipFreeAsync(part, st);
    if (out) (void)hipFreeAsync(out, st);
  };
  hipError_t e = hipMallocAsync((void **)&q, std::max<long long>(n, 1) * sizeof(float), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&part, 3 * kMaxPartials * sizeof(double), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&out, 3 * sizeof(double), st);
  if (e != hipSuccess) {
    release();
    lmh::set_error("lm_cost temporaries: %s", hipGetErrorString(e));
    return LM_ENOMEM;
  }
  int rc = LM_OK;
  const int nb_log = (int)std::min<long long>(kMaxPartials, std::max<long long>(1, (n + kBlock - 1) / kBlock));
  const int nb_img = (int)std::min<long long>(kMaxPartials, (nv + kBlock - 1) / kBlock);
  {
    lmh::BrickImage b;
    rc = b.alloc(gd, st);
    if (rc == LM_OK) rc = lmk::launch_to_layout(gd.n, gd.lay, 1, x, b.p, st);
    if (rc == LM_OK && n > 0) rc = lmk::launch_fwd(gd, b.p, ev, n, q, st);
  }
  if (rc == LM_OK) {
    hipLaunchKernelGGL(k_log_partials, dim3(nb_log), dim3(kBlock), 0, st, q, s, (long long)n, part);
    hipLaunchKernelGGL(k_image_partials, dim3(nb_img), dim3(kBlock), 0, st, x, g, gd.n[0], gd.n[1], gd.n[2],
                       part + kMaxPartials, part + 2 * kMaxPartials);
    hipLaunchKernelGGL(k_sum_terms, dim3(1), dim3(kBlock), 0, st, part, nb_log, nb_img, out);
    e = hipGetLastError();
    double h[3] = {0.0, 0.0, 0.0};
    if (e == hipSuccess) e = hipMemcpyAsync(h, out, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      lmh::set_error("lm_cost: %s", hipGetErrorString(e));
      rc = LM_EHIP;
    } else {
      if (terms) {
        terms[0] = h[0];
        terms[1] = h[1];
        terms[2] = h[2];
      }
      if (cost) *cost = h[0] - h[1] + beta * h[2];
    }
  }
  release();
  return rc;
}

}  // extern "C"
