// Listmode EM-TV (Algorithm 3 of the paper), the warm start of LM-SPDHG:
// per subset an EM step z = x n / g P_i^T (1 / (P_i x + s_i)), the weights
// w = g / (beta x), and the weighted TV denoising
//   x+ = argmin_{u >= 0} sum_j w_j / 2 (u_j - z_j)^2 + ||K u||_{2,1}
// solved by the accelerated primal-dual algorithm of Chambolle & Pock (J.
// Math. Imaging Vis. 40, 2011, Algorithm 2).
//
// The EM step reuses the projector pair (bricked image, the events of the
// subset stored contiguously).  The denoising works on row-major images:
// each of its iterations is one pass for the dual step (forward
// differences of ubar, projection onto the unit balls) and one for the
// primal step (adjoint stencil, weighted prox, extrapolation); both stream
// whole images and are bound by HBM bandwidth.  The step sizes of all
// iterations are computed on the device from the smallest finite weight,
// so a call never waits for the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "lm_host.hpp"
#include "lm_image.hpp"

namespace {

using lmk::GeomDev;

constexpr int kBlock = 256;
constexpr unsigned kInfBits = 0x7f800000u;  // +inf as float bits
constexpr long long kMaxGrid = 1LL << 20;   // grid-stride loops beyond this

inline unsigned grid_for(long long n) {
  return (unsigned)std::min<long long>((n + kBlock - 1) / kBlock, kMaxGrid);
}

// Subset i = {e : e mod n = i} stored contiguously: subset i starts at
// i (N div n) + min(i, N mod n) and holds its events in list order.
__host__ __device__ inline long long subset_start(long long N, int nsub, int i) {
  const long long r = N % nsub;
  return (long long)i * (N / nsub) + (i < r ? i : r);
}

__global__ __launch_bounds__(kBlock) void k_subset_order(const int16_t *__restrict__ ev, const float *__restrict__ s,
                                                         long long N, int nsub, int16_t *__restrict__ ev_out,
                                                         float *__restrict__ s_out) {
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < N; e += (long long)gridDim.x * kBlock) {
    const int i = (int)(e % nsub);
    const long long d = subset_start(N, nsub, i) + e / nsub;
#pragma unroll
    for (int c = 0; c < 5; ++c) ev_out[5 * d + c] = ev[5 * e + c];
    s_out[d] = s[e];
  }
}

// EM quotient, in place: q_e <- 1 / (q_e + s_e), 0 where q_e + s_e <= 0.
__global__ __launch_bounds__(kBlock) void k_em_quotient(float *__restrict__ q, const float *__restrict__ s,
                                                        long long m) {
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < m; e += (long long)gridDim.x * kBlock) {
    const float d = q[e] + s[e];
    q[e] = d > 0.0f ? 1.0f / d : 0.0f;
  }
}

__global__ void k_fill_u32(unsigned *__restrict__ p, long long n, unsigned v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// EM image z = x n bp / g (0 where g = 0).  With beta > 0 also the weights
// w = g / (beta x) (inf where x = 0), the start of the denoising (u = ubar
// = z, q = 0) and the smallest weight of each block in part[blockIdx.x]
// (as float bits: non-negative floats order like their bits).  With
// beta = 0, x <- z.
__global__ __launch_bounds__(kBlock) void k_em_image(float *__restrict__ x, const float *__restrict__ bp,
                                                     const float *__restrict__ g, long long nv, float nsub,
                                                     float beta, float *__restrict__ z, float *__restrict__ w,
                                                     float *__restrict__ u, float *__restrict__ ubar,
                                                     float *__restrict__ q, unsigned *__restrict__ part) {
  __shared__ unsigned red[kBlock / 64];
  unsigned lo = kInfBits;
  for (long long j = (long long)blockIdx.x * kBlock + threadIdx.x; j < nv; j += (long long)gridDim.x * kBlock) {
    const float xj = x[j], gj = g[j];
    const float zj = gj > 0.0f ? xj * nsub * bp[j] / gj : 0.0f;
    if (beta > 0.0f) {
      const float wj = xj > 0.0f ? gj / (beta * xj) : INFINITY;
      z[j] = zj;
      w[j] = wj;
      u[j] = zj;
      ubar[j] = zj;
      q[j] = 0.0f;
      q[nv + j] = 0.0f;
      q[2 * nv + j] = 0.0f;
      lo = min(lo, __float_as_uint(wj));
    } else {
      x[j] = zj;
    }
  }
  if (beta <= 0.0f) return;
  for (int o = 32; o > 0; o >>= 1) lo = min(lo, (unsigned)__shfl_xor((int)lo, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lo;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kBlock / 64; ++i) lo = min(lo, red[i]);
    part[blockIdx.x] = lo;
  }
}

// Step sizes of the accelerated iterations: tau_0 = sigma_0 = 1/||K||,
// theta_k = 1 / sqrt(1 + 2 gam tau_k), tau_{k+1} = theta_k tau_k,
// sigma_{k+1} = sigma_k / theta_k, with gam the smallest finite weight
// (0 if every weight is infinite or the smallest is 0), reduced here from
// the npart block minima.  One block of kBlock threads.
__global__ __launch_bounds__(kBlock) void k_pd_schedule(const unsigned *__restrict__ part, int npart, double tau0,
                                                        int iters, float4 *__restrict__ sched) {
  __shared__ unsigned red[kBlock / 64];
  unsigned lo = kInfBits;
  for (int i = threadIdx.x; i < npart; i += kBlock) lo = min(lo, part[i]);
  for (int o = 32; o > 0; o >>= 1) lo = min(lo, (unsigned)__shfl_xor((int)lo, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lo;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int i = 1; i < kBlock / 64; ++i) lo = min(lo, red[i]);
  const double gam = lo < kInfBits ? (double)__uint_as_float(lo) : 0.0;
  double tau = tau0, sigma = tau0;
  for (int k = 0; k < iters; ++k) {
    const double theta = 1.0 / sqrt(1.0 + 2.0 * gam * tau);
    sched[k] = make_float4((float)tau, (float)sigma, (float)theta, 0.0f);
    tau *= theta;
    sigma /= theta;
  }
}

// Dual step: q <- projection of q + sigma_k K ubar onto the unit ball of
// each voxel (K = forward differences, zero in the last layer).
__global__ __launch_bounds__(kBlock) void k_pd_dual(const float *__restrict__ ubar, float *__restrict__ q, int nx,
                                                    int ny, int nz, const float4 *__restrict__ sched, int k) {
  // images have at most 512^3 voxels: 32-bit indices, also for the three
  // components of q
  const unsigned nxy = (unsigned)nx * ny, nv = nxy * nz;
  const float sigma = sched[k].y;
  for (unsigned j = blockIdx.x * kBlock + threadIdx.x; j < nv; j += gridDim.x * kBlock) {
    const unsigned row = j / nx;
    const int ix = (int)(j - row * nx), iy = (int)(row % ny), iz = (int)(row / ny);
    const float c = ubar[j];
    const float gx = ix + 1 < nx ? ubar[j + 1] - c : 0.0f;
    const float gy = iy + 1 < ny ? ubar[j + nx] - c : 0.0f;
    const float gz = iz + 1 < nz ? ubar[j + nxy] - c : 0.0f;
    const float a = fmaf(sigma, gx, q[j]), b = fmaf(sigma, gy, q[nv + j]), d = fmaf(sigma, gz, q[2 * nv + j]);
    const float r = 1.0f / fmaxf(1.0f, sqrtf(a * a + b * b + d * d));
    q[j] = a * r;
    q[nv + j] = b * r;
    q[2 * nv + j] = d * r;
  }
}

// Primal step and extrapolation: v = u - tau_k K^T q,
// u+ = max(0, (v + tau_k w z) / (1 + tau_k w)) (u+ = z where w = inf),
// ubar = u+ + theta_k (u+ - u).  u is read and written at the thread's own
// voxel only; u_out may be u (or, in the last iteration, the caller's x).
__global__ __launch_bounds__(kBlock) void k_pd_primal(const float *u, const float *__restrict__ q,
                                                      const float *__restrict__ z, const float *__restrict__ w,
                                                      float *u_out, float *__restrict__ ubar, int nx, int ny, int nz,
                                                      const float4 *__restrict__ sched, int k) {
  const unsigned nxy = (unsigned)nx * ny, nv = nxy * nz;
  const float4 st = sched[k];
  const float tau = st.x, theta = st.z;
  for (unsigned j = blockIdx.x * kBlock + threadIdx.x; j < nv; j += gridDim.x * kBlock) {
    const unsigned row = j / nx;
    const int ix = (int)(j - row * nx), iy = (int)(row % ny), iz = (int)(row / ny);
    // (K^T q)_j = sum over axes of q_a[j - e_a] (if j has a lower neighbour)
    // minus q_a[j] (unless j is in the last layer)
    float kt = 0.0f;
    if (ix > 0) kt += q[j - 1];
    if (ix + 1 < nx) kt -= q[j];
    if (iy > 0) kt += q[nv + j - nx];
    if (iy + 1 < ny) kt -= q[nv + j];
    if (iz > 0) kt += q[2 * nv + j - nxy];
    if (iz + 1 < nz) kt -= q[2 * nv + j];
    const float uj = u[j], zj = z[j], wj = w[j];
    float up;
    if (isinf(wj)) {
      up = zj;
    } else {
      const float v = fmaf(-tau, kt, uj);
      const float tw = tau * wj;
      up = fmaxf(0.0f, fmaf(tw, zj, v) / (1.0f + tw));
    }
    u_out[j] = up;
    ubar[j] = fmaf(theta, up - uj, up);
  }
}

// Stream-ordered device temporaries of one call, freed (stream-ordered)
// when the call returns.
struct Temps {
  hipStream_t st;
  void *p[16] = {};
  int n = 0;
  explicit Temps(hipStream_t s) : st(s) {}
  template <class T>
  int get(T **out, long long count) {
    *out = nullptr;
    if (count <= 0) return LM_OK;
    void *q = nullptr;
    const hipError_t e = hipMallocAsync(&q, (size_t)count * sizeof(T), st);
    if (e != hipSuccess) {
      lmh::set_error("lm_emtv temporary of %lld bytes: %s", (long long)(count * sizeof(T)), hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? LM_ENOMEM : LM_EHIP;
    }
    p[n++] = q;
    *out = static_cast<T *>(q);
    return LM_OK;
  }
  ~Temps() {
    for (int i = 0; i < n; ++i) (void)hipFreeAsync(p[i], st);  // a release error has no caller to go to
  }
};

// Largest singular value of K (forward differences with a zero last layer
// along each axis): sqrt(sum_a 4 sin^2(pi (N_a - 1) / (2 N_a))).
double knorm(const int n[3]) {
  double s = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double t = std::sin(M_PI * (n[a] - 1) / (2.0 * n[a]));
    s += 4.0 * t * t;
  }
  return std::sqrt(s);
}

}  // namespace

extern "C" {

int lm_emtv(const lm_geom *G, const int16_t *ev, const float *s, int64_t n, int32_t n_subsets, int32_t n_iter,
            const float *g, float beta, int32_t denoise_iter, float *x, void *stream) {
  lmh::clear_error();
  GeomDev gd;
  if (int rc = lmh::make_geom(G, &gd)) return rc;
  LM_REQUIRE(n >= 0, LM_EINVAL, "negative event count");
  LM_REQUIRE(n_subsets >= 1, LM_EINVAL, "n_subsets must be >= 1");
  LM_REQUIRE(n_iter >= 0 && denoise_iter >= 0, LM_EINVAL, "negative iteration count");
  LM_REQUIRE(beta >= 0.0f && std::isfinite(beta), LM_EINVAL, "beta must be finite and >= 0");
  LM_REQUIRE(g && x, LM_EINVAL, "NULL image");
  LM_REQUIRE(n == 0 || (ev && s), LM_EINVAL, "NULL event list");
  if (n_iter == 0) return LM_OK;
  hipStream_t st = lmh::as_stream(stream);
  const long long nv = lmh::nvox_of(gd.n);
  GeomDev gb = gd;
  gb.lay = lmh::brick_layout(gd.n);
  const long long nb = lmk::layout_size(gb.lay);
  const long long m_max = (n + n_subsets - 1) / n_subsets;
  const bool denoise = beta > 0.0f;
  const int iters = denoise ? denoise_iter : 0;

  Temps t(st);
  int16_t *evs = nullptr;
  float *ss = nullptr, *qe = nullptr, *xb = nullptr, *bpb = nullptr, *bp = nullptr;
  float *z = nullptr, *w = nullptr, *u = nullptr, *ubar = nullptr, *q3 = nullptr;
  float4 *sched = nullptr;
  unsigned *part = nullptr;
  const unsigned img_grid = grid_for(nv);
  if (int rc = t.get(&evs, 5 * n)) return rc;
  if (int rc = t.get(&ss, n)) return rc;
  if (int rc = t.get(&qe, m_max)) return rc;
  if (int rc = t.get(&xb, nb)) return rc;
  if (int rc = t.get(&bpb, nb)) return rc;
  if (int rc = t.get(&bp, nv)) return rc;
  if (denoise) {
    if (int rc = t.get(&z, nv)) return rc;
    if (int rc = t.get(&w, nv)) return rc;
    if (int rc = t.get(&u, nv)) return rc;
    if (int rc = t.get(&ubar, nv)) return rc;
    if (int rc = t.get(&q3, 3 * nv)) return rc;
    if (int rc = t.get(&part, img_grid)) return rc;
    if (int rc = t.get(&sched, std::max(iters, 1))) return rc;
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_subset_order, dim3(grid_for(n)), dim3(kBlock), 0, st, ev, s, (long long)n, (int)n_subsets,
                       evs, ss);
    LM_TRY_HIP(hipGetLastError());
  }
  const double tau0 = 1.0 / knorm(gd.n);
  for (int it = 0; it < n_iter; ++it) {
    for (int i = 0; i < n_subsets; ++i) {
      const long long o = subset_start(n, n_subsets, i);
      const long long m = subset_start(n, n_subsets, i + 1) - o;
      // EM step: bp = P_i^T (1 / (P_i x + s_i)) on the bricked image
      hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(nb)), dim3(kBlock), 0, st, (unsigned *)bpb, nb, 0u);
      LM_TRY_HIP(hipGetLastError());
      if (m > 0) {
        if (int rc = lmk::launch_to_layout(gd.n, gb.lay, 1, x, xb, st)) return rc;
        if (int rc = lmk::launch_fwd(gb, xb, evs + 5 * o, m, qe, st)) return rc;
        hipLaunchKernelGGL(k_em_quotient, dim3(grid_for(m)), dim3(kBlock), 0, st, qe, ss + o, m);
        LM_TRY_HIP(hipGetLastError());
        if (int rc = lmk::launch_back(gb, qe, evs + 5 * o, m, bpb, st)) return rc;
      }
      if (int rc = lmk::launch_from_layout(gd.n, gb.lay, 1, bpb, bp, st)) return rc;
      hipLaunchKernelGGL(k_em_image, dim3(img_grid), dim3(kBlock), 0, st, x, bp, g, nv, (float)n_subsets, beta, z,
                         w, u, ubar, q3, part);
      LM_TRY_HIP(hipGetLastError());
      if (!denoise) continue;
      if (iters == 0) {
        LM_TRY_HIP(hipMemcpyAsync(x, z, (size_t)nv * sizeof(float), hipMemcpyDeviceToDevice, st));
        continue;
      }
      hipLaunchKernelGGL(k_pd_schedule, dim3(1), dim3(kBlock), 0, st, part, (int)img_grid, tau0, iters, sched);
      LM_TRY_HIP(hipGetLastError());
      for (int k = 0; k < iters; ++k) {
        hipLaunchKernelGGL(k_pd_dual, dim3(grid_for(nv)), dim3(kBlock), 0, st, ubar, q3, gd.n[0], gd.n[1], gd.n[2],
                           sched, k);
        LM_TRY_HIP(hipGetLastError());
        float *dst = k + 1 == iters ? x : u;
        hipLaunchKernelGGL(k_pd_primal, dim3(grid_for(nv)), dim3(kBlock), 0, st, u, q3, z, w, dst, ubar, gd.n[0],
                           gd.n[1], gd.n[2], sched, k);
        LM_TRY_HIP(hipGetLastError());
      }
    }
  }
  return LM_OK;
}

}  // extern "C"
