// LM-SPDHG plans on gfx950: event preprocessing (the event counts, the
// initialisation and the split into sublists of Algorithm 2), step sizes
// (Eq. lm_stepsizes) and the update loop of Algorithm 2, plus the C ABI of
// plans and the library's error reporting.
//
// A plan owns every per-event list and image of the state in HBM; the only
// host->device traffic during the iterations is kernel launches.
//
// Event counts mu_e use an open-addressing hash table of the canonical bin
// key (unordered crystal pair, TOF bin with the sign flipped when the pair
// is swapped): one 64-bit compare-and-swap insertion plus an integer atomic
// count per event, then a lookup.  Counts are exact integers.
//
// Subsets are interleaved (event e goes to subset e mod n); the plan stores
// the events of each subset contiguously so one launch streams one subset.
//
// Optional parts of the model, set before the initialisation (or, for the
// prior, at any time): per-event attenuation x normalisation factors, folded
// exactly into the stored s and mu; an image-space resolution model B
// (x blurred before each data update, its back projection after); the
// directional TV prior in place of TV.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "lm_blur.hpp"
#include "lm_device.hpp"
#include "lm_dtv.hpp"
#include "lm_host.hpp"
#include "lm_image.hpp"
#include "lm_tiles.hpp"

// --------------------------------------------------------------------------
// error reporting

namespace {
thread_local std::string g_err;
}

namespace lmh {
void set_error(const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}
void clear_error() { g_err.clear(); }
}  // namespace lmh

extern "C" const char *lm_last_error(void) { return g_err.c_str(); }

// --------------------------------------------------------------------------
// plan

struct lm_plan {
  lm_geom G;
  lmk::GeomDev g;
  long long n = 0;       // events
  int nsub = 0;
  long long nvox = 0;    // voxels of the image
  lmk::Layout lay;       // brick layout of the plan's images
  long long ne = 0;      // elements of one image in that layout (with padding)
  int ncomp = 3;         // components of w (2 for a single-slice image)
  double gamma = 0, rho = 0, beta = 0, knorm = 0, Sp = 0;
  std::vector<int> off;  // host copy of subset offsets [nsub + 1]
  // device buffers (sorted order unless noted)
  int4 *rec = nullptr;   // {id1, id2, k, bits of s}
  float *S = nullptr, *mu = nullptr, *P1 = nullptr, *tmp = nullptr;
  float *c = nullptr;    // complement of the dual, c = 1 - y
  int *perm = nullptr, *off_d = nullptr;
  // images, brick layout
  float *gimg = nullptr, *T = nullptr, *z = nullptr, *zbar = nullptr, *dz = nullptr;
  float *w = nullptr, *wn = nullptr, *xint = nullptr, *xalt = nullptr;
  // directional TV (lm_plan_set_prior_image): xi and D (w_new - w), ncomp
  // components each; dtv selects that prior over TV
  float *xi_dtv = nullptr, *pd = nullptr;
  bool dtv = false;
  // per-event multiplicative factors (lm_plan_set_event_factors), sorted
  // order; folded into s and mu, kept to return the event counts
  float *mfac = nullptr;
  // resolution model (lm_plan_set_resolution): B x for the data updates,
  // B dz after them, and two temporaries of the separable passes
  lmk::Blur blur{};
  float *xb = nullptr, *dzb = nullptr, *bt1 = nullptr, *bt2 = nullptr;
  // data updates by image tile (3D plans whose segment lists fit)
  lmk::TilePlan tiles;
  // the plan computed g = G^T 1 itself (lm_plan_create with g = NULL); g0
  // keeps that image when a resolution model later replaces g by B g0
  bool g_internal = false;
  float *g0 = nullptr;
  std::vector<void *> allocs;
  bool initialized = false;
  long long u = 0;
  hipStream_t last = nullptr;
  // optional per-kernel timing of the update loop
  int timing = 0;                                  // time every timing-th launch of a class (0: off)
  long long t_seen[LM_K_COUNT] = {0};              // launches of each class since the reset
  std::vector<hipEvent_t> ev_pool;                 // free events
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  double t_ms[LM_K_COUNT] = {0};
  long long t_n[LM_K_COUNT] = {0};
  bool trace = false;                              // roctx ranges per epoch call and update
};

namespace {

// A roctx range from construction to destruction (when on), so that early
// returns close it.
struct TraceRange {
  bool on;
  TraceRange(bool on_, const char *name) : on(on_) {
    if (on) roctxRangePushA(name);
  }
  ~TraceRange() {
    if (on) roctxRangePop();
  }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace

namespace {

constexpr int kBlock = 256;
inline unsigned grid_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

constexpr unsigned long long kEmpty = ~0ULL;

// The 64-bit finaliser ("fmix64") of Austin Appleby's public-domain
// MurmurHash3, with its published constants: every input bit affects every
// output bit, so nearby bin keys spread over the table.
__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}

__device__ __forceinline__ unsigned long long bin_key(const lmk::GeomDev &g, int id1, int id2, int k) {
  if (id1 > id2) {
    const int t = id1;
    id1 = id2;
    id2 = t;
    k = -k;
  }
  return ((unsigned long long)id1 * (unsigned long long)g.n_det + (unsigned long long)id2) *
             (unsigned long long)g.n_tof +
         (unsigned long long)(k + g.kmax);
}

__global__ void k_count_bad(lmk::GeomDev g, const int16_t *ev, long long n, unsigned long long *bad) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int id1, id2, k;
  const bool ok = (e >= n) || lmk::decode_event(g, ev + 5 * e, id1, id2, k);
  const unsigned long long m = __ballot(!ok);
  if ((threadIdx.x % 64) == 0 && m) atomicAdd(bad, (unsigned long long)__popcll(m));
}

// Insert every event's bin key; slot[e] receives the table slot.
__global__ void k_hash_insert(lmk::GeomDev g, const int16_t *ev, long long n, unsigned long long *keys,
                              unsigned *cnt, unsigned mask, unsigned *slot) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  int id1, id2, k;
  lmk::decode_event(g, ev + 5 * e, id1, id2, k);  // validated before
  const unsigned long long key = bin_key(g, id1, id2, k);
  unsigned h = (unsigned)mix64(key) & mask;
  for (;;) {
    const unsigned long long prev = atomicCAS(keys + h, kEmpty, key);
    if (prev == kEmpty || prev == key) {
      atomicAdd(cnt + h, 1u);
      slot[e] = h;
      return;
    }
    h = (h + 1) & mask;
  }
}

// Gather the events into subset order: event e -> position off[e mod n] + e / n.
__global__ void k_layout(lmk::GeomDev g, const int16_t *ev, const float *s, long long n, int nsub,
                         const unsigned *cnt, const unsigned *slot, int4 *rec, float *mu, int *perm) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const long long q = n / nsub, rem = n % nsub;
  const long long i = e % nsub;
  const long long pos = i * q + (i < rem ? i : rem) + e / nsub;
  int id1, id2, k;
  lmk::decode_event(g, ev + 5 * e, id1, id2, k);
  rec[pos] = make_int4(id1, id2, k, __float_as_int(s[e]));
  mu[pos] = (float)cnt[slot[e]];
  perm[pos] = (int)e;
}

__global__ void k_fill(float *p, float v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// S_e = gamma rho / (P^LM 1)_e (Eq. lm_stepsizes), 0 where the LOR misses
// the image: (P^LM 1)_e <= p1_min, 1e-6 of the smallest voxel size (in mm,
// the unit of P^LM 1), so that a LOR that meets the image only within
// rounding (a corner weight of 1e-12 at an edge) carries no dual step.
constexpr double kP1Floor = 1e-6;

__global__ void k_step_S(const float *P1, float *S, float gr, float p1_min, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) S[i] = P1[i] > p1_min ? gr / P1[i] : 0.0f;
}

inline float p1_floor(const lm_geom &G) {
  return (float)(kP1Floor * std::min(G.h[0], std::min(G.h[1], G.h[2])));
}

// T_j = rho / (2 gamma max(g_j, ||K||)).
__global__ void k_step_T(const float *g, float *T, float c, float knorm, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) T[i] = c / fmaxf(g[i], knorm);
}

// y = 1 - mu / (P x0 + s), kept as c = 1 - y = mu / (P x0 + s) (in place on
// the forward values), and the back projection weights v = (y - 1) / mu.
__global__ void k_init_dual(float *c, const int4 *rec, const float *mu, float *v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float q = c[i] + __int_as_float(rec[i].w);
  c[i] = mu[i] / q;
  v[i] = -1.0f / q;  // (y - 1) / mu
}

// out[perm[j]] = a + b in[j] (sorted -> caller order)
__global__ void k_scatter_f(const float *in, const int *perm, float *out, long long n, float a = 0.0f,
                            float b = 1.0f) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[perm[j]] = fmaf(b, in[j], a);
}
__global__ void k_scatter_mu(const float *in, const int *perm, int *out, long long n) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[perm[j]] = (int)in[j];
}
// the same for a plan with factors: the stored mu / m times m, rounded
__global__ void k_scatter_mu_fac(const float *in, const float *m, const int *perm, int *out, long long n) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[perm[j]] = (int)rintf(in[j] * m[j]);
}

// z += a
__global__ void k_add(float *z, const float *a, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] += a[i];
}

// Counts factors that are not positive and finite.
__global__ void k_check_factors(const float *m, long long n, unsigned long long *bad) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n && !(m[e] > 0.0f && m[e] < INFINITY)) atomicAdd(bad, 1ULL);
}

// Folds the factor of each event into the stored lists: s -> s / m and
// mu -> mu / m (sorted position j holds caller event perm[j]).
__global__ void k_apply_factors(const float *m, const int *perm, int4 *rec, float *mu, float *mfac, long long n) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const float f = m[perm[j]];
  int4 r = rec[j];
  r.w = __float_as_int(__int_as_float(r.w) / f);
  rec[j] = r;
  mu[j] = mu[j] / f;
  mfac[j] = f;
}
// out[j] = in[perm[j]] (caller -> sorted order)
__global__ void k_gather_f(const float *in, const int *perm, float *out, long long n) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = in[perm[j]];
}
// Subset of every caller event as stored: stored position j lies in subset
// i with off[i] <= j < off[i+1]; out[perm[j]] = i.
__global__ void k_subset_ids(const int *off, const int *perm, int *out, int nsub, long long n) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int lo = 0, hi = nsub;  // invariant: off[lo] <= j < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= j)
      lo = mid;
    else
      hi = mid;
  }
  out[perm[j]] = lo;
}

unsigned long long hash_capacity(long long n) {
  unsigned long long c = 1024;
  while (c < 2ULL * (unsigned long long)n) c <<= 1;
  return c;
}

double exact_knorm(const int n[3]) {
  double s = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double N = n[a];
    const double v = std::sin(M_PI * (N - 1.0) / (2.0 * N));
    s += 4.0 * v * v;
  }
  return std::sqrt(s);
}

struct Sizes {
  size_t persistent, temporary;
};

Sizes plan_sizes(long long n, int nsub, long long nvox, long long ne, int ncomp) {
  Sizes s;
  const size_t N = (size_t)n, E = (size_t)ne;
  s.persistent = N * (sizeof(int4) + 5 * sizeof(float) + sizeof(int)) + (size_t)(nsub + 1) * sizeof(int) +
                 E * sizeof(float) * (7 + 2 * (size_t)ncomp);
  const size_t cap = hash_capacity(n);
  s.temporary = cap * (sizeof(unsigned long long) + sizeof(unsigned)) + N * sizeof(unsigned) +
                E * sizeof(float) + 64;
  return s;
}

template <class T>
int dalloc(lm_plan *p, T **ptr, size_t count) {
  void *q = nullptr;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  const hipError_t e = hipMallocAsync(&q, bytes, p->last);
  if (e != hipSuccess) {
    lmh::set_error("hipMallocAsync(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    return LM_ENOMEM;
  }
  p->allocs.push_back(q);
  *ptr = static_cast<T *>(q);
  return LM_OK;
}

// Device memory is allocated and freed stream-ordered (hipMallocAsync /
// hipFreeAsync on the plan's last stream): neither implies a device-wide
// synchronisation, so plans of other streams keep running meanwhile.
// Release errors are not reported: the plan is gone either way.
void free_plan(lm_plan *p) {
  for (void *q : p->allocs) (void)hipFreeAsync(q, p->last);
  p->allocs.clear();
  for (auto &e : p->ev_pending) {
    (void)hipEventDestroy(e.second.first);
    (void)hipEventDestroy(e.second.second);
  }
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  delete p;
}

// Times one launcher call when the plan's timing is enabled.
template <class F>
int timed(lm_plan *p, int cls, hipStream_t st, F &&launch) {
  if (!p->timing || (p->t_seen[cls]++ % p->timing) != 0) return launch();
  hipEvent_t e[2];
  for (int i = 0; i < 2; ++i) {
    if (p->ev_pool.empty()) {
      LM_TRY_HIP(hipEventCreate(&e[i]));
    } else {
      e[i] = p->ev_pool.back();
      p->ev_pool.pop_back();
    }
  }
  LM_TRY_HIP(hipEventRecord(e[0], st));
  const int rc = launch();
  LM_TRY_HIP(hipEventRecord(e[1], st));
  p->ev_pending.push_back({cls, {e[0], e[1]}});
  return rc;
}

}  // namespace

// --------------------------------------------------------------------------
// C ABI

extern "C" {

int lm_plan_bytes(const lm_geom *G, int64_t n_ev, int32_t n_sub, size_t *bytes) {
  return lm_plan_bytes_ex(G, n_ev, n_sub, 0, bytes);
}

int lm_plan_bytes_ex(const lm_geom *G, int64_t n_ev, int32_t n_sub, int32_t parts, size_t *bytes) {
  lmh::clear_error();
  lmk::GeomDev g;
  if (int rc = lmh::make_geom(G, &g)) return rc;
  LM_REQUIRE(n_ev >= 0 && n_sub >= 1 && bytes, LM_EINVAL, "bad arguments");
  LM_REQUIRE((parts & ~(LM_PART_DTV | LM_PART_FACTORS | LM_PART_RESOLUTION)) == 0, LM_EINVAL,
             "unknown plan parts 0x%x", (unsigned)parts);
  const int ncomp = G->n[2] > 1 ? 3 : 2;
  const long long E = lmk::layout_size(lmh::brick_layout(G->n));
  const Sizes s = plan_sizes(n_ev, n_sub, lmh::nvox_of(G->n), E, ncomp);
  lmk::GeomDev gb = g;
  gb.lay = lmh::brick_layout(G->n);
  size_t extra = lmk::tile_bytes_bound(gb, n_ev, n_sub);
  // allocations of the optional parts (each with the one-element minimum of
  // the plan's allocator)
  if (parts & LM_PART_DTV) extra += 2 * (size_t)E * ncomp * sizeof(float);
  if (parts & LM_PART_FACTORS) extra += (size_t)std::max<int64_t>(n_ev, 1) * sizeof(float);
  if (parts & LM_PART_RESOLUTION) extra += 5 * (size_t)E * sizeof(float);  // B x, B dz, 2 temporaries, g0
  *bytes = s.persistent + s.temporary + extra;
  return LM_OK;
}

int lm_plan_create(const lm_geom *G, const int16_t *ev, const float *s, int64_t n, int32_t n_sub,
                   const float *g_in, double gamma, double rho, double beta, double knorm, void *stream,
                   lm_plan **out) {
  lmh::clear_error();
  LM_REQUIRE(out != nullptr, LM_EINVAL, "NULL output");
  *out = nullptr;
  lmk::GeomDev g;
  if (int rc = lmh::make_geom(G, &g)) return rc;
  LM_REQUIRE(n >= 0 && n < (1LL << 31), LM_EINVAL, "event count %lld outside [0, 2^31)", (long long)n);
  LM_REQUIRE(n_sub >= 1, LM_EINVAL, "need at least one subset");
  LM_REQUIRE(n == 0 || (ev && s), LM_EINVAL, "NULL events or contamination");
  LM_REQUIRE(gamma > 0.0 && rho > 0.0 && beta >= 0.0 && std::isfinite(gamma) && std::isfinite(rho) &&
                 std::isfinite(beta),
             LM_EINVAL, "gamma and rho must be positive, beta non-negative");
  hipStream_t st = lmh::as_stream(stream);

  // validate before allocating anything
  if (n > 0) {
    unsigned long long *bad = nullptr;
    LM_TRY_HIP(hipMallocAsync((void **)&bad, sizeof(unsigned long long), st));
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(unsigned long long), st);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_count_bad, dim3(grid_for(n)), dim3(kBlock), 0, st, g, ev, (long long)n, bad);
      e = hipGetLastError();
    }
    unsigned long long hb = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, sizeof(hb), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFreeAsync(bad, st);
    LM_TRY_HIP(e);
    LM_REQUIRE(hb == 0, LM_ERANGE, "%llu events have a crystal, ring or TOF index out of range", hb);
  }

  lm_plan *p = new lm_plan();
  p->G = *G;
  p->g = g;
  p->n = n;
  p->nsub = n_sub;
  p->nvox = lmh::nvox_of(G->n);
  p->lay = lmh::brick_layout(G->n);
  p->ne = lmk::layout_size(p->lay);
  p->g.lay = p->lay;  // the plan's kernels address bricked images
  p->ncomp = G->n[2] > 1 ? 3 : 2;
  p->gamma = gamma;
  p->rho = rho;
  p->beta = beta;
  p->knorm = knorm > 0.0 ? knorm : exact_knorm(G->n);
  p->Sp = gamma * rho / p->knorm;
  p->last = st;
  p->off.resize(n_sub + 1);
  {
    const long long q = n / n_sub, rem = n % n_sub;
    for (int i = 0; i <= n_sub; ++i) p->off[i] = (int)(i * q + std::min<long long>(i, rem));
  }
  const long long N = n, E = p->ne;
  int rc = LM_OK;
  auto fail = [&](int code) {
    free_plan(p);
    return code;
  };
  if ((rc = dalloc(p, &p->rec, N)) || (rc = dalloc(p, &p->S, N)) || (rc = dalloc(p, &p->mu, N)) ||
      (rc = dalloc(p, &p->c, N)) || (rc = dalloc(p, &p->P1, N)) || (rc = dalloc(p, &p->tmp, N)) ||
      (rc = dalloc(p, &p->perm, N)) || (rc = dalloc(p, &p->off_d, n_sub + 1)) ||
      (rc = dalloc(p, &p->gimg, E)) || (rc = dalloc(p, &p->T, E)) || (rc = dalloc(p, &p->z, E)) ||
      (rc = dalloc(p, &p->zbar, E)) || (rc = dalloc(p, &p->dz, E)) || (rc = dalloc(p, &p->xint, E)) ||
      (rc = dalloc(p, &p->xalt, E)) ||
      (rc = dalloc(p, &p->w, E * p->ncomp)) || (rc = dalloc(p, &p->wn, E * p->ncomp)))
    return fail(rc);

  // temporaries: hash table, slots, ones image (bricks)
  const unsigned long long cap = hash_capacity(N);
  unsigned long long *keys = nullptr;
  unsigned *cnt = nullptr, *slot = nullptr;
  float *ones = nullptr;
  hipError_t e = hipMallocAsync((void **)&keys, cap * sizeof(unsigned long long), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&cnt, cap * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&slot, std::max<long long>(N, 1) * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&ones, E * sizeof(float), st);
  auto free_tmp = [&]() {  // release errors are not reported
    if (keys) (void)hipFreeAsync(keys, st);
    if (cnt) (void)hipFreeAsync(cnt, st);
    if (slot) (void)hipFreeAsync(slot, st);
    if (ones) (void)hipFreeAsync(ones, st);
  };
  if (e != hipSuccess) {
    free_tmp();
    lmh::set_error("temporary allocation failed: %s", hipGetErrorString(e));
    return fail(LM_ENOMEM);
  }
  auto step = [&](hipError_t he, const char *what) {
    if (he != hipSuccess && rc == LM_OK) {
      lmh::set_error("%s: %s", what, hipGetErrorString(he));
      rc = LM_EHIP;
    }
  };
  step(hipMemcpyAsync(p->off_d, p->off.data(), (n_sub + 1) * sizeof(int), hipMemcpyHostToDevice, st), "offsets");
  // every image starts at zero, padding included (padding stays zero)
  for (float *img : {p->gimg, p->T, p->z, p->zbar, p->dz, p->xint, p->xalt})
    step(hipMemsetAsync(img, 0, E * sizeof(float), st), "zero images");
  for (float *img : {p->w, p->wn}) step(hipMemsetAsync(img, 0, E * p->ncomp * sizeof(float), st), "zero w");
  if (N > 0) {
    step(hipMemsetAsync(keys, 0xFF, cap * sizeof(unsigned long long), st), "hash init");
    step(hipMemsetAsync(cnt, 0, cap * sizeof(unsigned), st), "hash init");
    hipLaunchKernelGGL(k_hash_insert, dim3(grid_for(N)), dim3(kBlock), 0, st, g, ev, N, keys, cnt,
                       (unsigned)(cap - 1), slot);
    step(hipGetLastError(), "hash insert");
    hipLaunchKernelGGL(k_layout, dim3(grid_for(N)), dim3(kBlock), 0, st, g, ev, s, N, n_sub, cnt, slot, p->rec,
                       p->mu, p->perm);
    step(hipGetLastError(), "layout");
  }
  // P^LM 1 and S
  hipLaunchKernelGGL(k_fill, dim3(grid_for(E)), dim3(kBlock), 0, st, ones, 1.0f, E);
  step(hipGetLastError(), "fill");
  if (rc == LM_OK && N > 0) rc = lmk::launch_fwd_rec(p->g, ones, p->rec, N, p->P1, st);
  if (N > 0) {
    hipLaunchKernelGGL(k_step_S, dim3(grid_for(N)), dim3(kBlock), 0, st, p->P1, p->S, (float)(gamma * rho),
                       p1_floor(p->G), N);
    step(hipGetLastError(), "step S");
  }
  // sensitivity (row-major, from the caller or lm_sens) into bricks, and T
  if (g_in) {
    if (rc == LM_OK) rc = lmk::launch_to_layout(G->n, p->lay, 1, g_in, p->gimg, st);
  } else {
    step(hipMemsetAsync(p->gimg, 0, E * sizeof(float), st), "zero g");
    if (rc == LM_OK) rc = lmk::launch_sens(p->g, p->gimg, st);  // bricked geometry
    p->g_internal = true;
  }
  hipLaunchKernelGGL(k_step_T, dim3(grid_for(E)), dim3(kBlock), 0, st, p->gimg, p->T, (float)(rho / (2.0 * gamma)),
                     (float)p->knorm, E);
  step(hipGetLastError(), "step T");
  // the tile lists of the data updates (synchronous; the per-event path
  // stays when they do not fit)
  if (rc == LM_OK && N > 0) rc = lmk::build_tiles(p->g, p->rec, p->off, p->tiles, p->allocs, st);
  step(hipStreamSynchronize(st), "plan create");
  free_tmp();
  if (rc != LM_OK) return fail(rc);
  *out = p;
  return LM_OK;
}

int lm_spdhg_init(lm_plan *p, const float *x0, void *stream) {
  lmh::clear_error();
  LM_REQUIRE(p && x0, LM_EINVAL, "NULL plan or image");
  hipStream_t st = lmh::as_stream(stream);
  p->last = st;
  const long long N = p->n, E = p->ne;
  if (int rc = lmk::launch_to_layout(p->G.n, p->lay, 1, x0, p->xint, st)) return rc;
  LM_TRY_HIP(hipMemcpyAsync(p->z, p->gimg, E * sizeof(float), hipMemcpyDeviceToDevice, st));
  if (N > 0 && !p->blur.on) {
    if (int rc = lmk::launch_fwd_rec(p->g, p->xint, p->rec, N, p->c, st)) return rc;
    hipLaunchKernelGGL(k_init_dual, dim3(grid_for(N)), dim3(kBlock), 0, st, p->c, p->rec, p->mu, p->tmp, N);
    LM_TRY_HIP(hipGetLastError());
    if (int rc = lmk::launch_back_rec(p->g, p->tmp, p->rec, N, p->z, st)) return rc;
  } else if (N > 0) {
    // P = G B: y from G (B x0); z gains B G^T((y - 1) / mu)
    if (int rc = lmk::launch_blur(p->G.n, p->lay, E, p->blur, p->xint, p->xb, p->bt1, p->bt2, st)) return rc;
    if (int rc = lmk::launch_fwd_rec(p->g, p->xb, p->rec, N, p->c, st)) return rc;
    hipLaunchKernelGGL(k_init_dual, dim3(grid_for(N)), dim3(kBlock), 0, st, p->c, p->rec, p->mu, p->tmp, N);
    LM_TRY_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_fill, dim3(grid_for(E)), dim3(kBlock), 0, st, p->dz, 0.0f, E);
    LM_TRY_HIP(hipGetLastError());
    if (int rc = lmk::launch_back_rec(p->g, p->tmp, p->rec, N, p->dz, st)) return rc;
    if (int rc = lmk::launch_blur(p->G.n, p->lay, E, p->blur, p->dz, p->dzb, p->bt1, p->bt2, st)) return rc;
    hipLaunchKernelGGL(k_add, dim3(grid_for(E)), dim3(kBlock), 0, st, p->z, p->dzb, E);
    LM_TRY_HIP(hipGetLastError());
  }
  LM_TRY_HIP(hipMemcpyAsync(p->zbar, p->z, E * sizeof(float), hipMemcpyDeviceToDevice, st));
  LM_TRY_HIP(hipMemsetAsync(p->w, 0, E * p->ncomp * sizeof(float), st));
  LM_TRY_HIP(hipMemsetAsync(p->wn, 0, E * p->ncomp * sizeof(float), st));
  LM_TRY_HIP(hipMemsetAsync(p->dz, 0, E * sizeof(float), st));
  p->u = 0;
  p->initialized = true;
  return LM_OK;
}

int lm_spdhg_epoch(lm_plan *p, float *x, const int32_t *seq, int32_t n_updates, void *stream) {
  lmh::clear_error();
  LM_REQUIRE(p && x, LM_EINVAL, "NULL plan or image");
  LM_REQUIRE(p->initialized, LM_ESTATE, "lm_spdhg_init has not been called");
  LM_REQUIRE(n_updates >= 0 && (n_updates == 0 || seq), LM_EINVAL, "bad update sequence");
  for (int u = 0; u < n_updates; ++u)
    LM_REQUIRE(seq[u] >= 0 && seq[u] <= p->nsub, LM_EINVAL, "seq[%d] = %d outside [0, %d]", u, seq[u], p->nsub);
  if (n_updates == 0) return LM_OK;
  const TraceRange epoch_range(p->trace, "lm_spdhg_epoch");
  hipStream_t st = lmh::as_stream(stream);
  p->last = st;
  const long long E = p->ne;
  const float inv_p_data = 2.0f * (float)p->nsub;  // 1 / p_k, p_k = 1 / (2n)
  const float inv_p_prior = 2.0f;                  // 1 / p_prior, p_prior = 1/2
  float *xi = p->xint;
  if (int rc = timed(p, LM_K_PRIMAL, st, [&] {
        int r = lmk::launch_to_layout(p->G.n, p->lay, 1, x, xi, st);
        return r ? r : lmk::launch_primal(xi, p->T, p->zbar, E, st);
      }))
    return rc;
  char range_name[48] = "prior update";
  for (int u = 0; u < n_updates; ++u) {
    const int i = seq[u];
    const bool fuse = u + 1 < n_updates;
    if (p->trace) {
      if (i < p->nsub) std::snprintf(range_name, sizeof range_name, "data update, subset %d", i);
      else std::snprintf(range_name, sizeof range_name, "prior update");
    }
    const TraceRange update_range(p->trace, range_name);
    if (i < p->nsub) {
      const long long o = p->off[i], c = p->off[i + 1] - p->off[i];
      if (p->tiles.on && !p->blur.on) {
        // by tile: forward, prox and records, then the back projection
        // fused with z / zbar and the next primal step
        if (int rc = timed(p, LM_K_DATA, st, [&] {
              return lmk::launch_tile_fwd(p->g, p->tiles, xi, p->rec, p->S, p->mu, p->c, o, c, st);
            }))
          return rc;
        if (int rc = timed(p, LM_K_DUAL_IMAGE, st, [&] {
              return lmk::launch_tile_back(p->g, p->tiles, i, p->z, xi, p->T, p->zbar, nullptr, inv_p_data, fuse,
                                           st);
            }))
          return rc;
      } else if (p->tiles.on) {
        // P = G B by tile: the update projects B x and writes its whole back
        // projection to dz, which the blur passes take to z
        if (int rc = timed(p, LM_K_DATA, st, [&] {
              int r = lmk::launch_blur(p->G.n, p->lay, E, p->blur, xi, p->xb, p->bt1, p->bt2, st);
              if (!r) r = lmk::launch_tile_fwd(p->g, p->tiles, p->xb, p->rec, p->S, p->mu, p->c, o, c, st);
              return r ? r : lmk::launch_tile_back(p->g, p->tiles, i, p->z, xi, p->T, p->zbar, p->dz, inv_p_data,
                                                   fuse, st);
            }))
          return rc;
        if (int rc = timed(p, LM_K_DUAL_IMAGE, st, [&] {
              return lmk::launch_blur_dual_image(p->G.n, p->lay, E, p->blur, p->dz, p->bt1, p->bt2, p->z, xi, p->T,
                                                 p->zbar, inv_p_data, fuse, st);
            }))
          return rc;
      } else if (!p->blur.on) {
        if (int rc = timed(p, LM_K_DATA, st, [&] {
              return lmk::launch_data_update(p->g, xi, p->rec + o, p->S + o, p->mu + o, p->c + o, p->dz, c, st);
            }))
          return rc;
        if (int rc = timed(p, LM_K_DUAL_IMAGE, st, [&] {
              return lmk::launch_dual_image(p->z, p->dz, xi, p->T, p->zbar, inv_p_data, fuse, E, st);
            }))
          return rc;
      } else {
        // P = G B: the update projects B x; z takes B of its back projection
        if (int rc = timed(p, LM_K_DATA, st, [&] {
              int r = lmk::launch_blur(p->G.n, p->lay, E, p->blur, xi, p->xb, p->bt1, p->bt2, st);
              return r ? r : lmk::launch_data_update(p->g, p->xb, p->rec + o, p->S + o, p->mu + o, p->c + o, p->dz,
                                                     c, st);
            }))
          return rc;
        if (int rc = timed(p, LM_K_DUAL_IMAGE, st, [&] {
              return lmk::launch_blur_dual_image(p->G.n, p->lay, E, p->blur, p->dz, p->bt1, p->bt2, p->z, xi, p->T,
                                                 p->zbar, inv_p_data, fuse, st);
            }))
          return rc;
      }
    } else if (p->dtv && !lmk::prior_march_ok(p->lay, p->ncomp)) {
      // K = D grad on one slice: the dual step, then the adjoint fused with
      // z / zbar and the next primal step (in place)
      if (int rc = timed(p, LM_K_TV, st, [&] {
            return lmk::launch_dtv_prior(p->G.n, p->lay, p->ncomp, E, xi, p->w, p->wn, p->xi_dtv, p->pd, p->z,
                                         p->T, p->zbar, (float)p->Sp, (float)p->beta, inv_p_prior, fuse, st);
          }))
        return rc;
      std::swap(p->w, p->wn);
    } else {
      // TV, or DTV (K = D grad) in 3D: one pass
      if (int rc = timed(p, LM_K_TV, st, [&] {
            return lmk::launch_tv_fused(p->G.n, p->lay, p->ncomp, xi, p->w, p->dtv ? p->xi_dtv : nullptr, p->wn,
                                        p->z, p->xalt, p->T, p->zbar, (float)p->Sp, (float)p->beta, inv_p_prior,
                                        fuse, st);
          }))
        return rc;
      std::swap(p->w, p->wn);
      if (fuse) std::swap(p->xint, p->xalt);  // the next primal step's x
      xi = p->xint;
    }
    ++p->u;
  }
  if (int rc = timed(p, LM_K_PRIMAL, st, [&] { return lmk::launch_from_layout(p->G.n, p->lay, 1, xi, x, st); }))
    return rc;
  return LM_OK;
}

int lm_plan_set_event_factors(lm_plan *p, const float *m, void *stream) {
  lmh::clear_error();
  LM_REQUIRE(p && m, LM_EINVAL, "NULL plan or factors");
  LM_REQUIRE(!p->initialized, LM_ESTATE, "event factors must be set before lm_spdhg_init");
  LM_REQUIRE(!p->mfac, LM_ESTATE, "event factors are already set");
  LM_REQUIRE(!p->g_internal, LM_ESTATE,
             "the plan computed g = P^T 1 itself; with factors g must be the sensitivity of diag(m) P over all "
             "LORs, which the event list cannot give: pass it to lm_plan_create");
  const long long N = p->n;
  if (N == 0) return LM_OK;
  hipStream_t st = lmh::as_stream(stream);
  p->last = st;
  unsigned long long *d = nullptr, h = 0;
  LM_TRY_HIP(hipMallocAsync((void **)&d, sizeof(*d), st));
  hipError_t e = hipMemsetAsync(d, 0, sizeof(*d), st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_check_factors, dim3(grid_for(N)), dim3(kBlock), 0, st, m, N, d);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFreeAsync(d, st);
  LM_TRY_HIP(e);
  LM_REQUIRE(h == 0, LM_ERANGE, "%llu event factors are not positive and finite", h);
  if (int rc = dalloc(p, &p->mfac, (size_t)N)) return rc;
  hipLaunchKernelGGL(k_apply_factors, dim3(grid_for(N)), dim3(kBlock), 0, st, m, p->perm, p->rec, p->mu, p->mfac, N);
  LM_TRY_HIP(hipGetLastError());
  LM_TRY_HIP(hipStreamSynchronize(st));
  return LM_OK;
}

int lm_plan_set_resolution(lm_plan *p, const double fwhm_vox[3], void *stream) {
  lmh::clear_error();
  LM_REQUIRE(p && fwhm_vox, LM_EINVAL, "NULL plan or FWHM");
  LM_REQUIRE(!p->initialized, LM_ESTATE, "the resolution model must be set before lm_spdhg_init");
  lmk::Blur b;
  if (int rc = lmk::make_blur(fwhm_vox, &b)) return rc;
  hipStream_t st = lmh::as_stream(stream);
  p->last = st;
  const long long N = p->n, E = p->ne;
  if (b.on && !p->xb) {
    int rc;
    if ((rc = dalloc(p, &p->xb, (size_t)E)) || (rc = dalloc(p, &p->dzb, (size_t)E)) ||
        (rc = dalloc(p, &p->bt1, (size_t)E)) || (rc = dalloc(p, &p->bt2, (size_t)E)))
      return rc;
  }
  p->blur = b;
  // P^LM 1 and S_e = gamma rho / (P^LM 1)_e of the operator G B
  if (N > 0) {
    float *ones = b.on ? p->dzb : p->dz;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(E)), dim3(kBlock), 0, st, ones, 1.0f, E);
    LM_TRY_HIP(hipGetLastError());
    const float *src = ones;
    if (b.on) {
      if (int rc = lmk::launch_blur(p->G.n, p->lay, E, b, ones, p->xb, p->bt1, p->bt2, st)) return rc;
      src = p->xb;
    }
    if (int rc = lmk::launch_fwd_rec(p->g, src, p->rec, N, p->P1, st)) return rc;
    hipLaunchKernelGGL(k_step_S, dim3(grid_for(N)), dim3(kBlock), 0, st, p->P1, p->S, (float)(p->gamma * p->rho),
                       p1_floor(p->G), N);
    LM_TRY_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_fill, dim3(grid_for(E)), dim3(kBlock), 0, st, ones, 0.0f, E);
    LM_TRY_HIP(hipGetLastError());
  }
  if (p->g_internal) {
    // the plan's own g = G^T 1 becomes the sensitivity of G B, B G^T 1 (B is
    // symmetric), and T follows it
    if (!p->g0) {
      if (int rc = dalloc(p, &p->g0, (size_t)E)) return rc;
      LM_TRY_HIP(hipMemcpyAsync(p->g0, p->gimg, E * sizeof(float), hipMemcpyDeviceToDevice, st));
    }
    if (b.on) {
      if (int rc = lmk::launch_blur(p->G.n, p->lay, E, b, p->g0, p->gimg, p->bt1, p->bt2, st)) return rc;
    } else {
      LM_TRY_HIP(hipMemcpyAsync(p->gimg, p->g0, E * sizeof(float), hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL(k_step_T, dim3(grid_for(E)), dim3(kBlock), 0, st, p->gimg, p->T,
                       (float)(p->rho / (2.0 * p->gamma)), (float)p->knorm, E);
    LM_TRY_HIP(hipGetLastError());
  }
  LM_TRY_HIP(hipStreamSynchronize(st));
  return LM_OK;
}

int lm_plan_set_prior_image(lm_plan *p, const float *v, double eta, void *stream) {
  lmh::clear_error();
  LM_REQUIRE(p, LM_EINVAL, "NULL plan");
  if (!v) {
    p->dtv = false;
    return LM_OK;
  }
  LM_REQUIRE(eta > 0.0 && std::isfinite(eta), LM_EINVAL, "eta must be positive and finite");
  hipStream_t st = lmh::as_stream(stream);
  p->last = st;
  if (!p->xi_dtv) {
    if (int rc = dalloc(p, &p->xi_dtv, (size_t)(p->ne * p->ncomp))) return rc;
    if (int rc = dalloc(p, &p->pd, (size_t)(p->ne * p->ncomp))) return rc;
  }
  if (int rc = lmk::launch_dtv_field(p->G.n, p->lay, p->ncomp, p->ne, v, (float)eta, p->xi_dtv, st)) return rc;
  p->dtv = true;
  return LM_OK;
}

int lm_plan_info(const lm_plan *p, int64_t *n_ev, int32_t *n_sub, int64_t *nvox) {
  lmh::clear_error();
  LM_REQUIRE(p, LM_EINVAL, "NULL plan");
  if (n_ev) *n_ev = p->n;
  if (n_sub) *n_sub = p->nsub;
  if (nvox) *nvox = p->nvox;
  return LM_OK;
}

int lm_plan_get_lists(const lm_plan *p, float *y, int32_t *mu, int32_t *subset, float *p1, void *stream) {
  lmh::clear_error();
  LM_REQUIRE(p, LM_EINVAL, "NULL plan");
  hipStream_t st = lmh::as_stream(stream);
  const long long N = p->n;
  if (N == 0) return LM_OK;
  if (y) {
    hipLaunchKernelGGL(k_scatter_f, dim3(grid_for(N)), dim3(kBlock), 0, st, p->c, p->perm, y, N, 1.0f, -1.0f);
    LM_TRY_HIP(hipGetLastError());
  }
  if (mu) {
    if (p->mfac)
      hipLaunchKernelGGL(k_scatter_mu_fac, dim3(grid_for(N)), dim3(kBlock), 0, st, p->mu, p->mfac, p->perm, mu, N);
    else
      hipLaunchKernelGGL(k_scatter_mu, dim3(grid_for(N)), dim3(kBlock), 0, st, p->mu, p->perm, mu, N);
    LM_TRY_HIP(hipGetLastError());
  }
  if (subset) {
    hipLaunchKernelGGL(k_subset_ids, dim3(grid_for(N)), dim3(kBlock), 0, st, p->off_d, p->perm, subset, p->nsub, N);
    LM_TRY_HIP(hipGetLastError());
  }
  if (p1) {
    hipLaunchKernelGGL(k_scatter_f, dim3(grid_for(N)), dim3(kBlock), 0, st, p->P1, p->perm, p1, N);
    LM_TRY_HIP(hipGetLastError());
  }
  return LM_OK;
}

int lm_plan_get_layout(const lm_plan *p, int32_t *perm, int32_t *offsets, void *stream) {
  lmh::clear_error();
  LM_REQUIRE(p, LM_EINVAL, "NULL plan");
  hipStream_t st = lmh::as_stream(stream);
  if (perm && p->n > 0)
    LM_TRY_HIP(hipMemcpyAsync(perm, p->perm, p->n * sizeof(int), hipMemcpyDeviceToDevice, st));
  if (offsets)
    LM_TRY_HIP(hipMemcpyAsync(offsets, p->off_d, (p->nsub + 1) * sizeof(int), hipMemcpyDeviceToDevice, st));
  return LM_OK;
}

int lm_plan_get_images(const lm_plan *p, float *g, float *T, void *stream) {
  lmh::clear_error();
  LM_REQUIRE(p, LM_EINVAL, "NULL plan");
  hipStream_t st = lmh::as_stream(stream);
  if (g)
    if (int rc = lmk::launch_from_layout(p->G.n, p->lay, 1, p->gimg, g, st)) return rc;
  if (T)
    if (int rc = lmk::launch_from_layout(p->G.n, p->lay, 1, p->T, T, st)) return rc;
  return LM_OK;
}

int lm_plan_get_state(const lm_plan *p, float *z, float *zbar, float *w, float *c, int64_t *u, void *stream) {
  lmh::clear_error();
  LM_REQUIRE(p, LM_EINVAL, "NULL plan");
  LM_REQUIRE(p->initialized, LM_ESTATE, "plan not initialised");
  hipStream_t st = lmh::as_stream(stream);
  const long long V = p->nvox;
  if (z)
    if (int rc = lmk::launch_from_layout(p->G.n, p->lay, 1, p->z, z, st)) return rc;
  if (zbar)
    if (int rc = lmk::launch_from_layout(p->G.n, p->lay, 1, p->zbar, zbar, st)) return rc;
  if (w) {
    if (int rc = lmk::launch_from_layout(p->G.n, p->lay, p->ncomp, p->w, w, st)) return rc;
    if (p->ncomp < 3) LM_TRY_HIP(hipMemsetAsync(w + V * p->ncomp, 0, V * (3 - p->ncomp) * sizeof(float), st));
  }
  if (c && p->n > 0) {
    hipLaunchKernelGGL(k_scatter_f, dim3(grid_for(p->n)), dim3(kBlock), 0, st, p->c, p->perm, c, p->n, 0.0f, 1.0f);
    LM_TRY_HIP(hipGetLastError());
  }
  if (u) *u = p->u;
  return LM_OK;
}

int lm_plan_set_state(lm_plan *p, const float *z, const float *zbar, const float *w, const float *c, int64_t u,
                      void *stream) {
  lmh::clear_error();
  LM_REQUIRE(p && z && zbar && w && (c || p->n == 0), LM_EINVAL, "NULL argument");
  LM_REQUIRE(u >= 0, LM_EINVAL, "negative update counter");
  hipStream_t st = lmh::as_stream(stream);
  p->last = st;
  if (int rc = lmk::launch_to_layout(p->G.n, p->lay, 1, z, p->z, st)) return rc;
  if (int rc = lmk::launch_to_layout(p->G.n, p->lay, 1, zbar, p->zbar, st)) return rc;
  if (int rc = lmk::launch_to_layout(p->G.n, p->lay, p->ncomp, w, p->w, st)) return rc;
  if (p->n > 0) {
    hipLaunchKernelGGL(k_gather_f, dim3(grid_for(p->n)), dim3(kBlock), 0, st, c, p->perm, p->c, p->n);
    LM_TRY_HIP(hipGetLastError());
  }
  LM_TRY_HIP(hipMemsetAsync(p->dz, 0, p->ne * sizeof(float), st));
  p->u = u;
  p->initialized = true;
  return LM_OK;
}

int lm_plan_set_tracing(lm_plan *p, int on) {
  lmh::clear_error();
  LM_REQUIRE(p, LM_EINVAL, "NULL plan");
  p->trace = on != 0;
  return LM_OK;
}

int lm_plan_timing(lm_plan *p, int every) {
  lmh::clear_error();
  LM_REQUIRE(p, LM_EINVAL, "NULL plan");
  LM_REQUIRE(every >= 0, LM_EINVAL, "negative timing stride %d", every);
  for (auto &e : p->ev_pending) {
    p->ev_pool.push_back(e.second.first);
    p->ev_pool.push_back(e.second.second);
  }
  p->ev_pending.clear();
  for (int k = 0; k < LM_K_COUNT; ++k) {
    p->t_ms[k] = 0.0;
    p->t_n[k] = 0;
    p->t_seen[k] = 0;
  }
  p->timing = every;
  return LM_OK;
}

int lm_plan_get_timing(lm_plan *p, double *ms, int64_t *launches) {
  lmh::clear_error();
  LM_REQUIRE(p, LM_EINVAL, "NULL plan");
  for (auto &e : p->ev_pending) {
    LM_TRY_HIP(hipEventSynchronize(e.second.second));
    float t = 0.0f;
    LM_TRY_HIP(hipEventElapsedTime(&t, e.second.first, e.second.second));
    p->t_ms[e.first] += t;
    p->t_n[e.first] += 1;
    p->ev_pool.push_back(e.second.first);
    p->ev_pool.push_back(e.second.second);
  }
  p->ev_pending.clear();
  for (int k = 0; k < LM_K_COUNT; ++k) {
    if (ms) ms[k] = p->t_ms[k];
    if (launches) launches[k] = p->t_n[k];
  }
  return LM_OK;
}

int lm_plan_destroy(lm_plan *p) {
  lmh::clear_error();
  if (!p) return LM_OK;
  hipError_t e = hipStreamSynchronize(p->last);
  free_plan(p);
  LM_TRY_HIP(e);
  return LM_OK;
}

}  // extern "C"
