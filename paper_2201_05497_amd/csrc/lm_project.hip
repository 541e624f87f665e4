// Listmode TOF Joseph projector kernels for gfx950 and their C ABI entry
// points: lm_fwd, lm_back, lm_sens, lm_validate_events, plus the fused
// subset update of LM-SPDHG used by the plan code.
//
// The forward operator is the paper's listmode operator (Eq. lmop): one
// row of the TOF system matrix per event.  The fused update evaluates, for
// every event of a subset, the forward value, the dual prox (Eq. proxD with
// d = mu_e) and back-projects the scaled dual increment (the data-subset
// branch of Algorithm 2) in a single pass, so the samples of the forward pass are reused
// from registers by the back projection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "lm_device.hpp"
#include "lm_host.hpp"
#include "lm_image.hpp"

using namespace lmk;

namespace {

constexpr int kBlock = 256;

// Event sources: the caller's int16[5] records, the plan's int4 records,
// or the caller's records in a given order (out[order[e]] for the e-th).
// kXcdOrder: the blocks of a launch take the list in eight contiguous
// parts, one per XCD (blocks are dealt to the XCDs round robin), so that
// the events of a part share that XCD's L2.
struct CallerEvents {
  static constexpr bool kXcdOrder = false;
  const int16_t *ev;
  CallerEvents offset(long long o) const { return CallerEvents{ev + 5 * o}; }
  __device__ __forceinline__ bool get(const GeomDev &g, long long e, int &id1, int &id2, int &k) const {
    return decode_event(g, ev + 5 * e, id1, id2, k);
  }
  __device__ __forceinline__ long long slot(long long e) const { return e; }
};
struct PlanEvents {
  static constexpr bool kXcdOrder = false;
  const int4 *rec;
  PlanEvents offset(long long o) const { return PlanEvents{rec + o}; }
  __device__ __forceinline__ bool get(const GeomDev &, long long e, int &id1, int &id2, int &k) const {
    const int4 r = rec[e];
    id1 = r.x;
    id2 = r.y;
    k = r.z;
    return true;
  }
  __device__ __forceinline__ long long slot(long long e) const { return e; }
};
struct SortedEvents {
  static constexpr bool kXcdOrder = true;
  const int16_t *ev;
  const unsigned *order;
  SortedEvents offset(long long o) const { return SortedEvents{ev, order + o}; }
  __device__ __forceinline__ bool get(const GeomDev &g, long long e, int &id1, int &id2, int &k) const {
    return decode_event(g, ev + 5 * (long long)order[e], id1, id2, k);
  }
  __device__ __forceinline__ long long slot(long long e) const { return order[e]; }
};

// Lanes per event of the forward projector, and events per launch (2^19
// blocks).
constexpr int kFwdLanes = 8;
constexpr long long kFwdLaunch = 1LL << 27;

// Forward projection.  A wavefront takes 64 consecutive events of the
// source: lane e first sets up the ray of event e (the double-precision
// set-up runs once per event rather than once per lane of a group) and
// stores it in LDS; then, in eight rounds, each group of kFwdLanes = 8 lanes
// walks the planes of one event (lane l of the group from the brick
// boundary at or below the first plane, every 8th plane), and lane e of the
// wavefront collects event e's sum for one store per lane.
template <class Src>
__global__ __launch_bounds__(kBlock) void k_fwd(GeomDev g, const int *skip, const float *__restrict__ x, Src src,
                                                long long n, float *__restrict__ out) {
  static_assert(kFwdLanes == 8, "eight groups of eight lanes per wavefront");
  __shared__ RayPack rays[kBlock];
  if (skip && *skip) return;  // the list went to the path by line
  const int lane = threadIdx.x & 63;
  const int wbase = threadIdx.x & ~63;
  long long blk = blockIdx.x;
  if constexpr (Src::kXcdOrder) {  // gridDim.x is a multiple of 8
    const long long per = gridDim.x / 8;
    blk = (blk % 8) * per + blk / 8;
  }
  if (blk * kBlock + wbase >= n) return;  // the whole wavefront is past the end
  const long long e = blk * kBlock + threadIdx.x;
  {
    // every field defined on every path: lanes past the end and invalid
    // events store an empty ray, and only valid events reach the set-up
    // (which reads the crystal table at the decoded ids)
    RayPack pk = empty_ray();
    int id1 = 0, id2 = 0, k = 0;
    if (e < n && src.get(g, e, id1, id2, k)) pk = pack_ray(setup_ray(g, id1, id2, k, W_BIN, 1 << 20));
    rays[threadIdx.x] = pk;
  }
  // LDS operations of one wavefront complete in order; the fences keep the
  // compiler from moving the reads above the writes
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const float D = tof_bin_width(g);
  const int gl = lane & 7, grp = lane >> 3;
  float mine = 0.0f, L = 0.0f;
  for (int round = 0; round < 8; ++round) {
    const RayPack pk = rays[wbase + 8 * round + grp];
    float acc = 0.0f;
    if (pk.p.y > 0) acc = g.tof_on ? fwd_walk<true>(g, x, pk, D, gl) : fwd_walk<false>(g, x, pk, D, gl);
    acc = group_sum<8>(acc);
    // lanes 8 round .. 8 round + 7 take the sums of groups 0 .. 7
    const float got = __shfl(acc, 8 * gl);
    if (grp == round) mine = got;
  }
  L = __int_as_float(rays[threadIdx.x].q.w);
  if (e < n) out[src.slot(e)] = L * mine;
}

// Per-wavefront LDS staging of the interleaved scatter (4 wavefronts per
// block, 4 corners x 64 lanes each).
struct Stage {
  int idx[kBlock / 64][256];
  float val[kBlock / 64][256];
};

// Back projection: one event per wavefront, the scatter of every 64 planes
// interleaved over corners; the grid strides over the list.  With `skip`
// set the kernel does nothing when *skip is non-zero (the list went to the
// transaxial-line path instead).
template <class Src>
__global__ __launch_bounds__(kBlock) void k_back(GeomDev g, const int *skip, const float *__restrict__ v, Src src,
                                                 long long n, float *img) {
  __shared__ Stage st;
  if (skip && *skip) return;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const long long stride = (long long)gridDim.x * (kBlock / 64);
  for (long long e = (long long)blockIdx.x * (kBlock / 64) + wv; e < n; e += stride) {
    const float ve = v[e];
    if (ve == 0.0f) continue;
    int id1, id2, k;
    if (!src.get(g, e, id1, id2, k)) continue;
    const Ray r = setup_ray(g, id1, id2, k, W_BIN, 1 << 20);
    const float c = r.L * ve;
    const int off = brick_offset(g.lay, r);
    for (int j0 = -off; j0 < r.nplanes; j0 += 64) {
      const int j = j0 + lane;
      Sample s = sample_at(g, r, j, g.tof_on);
      const float cs = (j >= 0 && j < r.nplanes) ? c * s.w : 0.0f;
      scatter_interleaved(g, img, r, s, cs, lane, st.idx[wv], st.val[wv]);
    }
  }
}

// Sensitivity: every unordered pair (id1 < id2) of crystals, weight summed
// over all TOF bins, one pair per wavefront, the grid striding over the
// pairs; nothing when *skip is non-zero (the pairs went to the line path).
__global__ __launch_bounds__(kBlock) void k_sens(GeomDev g, const int *skip, long long npairs, float *img) {
  __shared__ Stage st;
  if (skip && *skip) return;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const long long nd = g.n_det;
  const long long stride = (long long)gridDim.x * (kBlock / 64);
  for (long long p = (long long)blockIdx.x * (kBlock / 64) + wv; p < npairs; p += stride) {
    // row i holds pairs (i, i+1..nd-1); first index of row i is i*nd - i(i+1)/2
    const double b = 2.0 * nd - 1.0;
    long long i = (long long)floor((b - sqrt(b * b - 8.0 * (double)p)) * 0.5);
    auto first = [&](long long r) { return r * nd - r * (r + 1) / 2; };
    if (i < 0) i = 0;
    while (i > 0 && first(i) > p) --i;
    while (i + 1 < nd && first(i + 1) <= p) ++i;
    const long long jdx = i + 1 + (p - first(i));
    const Ray r = setup_ray(g, (int)i, (int)jdx, 0, W_SUM, 1 << 20);
    const int off = brick_offset(g.lay, r);
    for (int j0 = -off; j0 < r.nplanes; j0 += 64) {
      const int j = j0 + lane;
      Sample s = sample_at(g, r, j, g.tof_on);
      const float cs = (j >= 0 && j < r.nplanes) ? r.L * s.w : 0.0f;
      scatter_interleaved(g, img, r, s, cs, lane, st.idx[wv], st.val[wv]);
    }
  }
}

// Fused subset update (the data-subset branch of Algorithm 2) for the events
// of one subset, stored contiguously in the plan's order, one event per
// wavefront:
//   q = (P x)_e + s_e;  y+ = prox(y_e + S_e q) with d = mu_e;
//   dz += P^T((y+ - y_e)/mu_e);  y_e = y+.
// The dual is kept as its complement c = 1 - y (y tends to 1 on LORs with
// large expected counts, where 1 - y would cancel), and the increment is
// evaluated in the cancellation-free form
//   y+ - y = 2 S (q c - mu) / (S q + c + sqrt((S q - c)^2 + 4 S mu)),
// algebraically identical to Eq. proxD minus y; c+ = c - (y+ - y).  The
// samples of the forward pass stay in registers for the back projection.
template <int JMAX>
__global__ __launch_bounds__(kBlock) void k_data_update(GeomDev g, const float *__restrict__ x,
                                                        const int4 *__restrict__ rec,
                                                        const float *__restrict__ S,
                                                        const float *__restrict__ mu,
                                                        float *__restrict__ cdual, float *dz, long long n) {
  __shared__ Stage st;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const long long e = (long long)blockIdx.x * (kBlock / 64) + wv;
  if (e >= n) return;
  const int4 rc = rec[e];
  const float Se = S[e];
  if (Se == 0.0f) return;  // LOR misses the image: the prox leaves y unchanged
  const Ray r = setup_ray(g, rc.x, rc.y, rc.z, W_BIN, JMAX * 64 - kMaxBrickOffset);
  const int off = brick_offset(g.lay, r);
  Sample cache[JMAX];
  float acc = 0.0f;
#pragma unroll
  for (int jj = 0; jj < JMAX; ++jj) {
    const int j = lane + jj * 64 - off;
    cache[jj] = sample_at(g, r, j, g.tof_on);
    if (j >= 0 && j < r.nplanes) {
      acc = fmaf(cache[jj].w, gather(g, x, r, cache[jj]), acc);
    } else {
      cache[jj].w = 0.0f;
    }
  }
  acc = group_sum<64>(acc);
  const float q = fmaf(r.L, acc, __int_as_float(rc.w));
  const float c = cdual[e], me = mu[e];
  const float sq = Se * q;
  const float t = sq - c;
  const float rt = sqrtf(fmaf(t, t, 4.0f * Se * me));
  const float dy = 2.0f * Se * fmaf(q, c, -me) / (sq + c + rt);
  if (lane == 0) cdual[e] = c - dy;
  if (dy == 0.0f) return;
  const float cf = r.L * (dy / me);
#pragma unroll
  for (int jj = 0; jj < JMAX; ++jj) {
    if (jj * 64 - off < r.nplanes) {
      const float cs = (cache[jj].w != 0.0f) ? cf * cache[jj].w : 0.0f;
      scatter_interleaved(g, dz, r, cache[jj], cs, lane, st.idx[wv], st.val[wv]);
    }
  }
}

// Counts events with an out-of-range crystal, ring or TOF index.
__global__ void k_validate(GeomDev g, const int16_t *ev, long long n, unsigned long long *bad) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int id1, id2, k;
  const bool ok = (e >= n) || decode_event(g, ev + 5 * e, id1, id2, k);
  const unsigned long long m = __ballot(!ok);
  if ((threadIdx.x % 64) == 0 && m) atomicAdd(bad, (unsigned long long)__popcll(m));
}


inline unsigned blocks_for(long long n, int lpe) {
  const long long per = kBlock / lpe;
  return (unsigned)((n + per - 1) / per);
}

// A launch covers at most 2^22 blocks (2^30 work-items): the total number
// of work-items of one dispatch must stay below 2^32.  Larger inputs are
// processed in consecutive launches on the same stream.
constexpr long long kMaxBlocks = 1LL << 22;
inline long long chunk_items(int lpe) { return kMaxBlocks * (kBlock / lpe); }

}  // namespace

// --------------------------------------------------------------------------
// geometry and launch policy

namespace lmh {

int make_geom(const lm_geom *G, lmk::GeomDev *o) {
  LM_REQUIRE(G != nullptr, LM_EINVAL, "lm_geom is NULL");
  LM_REQUIRE(G->det != nullptr, LM_EINVAL, "lm_geom.det is NULL");
  LM_REQUIRE(G->n_cry > 0 && G->n_ring > 0, LM_EINVAL, "n_cry and n_ring must be positive");
  LM_REQUIRE((long long)G->n_cry * G->n_ring < (1LL << 30), LM_EINVAL, "too many crystals");
  for (int a = 0; a < 3; ++a) {
    LM_REQUIRE(G->n[a] >= 1 && G->n[a] <= kMaxDim, LM_EINVAL, "image size n[%d]=%d outside 1..%d", a,
               G->n[a], kMaxDim);
    LM_REQUIRE(G->h[a] > 0.0 && std::isfinite(G->h[a]), LM_EINVAL, "voxel size h[%d] must be > 0", a);
  }
  LM_REQUIRE(G->n_tof >= 1 && (G->n_tof % 2) == 1 && G->n_tof < 32767, LM_EINVAL,
             "n_tof must be odd and positive");
  if (G->tof_on) {
    LM_REQUIRE(G->tof_bin > 0.0 && G->tof_fwhm > 0.0 && G->tof_nsigma > 0.0, LM_EINVAL,
               "TOF bin, FWHM and truncation must be positive");
  }
  o->det = G->det;
  o->n_cry = G->n_cry;
  o->n_ring = G->n_ring;
  o->n_det = G->n_cry * G->n_ring;
  for (int a = 0; a < 3; ++a) {
    o->n[a] = G->n[a];
    o->h[a] = G->h[a];
    o->c0[a] = -0.5 * (G->n[a] - 1) * G->h[a];
  }
  o->lay = lmh::row_major(G->n);
  o->n_tof = G->n_tof;
  o->kmax = (G->n_tof - 1) / 2;
  o->tof_on = G->tof_on ? 1 : 0;
  const double sigma = G->tof_fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
  o->tof_bin = G->tof_bin;
  o->inv_sr2 = G->tof_on ? 1.0 / (sigma * std::sqrt(2.0)) : 0.0;
  o->half_win = G->tof_on ? G->tof_nsigma * sigma + 0.5 * G->tof_bin : 0.0;
  o->vclip = (float)(G->tof_nsigma / std::sqrt(2.0));
  o->inv_norm = (float)(1.0 / (2.0 * std::erf(G->tof_nsigma / std::sqrt(2.0))));
  return LM_OK;
}

int max_planes(const lmk::GeomDev &g, int mode) {
  const int nmax = std::max(g.n[0], std::max(g.n[1], g.n[2]));
  if (!g.tof_on || mode == lmk::W_SUM) return nmax;
  const double hmin = std::min(g.h[0], std::min(g.h[1], g.h[2]));
  // the LOR advances at least h_a along t per plane; +3 covers the margins
  const long long b = (long long)std::ceil(2.0 * g.half_win / hmin) + 3;
  return (int)std::min<long long>(b, nmax);
}


}  // namespace lmh

// --------------------------------------------------------------------------
// launchers

namespace lmk {

template <class Src>
static int fwd_impl(const GeomDev &g, const float *x, Src src, long long n, float *out, hipStream_t st,
                    const int *skip = nullptr) {
  if (n == 0) return LM_OK;
  for (long long o = 0; o < n; o += kFwdLaunch) {
    const long long m = std::min(kFwdLaunch, n - o);
    unsigned nb = blocks_for(m, 1);
    if (Src::kXcdOrder) nb = (nb + 7) / 8 * 8;
    // sorted sources write out[order[e]]: out is the whole list's
    hipLaunchKernelGGL((k_fwd<Src>), dim3(nb), dim3(kBlock), 0, st, g, skip, x, src.offset(o), m,
                       Src::kXcdOrder ? out : out + o);
    LM_TRY_HIP(hipGetLastError());
  }
  return LM_OK;
}

// Grid of the grid-stride scattering kernels: enough wavefronts to fill the
// chip many times over, few enough that a launch whose work went to another
// path costs next to nothing.
constexpr long long kStrideBlocks = 1LL << 16;

template <class Src>
static int back_impl(const GeomDev &g, const int *skip, const float *v, Src src, long long n, float *img,
                     hipStream_t st) {
  if (n == 0) return LM_OK;
  const long long nb = std::min<long long>(kStrideBlocks, blocks_for(n, 64));
  hipLaunchKernelGGL((k_back<Src>), dim3((unsigned)nb), dim3(kBlock), 0, st, g, skip, v, src, n, img);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

// A device flag (one int), allocated and freed stream-ordered.
struct DevFlag {
  int *p = nullptr;
  hipStream_t st = nullptr;
  int alloc(hipStream_t s) {
    st = s;
    const hipError_t e = hipMallocAsync((void **)&p, sizeof(int), s);
    if (e != hipSuccess) {
      p = nullptr;
      lmh::set_error("flag temporary: %s", hipGetErrorString(e));
      return LM_ENOMEM;
    }
    return LM_OK;
  }
  ~DevFlag() {
    if (p) (void)hipFreeAsync(p, st);  // a release error has no caller to go to
  }
};

int launch_fwd(const GeomDev &g, const float *x, const int16_t *ev, long long n, float *out, hipStream_t st) {
  return fwd_impl(g, x, CallerEvents{ev}, n, out, st);
}
int launch_back(const GeomDev &g, const float *v, const int16_t *ev, long long n, float *img, hipStream_t st) {
  if (n == 0) return LM_OK;
  DevFlag cyl;
  bool queued = false;
  if (lines_possible(g)) {
    if (int rc = cyl.alloc(st)) return rc;
    if (int rc = launch_cylindrical(g, cyl.p, st)) return rc;
    if (int rc = launch_back_lines(g, cyl.p, v, ev, n, img, st, queued)) return rc;
  }
  // the per-event kernel takes the list when the line path was not queued,
  // or was queued on a scanner that is not cylindrical
  return back_impl(g, queued ? cyl.p : nullptr, v, CallerEvents{ev}, n, img, st);
}
int launch_fwd_rec(const GeomDev &g, const float *x, const int4 *rec, long long n, float *out, hipStream_t st) {
  return fwd_impl(g, x, PlanEvents{rec}, n, out, st);
}
int launch_back_rec(const GeomDev &g, const float *v, const int4 *rec, long long n, float *img, hipStream_t st) {
  return back_impl(g, nullptr, v, PlanEvents{rec}, n, img, st);
}

int launch_sens(const GeomDev &g, float *img, hipStream_t st) {
  const long long nd = g.n_det;
  const long long npairs = nd * (nd - 1) / 2;
  const long long nb = std::min<long long>(kStrideBlocks, blocks_for(npairs, 64));
  if (!lines_possible(g)) {
    hipLaunchKernelGGL(k_sens, dim3((unsigned)nb), dim3(kBlock), 0, st, g, nullptr, npairs, img);
    LM_TRY_HIP(hipGetLastError());
    return LM_OK;
  }
  DevFlag cyl;
  if (int rc = cyl.alloc(st)) return rc;
  if (int rc = launch_cylindrical(g, cyl.p, st)) return rc;
  if (int rc = launch_sens_lines(g, cyl.p, img, st)) return rc;
  hipLaunchKernelGGL(k_sens, dim3((unsigned)nb), dim3(kBlock), 0, st, g, cyl.p, npairs, img);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_data_update(const GeomDev &g, const float *x, const int4 *rec, const float *S, const float *mu,
                       float *cdual, float *dz, long long n, hipStream_t st) {
  if (n == 0) return LM_OK;
  // the lanes of an event start up to kMaxBrickOffset planes before its
  // first plane
  const int planes = lmh::max_planes(g, W_BIN) + kMaxBrickOffset;
  const int jneed = (planes + 63) / 64;
#define LM_DU(J_)                                                                                       \
  if (jneed <= J_) {                                                                                    \
    for (long long o = 0; o < n; o += chunk_items(64)) {                                                \
      const long long m = std::min(chunk_items(64), n - o);                                             \
      hipLaunchKernelGGL((k_data_update<J_>), dim3(blocks_for(m, 64)), dim3(kBlock), 0, st, g, x, rec + o, \
                         S + o, mu + o, cdual + o, dz, m);                                              \
      LM_TRY_HIP(hipGetLastError());                                                                    \
    }                                                                                                   \
    return LM_OK;                                                                                       \
  }
  LM_DU(1) LM_DU(2) LM_DU(3) LM_DU(4) LM_DU(6) LM_DU(9)
#undef LM_DU
  lmh::set_error("no update kernel for %d planes per event", planes);
  return LM_EINVAL;
}

}  // namespace lmk

// --------------------------------------------------------------------------
// Scratch of lm_fwd_noalloc: the bricked copy of the caller's image lives in
// a file-scope device array (64 MiB on every device the library runs on,
// held until the process ends) instead of a stream-ordered allocation.  In
// host code `scratch` names a host-side stand-in, not device memory: kernels
// get the address that hipGetSymbolAddress returns for the device.

constexpr long long kNoAllocScratchFloats = 1LL << 24;
static __device__ __align__(256) float scratch[kNoAllocScratchFloats];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (which must be the
// device of `st`), looked up once per device with that device current.
int noalloc_scratch(hipStream_t st, float **out) {
  int dev = -1;
  LM_TRY_HIP(hipGetDevice(&dev));
  LM_REQUIRE(dev >= 0 && dev < kMaxDevices, LM_EINVAL, "device %d beyond the %d the library serves", dev,
             kMaxDevices);
  if (st != nullptr) {
    hipDevice_t sdev = -1;
    LM_TRY_HIP(hipStreamGetDevice(st, &sdev));
    LM_REQUIRE(sdev == dev, LM_EINVAL, "stream of device %d, but device %d is current", (int)sdev, dev);
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *ptr = nullptr;
    LM_TRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<float *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return LM_OK;
}

}  // namespace

// --------------------------------------------------------------------------
// C ABI

extern "C" {

int lm_fwd(const lm_geom *G, const float *x, const int16_t *ev, int64_t n, float *out, void *stream) {
  lmh::clear_error();
  GeomDev g;
  if (int rc = lmh::make_geom(G, &g)) return rc;
  LM_REQUIRE(n >= 0, LM_EINVAL, "negative event count");
  LM_REQUIRE(n == 0 || (x && ev && out), LM_EINVAL, "NULL array");
  if (n == 0) return LM_OK;
  hipStream_t st = lmh::as_stream(stream);
  lmh::BrickImage b;
  if (int rc = b.alloc(g, st)) return rc;
  if (int rc = lmk::launch_to_layout(g.n, g.lay, 1, x, b.p, st)) return rc;
  // a long list is sorted by transaxial crystal pair and projected line by
  // line on a cylindrical scanner, else per event in the sorted order (so
  // that the events of a line share cache lines)
  unsigned *order = nullptr, *off = nullptr;
  if (int rc = lmk::sort_events_by_line(g, ev, n, &order, &off, st)) return rc;
  if (!order) return launch_fwd(g, b.p, ev, n, out, st);
  int rc = LM_OK;
  {
    DevFlag cyl;
    bool queued = false;
    if (lines_possible(g)) {
      rc = cyl.alloc(st);
      if (rc == LM_OK) rc = launch_cylindrical(g, cyl.p, st);
      if (rc == LM_OK) rc = launch_fwd_lines(g, cyl.p, b.p, ev, order, off, n, out, st, queued);
    }
    if (rc == LM_OK) rc = fwd_impl(g, b.p, SortedEvents{ev, order}, n, out, st, queued ? cyl.p : nullptr);
  }
  (void)hipFreeAsync(order, st);  // release errors have no caller to go to
  (void)hipFreeAsync(off, st);
  return rc;
}

int lm_fwd_noalloc(const lm_geom *G, const float *x, const int16_t *ev, int64_t n, float *out, void *stream) {
  lmh::clear_error();
  GeomDev g;
  if (int rc = lmh::make_geom(G, &g)) return rc;
  LM_REQUIRE(n >= 0, LM_EINVAL, "negative event count");
  LM_REQUIRE(n == 0 || (x && ev && out), LM_EINVAL, "NULL array");
  g.lay = lmh::brick_layout(g.n);
  const long long need = layout_size(g.lay);
  LM_REQUIRE(need <= kNoAllocScratchFloats, LM_EINVAL,
             "the image takes %lld floats in brick layout, beyond the %lld of lm_fwd_noalloc's scratch", need,
             kNoAllocScratchFloats);
  if (n == 0) return LM_OK;
  hipStream_t st = lmh::as_stream(stream);
  float *scr = nullptr;
  if (int rc = noalloc_scratch(st, &scr)) return rc;
  if (int rc = lmk::launch_to_layout(g.n, g.lay, 1, x, scr, st)) return rc;
  return launch_fwd(g, scr, ev, n, out, st);
}

int lm_back(const lm_geom *G, const float *v, const int16_t *ev, int64_t n, float *img, void *stream) {
  lmh::clear_error();
  GeomDev g;
  if (int rc = lmh::make_geom(G, &g)) return rc;
  LM_REQUIRE(n >= 0, LM_EINVAL, "negative event count");
  LM_REQUIRE(n == 0 || (v && ev && img), LM_EINVAL, "NULL array");
  if (n == 0) return LM_OK;
  hipStream_t st = lmh::as_stream(stream);
  lmh::BrickImage b;
  if (int rc = b.alloc(g, st)) return rc;
  if (int rc = lmk::launch_to_layout(g.n, g.lay, 1, img, b.p, st)) return rc;
  if (int rc = launch_back(g, v, ev, n, b.p, st)) return rc;
  return lmk::launch_from_layout(g.n, g.lay, 1, b.p, img, st);
}

int lm_sens(const lm_geom *G, float *img, void *stream) {
  lmh::clear_error();
  GeomDev g;
  if (int rc = lmh::make_geom(G, &g)) return rc;
  LM_REQUIRE(img != nullptr, LM_EINVAL, "NULL image");
  hipStream_t st = lmh::as_stream(stream);
  lmh::BrickImage b;
  if (int rc = b.alloc(g, st)) return rc;
  if (int rc = lmk::launch_to_layout(g.n, g.lay, 1, img, b.p, st)) return rc;
  if (int rc = launch_sens(g, b.p, st)) return rc;
  return lmk::launch_from_layout(g.n, g.lay, 1, b.p, img, st);
}

int lm_validate_events(const lm_geom *G, const int16_t *ev, int64_t n, int64_t *n_bad, void *stream) {
  lmh::clear_error();
  GeomDev g;
  if (int rc = lmh::make_geom(G, &g)) return rc;
  LM_REQUIRE(n >= 0 && n_bad != nullptr, LM_EINVAL, "bad arguments");
  *n_bad = 0;
  if (n == 0) return LM_OK;
  LM_REQUIRE(ev != nullptr, LM_EINVAL, "NULL events");
  hipStream_t st = lmh::as_stream(stream);
  unsigned long long *d = nullptr;
  LM_TRY_HIP(hipMallocAsync((void **)&d, sizeof(unsigned long long), st));
  hipError_t e = hipMemsetAsync(d, 0, sizeof(unsigned long long), st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_validate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, ev, (long long)n, d);
    e = hipGetLastError();
  }
  unsigned long long h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFreeAsync(d, st);
  LM_TRY_HIP(e);
  *n_bad = (int64_t)h;
  return LM_OK;
}

}  // extern "C"
