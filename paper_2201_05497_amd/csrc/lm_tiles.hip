// The data update of LM-SPDHG (Algorithm 2, data-subset branch: forward
// projection, dual prox of Eq. proxD, back projection of the dual
// increments, z / zbar step) by image tile, for 3D plans.
//
// The per-event kernel (k_data_update) adds each event's back projection
// into dz with FP32 atomics.  On gfx950 those atomics are executed beyond
// the L2 at about 2e10 requests/s, one request per 64-byte sector that the
// lanes of an instruction share: ~47 requests per event, most of a data
// update's time.  Here the subsets are fixed when the plan is created, so
// the back projection of every subset is binned once by 8x8x8-voxel tile
// (2x2x2 bricks): a "segment" is an event whose samples reach a tile, the
// tile of its samples on 8 consecutive planes along its dominant axis.  An
// update then runs in two kernels:
//
//   phase 1, per event (8 lanes per event, as the forward projector):
//     q = (P x)_e + s_e, the dual prox, c = 1 - y updated, and one
//     record per segment of the event (the in-plane coordinates of its
//     samples relative to the tile's first plane; for each of the tile's 8
//     planes the sample's value cf w_j with cf = L dy / mu, the tile-local
//     index of its first corner and which corners fall in the tile; 64
//     bytes, one memory sector), the records of an event in a row;
//   phase 2, one workgroup per tile: every wavefront takes the tile's
//     records two at a time through the tile's list of record numbers
//     (lanes = 8 planes x 4 bilinear corners per record; the list entries
//     two steps ahead and the records one step ahead are loaded while the
//     current ones are added)
//     into its own LDS copies of the tile with plain read-add-writes (the
//     32 lanes of a record touch distinct voxels); the copies are summed and
//     the tile's voxels, loaded at the start, take the z / zbar step and the
//     fused primal step of the next update.  No global atomics, and dz never
//     goes to memory.
//
// The per-sample arithmetic (bilinear weights, TOF weights, their
// products) is that of the per-event kernels; the back projection takes a
// sample's in-plane coordinate as G + p V from the tile's first plane
// instead of F + j V from the ray's, which can differ by a rounding (1e-7
// of a voxel), so results differ from the per-event kernels by that and by
// the order of the float32 additions.  Where the two place a coordinate on
// opposite sides of a voxel boundary, the corner that changes has a
// weight of that size, and the tile list (built from F + j V) may lack its
// tile: such a corner is dropped.
// Tiles are launched hottest first (most segments over all subsets), so
// the long ones do not trail at the end of a launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "lm_device.hpp"
#include "lm_host.hpp"
#include "lm_tiles.hpp"

using namespace lmk;

static_assert(sizeof(TileRec) == 64, "a record is one 64-byte memory sector");

namespace {

constexpr int kTE = 8;                 // tile edge, voxels
constexpr int kTV = kTE * kTE * kTE;   // voxels per tile
constexpr int kWaves2 = 4;             // wavefronts per phase-2 workgroup
constexpr int kBlock2 = 64 * kWaves2;
constexpr int kVoxPerThread = kTV / kBlock2;  // voxels of the tile per phase-2 thread
static_assert(kBlock2 <= kTV && kTV % kBlock2 == 0, "phase-2 threads cover the tile's voxels evenly");
constexpr int kLanes1 = 8;             // lanes per event in phase 1
constexpr int kBlock1 = 256;
constexpr int kMaxJ8 = 16;             // phase 1 caches up to 16 samples per lane
// The tile path runs when the largest subset has at least this many events
// per tile: a workgroup's fixed cost (its LDS copies, the latency of its
// first records and of its voxels) must be shared by enough segments.  On
// the 200x200x96 image (7500 tiles) with 4.5e4 events per subset (6 per
// tile) a data update takes 81 us by tile (45 us phase 1, 35 us phase 2)
// against 137 us per event (118 us, then 19 us for the z / zbar pass).
// Phase 2 runs workgroups of 4 wavefronts (8 LDS copies of the tile, 16
// KB; each thread owns two of the tile's voxels): a wavefront's fixed work
// (clearing its share of the copies, loading and finishing its voxels) is
// shared by about 20 records on that image.  With 8 wavefronts phase 2
// took 43.9 us per update, with 4 35.8 us, with 2 44.1 us.
constexpr long long kMinEventsPerTile = 4;

// Calls f(tile) for every tile that a corner of a sample of ray r on planes
// [8 ta, 8 ta + 7] can reach, for every ta the ray visits.  The coordinate
// of a sample, fmaf(j, V, F), is monotonic in j, so its range over a chunk
// of planes is that of the chunk's end samples.
template <class F>
__device__ __forceinline__ void for_each_segment(const Ray &r, const TileGeom &tg, F f) {
  if (r.nplanes <= 0) return;
  const int a = r.a;
  const int last = r.m0 + r.nplanes - 1;
  for (int ta = r.m0 / kTE; ta <= last / kTE; ++ta) {
    const int jlo = max(0, ta * kTE - r.m0), jhi = min(r.nplanes - 1, ta * kTE + kTE - 1 - r.m0);
    const float u1a = fmaf((float)jlo, r.V1, r.F1), u1b = fmaf((float)jhi, r.V1, r.F1);
    const float u2a = fmaf((float)jlo, r.V2, r.F2), u2b = fmaf((float)jhi, r.V2, r.F2);
    const int f1a = r.I1 + (int)floorf(u1a), f1b = r.I1 + (int)floorf(u1b);
    const int f2a = r.I2 + (int)floorf(u2a), f2b = r.I2 + (int)floorf(u2b);
    const int lo1 = max(min(f1a, f1b), 0), hi1 = min(max(f1a, f1b) + 1, r.n1 - 1);
    const int lo2 = max(min(f2a, f2b), 0), hi2 = min(max(f2a, f2b) + 1, r.n2 - 1);
    if (lo1 > hi1 || lo2 > hi2) continue;
    for (int t1 = lo1 / kTE; t1 <= hi1 / kTE; ++t1)
      for (int t2 = lo2 / kTE; t2 <= hi2 / kTE; ++t2) {
        const int tx = a == 0 ? ta : t1;
        const int ty = a == 0 ? t1 : (a == 1 ? ta : t2);
        const int tz = a == 2 ? ta : t2;
        f((tz * tg.nty + ty) * tg.ntx + tx);
      }
  }
}

// The subset stored at position e: the last i with sub[i] <= e (sub: the
// nsub + 1 first positions of the subsets, non-decreasing, sub[nsub] = n).
__device__ __forceinline__ int subset_at(const long long *sub, int nsub, long long e) {
  int lo = 0, hi = nsub - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sub[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Segments of every stored event, all subsets in one launch: per (subset,
// tile) and per event.
__global__ __launch_bounds__(256) void k_tile_count(GeomDev g, TileGeom tg, int maxp, const int4 *rec, long long e0,
                                                    long long n, const long long *sub, int nsub, unsigned *cnt,
                                                    unsigned *ecnt) {
  const long long e = e0 + (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  unsigned *c = cnt + (long long)subset_at(sub, nsub, e) * tg.ntiles;
  const int4 rc = rec[e];
  const Ray r = setup_ray(g, rc.x, rc.y, rc.z, W_BIN, maxp);
  unsigned q = 0;
  for_each_segment(r, tg, [&](int t) {
    atomicAdd(c + t, 1u);
    ++q;
  });
  ecnt[e] = q;
}

// Lists, per (subset, tile), the records of the subset's segments that fall
// in the tile (rank from an atomic counter: the order inside a tile is not
// fixed).  Records are numbered in event order from the subset's first
// event: event e's q-th segment is record eoff[e] - eoff[sub[i]] + q.
__global__ __launch_bounds__(256) void k_tile_place(GeomDev g, TileGeom tg, int maxp, const int4 *rec, long long e0,
                                                    long long n, const long long *sub, int nsub, const long long *off,
                                                    unsigned *fill, const unsigned long long *eoff, unsigned *seg) {
  const long long e = e0 + (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const int i = subset_at(sub, nsub, e);
  const long long *o = off + (long long)i * tg.ntiles;
  unsigned *f = fill + (long long)i * tg.ntiles;
  const int4 rc = rec[e];
  const Ray r = setup_ray(g, rc.x, rc.y, rc.z, W_BIN, maxp);
  unsigned q = (unsigned)(eoff[e] - eoff[sub[i]]);
  for_each_segment(r, tg, [&](int t) { seg[o[t] + atomicAdd(f + t, 1u)] = q++; });
}

// Exclusive prefix sum of cnt[0 .. n) into off[0 .. n] (64-bit); one block
// of 1024 threads, each summing a contiguous segment.
__global__ __launch_bounds__(1024) void k_scan64(const unsigned *cnt, long long n, long long *off) {
  __shared__ long long part[1024];
  const int t = threadIdx.x;
  const long long seg = (n + 1023) / 1024;
  const long long a = min(n, t * seg), b = min(n, a + seg);
  long long sum = 0;
  for (long long i = a; i < b; ++i) sum += cnt[i];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const long long add = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  long long run = part[t] - sum;
  for (long long i = a; i < b; ++i) {
    off[i] = run;
    run += cnt[i];
  }
  if (t == 1023) off[n] = part[1023];
}

// Exclusive prefix sum of a long list in three launches: sums of blocks of
// kScanB entries, their prefix (k_scan64), then the prefix inside each block.
constexpr int kScanB = 1024;

__global__ __launch_bounds__(kScanB) void k_block_sums(const unsigned *in, long long n, unsigned *bsum) {
  __shared__ unsigned red[kScanB];
  const long long i = (long long)blockIdx.x * kScanB + threadIdx.x;
  red[threadIdx.x] = i < n ? in[i] : 0u;
  __syncthreads();
  for (int o = kScanB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kScanB) void k_block_scan(const unsigned *in, long long n, const long long *boff,
                                                       unsigned long long *out) {
  __shared__ unsigned long long s[kScanB];
  const int t = threadIdx.x;
  const long long i = (long long)blockIdx.x * kScanB + t;
  const unsigned v = i < n ? in[i] : 0u;
  s[t] = v;
  __syncthreads();
  for (int o = 1; o < kScanB; o <<= 1) {  // inclusive scan
    const unsigned long long add = t >= o ? s[t - o] : 0ull;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  if (i < n) out[i] = (unsigned long long)boff[blockIdx.x] + s[t] - v;
  if (i == n - 1) out[n] = (unsigned long long)boff[blockIdx.x] + s[t];
}

// A ray of phase 1 as the lanes of its event's group read it from LDS.
struct TileRay {
  int4 p;    // {m0, nplanes, a, I1}
  int4 q;    // {I2, F1, V1, F2} (floats as bits)
  float4 r;  // {V2, A, B, L}
};

// Phase 1: per event (8 lanes), the forward projection, the dual prox (the
// cancellation-free form of k_data_update), and the event's segment
// records.  Lane l takes the planes m = 8 c + l of the 8-plane chunks c the
// ray visits, so the values of a chunk's 8 planes sit in the 8 lanes.
// The double-precision set-up of the block's 32 rays runs once per ray, in
// the first wavefront (one ray per lane), instead of in every lane of each
// group; the other wavefronts wait for it at the barrier.  With TAB the
// TOF weights come from the geometry's table (copied to LDS), otherwise
// from erfc.
template <int J8, bool TAB>
__global__ __launch_bounds__(kBlock1) void k_tile_fwd(GeomDev g, TileGeom tg, int maxp, const float *__restrict__ x,
                                                      const int4 *__restrict__ rec, const float *__restrict__ S,
                                                      const float *__restrict__ mu, float *__restrict__ cdual,
                                                      long long n, const unsigned long long *__restrict__ eoff,
                                                      TileRec *__restrict__ out, TofTab tt,
                                                      const float4 *__restrict__ tab) {
  constexpr int kEv = kBlock1 / kLanes1;  // events per block
  __shared__ TileRay rays[kEv];
  extern __shared__ float4 stab[];  // TAB: tof_tab_size(tt) intervals (dynamic LDS)
  const long long e_first = (long long)blockIdx.x * kEv;
  if (threadIdx.x < kEv) {
    const long long e = e_first + threadIdx.x;
    Ray r{};
    if (e < n) {
      const int4 rc = rec[e];
      r = setup_ray(g, rc.x, rc.y, rc.z, W_BIN, maxp);
    }
    TileRay t;
    t.p = make_int4(r.m0, r.nplanes, r.a, r.I1);
    t.q = make_int4(r.I2, __float_as_int(r.F1), __float_as_int(r.V1), __float_as_int(r.F2));
    t.r = make_float4(r.V2, r.A, r.B, r.L);
    rays[threadIdx.x] = t;
  }
  if constexpr (TAB) {
    const int nt = tof_tab_size(tt);
    for (int i = threadIdx.x; i < nt; i += kBlock1) stab[i] = tab[i];
  }
  __syncthreads();
  const int lane = threadIdx.x % kLanes1;
  const long long e = e_first + threadIdx.x / kLanes1;
  if (e >= n) return;
  Ray r{};
  {
    const TileRay t = rays[threadIdx.x / kLanes1];
    r.m0 = t.p.x;
    r.nplanes = t.p.y;
    r.a = t.p.z;
    r.I1 = t.p.w;
    r.I2 = t.q.x;
    r.F1 = __int_as_float(t.q.y);
    r.V1 = __int_as_float(t.q.z);
    r.F2 = __int_as_float(t.q.w);
    r.V2 = t.r.x;
    r.A = t.r.y;
    r.B = t.r.z;
    r.L = t.r.w;
  }
  const int b1 = (r.a == 0) ? 1 : 0, b2 = (r.a == 2) ? 1 : 2;
  r.n1 = sel3(b1, g.n[0], g.n[1], g.n[2]);
  r.n2 = sel3(b2, g.n[0], g.n[1], g.n[2]);
  const float Se = S[e];
  const float s_e = __int_as_float(rec[e].w);
  const int off8 = r.m0 & (kTE - 1);
  float wj[J8];
  float acc = 0.0f;
  {
    const AxisTerm ta = axis_term(g.lay, r.a), t1 = axis_term(g.lay, b1), t2 = axis_term(g.lay, b2);
    const TofTab tu = tof_tab_uniform(tt);
    const float D = tof_bin_width(g);
    // plane term of the lane's first plane m0 - off8 + lane, advanced by a
    // chunk of 8 planes (two bricks) per step
    int fa = axis_index(ta, r.m0 - off8 + lane);
    const int fa_step = (kTE >> ta.s) * ta.bs;
    // one sample's loads at a time: issuing every sample's gathers first
    // (40 loads in flight, 99 VGPRs) lowered the occupancy and made the
    // kernel slower (48.3 against 45.1 us per C2 update)
#pragma unroll
    for (int jj = 0; jj < J8; ++jj, fa += fa_step) {
      const int j = lane + jj * kLanes1 - off8;
      wj[jj] = 0.0f;
      if (Se != 0.0f && j >= 0 && j < r.nplanes) {
        const float u1 = fmaf((float)j, r.V1, r.F1), u2 = fmaf((float)j, r.V2, r.F2);
        const float fl1 = floorf(u1), fl2 = floorf(u2);
        // the loads first: the TOF weight's arithmetic runs while they are
        // in flight; corners outside the image read as zero, the same
        // values as gather()
        const float v = gather_terms(x, t1, t2, r.n1, r.n2, fa, r.I1 + (int)fl1, r.I2 + (int)fl2, u1 - fl1,
                                     u2 - fl2);
        float w = 1.0f;
        if (g.tof_on) {
          const float vh = fmaf(-(float)j, r.B, r.A);
          if constexpr (TAB) w = tof_weight_tab(tu, stab, vh);
          else w = tof_weight(vh, vh - D, g.vclip, g.inv_norm);
        }
        wj[jj] = w;
        acc = fmaf(w, v, acc);
      }
    }
  }
  acc = group_sum<kLanes1>(acc);
  float cf = 0.0f;
  if (Se != 0.0f) {  // LOR misses the image: the prox leaves y unchanged
    const float q = fmaf(r.L, acc, s_e);
    const float c = cdual[e], me = mu[e];
    const float sq = Se * q;
    const float t = sq - c;
    const float rt = sqrtf(fmaf(t, t, 4.0f * Se * me));
    const float dy = 2.0f * Se * fmaf(q, c, -me) / (sq + c + rt);
    if (lane == 0) cdual[e] = c - dy;
    if (dy != 0.0f) cf = r.L * (dy / me);
  }
  if (r.nplanes <= 0) return;
  // the records, in the order of for_each_segment; lane p writes the entry
  // of plane p of each
  TileRec *o = out + (eoff[e] - eoff[0]);  // the event's records, in a row
  const int last = r.m0 + r.nplanes - 1;
  // strides of the two other axes and of the dominant one in a tile's
  // row-major index
  const int d1 = r.a == 0 ? kTE : 1, d2 = r.a == 2 ? kTE : kTE * kTE;
  const int dm = r.a == 0 ? 1 : (r.a == 1 ? kTE : kTE * kTE);
#pragma unroll
  for (int jj = 0; jj < J8; ++jj) {
    const int ta = r.m0 / kTE + jj;
    if (ta > last / kTE) break;
    const int jlo = max(0, ta * kTE - r.m0), jhi = min(r.nplanes - 1, ta * kTE + kTE - 1 - r.m0);
    const float u1a = fmaf((float)jlo, r.V1, r.F1), u1b = fmaf((float)jhi, r.V1, r.F1);
    const float u2a = fmaf((float)jlo, r.V2, r.F2), u2b = fmaf((float)jhi, r.V2, r.F2);
    const int f1a = r.I1 + (int)floorf(u1a), f1b = r.I1 + (int)floorf(u1b);
    const int f2a = r.I2 + (int)floorf(u2a), f2b = r.I2 + (int)floorf(u2b);
    const int lo1 = max(min(f1a, f1b), 0), hi1 = min(max(f1a, f1b) + 1, r.n1 - 1);
    const int lo2 = max(min(f2a, f2b), 0), hi2 = min(max(f2a, f2b) + 1, r.n2 - 1);
    if (lo1 > hi1 || lo2 > hi2) continue;
    // the chunk's coordinates relative to its first plane (ray coordinates
    // at plane ta * 8, before adding I1, I2), and this lane's sample on
    // plane ta * 8 + lane as phase 2 will compute it (j outside [0,
    // nplanes) has wj = 0 and adds nothing)
    const float jb = (float)(ta * kTE - r.m0);
    const float G1 = fmaf(jb, r.V1, r.F1), G2 = fmaf(jb, r.V2, r.F2);
    const float v = (wj[jj] != 0.0f) ? cf * wj[jj] : 0.0f;
    const float u1 = fmaf((float)lane, r.V1, G1), u2 = fmaf((float)lane, r.V2, G2);
    const int c1 = r.I1 + (int)floorf(u1), c2 = r.I2 + (int)floorf(u2);
    // corners 0 and +1 along each other axis inside the image
    const int in1 = (c1 >= 0 && c1 < r.n1 ? 1 : 0) | (c1 + 1 >= 0 && c1 + 1 < r.n1 ? 2 : 0);
    const int in2 = (c2 >= 0 && c2 < r.n2 ? 1 : 0) | (c2 + 1 >= 0 && c2 + 1 < r.n2 ? 2 : 0);
    for (int t1 = lo1 / kTE; t1 <= hi1 / kTE; ++t1)
      for (int t2 = lo2 / kTE; t2 <= hi2 / kTE; ++t2, ++o) {
        const int l1 = c1 - t1 * kTE, l2 = c2 - t2 * kTE;
        // ... and inside the tile
        const int m1 = in1 & (((unsigned)l1 < (unsigned)kTE ? 1 : 0) | ((unsigned)(l1 + 1) < (unsigned)kTE ? 2 : 0));
        const int m2 = in2 & (((unsigned)l2 < (unsigned)kTE ? 1 : 0) | ((unsigned)(l2 + 1) < (unsigned)kTE ? 2 : 0));
        // bit b1 + 2 b2 set when corner (b1, b2) is inside
        int mask = ((m1 & 1) ? 1 : 0) | ((m1 & 2) ? 2 : 0);
        mask = ((m2 & 1) ? mask : 0) | ((m2 & 2) ? mask << 2 : 0);
        if (v == 0.0f) mask = 0;
        // corner 0 at (lane, l1, l2) along (a, axis 1, axis 2): with a corner
        // inside, l1 and l2 are in [-1, 7], the index in [-72, 511]
        const int at0 = lane * dm + l1 * d1 + l2 * d2;
        if (lane == 0) o->h = make_float4(G1, r.V1, G2, r.V2);
        o->v[lane] = v;
        o->meta[lane] = mask ? (unsigned short)((at0 + 128) | (mask << 10) | (r.a << 14)) : (unsigned short)0;
      }
  }
}

struct SegLane {
  float4 h;
  float v;
  unsigned meta;
};

__device__ __forceinline__ SegLane load_seg(const TileRec *__restrict__ recs, unsigned k, int jp) {
  SegLane s;
  const TileRec *r = recs + k;
  s.h = r->h;
  s.v = r->v[jp];
  s.meta = r->meta[jp];
  return s;
}

// What a phase-2 lane needs of its bilinear corner, fixed for the kernel:
// the corner's offset from corner 0 in the tile's row-major index for each
// dominant axis a of a record (minus the bias 128 of the index stored in
// meta), the corner's weight as (b1 + s1 f1) (b2 + s2 f2), which is f or
// 1 - f along each axis, and the corner's bit of the mask in meta.
struct CornerLane {
  int off0, off1, off2;
  float s1, b1, s2, b2;
  unsigned bit;
};

__device__ __forceinline__ CornerLane corner_lane(int corner) {
  CornerLane c;
  // strides of the two other axes in the tile's index (x fastest): a = 0
  // (y, z), a = 1 (x, z), a = 2 (x, y)
  const int c1 = corner & 1, c2 = (corner >> 1) & 1;
  c.off0 = c1 * kTE + c2 * kTE * kTE - 128;
  c.off1 = c1 * 1 + c2 * kTE * kTE - 128;
  c.off2 = c1 * 1 + c2 * kTE - 128;
  c.s1 = c1 ? 1.0f : -1.0f;
  c.b1 = c1 ? 0.0f : 1.0f;
  c.s2 = c2 ? 1.0f : -1.0f;
  c.b2 = c2 ? 0.0f : 1.0f;
  c.bit = 1u << (10 + corner);
  return c;
}

// The voxel of lane (plane jp, corner) for record s: its tile-local
// row-major index (li + 8 lj + 64 lk) and value, or add = 0.  The sample's
// coordinates are computed as phase 1 computed them for its corner mask.
__device__ __forceinline__ void seg_voxel(const SegLane &s, float fjp, const CornerLane &cl, float &add, int &at) {
  const unsigned mt = s.meta;
  const unsigned a = mt >> 14;
  at = (int)(mt & 1023u) + (a == 0 ? cl.off0 : (a == 1 ? cl.off1 : cl.off2));
  const float u1 = fmaf(fjp, s.h.y, s.h.x), u2 = fmaf(fjp, s.h.w, s.h.z);
  const float f1 = u1 - floorf(u1), f2 = u2 - floorf(u2);
  const float wc = fmaf(cl.s1, f1, cl.b1) * fmaf(cl.s2, f2, cl.b2);
  add = (mt & cl.bit) ? s.v * wc : 0.0f;
}

// Phase 2: one workgroup per tile; recs are the subset's records, seg the
// record numbers of every tile, off the subset's per-tile ranges of seg.
// The LDS copies are cleared with 16-byte stores.
// Each wavefront takes records two at a time (one per half), unrolled by
// two with alternating buffers so that the next records' loads are in
// flight while the current ones are added.
__global__ __launch_bounds__(kBlock2) void k_tile_back(GeomDev g, TileGeom tg, const int *__restrict__ order,
                                                       const long long *__restrict__ off,
                                                       const unsigned *__restrict__ seg,
                                                       const TileRec *__restrict__ recs, float *__restrict__ z,
                                                       float *__restrict__ x, const float *__restrict__ T,
                                                       float *__restrict__ zbar, float *__restrict__ dz_out,
                                                       float inv_p, int fuse) {
  __shared__ __align__(16) float acc[2 * kWaves2][kTV];
  const int tile = order[blockIdx.x];
  const int tx = tile % tg.ntx, ty = (tile / tg.ntx) % tg.nty, tz = tile / (tg.ntx * tg.nty);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, half = lane >> 5, hl = lane & 31;
  const int jp = hl >> 2;
  const CornerLane cl = corner_lane(hl & 3);
  const float fjp = (float)jp;
  // the thread's voxels v = threadIdx.x + kBlock2 q of the tile (threads in
  // the plan's brick order); their image values are loaded now and used at
  // the end
  const Layout &L = g.lay;
  bool mine_vox[kVoxPerThread];
  long long gi[kVoxPerThread];
  float xv[kVoxPerThread], zv[kVoxPerThread], Tv[kVoxPerThread];
#pragma unroll
  for (int q = 0; q < kVoxPerThread; ++q) {
    const int v = threadIdx.x + kBlock2 * q;
    const int b = (v >> 6) & 7, bi = tx * 2 + (b & 1), bj = ty * 2 + ((b >> 1) & 1), bk = tz * 2 + (b >> 2);
    mine_vox[q] = bi < L.nbx && bj < L.nby && bk < L.nbz;
    gi[q] = ((((long long)bk * L.nby + bj) * L.nbx + bi) << 6) | (v & 63);
    xv[q] = zv[q] = Tv[q] = 0.0f;
    if (mine_vox[q] && !dz_out) {
      zv[q] = z[gi[q]];
      if (fuse) {
        xv[q] = x[gi[q]];
        Tv[q] = T[gi[q]];
      }
    }
  }
  float4 *all = reinterpret_cast<float4 *>(&acc[0][0]);
  for (int i = threadIdx.x; i < 2 * kWaves2 * kTV / 4; i += kBlock2) all[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  __syncthreads();
  float *mine = acc[2 * wv + half];
  const long long s0 = off[tile];
  const int cnt = (int)(off[tile + 1] - s0);
  const unsigned *tseg = seg + s0;
  constexpr int kStep = 2 * kWaves2;
  const int k0 = 2 * wv + half;
  if (cnt > 0) {
    // indices are clamped to the last record so that every load is valid;
    // records past the end are not added
    auto idx = [&](int k) { return tseg[min(k, cnt - 1)]; };
    // in issue order, an index is loaded before the records that are in
    // flight when it is needed, so waiting for it leaves them in flight
    unsigned iB = idx(k0 + kStep);
    SegLane A = load_seg(recs, idx(k0), jp);
    unsigned iC = idx(k0 + 2 * kStep);
    for (int k = k0; k - k0 < cnt; k += 2 * kStep) {
      const SegLane B = load_seg(recs, iB, jp);
      const unsigned iD = idx(k + 3 * kStep);
      float add;
      int at;
      seg_voxel(A, fjp, cl, add, at);
      // the 32 lanes of a record touch distinct voxels of their own copy; a
      // lane may read a word another lane of the wavefront wrote before,
      // which the wavefront's in-order LDS operations deliver once the
      // compiler keeps the order (the fences)
      if (k < cnt && add != 0.0f) mine[at] += add;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      A = load_seg(recs, iC, jp);
      iC = idx(k + 4 * kStep);
      seg_voxel(B, fjp, cl, add, at);
      if (k + kStep < cnt && add != 0.0f) mine[at] += add;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      iB = iD;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kVoxPerThread; ++q) {
    if (!mine_vox[q]) continue;
    // voxel v of the brick-ordered tile: row-major position in the copies
    const int v = threadIdx.x + kBlock2 * q;
    const int b = (v >> 6) & 7;
    const int lv = (b & 1) * 4 + (v & 3) + kTE * (((b >> 1) & 1) * 4 + ((v >> 2) & 3)) +
                   kTE * kTE * ((b >> 2) * 4 + ((v >> 4) & 3));
    float d = 0.0f;
#pragma unroll
    for (int c = 0; c < 2 * kWaves2; ++c) d += acc[c][lv];
    if (dz_out) {
      dz_out[gi[q]] = d;
      continue;
    }
    const float zn = zv[q] + d;
    const float zb = fmaf(d, inv_p, zn);
    z[gi[q]] = zn;
    if (fuse)
      x[gi[q]] = fmaxf(0.0f, fmaf(-Tv[q], zb, xv[q]));
    else
      zbar[gi[q]] = zb;
  }
}

inline unsigned blocks(long long n, int per) { return (unsigned)((n + per - 1) / per); }

// events per launch of the per-event set-up kernels (a dispatch covers at
// most 2^30 work-items)
constexpr long long kChunk = 1LL << 28;

}  // namespace

namespace lmk {

TileGeom tile_geom(const int n[3]) {
  TileGeom t;
  t.ntx = (n[0] + kTE - 1) / kTE;
  t.nty = (n[1] + kTE - 1) / kTE;
  t.ntz = (n[2] + kTE - 1) / kTE;
  t.ntiles = t.ntx * t.nty * t.ntz;
  return t;
}

// 3D plans (4x4x4 bricks) whose events visit few enough planes for the
// register cache of phase 1.
static int j8_for(int maxp) { return (maxp + kTE - 1 + kLanes1 - 1) / kLanes1; }

bool tiles_supported(const GeomDev &g) {
  if (g.n[2] < 2 || g.lay.sx != 2 || g.lay.sy != 2 || g.lay.sz != 2) return false;
  return j8_for(lmh::max_planes(g, W_BIN)) <= kMaxJ8;
}

size_t tile_bytes_bound(const GeomDev &g, long long n, int nsub) {
  if (!tiles_supported(g) || n <= 0) return 0;
  const TileGeom tg = tile_geom(g.n);
  if ((n + nsub - 1) / nsub < kMinEventsPerTile * tg.ntiles) return 0;
  const int maxp = lmh::max_planes(g, W_BIN);
  // tiles a chunk of 8 planes along axis a can reach along axis b: the
  // corners span at most 7 h_a / h_b + 3 voxels
  long long per_chunk = 1;
  for (int a = 0; a < 3; ++a) {
    long long m = 1;
    for (int b = 0; b < 3; ++b) {
      if (b == a) continue;
      const long long span = (long long)std::floor(7.0 * g.h[a] / g.h[b]) + 3;
      m *= (span + kTE - 2) / kTE + 1;
    }
    per_chunk = std::max(per_chunk, m);
  }
  const long long per_event = ((maxp + kTE - 2) / kTE + 1) * per_chunk;
  const long long nmax = (n + nsub - 1) / nsub;
  const long long nbin = (long long)nsub * tg.ntiles;
  const size_t kept = (size_t)(n * per_event) * sizeof(unsigned) + (size_t)(n + 1) * sizeof(unsigned long long) +
                      (size_t)(nbin + 1) * sizeof(long long) + (size_t)tg.ntiles * sizeof(int) +
                      (size_t)(nmax * per_event) * sizeof(TileRec) + (size_t)kTofTabMax * sizeof(float4);
  const size_t temporary = (size_t)nbin * sizeof(unsigned) + (size_t)n * sizeof(unsigned) +
                           (size_t)((n + kScanB - 1) / kScanB) * (sizeof(unsigned) + sizeof(long long) + 8);
  return kept + temporary;
}

int build_tiles(const GeomDev &g, const int4 *rec, const std::vector<int> &off, TilePlan &tp,
                std::vector<void *> &owned, hipStream_t st) {
  tp = TilePlan{};
  if (!tiles_supported(g)) return LM_OK;
  const int nsub = (int)off.size() - 1;
  const long long N = off.back();
  if (N == 0) return LM_OK;
  const TileGeom tg = tile_geom(g.n);
  long long nlargest = 0;
  for (int i = 0; i < nsub; ++i) nlargest = std::max<long long>(nlargest, off[i + 1] - off[i]);
  if (nlargest < kMinEventsPerTile * tg.ntiles) return LM_OK;
  const int maxp = lmh::max_planes(g, W_BIN);
  const long long nbin = (long long)nsub * tg.ntiles;
  const long long nblk = (N + kScanB - 1) / kScanB;
  // temporaries: counts per (subset, tile) and per event, block sums, the
  // subsets' first positions
  unsigned *cnt = nullptr, *ecnt = nullptr, *bsum = nullptr;
  long long *boff = nullptr, *sub = nullptr;
  // kept by the plan
  long long *soff = nullptr;
  unsigned long long *eoff = nullptr;
  unsigned *seg = nullptr;
  int *ord = nullptr;
  TileRec *recs = nullptr;
  std::vector<void *> tmp;
  auto drop = [&](bool keep_error) {
    for (void *q : tmp) (void)hipFreeAsync(q, st);
    for (void *q : {(void *)soff, (void *)eoff, (void *)seg, (void *)ord, (void *)recs})
      if (q) (void)hipFreeAsync(q, st);
    if (!keep_error) (void)hipGetLastError();
  };
  auto get = [&](auto **ptr, size_t bytes, bool temporary) {
    const hipError_t e = hipMallocAsync((void **)ptr, std::max<size_t>(bytes, 1), st);
    if (e == hipSuccess && temporary) tmp.push_back(*ptr);
    return e;
  };
  hipError_t e = get(&cnt, nbin * sizeof(unsigned), true);
  if (e == hipSuccess) e = get(&ecnt, N * sizeof(unsigned), true);
  if (e == hipSuccess) e = get(&bsum, nblk * sizeof(unsigned), true);
  if (e == hipSuccess) e = get(&boff, (nblk + 1) * sizeof(long long), true);
  if (e == hipSuccess) e = get(&sub, (nsub + 1) * sizeof(long long), true);
  if (e == hipSuccess) e = get(&soff, (nbin + 1) * sizeof(long long), false);
  if (e == hipSuccess) e = get(&eoff, (N + 1) * sizeof(unsigned long long), false);
  if (e != hipSuccess) {
    drop(false);
    return LM_OK;  // no room: the per-event path
  }
  auto fail = [&](hipError_t he) {
    drop(true);
    lmh::set_error("tile binning: %s", hipGetErrorString(he));
    return LM_EHIP;
  };
  // the host copy stays alive until the synchronisation below
  const std::vector<long long> hsub(off.begin(), off.end());
  if ((e = hipMemcpyAsync(sub, hsub.data(), (nsub + 1) * sizeof(long long), hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemsetAsync(cnt, 0, nbin * sizeof(unsigned), st)) != hipSuccess)
    return fail(e);
  for (long long e0 = 0; e0 < N; e0 += kChunk)
    hipLaunchKernelGGL(k_tile_count, dim3(blocks(std::min(kChunk, N - e0), 256)), dim3(256), 0, st, g, tg, maxp,
                       rec, e0, N, sub, nsub, cnt, ecnt);
  hipLaunchKernelGGL(k_scan64, dim3(1), dim3(1024), 0, st, cnt, nbin, soff);
  hipLaunchKernelGGL(k_block_sums, dim3((unsigned)nblk), dim3(kScanB), 0, st, ecnt, N, bsum);
  hipLaunchKernelGGL(k_scan64, dim3(1), dim3(1024), 0, st, bsum, nblk, boff);
  hipLaunchKernelGGL(k_block_scan, dim3((unsigned)nblk), dim3(kScanB), 0, st, ecnt, N, boff, eoff);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  // per-tile loads over all subsets (launch order) and the largest subset's segments
  std::vector<long long> hoff((size_t)nbin + 1);
  if ((e = hipMemcpyAsync(hoff.data(), soff, (nbin + 1) * sizeof(long long), hipMemcpyDeviceToHost, st)) !=
      hipSuccess)
    return fail(e);
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail(e);
  const long long total = hoff[nbin];
  long long rec_max = 0;
  for (int i = 0; i < nsub; ++i)
    rec_max = std::max(rec_max, hoff[(size_t)(i + 1) * tg.ntiles] - hoff[(size_t)i * tg.ntiles]);
  if (rec_max >= (1LL << 32)) {
    drop(false);
    return LM_OK;  // record numbers relative to a subset must fit 32 bits
  }
  std::vector<long long> load(tg.ntiles, 0);
  for (long long b = 0; b < nbin; ++b) load[b % tg.ntiles] += hoff[b + 1] - hoff[b];
  std::vector<int> order(tg.ntiles);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return load[a] > load[b]; });
  e = get(&seg, total * sizeof(unsigned), false);
  if (e == hipSuccess) e = get(&ord, tg.ntiles * sizeof(int), false);
  if (e == hipSuccess) e = get(&recs, rec_max * sizeof(TileRec), false);
  if (e != hipSuccess) {
    drop(false);
    return LM_OK;  // no room for the segments: the per-event path
  }
  if ((e = hipMemcpyAsync(ord, order.data(), tg.ntiles * sizeof(int), hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemsetAsync(cnt, 0, nbin * sizeof(unsigned), st)) != hipSuccess)
    return fail(e);
  for (long long e0 = 0; e0 < N; e0 += kChunk)
    hipLaunchKernelGGL(k_tile_place, dim3(blocks(std::min(kChunk, N - e0), 256)), dim3(256), 0, st, g, tg, maxp,
                       rec, e0, N, sub, nsub, soff, cnt, eoff, seg);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  // the host order vector dies with this call
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return fail(e);
  for (void *q : tmp) (void)hipFreeAsync(q, st);
  for (void *q : {(void *)soff, (void *)eoff, (void *)seg, (void *)ord, (void *)recs}) owned.push_back(q);
  // phase 1 reads the TOF weights from a table where the geometry has one
  TofTab tt{};
  float4 *tab = nullptr;
  if (int rc = build_tof_table(g, tt, &tab, st)) return rc;
  if (tab) owned.push_back(tab);
  tp.tt = tt;
  tp.tab = tab;
  tp.on = true;
  tp.tg = tg;
  tp.maxp = maxp;
  tp.nseg = total;
  tp.rec_max = rec_max;
  tp.seg_off = soff;
  tp.eoff = eoff;
  tp.seg = seg;
  tp.order = ord;
  tp.rec = recs;
  return LM_OK;
}

int launch_tile_fwd(const GeomDev &g, const TilePlan &tp, const float *x, const int4 *rec, const float *S,
                    const float *mu, float *cdual, long long o, long long n, hipStream_t st) {
  if (n == 0) return LM_OK;
  const int jneed = j8_for(tp.maxp);
  const size_t tab_lds = tp.tab ? (size_t)tof_tab_size(tp.tt) * sizeof(float4) : 0;
#define LM_TF(J_)                                                                                               \
  if (jneed <= J_) {                                                                                            \
    if (tp.tab)                                                                                                 \
      hipLaunchKernelGGL((k_tile_fwd<J_, true>), dim3(blocks(n, kBlock1 / kLanes1)), dim3(kBlock1), tab_lds, st, \
                         g,                                                                                     \
                         tp.tg, tp.maxp, x, rec + o, S + o, mu + o, cdual + o, n, tp.eoff + o, tp.rec, tp.tt,   \
                         tp.tab);                                                                               \
    else                                                                                                        \
      hipLaunchKernelGGL((k_tile_fwd<J_, false>), dim3(blocks(n, kBlock1 / kLanes1)), dim3(kBlock1), 0, st, g,  \
                         tp.tg, tp.maxp, x, rec + o, S + o, mu + o, cdual + o, n, tp.eoff + o, tp.rec, tp.tt,   \
                         tp.tab);                                                                               \
    LM_TRY_HIP(hipGetLastError());                                                                              \
    return LM_OK;                                                                                               \
  }
  LM_TF(8) LM_TF(10) LM_TF(12) LM_TF(14) LM_TF(16)
#undef LM_TF
  lmh::set_error("no tile update kernel for %d planes per event", tp.maxp);
  return LM_EINVAL;
}

int launch_tile_back(const GeomDev &g, const TilePlan &tp, int subset, float *z, float *x, const float *T,
                     float *zbar, float *dz_out, float inv_p, bool fuse, hipStream_t st) {
  const long long *off = tp.seg_off + (long long)subset * tp.tg.ntiles;
  hipLaunchKernelGGL(k_tile_back, dim3(tp.tg.ntiles), dim3(kBlock2), 0, st, g, tp.tg, tp.order, off, tp.seg, tp.rec,
                     z, x, T, zbar, dz_out, inv_p, fuse ? 1 : 0);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

}  // namespace lmk
