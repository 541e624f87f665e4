// Back projection organised by transaxial line, for cylindrical scanners
// (crystal c of ring r at (x_c, y_c, z_r)): the sensitivity image P^T 1,
// and lm_back of long event lists after a counting sort by line.
//
// Every line of response between crystals c1 != c2 of any two rings has the
// same transaxial projection, so when its dominant axis is transaxial it
// meets the image planes at the same transaxial positions: only its z
// coordinate, its length and its TOF window depend on the rings.  A
// wavefront owns one transaxial line, 64 consecutive planes (lane l: plane
// M0 + l) and a part of 16 z planes, and accumulates the contributions of
// the line's LORs into LDS columns acc[corner][z][lane] (the two transaxial
// corners of the lane's plane over the part), each lane only touching its
// own column.  The columns are added to the image once per wavefront, so
// the image sees one atomic per touched voxel and line instead of one per
// LOR and voxel.  LORs whose dominant axis is z (short transaxial chords,
// large ring differences) keep the per-LOR projector.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "lm_device.hpp"
#include "lm_host.hpp"
#include "lm_sort.hpp"

using namespace lmk;

namespace {

constexpr int kLanes = 64;

// Transaxial part of a line from crystal c1 to crystal c2 of ring 0 and the
// lane's plane on it.
struct LineLane {
  int a;            // dominant transaxial axis (0: x, 1: y)
  int nb;           // image size along the other transaxial axis
  float fdx, fdy;   // float32 transaxial differences (dominant-axis decisions)
  double dxy2;      // squared transaxial length
  double ha_over_da;  // h_a / |d_a|
  bool active;      // the lane's plane lies on the LOR (lam in [0, 1])
  int m;            // the lane's plane
  double lam;       // LOR parameter at the plane
  int i1;           // lower transaxial corner (may be -1 or nb - 1)
  float f1;         // its fractional weight
};

// Pair index p of the row-major upper triangle of an n x n matrix (c1 < c2).
__device__ __forceinline__ void pair_of(long long p, int n, int &c1, int &c2) {
  const double b = 2.0 * n - 1.0;
  long long i = (long long)floor((b - sqrt(b * b - 8.0 * (double)p)) * 0.5);
  auto first = [&](long long r) { return r * n - r * (r + 1) / 2; };
  if (i < 0) i = 0;
  while (i > 0 && first(i) > p) --i;
  while (i + 1 < n && first(i + 1) <= p) ++i;
  c1 = (int)i;
  c2 = (int)(i + 1 + (p - first(i)));
}

__device__ __forceinline__ LineLane line_lane(const GeomDev &g, int c1, int c2, int m0, int lane) {
  LineLane q;
  const float *d1 = g.det + 3 * c1, *d2 = g.det + 3 * c2;
  q.fdx = d2[0] - d1[0];
  q.fdy = d2[1] - d1[1];
  q.a = (fabsf(q.fdy) > fabsf(q.fdx)) ? 1 : 0;
  const int b = 1 - q.a;
  const double p1a = q.a ? d1[1] : d1[0], da = q.a ? (double)d2[1] - d1[1] : (double)d2[0] - d1[0];
  const double p1b = b ? d1[1] : d1[0], db = b ? (double)d2[1] - d1[1] : (double)d2[0] - d1[0];
  const double dx = (double)d2[0] - d1[0], dy = (double)d2[1] - d1[1];
  q.dxy2 = dx * dx + dy * dy;
  const double ha = g.h[q.a], c0a = g.c0[q.a], hb = g.h[b], c0b = g.c0[b];
  const int na = g.n[q.a];
  q.nb = g.n[b];
  q.ha_over_da = ha / fabs(da);
  q.m = m0 + lane;
  q.active = false;
  q.lam = 0.0;
  q.i1 = -2;
  q.f1 = 0.0f;
  if (da == 0.0 || q.m >= na) return q;
  const double lam0 = (c0a - p1a) / da, dlam = ha / da;
  const double m_at0 = -lam0 / dlam, m_at1 = (1.0 - lam0) / dlam;
  const double mlo = ceil(fmin(m_at0, m_at1)), mhi = floor(fmax(m_at0, m_at1));
  if ((double)q.m < mlo || (double)q.m > mhi) return q;
  q.lam = lam0 + q.m * dlam;
  const double u1 = (p1b + q.lam * db - c0b) / hb;
  const double fl = floor(u1);
  if (fl < -1.0 || fl > (double)q.nb - 1.0) return q;  // both corners outside
  q.i1 = (int)fl;
  q.f1 = (float)(u1 - fl);
  q.active = true;
  return q;
}

// Per-LOR coefficients of a line's LOR (rings at z1, z2; TOF centre tc and
// half-width `edge` of the weight's bin range; value v): with the lane's
// LOR parameter lam, the TOF argument is vh = A - lam B (units of
// sigma sqrt 2), vl = vh - D, and the z coordinate in voxels is az + lam bz.
struct Lor {
  double A, B, az, bz;
  float D, c;  // c = v L
};

// The z coefficients first (cheap, they decide whether the LOR touches a
// wavefront's z part), then the rest.
__device__ __forceinline__ void lor_z(const GeomDev &g, double ihz, double z1, double z2, Lor &o) {
  o.az = (z1 - g.c0[2]) * ihz;
  o.bz = (z2 - z1) * ihz;
}

__device__ __forceinline__ void lor_rest(const GeomDev &g, const LineLane &q, double z1, double z2, double tc,
                                         double edge, float v, Lor &o) {
  const double dz = z2 - z1;
  const double dn = sqrt(q.dxy2 + dz * dz);
  // t(lam) = (lam - 1/2) dn, vh = (tc + edge - t) / (sigma sqrt 2)
  o.A = (tc + edge + 0.5 * dn) * g.inv_sr2;
  o.B = dn * g.inv_sr2;
  o.D = (float)(2.0 * edge * g.inv_sr2);
  o.c = v * (float)(q.ha_over_da * dn);
}

// A wavefront's share of the columns: z in [zlo, zlo + zc), acc[cb][z - zlo][lane].
struct ZPart {
  int zlo, zc;
};

// Adds one LOR's samples at the lane's plane to the lane's column.  With a
// TOF table (single bins) the weight is read from it; otherwise wfull is the
// weight of a sample whose TOF argument covers the whole truncated Gaussian
// (vh >= vclip and vl <= -vclip), the same value tof_weight gives for it, so
// that such samples skip the two erfc evaluations.
template <bool TAB>
__device__ __forceinline__ void add_lor(const GeomDev &g, const LineLane &q, const Lor &o, const ZPart &zp,
                                        float wfull, const TofTab &tt, const float4 *tab, float *acc, int nz,
                                        int lane) {
  if (!q.active) return;
  float c = o.c;
  if (g.tof_on) {
    const float vh = (float)fma(-q.lam, o.B, o.A);
    if constexpr (TAB) {
      c *= tof_weight_tab(tt, tab, vh);
    } else {
      const float vl = vh - o.D;
      c *= (vh >= g.vclip && vl <= -g.vclip) ? wfull : tof_weight(vh, vl, g.vclip, g.inv_norm);
    }
  }
  if (c == 0.0f) return;
  const double u2 = fma(q.lam, o.bz, o.az);
  const double fl = floor(u2);
  if (fl < -1.0 || fl > (double)nz - 1.0) return;
  const int k0 = (int)fl;
  const float f2 = (float)(u2 - fl);
  // the four corners are distinct entries of the lane's own column (no
  // other lane or wavefront touches it): all reads first, then all writes,
  // so that their LDS latencies overlap
  bool ok[4];
  float *ad[4];
  float w[4], old[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int cb = t >> 1, cz = t & 1;
    const int kz = k0 + cz - zp.zlo;
    ok[t] = (unsigned)(q.i1 + cb) < (unsigned)q.nb && (unsigned)kz < (unsigned)zp.zc && k0 + cz < nz;
    ad[t] = acc + ((cb * zp.zc + (ok[t] ? kz : 0)) * kLanes + lane);
    w[t] = c * (cb ? q.f1 : 1.0f - q.f1) * (cz ? f2 : 1.0f - f2);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) old[t] = ok[t] ? *ad[t] : 0.0f;
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (ok[t]) *ad[t] = old[t] + w[t];
}

// Adds the lane's columns to the image: one atomic per non-zero voxel.
__device__ __forceinline__ void flush(const GeomDev &g, const LineLane &q, const ZPart &zp, const float *acc,
                                      float *img, int lane) {
  const Layout &L = g.lay;
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int ib = q.i1 + cb;
    const bool ok = q.active && (unsigned)ib < (unsigned)q.nb;
    const int i = q.a == 0 ? q.m : ib, j = q.a == 0 ? ib : q.m;
    const int base = ok ? vidx(L, i, j, 0) : 0;
    for (int kz = 0; kz < zp.zc; ++kz) {
      const float v = acc[(cb * zp.zc + kz) * kLanes + lane];
      if (ok && v != 0.0f) atomicAdd(img + (base + vidx(L, 0, 0, zp.zlo + kz)), v);
    }
  }
}

// Lane j's value of x (j uniform).
__device__ __forceinline__ double readlane_f64(double x, int j) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, j);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), j);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Lane j's LOR coefficients (j uniform).
__device__ __forceinline__ Lor broadcast(const Lor &o, int j) {
  Lor r;
  r.A = readlane_f64(o.A, j);
  r.B = readlane_f64(o.B, j);
  r.az = readlane_f64(o.az, j);
  r.bz = readlane_f64(o.bz, j);
  r.D = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(o.D), j));
  r.c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(o.c), j));
  return r;
}

// z extent of a part: 2 x kZPart x 64 floats (8 KB) of LDS per wavefront,
// which allows 20 wavefronts per CU.  Measured on 5e8 events: parts of 8,
// 12, 16 and 32 planes took 439, 638, 364 and 438 ms (smaller parts test
// and add each event in more blocks, larger ones leave fewer wavefronts to
// hide the latency of each event's LDS updates).
constexpr int kZPart = 16;

// Sensitivity over the LORs of every line c1 < c2 whose dominant axis is
// transaxial: all ring pairs (r1, r2), the TOF weight summed over all bins.
// Block b (one wavefront): line b / (nchunk nzp), planes 64 chunk .. + 63
// with chunk = (b / nzp) % nchunk, and z part b % nzp.  A LOR whose z range
// over the chunk's planes misses the part is skipped on uniform values.
__global__ __launch_bounds__(kLanes) void k_sens_lines(GeomDev g, const int *cyl, long long p0, long long nlines,
                                                       int nchunk, int nzp, float *img) {
  __shared__ float acc[2 * kZPart * kLanes];
  if (!*cyl) return;
  const long long blk = (long long)blockIdx.x;
  const long long per_line = (long long)nchunk * nzp;
  if (blk / per_line >= nlines) return;
  const long long p = p0 + blk / per_line;
  const int chunk = (int)((blk / nzp) % nchunk), part = (int)(blk % nzp);
  const int lane = threadIdx.x;
  const int nz = g.n[2];
  ZPart zp;
  zp.zlo = part * kZPart;
  zp.zc = min(kZPart, nz - zp.zlo);
  int c1, c2;
  pair_of(p, g.n_cry, c1, c2);
  const LineLane q = line_lane(g, c1, c2, chunk * kLanes, lane);
  const unsigned long long act = __ballot(q.active);
  if (act == 0) return;  // the chunk misses the line
  // LOR parameter at the first and last active plane of the chunk
  const int la = __ffsll((long long)act) - 1, lb = 63 - __clzll((long long)act);
  const double lam_a = __shfl(q.lam, la), lam_b = __shfl(q.lam, lb);
  for (int i = lane; i < 2 * zp.zc * kLanes; i += kLanes) acc[i] = 0.0f;
  const double edge = (g.kmax + 0.5) * g.tof_bin;  // all bins: centre 0
  const float wfull = tof_weight(g.vclip, -g.vclip, g.vclip, g.inv_norm);
  const int nr = g.n_ring;
  const double ihz = 1.0 / g.h[2];
  auto zring = [&](int r) { return g.det[3 * (g.n_cry * r) + 2]; };
  for (int r1 = 0; r1 < nr; ++r1) {
    const float z1f = zring(r1);
    // The LOR (r1, r2) can touch the part when its corners over the chunk,
    // floor(u) - 1 .. floor(u) + 2 for u between ua and ub (one voxel of
    // margin on each side for rounding between the end planes), reach
    // [zlo, zlo + zc).  With z increasing with the ring (checked on the
    // host) both bounds grow with r2, so those r2 form one interval, found
    // by bisection on the same expressions.
    auto u_ends = [&](int r2, double &umin, double &umax) {
      Lor o;
      lor_z(g, ihz, z1f, zring(r2), o);
      const double ua = fma(lam_a, o.bz, o.az), ub = fma(lam_b, o.bz, o.az);
      umin = fmin(ua, ub);
      umax = fmax(ua, ub);
    };
    auto reaches_lo = [&](int r2) {  // floor(umax) + 2 >= zlo
      double umin, umax;
      u_ends(r2, umin, umax);
      return floor(umax) + 2.0 >= (double)zp.zlo;
    };
    auto below_hi = [&](int r2) {  // floor(umin) - 1 < zlo + zc
      double umin, umax;
      u_ends(r2, umin, umax);
      return floor(umin) - 1.0 < (double)(zp.zlo + zp.zc);
    };
    int lo = 0, hi = nr;  // first r2 with reaches_lo
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (reaches_lo(mid)) hi = mid; else lo = mid + 1;
    }
    const int r2a = lo;
    lo = r2a;
    hi = nr;  // first r2 >= r2a without below_hi
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (below_hi(mid)) lo = mid + 1; else hi = mid;
    }
    const int r2b = lo;
    // 64 ring pairs at a time: lane l sets up ring pair r2 = b + l, then
    // the wavefront adds them one after the other
    for (int b = r2a; b < r2b; b += kLanes) {
      const int r2 = b + lane;
      bool pass = false;
      Lor o;
      o.A = o.B = o.az = o.bz = 0.0;
      o.D = o.c = 0.0f;
      if (r2 < r2b) {
        const float z2f = zring(r2);
        pass = dominant_axis(q.fdx, q.fdy, z2f - z1f) != 2;  // z dominant: per-LOR path
        lor_z(g, ihz, z1f, z2f, o);
        lor_rest(g, q, z1f, z2f, 0.0, edge, 1.0f, o);
      }
      unsigned long long m = __ballot(pass);
      while (m) {
        const int j = __ffsll((long long)m) - 1;
        m &= m - 1;
        add_lor<false>(g, q, broadcast(o, j), zp, wfull, TofTab{}, nullptr, acc, nz, lane);
      }
    }
  }
  flush(g, q, zp, acc, img, lane);
}

// Stage for the per-LOR scatter (one wavefront per block).
struct Stage1 {
  int idx[256];
  float val[256];
};

// Sensitivity over the LORs the line kernel leaves out: those whose
// dominant axis is z.  Block p: crystals c1 <= c2 (the pair index of the
// upper triangle with its diagonal); ring pairs (r1, r2) for c1 < c2 and
// r1 < r2 for c1 = c2.
__global__ __launch_bounds__(kLanes) void k_sens_zdom(GeomDev g, const int *cyl, long long p0, long long np,
                                                      float *img) {
  __shared__ Stage1 st;
  if (!*cyl) return;
  const long long q = (long long)blockIdx.x;
  if (q >= np) return;
  const int lane = threadIdx.x;
  int c1, c2;
  // pairs with the diagonal: index p of an (n+1) x (n+1) upper triangle
  pair_of(p0 + q, g.n_cry + 1, c1, c2);
  c2 -= 1;
  const float *d1 = g.det + 3 * c1, *d2 = g.det + 3 * c2;
  const float fdx = d2[0] - d1[0], fdy = d2[1] - d1[1];
  const int nr = g.n_ring;
  for (long long rr0 = 0; rr0 < (long long)nr * nr; rr0 += kLanes) {
    const long long rr = rr0 + lane;
    bool zdom = false;
    int r1 = 0, r2 = 0;
    if (rr < (long long)nr * nr) {
      r1 = (int)(rr / nr);
      r2 = (int)(rr % nr);
      const float z1f = g.det[3 * (g.n_cry * r1) + 2], z2f = g.det[3 * (g.n_cry * r2) + 2];
      zdom = (c1 != c2 || r1 < r2) && dominant_axis(fdx, fdy, z2f - z1f) == 2;
    }
    unsigned long long mask = __ballot(zdom);
    while (mask) {
      const int src = __ffsll((long long)mask) - 1;
      mask &= mask - 1;
      const int s1 = __shfl(r1, src), s2 = __shfl(r2, src);
      const Ray r = setup_ray(g, c1 + g.n_cry * s1, c2 + g.n_cry * s2, 0, W_SUM, 1 << 20);
      const int off = brick_offset(g.lay, r);
      for (int j0 = -off; j0 < r.nplanes; j0 += kLanes) {
        const int j = j0 + lane;
        Sample s = sample_at(g, r, j, g.tof_on);
        const float cs = (j >= 0 && j < r.nplanes) ? r.L * s.w : 0.0f;
        scatter_interleaved(g, img, r, s, cs, lane, st.idx, st.val);
      }
    }
  }
}


// ---------------------------------------------------------------------------
// Back projection of a long event list by line: the events are counted and
// placed per line (a counting sort on the GPU), then one wavefront per
// (line, chunk, z part) accumulates its line's events as the sensitivity
// kernel does its ring pairs.  Events whose dominant axis is z take the
// per-event projector.

// An event on a line in the line's orientation (crystal c1 < c2): rings and
// TOF bin packed as r1 | r2 << 12 | (k + kmax) << 24, and its value.
struct LineRec {
  unsigned rk;
  float v;
};

// Line of a caller event; kPerEvent for an event the per-event projector
// takes (a z dominant axis, which includes both ends on one transaxial
// crystal), kNoEvent for one that contributes nothing (out of range, zero
// value, the same crystal twice).  rk as in LineRec.
constexpr int kNoEvent = -1, kPerEvent = -2;

__device__ __forceinline__ int event_line(const GeomDev &g, const int16_t *e, float v, unsigned &rk) {
  int id1, id2, k;
  if (!decode_event(g, e, id1, id2, k) || v == 0.0f) return kNoEvent;
  int c1 = e[0], r1 = e[1], c2 = e[2], r2 = e[3];
  if (c1 == c2) return r1 == r2 ? kNoEvent : kPerEvent;
  if (c1 > c2) {  // the line's orientation: swap the ends, mirror the TOF bin
    const int tc = c1, tr = r1;
    c1 = c2;
    r1 = r2;
    c2 = tc;
    r2 = tr;
    k = -k;
  }
  const float *d1 = g.det + 3 * c1, *d2 = g.det + 3 * c2;
  const float dz = g.det[3 * (g.n_cry * r2) + 2] - g.det[3 * (g.n_cry * r1) + 2];
  if (dominant_axis(d2[0] - d1[0], d2[1] - d1[1], dz) == 2) return kPerEvent;
  rk = (unsigned)r1 | ((unsigned)r2 << 12) | ((unsigned)(k + g.kmax) << 24);
  const long long n = g.n_cry;
  return (int)(c1 * n - (long long)c1 * (c1 + 1) / 2 + (c2 - c1 - 1));
}

// Line of every event (negative: not by line) and its record.
__global__ __launch_bounds__(256) void k_line_keys(GeomDev g, const int *cyl, const int16_t *ev, const float *v,
                                                   long long n, int *key, LineRec *rec) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= n || !*cyl) return;
  unsigned rk;
  const int L = event_line(g, ev + 5 * e, v[e], rk);
  key[e] = L;
  LineRec r;
  r.rk = rk;
  r.v = v[e];
  rec[e] = r;
}

// Back projection of the events of every line (records rec[off[L] ..
// off[L+1])); blocks as in k_sens_lines.  An event is skipped on uniform
// values when its TOF window or its z range misses the chunk and part.
__global__ __launch_bounds__(kLanes) void k_back_lines(GeomDev g, const int *cyl, const unsigned *off,
                                                       const LineRec *rec, long long p0, long long nlines, int nchunk,
                                                       int nzp, TofTab tt, const float4 *tab, float *img) {
  __shared__ float acc[2 * kZPart * kLanes];
  if (!*cyl) return;
  const long long blk = (long long)blockIdx.x;
  const long long per_line = (long long)nchunk * nzp;
  if (blk / per_line >= nlines) return;
  const long long p = p0 + blk / per_line;
  const unsigned e0 = off[p], e1 = off[p + 1];
  if (e0 == e1) return;
  const int chunk = (int)((blk / nzp) % nchunk), part = (int)(blk % nzp);
  const int lane = threadIdx.x;
  const int nz = g.n[2];
  ZPart zp;
  zp.zlo = part * kZPart;
  zp.zc = min(kZPart, nz - zp.zlo);
  int c1, c2;
  pair_of(p, g.n_cry, c1, c2);
  const LineLane q = line_lane(g, c1, c2, chunk * kLanes, lane);
  const unsigned long long act = __ballot(q.active);
  if (act == 0) return;
  const int la = __ffsll((long long)act) - 1, lb = 63 - __clzll((long long)act);
  const double lam_a = __shfl(q.lam, la), lam_b = __shfl(q.lam, lb);
  for (int i = lane; i < 2 * zp.zc * kLanes; i += kLanes) acc[i] = 0.0f;
  const double edge = 0.5 * g.tof_bin;
  const float wfull = tof_weight(g.vclip, -g.vclip, g.vclip, g.inv_norm);
  const TofTab tu = tof_tab_uniform(tt);
  const double ihz = 1.0 / g.h[2];
  // 64 events at a time: each lane loads one event and tests it (z range,
  // TOF window) for this chunk and part, then the wavefront adds the events
  // that pass, one after the other, with their coefficients broadcast.
  for (unsigned b0 = e0; b0 < e1; b0 += kLanes) {
    const unsigned e = b0 + lane;
    bool pass = false;
    Lor o;
    o.A = o.B = o.az = o.bz = 0.0;
    o.D = o.c = 0.0f;
    if (e < e1) {
      const LineRec r = rec[e];
      const int r1 = (int)(r.rk & 4095u), r2 = (int)((r.rk >> 12) & 4095u), k = (int)(r.rk >> 24) - g.kmax;
      const float z1f = g.det[3 * (g.n_cry * r1) + 2], z2f = g.det[3 * (g.n_cry * r2) + 2];
      lor_z(g, ihz, z1f, z2f, o);
      const double ua = fma(lam_a, o.bz, o.az), ub = fma(lam_b, o.bz, o.az);
      // z range inside the part (one voxel of margin)
      pass = !(floor(fmax(ua, ub)) + 2.0 < (double)zp.zlo ||
               floor(fmin(ua, ub)) - 1.0 >= (double)(zp.zlo + zp.zc));
      if (pass) {
        lor_rest(g, q, z1f, z2f, k * g.tof_bin, edge, r.v, o);
        if (g.tof_on) {
          // vh decreases along the line: every sample of the chunk lies
          // beyond one edge of the bin's truncated window (a margin for
          // rounding)
          const double vh_a = o.A - lam_a * o.B, vh_b = o.A - lam_b * o.B;
          if (fmin(vh_a, vh_b) - o.D >= g.vclip + 1e-3 || fmax(vh_a, vh_b) <= -g.vclip - 1e-3) pass = false;
        }
      }
    }
    unsigned long long m = __ballot(pass);
    while (m) {
      const int j = __ffsll((long long)m) - 1;
      m &= m - 1;
      if (tab)
        add_lor<true>(g, q, broadcast(o, j), zp, wfull, tu, tab, acc, nz, lane);
      else
        add_lor<false>(g, q, broadcast(o, j), zp, wfull, tu, tab, acc, nz, lane);
    }
  }
  flush(g, q, zp, acc, img, lane);
}

// The events the line pass leaves to the per-event projector (key
// kPerEvent).  Each wavefront reads the keys of 64 events at a time and
// projects the marked ones one after the other (a whole wavefront per
// event, as the plain back projection); the grid strides over the list.
__global__ __launch_bounds__(256) void k_back_zdom(GeomDev g, const int *cyl, const float *v, const int16_t *ev,
                                                   const int *key, long long n, float *img) {
  __shared__ Stage1 st[4];
  if (!*cyl) return;
  const int lane = threadIdx.x % kLanes, wv = threadIdx.x / kLanes;
  const long long nw = (long long)gridDim.x * 4;
  for (long long b0 = ((long long)blockIdx.x * 4 + wv) * kLanes; b0 < n; b0 += nw * kLanes) {
    const long long e = b0 + lane;
    unsigned long long m = __ballot(e < n && key[e] == kPerEvent);
    while (m) {
      const int jl = __ffsll((long long)m) - 1;
      m &= m - 1;
      const long long ej = b0 + jl;
      int id1, id2, k;
      decode_event(g, ev + 5 * ej, id1, id2, k);  // valid: the key is set only for valid events
      const Ray r = setup_ray(g, id1, id2, k, W_BIN, 1 << 20);
      const float c = r.L * v[ej];
      const int o = brick_offset(g.lay, r);
      for (int j0 = -o; j0 < r.nplanes; j0 += kLanes) {
        const int j = j0 + lane;
        Sample s = sample_at(g, r, j, g.tof_on);
        const float cs = (j >= 0 && j < r.nplanes) ? c * s.w : 0.0f;
        scatter_interleaved(g, img, r, s, cs, lane, st[wv].idx, st[wv].val);
      }
    }
  }
}

// The order of lm_fwd for a long list: the bucket of every event (its
// transaxial crystal pair c1 != c2 as line index; events of one crystal or
// out of range in bucket nlines), grouped by group_by_key.
__global__ __launch_bounds__(256) void k_fwd_keys(GeomDev g, const int16_t *ev, long long n, long long nlines,
                                                  unsigned *key) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const int c1 = ev[5 * e], c2 = ev[5 * e + 2];
  long long L = nlines;
  if ((unsigned)c1 < (unsigned)g.n_cry && (unsigned)c2 < (unsigned)g.n_cry && c1 != c2) {
    const long long lo = min(c1, c2), hi = max(c1, c2), nc = g.n_cry;
    L = lo * nc - lo * (lo + 1) / 2 + (hi - lo - 1);
  }
  key[e] = (unsigned)L;
}

// ---------------------------------------------------------------------------
// Forward projection of a long event list by line.  After the counting
// sort by transaxial crystal pair, one block takes the events of one line:
// it first interpolates the image across the line transaxially, plane by
// plane, into an LDS sheet s[m][z] = (1 - f1(m)) x(m, i1(m), z) + f1(m)
// x(m, i1(m) + 1, z) over the planes m the line crosses; the bilinear
// sample of any LOR of the line at plane m is then (1 - f2) s[m][k0] +
// f2 s[m][k0 + 1] with the LOR's own z coordinate k0 + f2, the same
// interpolation as the per-event projector (across the transaxial axis
// first, then along z).  Groups of 8 lanes walk the planes of one event
// each, so the image is read once per line instead of once per event.
// Events whose dominant axis is z (and, in extra blocks, the bucket of
// events of one crystal or out of range) take the per-event walk.

constexpr int kFwdLineBlock = 1024;                   // 16 wavefronts
constexpr int kFwdLineGroups = kFwdLineBlock / 8;     // events walked at once
constexpr int kFwdTailBlocks = 256;                   // blocks of the last bucket

// Transaxial geometry of a line in its orientation c1 < c2 (ring 0 crystals):
// planes m of the dominant transaxial axis a, LOR parameter lam(m) = lam0 + m
// dlam (0 at c1, 1 at c2), the other transaxial coordinate u1(m) = (p1b +
// lam db - c0b) / hb in voxels; planes [mlo, mlo + nm) have lam in [0, 1].
struct FwdLine {
  int a, nb, mlo, nm;
  double lam0, dlam, idlam, p1b, db, c0b, hb;
  double dxy2, ha_over_da;
};

__host__ __device__ __forceinline__ FwdLine fwd_line(const GeomDev &g, int c1, int c2) {
  FwdLine q;
  const float *d1 = g.det + 3 * c1, *d2 = g.det + 3 * c2;
  q.a = dominant_axis(d2[0] - d1[0], d2[1] - d1[1], 0.0f);
  const int b = 1 - q.a;
  const double p1a = q.a ? d1[1] : d1[0], da = q.a ? (double)d2[1] - d1[1] : (double)d2[0] - d1[0];
  q.p1b = b ? d1[1] : d1[0];
  q.db = b ? (double)d2[1] - d1[1] : (double)d2[0] - d1[0];
  const double dx = (double)d2[0] - d1[0], dy = (double)d2[1] - d1[1];
  q.dxy2 = dx * dx + dy * dy;
  const double ha = g.h[q.a], c0a = g.c0[q.a];
  q.c0b = g.c0[b];
  q.hb = g.h[b];
  q.nb = g.n[b];
  q.ha_over_da = ha / fabs(da);
  q.lam0 = (c0a - p1a) / da;
  q.dlam = ha / da;
  q.idlam = da / ha;  // plane ranges only (margins of one plane absorb its rounding)
  const double m_at0 = -q.lam0 / q.dlam, m_at1 = (1.0 - q.lam0) / q.dlam;
  const double lo = fmax(0.0, ceil(fmin(m_at0, m_at1))), hi = fmin((double)(g.n[q.a] - 1), floor(fmax(m_at0, m_at1)));
  q.mlo = (int)lo;
  q.nm = hi >= lo ? (int)(hi - lo) + 1 : 0;
  return q;
}

// The rows of the sheet are padded by one float so that the 8 lanes of a
// group, on 8 consecutive planes, read 8 different LDS banks.
__host__ __device__ __forceinline__ int sheet_row(int nz) { return nz + 1; }

size_t fwd_sheet_bytes(const GeomDev &g) {
  const size_t nm = (size_t)std::max(g.n[0], g.n[1]);
  return (nm * sheet_row(g.n[2]) + 3 * nm) * sizeof(float);
}

// TOF weights of the walks: none, the erfc evaluation, or the table.
enum TofMode { kTofNone = 0, kTofErfc = 1, kTofTable = 2 };

// LDS of a line block: the TOF table (when given), the sheet [plane][z]
// (rows of sheet_row(nz) floats), each plane's two transaxial corners as
// layout indices at z = 0 (-1: outside the image) and the fraction f1.
struct SheetLds {
  float4 *tab;
  int ntab;
  float *S;
  int *idx;
  float *f1;
};

__device__ __forceinline__ SheetLds sheet_lds(float4 *sh4, const GeomDev &g, int ntab) {
  const int nm_max = max(g.n[0], g.n[1]), row = sheet_row(g.n[2]);
  SheetLds L;
  L.tab = sh4;
  L.ntab = ntab;
  L.S = (float *)(sh4 + ntab);
  L.idx = (int *)(L.S + (size_t)nm_max * row);
  L.f1 = L.S + (size_t)nm_max * row + 2 * nm_max;
  return L;
}

// The transaxial corners of the line's planes (one plane per thread).
__device__ __forceinline__ void sheet_corners(const GeomDev &g, const FwdLine &q, const SheetLds &L, int tid) {
  const AxisTerm ta = axis_term(g.lay, q.a), tb = axis_term(g.lay, 1 - q.a);
  for (int mm = tid; mm < q.nm; mm += kFwdLineBlock) {
    const int m = q.mlo + mm;
    const double lam = fma((double)m, q.dlam, q.lam0);
    const double u1 = (q.p1b + lam * q.db - q.c0b) / q.hb;
    const double fl = floor(u1);
    const int i1 = (int)fl;
    const bool ok0 = fl >= 0.0 && fl <= (double)q.nb - 1.0, ok1 = fl >= -1.0 && fl <= (double)q.nb - 2.0;
    L.idx[2 * mm] = ok0 ? axis_index(ta, m) + axis_index(tb, i1) : -1;
    L.idx[2 * mm + 1] = ok1 ? axis_index(ta, m) + axis_index(tb, i1 + 1) : -1;
    L.f1[mm] = (float)(u1 - fl);
  }
}

// A LOR of a line (ring z's z1, z2 and TOF bin k in the line's orientation):
// the planes it can touch, m0 .. m1 (m1 < m0: none), its TOF argument vh0 +
// j dvh and z coordinate u20 + j du2 (voxels) at plane m0 + j, and its plane
// length L.  The TOF argument is stepped in float from its double value at
// m0 (|vh| stays below a few units, so its float error is a few 1e-7 sigma,
// as in the per-event walk); z takes one double FMA per sample (in float, j
// dz a few tens of voxels along would carry 1e-6 voxel errors).
struct LineLor {
  int m0, m1;
  float vh0, dvh;
  double u20, du2;
  float L;
};

__device__ __forceinline__ LineLor line_lor(const GeomDev &g, const FwdLine &q, float z1f, float z2f, int k, float D,
                                            double ihz) {
  const int nz = g.n[2];
  const double dz = (double)z2f - z1f;
  const double dn = sqrt(q.dxy2 + dz * dz);
  // vh(lam) = A - lam B (units of sigma sqrt 2), z(lam) = az + lam bz (voxels)
  const double A = (k * g.tof_bin + 0.5 * g.tof_bin + 0.5 * dn) * g.inv_sr2, B = dn * g.inv_sr2;
  const double az = ((double)z1f - g.c0[2]) * ihz, bz = dz * ihz;
  double lo = q.mlo, hi = q.mlo + q.nm - 1;
  if (g.tof_on) {  // vh in [-vclip, vclip + D], one plane of margin
    const double iB = 1.0 / B;
    const double ma = ((A - ((double)g.vclip + D)) * iB - q.lam0) * q.idlam;
    const double mb = ((A + (double)g.vclip) * iB - q.lam0) * q.idlam;
    lo = fmax(lo, floor(fmin(ma, mb)) - 1.0);
    hi = fmin(hi, ceil(fmax(ma, mb)) + 1.0);
  }
  if (bz != 0.0) {  // z in (-1, nz), one plane of margin
    const double ibz = 1.0 / bz;
    const double ma = ((-1.0 - az) * ibz - q.lam0) * q.idlam, mb = (((double)nz - az) * ibz - q.lam0) * q.idlam;
    lo = fmax(lo, floor(fmin(ma, mb)) - 1.0);
    hi = fmin(hi, ceil(fmax(ma, mb)) + 1.0);
  } else if (az <= -1.0 || az >= (double)nz) {
    hi = lo - 1.0;
  }
  LineLor o;
  o.L = (float)(q.ha_over_da * dn);
  o.vh0 = o.dvh = 0.0f;
  o.u20 = o.du2 = 0.0;
  if (hi >= lo) {
    o.m0 = (int)lo;
    o.m1 = (int)hi;
    const double lam_lo = fma(lo, q.dlam, q.lam0);
    o.vh0 = (float)(A - lam_lo * B);
    o.dvh = (float)(-q.dlam * B);
    o.u20 = fma(lam_lo, bz, az);
    o.du2 = q.dlam * bz;
  } else {
    o.m0 = q.mlo;
    o.m1 = q.mlo - 1;
  }
  return o;
}

// The TOF weight of a line walk's sample.
template <int TM>
__device__ __forceinline__ float line_weight(const GeomDev &g, const LineLor &o, int j, float D, const TofTab &tt,
                                             const float4 *tab) {
  if constexpr (TM == kTofErfc) {
    const float vh = fmaf((float)j, o.dvh, o.vh0);
    return tof_weight(vh, vh - D, g.vclip, g.inv_norm);
  } else if constexpr (TM == kTofTable) {
    return tof_weight_tab(tt, tab, fmaf((float)j, o.dvh, o.vh0));
  } else {
    return 1.0f;
  }
}

// The forward walk of one LOR of the line over its planes (lane gl of its
// group: m0 + gl, + 8, ...): the sum of w (lerp in z of the sheet).
template <int TM>
__device__ __forceinline__ float fwd_line_walk(const GeomDev &g, const FwdLine &q, const float *S, int nz,
                                               const LineLor &o, float D, const TofTab &tt, const float4 *tab, int gl) {
  const int row = sheet_row(nz);
  float acc = 0.0f;
  const float *sr = S + (o.m0 + gl - q.mlo) * row;
  for (int j = gl; j <= o.m1 - o.m0; j += 8, sr += 8 * row) {
    const float w = line_weight<TM>(g, o, j, D, tt, tab);
    const double u2 = fma((double)j, o.du2, o.u20);
    const double fl = floor(u2);
    const int k0 = (int)fl;
    const float f2 = (float)(u2 - fl);
    const bool ok0 = (unsigned)k0 < (unsigned)nz, ok1 = (unsigned)(k0 + 1) < (unsigned)nz;
    const float t0 = sr[ok0 ? k0 : 0], t1 = sr[ok1 ? k0 + 1 : 0];
    const float s0 = ok0 ? t0 : 0.0f, s1 = ok1 ? t1 : 0.0f;
    acc = fmaf(w, fmaf(f2, s1 - s0, s0), acc);
  }
  return acc;
}


// Per-event projection of event e by a group (the per-event projector's
// walk over the image x); 0 for an invalid event.
__device__ __forceinline__ float fwd_event(const GeomDev &g, const float *__restrict__ x, const int16_t *ev, float D,
                                           int gl) {
  int id1, id2, k;
  if (!decode_event(g, ev, id1, id2, k)) return 0.0f;
  const RayPack pk = pack_ray(setup_ray(g, id1, id2, k, W_BIN, 1 << 20));
  if (pk.p.y <= 0) return 0.0f;
  const float acc = g.tof_on ? fwd_walk<true>(g, x, pk, D, gl) : fwd_walk<false>(g, x, pk, D, gl);
  return __int_as_float(pk.q.w) * acc;
}

// Records of the sorted events of the lines (positions below off[nlines]):
// {e, r1 | r2 << 12 | (k + kmax) << 24} in the line's orientation (crystal
// c1 < c2: an event with c1 > c2 has its rings swapped and its TOF bin
// mirrored), or kNoRec for an event that does not decode.  The line kernel
// then reads its events in a row instead of gathering them through the
// sorted order.
constexpr unsigned kNoRec = ~0u;

__global__ __launch_bounds__(256) void k_fwd_recs(GeomDev g, const int *cyl, const int16_t *__restrict__ ev,
                                                  const unsigned *__restrict__ order, const unsigned *off,
                                                  long long nlines, uint2 *__restrict__ rec) {
  if (!*cyl) return;
  const unsigned pos = blockIdx.x * 256 + threadIdx.x;
  if (pos >= off[nlines]) return;
  const unsigned e = order[pos];
  const int16_t *r = ev + 5 * (size_t)e;
  int id1, id2, k;
  unsigned rk = kNoRec;
  if (decode_event(g, r, id1, id2, k)) {
    int r1 = r[1], r2 = r[3];
    if (r[0] > r[2]) {
      const int t = r1;
      r1 = r2;
      r2 = t;
      k = -k;
    }
    rk = (unsigned)r1 | ((unsigned)r2 << 12) | ((unsigned)(k + g.kmax) << 24);
  }
  rec[pos] = make_uint2(e, rk);
}

// Blocks b < 8 ceil(nlines / 8): the events of one line each, sorted
// positions off[L] .. off[L + 1] with L = (b % 8) ceil(nlines / 8) + b / 8
// (blocks are dealt to the XCDs round robin, so consecutive lines, which
// read nearby voxels, share an XCD's L2; blocks with L >= nlines do
// nothing); the kFwdTailBlocks blocks after them: the last bucket (events
// of one crystal, or out of range) by the per-event walk.  Does nothing
// unless *cyl is set.
__global__ __launch_bounds__(kFwdLineBlock) void k_fwd_lines(GeomDev g, const int *cyl, const float *__restrict__ x,
                                                             const int16_t *__restrict__ ev, const unsigned *order,
                                                             const uint2 *__restrict__ rec, const unsigned *off,
                                                             long long nlines, TofTab tt, const float4 *tab,
                                                             float *__restrict__ out) {
  extern __shared__ float4 sh4[];
  if (!*cyl) return;
  const int tid = threadIdx.x, grp = tid >> 3, gl = tid & 7;
  const float D = tof_bin_width(g);
  const long long per = (nlines + 7) / 8;
  long long blk = blockIdx.x;
  if (blk >= 8 * per) {  // the last bucket
    const unsigned t0 = off[nlines], t1 = off[nlines + 1];
    for (unsigned pos = t0 + (unsigned)((blk - 8 * per) * kFwdLineGroups + grp); pos < t1;
         pos += kFwdTailBlocks * kFwdLineGroups) {
      const unsigned e = order[pos];
      float acc = fwd_event(g, x, ev + 5 * (size_t)e, D, gl);
      acc = group_sum<8>(acc);
      if (gl == 0) out[e] = acc;
    }
    return;
  }
  blk = (blk % 8) * per + blk / 8;
  if (blk >= nlines) return;
  const unsigned e0 = off[blk], e1 = off[blk + 1];
  if (e0 == e1) return;
  int c1, c2;
  pair_of(blk, g.n_cry, c1, c2);
  const FwdLine q = fwd_line(g, c1, c2);
  const int nz = g.n[2], row = sheet_row(nz);
  const SheetLds L = sheet_lds(sh4, g, tab ? tof_tab_size(tt) : 0);
  for (int i = tid; i < L.ntab; i += kFwdLineBlock) L.tab[i] = tab[i];
  const TofTab tu = tof_tab_uniform(tt);
  sheet_corners(g, q, L, tid);
  __syncthreads();
  // cells (plane, z), planes fastest; 4 cells (8 loads) per thread in flight
  const AxisTerm tz = axis_term(g.lay, 2);
  const int ncell = q.nm * nz;
  for (int t0 = tid; t0 < ncell; t0 += 4 * kFwdLineBlock) {
    float x0[4], x1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = min(t0 + u * kFwdLineBlock, ncell - 1);
      const int mm = t % q.nm, k = t / q.nm;
      const int zi = axis_index(tz, k), j0 = L.idx[2 * mm], j1 = L.idx[2 * mm + 1];
      const float v0 = x[j0 >= 0 ? j0 + zi : 0], v1 = x[j1 >= 0 ? j1 + zi : 0];
      x0[u] = j0 >= 0 ? v0 : 0.0f;
      x1[u] = j1 >= 0 ? v1 : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u * kFwdLineBlock;
      if (t < ncell) {
        const int mm = t % q.nm, k = t / q.nm;
        L.S[mm * row + k] = fmaf(L.f1[mm], x1[u] - x0[u], x0[u]);
      }
    }
  }
  __syncthreads();
  const double ihz = 1.0 / g.h[2];
  for (unsigned pos = e0 + grp; pos < e1; pos += kFwdLineGroups) {
    const uint2 rr = rec[pos];
    const unsigned e = rr.x;
    float val = 0.0f;
    if (rr.y != kNoRec) {
      const int r1 = (int)(rr.y & 4095u), r2 = (int)((rr.y >> 12) & 4095u), k = (int)(rr.y >> 24) - g.kmax;
      const float z1f = g.det[3 * (g.n_cry * r1) + 2], z2f = g.det[3 * (g.n_cry * r2) + 2];
      const float *d1 = g.det + 3 * c1, *d2 = g.det + 3 * c2;
      if (dominant_axis(d2[0] - d1[0], d2[1] - d1[1], z2f - z1f) == 2) {
        float acc = fwd_event(g, x, ev + 5 * (size_t)e, D, gl);
        val = group_sum<8>(acc);
      } else {
        const LineLor o = line_lor(g, q, z1f, z2f, k, D, ihz);
        float acc = 0.0f;
        if (o.m1 >= o.m0) {
          if (!g.tof_on)
            acc = fwd_line_walk<kTofNone>(g, q, L.S, nz, o, D, tu, L.tab, gl);
          else if (L.ntab)
            acc = fwd_line_walk<kTofTable>(g, q, L.S, nz, o, D, tu, L.tab, gl);
          else
            acc = fwd_line_walk<kTofErfc>(g, q, L.S, nz, o, D, tu, L.tab, gl);
        }
        acc = group_sum<8>(acc);
        val = o.L * acc;
      }
    }
    if (gl == 0) out[e] = val;
  }
}


// Coefficients of the TOF table (one interval per thread; see TofTab):
// values and derivatives of the piece's own smooth expression at both ends
// of the interval, in double.
__global__ __launch_bounds__(256) void k_tof_table(TofTab t, double vc, double D, double inv_norm, float4 *tab) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= tof_tab_size(t)) return;
  int j;
  float start, end;
  if (i < t.n0) {
    j = i;
    start = t.b0;
    end = t.b1;
  } else if (i < t.n0 + t.n1) {
    j = i - t.n0;
    start = t.b1;
    end = t.b2;
  } else {
    j = i - t.n0 - t.n1;
    start = t.b2;
    end = t.b3;
  }
  // the evaluation maps s in [0, 1) to vh = start + (j + s) / kTofTabPerUnit
  const double a = start + (double)j / kTofTabPerUnit, b = start + (double)(j + 1) / kTofTabPerUnit;
  // the piece's expression (decided at the piece's middle, also for an
  // interval that runs past the piece's end)
  const double mid = 0.5 * ((double)start + (double)end);
  const bool up = mid < vc;       // the upper edge inside the truncation
  const bool lo = mid - D > -vc;  // the lower edge inside the truncation
  const double eu = erf(vc), el = erf(-vc);
  auto f = [&](double v) { return inv_norm * ((up ? erf(v) : eu) - (lo ? erf(v - D) : el)); };
  auto df = [&](double v) {
    const double two_over_sqrt_pi = 1.1283791670955126;
    return inv_norm * two_over_sqrt_pi * ((up ? exp(-v * v) : 0.0) - (lo ? exp(-(v - D) * (v - D)) : 0.0));
  };
  const double h = b - a, fa = f(a), fb = f(b), da = h * df(a), db = h * df(b);
  tab[i] = make_float4((float)fa, (float)da, (float)(3.0 * (fb - fa) - 2.0 * da - db),
                       (float)(2.0 * (fa - fb) + da + db));
}

// The scanner is cylindrical when crystal c of ring r sits at (x_c, y_c, z_r):
// the same transaxial position in every ring and one z per ring, with z_r
// increasing in r.  One block checks every crystal and writes flag[0] = 1
// (cylindrical) or 0; the kernels of the two paths read the flag, so the
// decision never waits for the host.
__global__ __launch_bounds__(256) void k_cylindrical(GeomDev g, int *flag) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  int b = 0;
  const float *d = g.det;
  for (int i = threadIdx.x; i < g.n_det; i += 256) {
    const int r = i / g.n_cry, c = i - r * g.n_cry;
    const float *p = d + 3 * (long long)i;
    if (p[0] != d[3 * c] || p[1] != d[3 * c + 1] || p[2] != d[3 * (long long)g.n_cry * r + 2]) b = 1;
    if (c == 0 && r > 0 && !(p[2] > d[3 * (long long)g.n_cry * (r - 1) + 2])) b = 1;
  }
  if (b) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) flag[0] = bad ? 0 : 1;
}

}  // namespace

namespace lmk {

bool lines_possible(const GeomDev &g) { return g.n_ring >= 2 && g.n_cry >= 2; }

int launch_cylindrical(const GeomDev &g, int *flag, hipStream_t st) {
  hipLaunchKernelGGL(k_cylindrical, dim3(1), dim3(256), 0, st, g, flag);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

// Sensitivity by transaxial line; its kernels do nothing unless *cyl is set.
int launch_sens_lines(const GeomDev &g, const int *cyl, float *img, hipStream_t st) {
  const int na_max = std::max(g.n[0], g.n[1]);
  const int nchunk = (na_max + kLanes - 1) / kLanes;
  const int nzp = (g.n[2] + kZPart - 1) / kZPart;
  const long long nlines = (long long)g.n_cry * (g.n_cry - 1) / 2;
  // at most 2^24 blocks of 64 work-items per launch
  const long long per = std::max<long long>(1, (1LL << 24) / ((long long)nchunk * nzp));
  for (long long p0 = 0; p0 < nlines; p0 += per) {
    const long long m = std::min(per, nlines - p0);
    hipLaunchKernelGGL(k_sens_lines, dim3((unsigned)(m * nchunk * nzp)), dim3(kLanes), 0, st, g, cyl, p0, m, nchunk,
                       nzp, img);
    LM_TRY_HIP(hipGetLastError());
  }
  const long long npz = (long long)g.n_cry * (g.n_cry + 1) / 2;  // c1 <= c2
  for (long long p0 = 0; p0 < npz; p0 += (1LL << 24)) {
    const long long m = std::min(1LL << 24, npz - p0);
    hipLaunchKernelGGL(k_sens_zdom, dim3((unsigned)m), dim3(kLanes), 0, st, g, cyl, p0, m, img);
    LM_TRY_HIP(hipGetLastError());
  }
  return LM_OK;
}


int sort_events_by_line(const GeomDev &g, const int16_t *ev, long long n, unsigned **order, unsigned **offsets,
                        hipStream_t st) {
  *order = nullptr;
  if (offsets) *offsets = nullptr;
  const long long nlines = (long long)g.n_cry * (g.n_cry - 1) / 2;
  if (g.n_cry < 2 || n < 64 * nlines || n >= (1LL << 31) || nlines + 1 > (long long)kGroupMaxBuckets) return LM_OK;
  unsigned *key = nullptr, *off = nullptr, *ord = nullptr;
  auto release = [&](bool keep) {  // release errors are not reported
    if (key) (void)hipFreeAsync(key, st);
    if (ord && !keep) (void)hipFreeAsync(ord, st);
    if (off && !(keep && offsets)) (void)hipFreeAsync(off, st);
  };
  hipError_t e = hipMallocAsync((void **)&key, n * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&off, (nlines + 2) * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&ord, n * sizeof(unsigned), st);
  if (e == hipErrorOutOfMemory) {
    release(false);
    (void)hipGetLastError();
    return LM_OK;  // the list is projected in its own order
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_fwd_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, ev, n, nlines, key);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    release(false);
    LM_TRY_HIP(e);
  }
  const int rc = group_by_key(key, (const unsigned *)nullptr, n, (unsigned)(nlines + 1), nullptr, ord, off, st);
  if (rc == LM_ENOMEM) {
    release(false);
    lmh::clear_error();
    return LM_OK;  // the list is projected in its own order
  }
  release(rc == LM_OK);
  if (rc != LM_OK) return rc;
  *order = ord;
  if (offsets) *offsets = off;
  return LM_OK;
}

// The largest LDS allocation of a block on the current device.
static int lds_per_block(int &bytes) {
  int dev = 0;
  LM_TRY_HIP(hipGetDevice(&dev));
  LM_TRY_HIP(hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  return LM_OK;
}

int build_tof_table(const GeomDev &g, TofTab &t, float4 **tab, hipStream_t st) {
  *tab = nullptr;
  if (!g.tof_on) return LM_OK;
  t = tof_tab_layout(g);
  const int n = tof_tab_size(t);
  if (n > kTofTabMax) return LM_OK;
  const hipError_t e = hipMallocAsync((void **)tab, (size_t)n * sizeof(float4), st);
  if (e == hipErrorOutOfMemory) {
    *tab = nullptr;
    (void)hipGetLastError();
    return LM_OK;
  }
  LM_TRY_HIP(e);
  const double vc = (g.half_win - 0.5 * g.tof_bin) * g.inv_sr2, D = g.tof_bin * g.inv_sr2;
  const double inv_norm = 1.0 / (2.0 * std::erf(vc));
  hipLaunchKernelGGL(k_tof_table, dim3((n + 255) / 256), dim3(256), 0, st, t, vc, D, inv_norm, *tab);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_fwd_lines(const GeomDev &g, const int *cyl, const float *x, const int16_t *ev, const unsigned *order,
                     const unsigned *off, long long n, float *out, hipStream_t st, bool &queued) {
  queued = false;
  // the records hold rings in 12 bits and the TOF bin in 8
  if (!lines_possible(g) || n == 0 || g.n_ring > 4096 || g.n_tof > 255 || n >= (1LL << 32)) return LM_OK;
  int lds_max = 0;
  if (int rc = lds_per_block(lds_max)) return rc;
  if (fwd_sheet_bytes(g) > (size_t)lds_max) return LM_OK;
  uint2 *rec = nullptr;
  {
    const hipError_t ea = hipMallocAsync((void **)&rec, (size_t)n * sizeof(uint2), st);
    if (ea == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      return LM_OK;  // the per-event walk in the sorted order
    }
    LM_TRY_HIP(ea);
  }
  const long long nlines = (long long)g.n_cry * (g.n_cry - 1) / 2;
  hipLaunchKernelGGL(k_fwd_recs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, cyl, ev, order, off, nlines,
                     rec);
  if (const hipError_t ek = hipGetLastError(); ek != hipSuccess) {
    (void)hipFreeAsync(rec, st);
    LM_TRY_HIP(ek);
  }
  TofTab tt{};
  float4 *tab = nullptr;
  if (int rc = build_tof_table(g, tt, &tab, st)) {
    (void)hipFreeAsync(rec, st);
    return rc;
  }
  size_t bytes = fwd_sheet_bytes(g) + (tab ? (size_t)tof_tab_size(tt) * sizeof(float4) : 0);
  if (bytes > (size_t)lds_max) {  // the sheet alone fits: erfc weights
    if (tab) (void)hipFreeAsync(tab, st);
    tab = nullptr;
    bytes = fwd_sheet_bytes(g);
  }
  const long long nb = 8 * ((nlines + 7) / 8) + kFwdTailBlocks;
  hipLaunchKernelGGL(k_fwd_lines, dim3((unsigned)nb), dim3(kFwdLineBlock), bytes, st, g, cyl, x, ev, order, rec, off,
                     nlines, tt, tab, out);
  const hipError_t e = hipGetLastError();
  if (tab) (void)hipFreeAsync(tab, st);  // release errors have no caller to go to
  (void)hipFreeAsync(rec, st);
  LM_TRY_HIP(e);
  queued = true;
  return LM_OK;
}

// Back projection of a long list by line: worth it when the lines carry
// many events each (the per-block flush costs about as many atomics as
// a few tens of events do on the per-event path).
constexpr long long kMinEventsPerLine = 64;

int launch_back_lines(const GeomDev &g, const int *cyl, const float *v, const int16_t *ev, long long n, float *img,
                      hipStream_t st, bool &queued) {
  queued = false;
  const long long nlines = (long long)g.n_cry * (g.n_cry - 1) / 2;
  if (!lines_possible(g) || g.n_ring > 4096 || g.n_tof > 255) return LM_OK;
  if (n < kMinEventsPerLine * nlines || n >= (1LL << 31) || nlines > (long long)kGroupMaxBuckets) return LM_OK;
  int *key = nullptr;
  unsigned *off = nullptr;
  LineRec *rec = nullptr, *recu = nullptr;
  auto release = [&]() {  // release errors are not reported
    if (key) (void)hipFreeAsync(key, st);
    if (off) (void)hipFreeAsync(off, st);
    if (rec) (void)hipFreeAsync(rec, st);
    if (recu) (void)hipFreeAsync(recu, st);
  };
  hipError_t e = hipMallocAsync((void **)&key, n * sizeof(int), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&off, (nlines + 1) * sizeof(unsigned), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&rec, n * sizeof(LineRec), st);
  if (e == hipSuccess) e = hipMallocAsync((void **)&recu, n * sizeof(LineRec), st);
  if (e == hipErrorOutOfMemory) {
    // no room for the sort: the per-event path needs no temporaries
    release();
    (void)hipGetLastError();
    return LM_OK;
  }
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_line_keys, dim3(grid), dim3(256), 0, st, g, cyl, ev, v, n, key, recu);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    // events of no line (negative keys) are dropped from the records
    static_assert(sizeof(LineRec) == sizeof(unsigned long long), "a record is one 64-bit payload");
    const int rc = group_by_key((const unsigned *)key, (const unsigned long long *)recu, n, (unsigned)nlines, cyl,
                                (unsigned long long *)rec, off, st);
    if (rc == LM_ENOMEM) {
      release();
      lmh::clear_error();
      return LM_OK;  // the per-event path
    }
    if (rc != LM_OK) {
      release();
      return rc;
    }
  }
  const int na_max = std::max(g.n[0], g.n[1]);
  const int nchunk = (na_max + kLanes - 1) / kLanes;
  const int nzp = (g.n[2] + kZPart - 1) / kZPart;
  const long long per = std::max<long long>(1, (1LL << 24) / ((long long)nchunk * nzp));
  TofTab tt{};
  float4 *tab = nullptr;
  if (e == hipSuccess) {
    if (int rc = build_tof_table(g, tt, &tab, st)) {
      release();
      return rc;
    }
  }
  for (long long p0 = 0; e == hipSuccess && p0 < nlines; p0 += per) {
    const long long m = std::min(per, nlines - p0);
    hipLaunchKernelGGL(k_back_lines, dim3((unsigned)(m * nchunk * nzp)), dim3(kLanes), 0, st, g, cyl, off, rec, p0,
                       m, nchunk, nzp, tt, tab, img);
    e = hipGetLastError();
  }
  if (tab) (void)hipFreeAsync(tab, st);  // a release error has no caller to go to
  if (e == hipSuccess) {
    // 4096 blocks of 4 wavefronts stride over the list
    const long long nb = std::min<long long>(4096, (n + 4 * kLanes - 1) / (4 * kLanes));
    hipLaunchKernelGGL(k_back_zdom, dim3((unsigned)nb), dim3(256), 0, st, g, cyl, v, ev, key, n, img);
    e = hipGetLastError();
  }
  release();
  LM_TRY_HIP(e);
  queued = true;
  return LM_OK;
}

}  // namespace lmk
