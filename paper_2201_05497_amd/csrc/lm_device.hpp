// Device core of the listmode TOF Joseph projector (gfx950).
//
// One event is handled by a group of LPE lanes of a 64-wide wavefront (8 in
// the forward projector, the whole wavefront in the kernels that scatter);
// the lanes of a group walk the image planes of the event's line of
// response, lane l taking planes m0 + l, m0 + l + LPE, ...
//
// The per-event set-up (dominant axis, plane range, interpolation and TOF
// coefficients) is done in double precision, once per event.  The
// per-sample arithmetic is float32 and works on small numbers only: the
// interpolation coordinate of a sample is written as an integer part fixed
// per event plus F + j*V with j the plane offset inside the event's range,
// and the TOF argument as A - j*B, so float32 rounding stays at the 1e-6
// level of a voxel or a TOF sigma.
//
// Voxel addresses go through a Layout: images are either row-major
// ([z][y][x], the caller's layout) or stored in bricks of 4x4x4 voxels (4x4x1
// for a single slice), 256 bytes each, so that the few planes a ray spends
// in a brick touch the same cache lines whatever the ray's direction.  The
// FP32 atomics of the back projection are executed beyond the L2, one
// request per memory sector that lanes of an instruction share, so the
// sectors one atomic instruction touches set its cost.
//
// The functions below except the atomic scatters and group_sum are
// __host__ __device__ so that the projector can also be exercised by a CPU
// build.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lmk {

// Voxel (i, j, k) -> linear index.  Bricks are 2^sx x 2^sy x 2^sz voxels;
// nbx, nby bricks per brick row and brick slice.  Row-major is the special
// case sx = sy = sz = 0 with nbx = nx, nby = ny.
struct Layout {
  int nbx, nby, nbz;
  int sx, sy, sz;    // log2 of the brick size along x, y, z
};

__host__ __device__ __forceinline__ int vidx(const Layout &L, int i, int j, int k) {
  const int b = ((k >> L.sz) * L.nby + (j >> L.sy)) * L.nbx + (i >> L.sx);
  const int mx = (1 << L.sx) - 1, my = (1 << L.sy) - 1, mz = (1 << L.sz) - 1;
  return (b << (L.sx + L.sy + L.sz)) | ((((k & mz) << L.sy) | (j & my)) << L.sx) | (i & mx);
}

// Inverse of vidx: position p of the layout -> voxel (i, j, k) (padding
// positions decode to coordinates beyond the image size).
__host__ __device__ __forceinline__ void vpos(const Layout &L, long long p, int &i, int &j, int &k) {
  const int sh = L.sx + L.sy + L.sz;
  const long long b = p >> sh;
  const int loc = (int)(p & ((1LL << sh) - 1));
  const int li = loc & ((1 << L.sx) - 1);
  const int lj = (loc >> L.sx) & ((1 << L.sy) - 1);
  const int lk = loc >> (L.sx + L.sy);
  const long long bi = b % L.nbx, bj = (b / L.nbx) % L.nby, bk = b / ((long long)L.nbx * L.nby);
  i = (int)(bi << L.sx) | li;
  j = (int)(bj << L.sy) | lj;
  k = (int)(bk << L.sz) | lk;
}

// Elements of an image stored with layout L (the padded brick grid).
__host__ __device__ __forceinline__ long long layout_size(const Layout &L) {
  return (long long)L.nbx * L.nby * L.nbz << (L.sx + L.sy + L.sz);
}

// Geometry in the form the kernels use (built on the host from lm_geom).
struct GeomDev {
  const float *det;  // [n_det][3]
  int n_cry, n_ring, n_det;
  int n[3];          // nx, ny, nz
  Layout lay;        // voxel addressing of the images the kernels see
  double h[3];
  double c0[3];      // coordinate of the centre of voxel 0 along each axis
  int n_tof, kmax;
  int tof_on;
  double tof_bin;
  double inv_sr2;    // 1 / (sigma sqrt 2)
  double half_win;   // nsigma*sigma + tof_bin/2: half support of a bin's weight
  float vclip;       // nsigma / sqrt 2
  float inv_norm;    // 1 / (2 erf(nsigma / sqrt 2))
};

// Per-event set-up of a LOR.
struct Ray {
  int nplanes;       // planes to visit (0: nothing)
  int m0;            // first plane along the dominant axis
  int a;             // dominant axis
  int n1, n2;        // image size along the two other axes
  int I1, I2;        // integer parts of the interpolation coordinates at m0
  float F1, V1, F2, V2;  // u_b(m0 + j) = I_b + F_b + j V_b
  double F1d, V1d, F2d, V2d;  // the same in double (the forward walk's coordinates)
  float A, B, D;     // TOF: vh(j) = A - j B, vl = vh - D (units of sigma sqrt 2)
  float L;           // plane length h_a |d| / |d_a|
};

enum WeightMode { W_BIN = 0, W_SUM = 1 };

template <class T>
__host__ __device__ __forceinline__ T sel3(int i, T x, T y, T z) {
  return i == 0 ? x : (i == 1 ? y : z);
}

__host__ __device__ __forceinline__ int dominant_axis(float dx, float dy, float dz) {
  float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
  int a = 0;
  float am = ax;
  if (ay > am) { a = 1; am = ay; }
  if (az > am) { a = 2; }
  return a;
}

// Sets up the LOR from crystal id1 to id2 with TOF bin k.  mode W_SUM sets
// up the weight summed over all TOF bins (the sensitivity image).
__host__ __device__ __forceinline__ Ray setup_ray(const GeomDev &g, int id1, int id2, int k, int mode,
                                                  int max_planes) {
  Ray r;
  r.nplanes = 0;
  r.m0 = r.a = r.n1 = r.n2 = r.I1 = r.I2 = 0;
  r.F1 = r.V1 = r.F2 = r.V2 = r.A = r.B = r.D = r.L = 0.0f;
  r.F1d = r.V1d = r.F2d = r.V2d = 0.0;
  const float *q1 = g.det + 3 * id1;
  const float *q2 = g.det + 3 * id2;
  const float f1x = q1[0], f1y = q1[1], f1z = q1[2];
  const float f2x = q2[0], f2y = q2[1], f2z = q2[2];
  const int a = dominant_axis(f2x - f1x, f2y - f1y, f2z - f1z);
  const float dfa = (a == 0) ? (f2x - f1x) : (a == 1) ? (f2y - f1y) : (f2z - f1z);
  if (dfa == 0.0f) return r;
  const int b1 = (a == 0) ? 1 : 0;
  const int b2 = (a == 2) ? 1 : 2;
  // components selected with conditionals (no runtime-indexed local
  // arrays, which would live in scratch memory)
  const double p1x = f1x, p1y = f1y, p1z = f1z;
  const double dx = (double)f2x - p1x, dy = (double)f2y - p1y, dz = (double)f2z - p1z;
  const double p1a = sel3(a, p1x, p1y, p1z), da = sel3(a, dx, dy, dz);
  const double p1b1 = sel3(b1, p1x, p1y, p1z), db1 = sel3(b1, dx, dy, dz);
  const double p1b2 = sel3(b2, p1x, p1y, p1z), db2 = sel3(b2, dx, dy, dz);
  const double dn = sqrt(dx * dx + dy * dy + dz * dz);
  const double ida = 1.0 / da;
  const double ha = sel3(a, g.h[0], g.h[1], g.h[2]);
  const double c0a = sel3(a, g.c0[0], g.c0[1], g.c0[2]);
  const double c0b1 = sel3(b1, g.c0[0], g.c0[1], g.c0[2]);
  const double c0b2 = sel3(b2, g.c0[0], g.c0[1], g.c0[2]);
  const double hb1 = sel3(b1, g.h[0], g.h[1], g.h[2]);
  const double hb2 = sel3(b2, g.h[0], g.h[1], g.h[2]);
  const int na = sel3(a, g.n[0], g.n[1], g.n[2]);
  const int nb1 = sel3(b1, g.n[0], g.n[1], g.n[2]);
  const int nb2 = sel3(b2, g.n[0], g.n[1], g.n[2]);
  // plane m has centre c0a + m ha and LOR parameter lam(m) = lam0 + m dlam
  const double lam0 = (c0a - p1a) * ida;
  const double dlam = ha * ida;
  // lam in [0, 1]
  double mlo_d, mhi_d;
  {
    double m_at0 = -lam0 / dlam, m_at1 = (1.0 - lam0) / dlam;
    mlo_d = fmin(m_at0, m_at1);
    mhi_d = fmax(m_at0, m_at1);
    mlo_d = ceil(mlo_d);
    mhi_d = floor(mhi_d);
  }
  // TOF support of the weight (one plane of margin on each side; outside
  // the support the weight evaluates to exactly zero anyway)
  double tc = 0.0, hw = 0.0;
  if (g.tof_on) {
    if (mode == W_BIN) {
      tc = k * g.tof_bin;
      hw = g.half_win;
    } else {
      tc = 0.0;
      hw = g.kmax * g.tof_bin + g.half_win;
    }
    // t(m) = (lam(m) - 1/2) dn  ->  lam in [1/2 + (tc-hw)/dn, 1/2 + (tc+hw)/dn]
    double la = 0.5 + (tc - hw) / dn, lb = 0.5 + (tc + hw) / dn;
    double ma = (la - lam0) / dlam, mb = (lb - lam0) / dlam;
    mlo_d = fmax(mlo_d, floor(fmin(ma, mb)) - 1.0);
    mhi_d = fmin(mhi_d, ceil(fmax(ma, mb)) + 1.0);
  }
  // interpolation coordinates u_b(m) = (p1_b + lam(m) d_b - c0b) / h_b
  const double U1 = (p1b1 + lam0 * db1 - c0b1) / hb1;
  const double V1 = dlam * db1 / hb1;
  const double U2 = (p1b2 + lam0 * db2 - c0b2) / hb2;
  const double V2 = dlam * db2 / hb2;
  // clip to the image box in the two other axes: u_b in (-1, n_b)
  {
    if (V1 != 0.0) {
      double ma = (-1.0 - U1) / V1, mb = (nb1 - U1) / V1;
      mlo_d = fmax(mlo_d, floor(fmin(ma, mb)) - 1.0);
      mhi_d = fmin(mhi_d, ceil(fmax(ma, mb)) + 1.0);
    } else if (U1 <= -1.0 || U1 >= nb1) {
      return r;
    }
    if (V2 != 0.0) {
      double ma = (-1.0 - U2) / V2, mb = (nb2 - U2) / V2;
      mlo_d = fmax(mlo_d, floor(fmin(ma, mb)) - 1.0);
      mhi_d = fmin(mhi_d, ceil(fmax(ma, mb)) + 1.0);
    } else if (U2 <= -1.0 || U2 >= nb2) {
      return r;
    }
  }
  mlo_d = fmax(mlo_d, 0.0);
  mhi_d = fmin(mhi_d, (double)(na - 1));
  if (mhi_d < mlo_d) return r;
  const int m0 = (int)mlo_d;
  int np = (int)mhi_d - m0 + 1;
  // max_planes (from max_planes() on the host) covers every plane of the
  // TOF support; the clamp can only drop a margin plane of zero weight
  if (np > max_planes) np = max_planes;
  r.nplanes = np;
  r.m0 = m0;
  r.a = a;
  r.n1 = nb1;
  r.n2 = nb2;
  const double u1 = U1 + m0 * V1, u2 = U2 + m0 * V2;
  const double i1 = floor(u1), i2 = floor(u2);
  r.I1 = (int)i1;
  r.I2 = (int)i2;
  r.F1d = u1 - i1;
  r.F2d = u2 - i2;
  r.V1d = V1;
  r.V2d = V2;
  r.F1 = (float)r.F1d;
  r.F2 = (float)r.F2d;
  r.V1 = (float)V1;
  r.V2 = (float)V2;
  r.L = (float)(ha * dn / fabs(da));
  // TOF: vh(j) = (tc + bin_hi - t(m0 + j)) / (sigma sqrt2), t(m) = (lam(m) - 1/2) dn
  // (inv_sr2 is 0 without TOF, which zeroes all three coefficients)
  const double t0 = (lam0 + m0 * dlam - 0.5) * dn;
  const double dt = dlam * dn;
  const double edge = (mode == W_BIN) ? 0.5 * g.tof_bin : (g.kmax + 0.5) * g.tof_bin;
  const float A = (float)((tc + edge - t0) * g.inv_sr2);
  const float B = (float)(dt * g.inv_sr2);
  const float D = (float)(2.0 * edge * g.inv_sr2);
  r.A = A;
  r.B = B;
  r.D = D;
  return r;
}

// Hardware reciprocal and base-2 exponential (about 1 ulp) on the GPU; the
// library functions in a CPU build.
__host__ __device__ __forceinline__ float rcp_approx(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
__host__ __device__ __forceinline__ float exp2_approx(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_exp2f(x);
#else
  return exp2f(x);
#endif
}

// erfc(x) for x >= 0: exp(-x^2) times a polynomial of degree 9 in
// t = 1 / (1 + x/2) fitted to erfcx(x) = exp(x^2) erfc(x) on [0, 6]
// (fit_erfcx.py beside this file derives the coefficients and prints the
// error: 1.3e-8 relative for the fit, 3.9e-7 for this float32 evaluation).
// The exponent carries the rounding errors of x^2 and of its product with
// log2(e), so that exp(-x^2) keeps its relative accuracy in the tail, where
// the TOF weights are differences of small erfc values.  Beyond x = 6
// (erfc < 2e-17) t is held at its value at 6.  About 20 instructions
// against some 45 of the library erfcf, which dominated the sample cost.
__host__ __device__ __forceinline__ float erfc_fit(float x) {
  const float t = rcp_approx(fmaf(0.5f, fminf(x, 6.0f), 1.0f));
  float p = -4.066043064e-02f;
  p = fmaf(p, t, 1.858535771e-01f);
  p = fmaf(p, t, -2.580647219e-01f);
  p = fmaf(p, t, -2.349973576e-02f);
  p = fmaf(p, t, 2.209694377e-01f);
  p = fmaf(p, t, 7.137612071e-02f);
  p = fmaf(p, t, 2.880340928e-01f);
  p = fmaf(p, t, 2.728175410e-01f);
  p = fmaf(p, t, 2.832332862e-01f);
  p = fmaf(p, t, -5.917991272e-05f);
  constexpr float kLog2eHi = 1.44269502f;      // log2(e) rounded to float
  constexpr float kLog2eLo = 1.925963e-08f;    // log2(e) - kLog2eHi
  const float hi = x * x;
  const float lo = fmaf(x, x, -hi);
  const float a = hi * kLog2eHi;
  const float da = fmaf(hi, kLog2eHi, -a) + fmaf(hi, kLog2eLo, lo * kLog2eHi);
  return p * (exp2_approx(-a) * fmaf(-da, 0.693147181f, 1.0f));
}

// Integral of the truncated, renormalised Gaussian between the bin edges
// vl < vh (in units of sigma sqrt 2): (erf(vh) - erf(vl)) / (2 erf(vclip))
// after clipping both to [-vclip, vclip], written with erfc of |v| so that
// tails do not cancel.
__host__ __device__ __forceinline__ float tof_weight(float vh, float vl, float vclip, float inv_norm) {
  vh = fminf(fmaxf(vh, -vclip), vclip);
  vl = fminf(fmaxf(vl, -vclip), vclip);
  const float eh = erfc_fit(fabsf(vh));
  const float el = erfc_fit(fabsf(vl));
  // selects rather than branches: el - eh on the positive side, its
  // negation eh - el on the negative side, 2 - el - eh across 0.  The
  // weight of a bin is never negative; where the two erfc values nearly
  // cancel (far tails) the rounding of their difference can be, and is
  // clamped.
  const float d = el - eh;
  const float same = (vl >= 0.0f) ? d : -d;
  const float across = (2.0f - el) - eh;
  const float w = (vl >= 0.0f || vh <= 0.0f) ? same : across;
  return fmaxf(w, 0.0f) * inv_norm;
}

// The weight of one TOF bin as a function of its upper edge vh alone (vl =
// vh - D, D the bin width; units of sigma sqrt 2), tabulated: it is
// inv_norm (erf(clamp(vh)) - erf(clamp(vh - D))) with clamp to [-vc, vc],
// non-zero on (-vc, vc + D) and smooth between the points where an edge
// meets the truncation (-vc, min(-vc + D, vc), max(-vc + D, vc), vc + D).
// Each of the three pieces is cut, from its start, into intervals of width
// exactly 1/64 (a power of two, so that the position (vh - start) * 64 is
// exact in float32; the last interval of a piece runs past its end and
// follows the piece's own smooth expression there) with a cubic Hermite
// interpolant of the exact values and derivatives (error below h^4 max |4th
// derivative| / 384, about 1e-9 of the peak weight; the float32
// coefficients and evaluation add about 1e-7).  Evaluating it is an LDS
// read and three FMAs instead of two erfc.  The table is built per geometry
// by build_tof_table.
constexpr int kTofTabMax = 1024;  // intervals
constexpr int kTofTabPerUnit = 64;

struct TofTab {
  float b0, b1, b2, b3;  // piece boundaries
  int n0, n1, n2;        // intervals of each piece (piece 1 starts at n0, piece 2 at n0 + n1)
};

// The table layout of a geometry with TOF (host).
inline TofTab tof_tab_layout(const GeomDev &g) {
  const double vc = (g.half_win - 0.5 * g.tof_bin) * g.inv_sr2, D = g.tof_bin * g.inv_sr2;
  const double c[4] = {-vc, fmin(-vc + D, vc), fmax(-vc + D, vc), vc + D};
  TofTab t;
  t.b0 = (float)c[0];
  t.b1 = (float)c[1];
  t.b2 = (float)c[2];
  t.b3 = (float)c[3];
  const float b[4] = {t.b0, t.b1, t.b2, t.b3};
  int n[3];
  for (int p = 0; p < 3; ++p) {
    const double w = (double)b[p + 1] - (double)b[p];
    n[p] = w > 0.0 ? (int)ceil(w * kTofTabPerUnit) : 1;
  }
  t.n0 = n[0];
  t.n1 = n[1];
  t.n2 = n[2];
  return t;
}

// The table layout held in registers, uniform over the wavefront (the
// evaluation selects among its fields per lane; with the struct in kernel
// argument memory the compiler would load the selected field per lane).
__device__ __forceinline__ TofTab tof_tab_uniform(const TofTab &t) {
  TofTab u;
  u.b0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(t.b0)));
  u.b1 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(t.b1)));
  u.b2 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(t.b2)));
  u.b3 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(t.b3)));
  u.n0 = __builtin_amdgcn_readfirstlane(t.n0);
  u.n1 = __builtin_amdgcn_readfirstlane(t.n1);
  u.n2 = __builtin_amdgcn_readfirstlane(t.n2);
  return u;
}

__host__ __device__ __forceinline__ int tof_tab_size(const TofTab &t) { return t.n0 + t.n1 + t.n2; }

// The tabulated weight at vh (0 outside (b0, b3)); tab: the coefficients
// {c0, c1, c2, c3} of c0 + s (c1 + s (c2 + s c3)) of every interval, s in
// [0, 1) the position inside the interval.
__device__ __forceinline__ float tof_weight_tab(const TofTab &t, const float4 *tab, float vh) {
  const bool p2 = vh >= t.b2, p1 = vh >= t.b1;
  const float start = p2 ? t.b2 : (p1 ? t.b1 : t.b0);
  const int base = p2 ? t.n0 + t.n1 : (p1 ? t.n0 : 0);
  const int nmax = p2 ? t.n2 : (p1 ? t.n1 : t.n0);
  const float u = (vh - start) * (float)kTofTabPerUnit;
  const int i = min(max((int)u, 0), nmax - 1);
  const float s = u - (float)i;
  const float4 c = tab[base + i];
  const float w = fmaf(fmaf(fmaf(c.w, s, c.z), s, c.y), s, c.x);
  // near the ends of the support the cubic of a weight that falls to 0 can
  // round below it
  return (vh > t.b0 && vh < t.b3) ? fmaxf(w, 0.0f) : 0.0f;
}

// One sample of a ray: plane, lower corner and weights.
struct Sample {
  int m;        // plane along the dominant axis
  int i1, i2;   // lower corner along the two other axes (may be out of range)
  float f1, f2; // fractional parts
  float w;      // TOF weight (1 without TOF); 0 = no sample
};

__host__ __device__ __forceinline__ Sample sample_at(const GeomDev &g, const Ray &r, int j, int tof_on) {
  Sample s;
  const float u1 = fmaf((float)j, r.V1, r.F1);
  const float u2 = fmaf((float)j, r.V2, r.F2);
  const float fl1 = floorf(u1), fl2 = floorf(u2);
  s.f1 = u1 - fl1;
  s.f2 = u2 - fl2;
  s.i1 = r.I1 + (int)fl1;
  s.i2 = r.I2 + (int)fl2;
  s.m = r.m0 + j;
  if (tof_on) {
    const float vh = fmaf(-(float)j, r.B, r.A);
    s.w = tof_weight(vh, vh - r.D, g.vclip, g.inv_norm);
  } else {
    s.w = 1.0f;
  }
  return s;
}

// Index of voxel (plane m, u1, u2) of a ray with dominant axis a.
__host__ __device__ __forceinline__ int ray_vidx(const Layout &L, int a, int m, int u1, int u2) {
  const int i = (a == 0) ? m : u1;
  const int j = (a == 0) ? u1 : ((a == 1) ? m : u2);
  const int k = (a == 2) ? m : u2;
  return vidx(L, i, j, k);
}

// Corner c (bit 0: +1 along the first other axis, bit 1: along the second)
// of a sample: its voxel index, or -1 outside the image, and its bilinear
// weight.
__host__ __device__ __forceinline__ int corner(const GeomDev &g, const Ray &r, const Sample &s, int c,
                                               float &wc) {
  const int u1 = s.i1 + (c & 1), u2 = s.i2 + (c >> 1);
  wc = ((c & 1) ? s.f1 : 1.0f - s.f1) * ((c & 2) ? s.f2 : 1.0f - s.f2);
  if ((unsigned)u1 >= (unsigned)r.n1 || (unsigned)u2 >= (unsigned)r.n2) return -1;
  return ray_vidx(g.lay, r.a, s.m, u1, u2);
}

// Bilinear gather of a sample (corners outside the image read as zero).
__host__ __device__ __forceinline__ float gather(const GeomDev &g, const float *__restrict__ img, const Ray &r,
                                                 const Sample &s) {
  float v[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float wc;
    const int ix = corner(g, r, s, c, wc);
    v[c] = (ix >= 0) ? img[ix] : 0.0f;
  }
  const float lo = fmaf(s.f1, v[1] - v[0], v[0]);
  const float hi = fmaf(s.f1, v[3] - v[2], v[2]);
  return fmaf(s.f2, hi - lo, lo);
}

// A voxel index of a layout is a sum of one term per axis: with brick
// coordinate c >> s and position c & mask inside the brick,
// vidx(L, i, j, k) = term(i) + term(j) + term(k), term(c) = (c >> s) * bs +
// ((c & mask) << w), bs the stride of one brick along the axis (in voxels)
// and w the in-brick shift.  The gathers below add the terms of the two
// other axes to the dominant axis' term; a corner one voxel further along an
// axis adds that axis' `step`, or `wrap` when it crosses into the next brick.
struct AxisTerm {
  int s, mask, w, bs;
  int step, wrap;
};

__host__ __device__ __forceinline__ AxisTerm axis_term(const Layout &L, int axis) {
  AxisTerm t;
  t.s = sel3(axis, L.sx, L.sy, L.sz);
  t.mask = (1 << t.s) - 1;
  t.w = sel3(axis, 0, L.sx, L.sx + L.sy);
  t.bs = sel3(axis, 1, L.nbx, L.nbx * L.nby) << (L.sx + L.sy + L.sz);
  t.step = 1 << t.w;
  t.wrap = t.bs - (t.mask << t.w);
  return t;
}

// term(c) for c >= 0.  Both factors stay below 2^24 for images of up to
// kMaxDim voxels per axis, so the product takes the 24-bit multiply.
__host__ __device__ __forceinline__ int axis_index(const AxisTerm &t, int c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return (int)__umul24((unsigned)(c >> t.s), (unsigned)t.bs) + ((c & t.mask) << t.w);
#else
  return (c >> t.s) * t.bs + ((c & t.mask) << t.w);
#endif
}

// Bilinear gather at plane term `fa` and lower corner (i1, i2) with
// fractions (f1, f2); the same values as gather() (corners outside the
// image read as zero), without branches: every corner is loaded, from
// voxel 0 in place of one outside the image, and its value selected.
__device__ __forceinline__ float gather_terms(const float *__restrict__ img, const AxisTerm &t1, const AxisTerm &t2,
                                              int n1, int n2, int fa, int i1, int i2, float f1, float f2) {
  const bool a0 = (unsigned)i1 < (unsigned)n1, a1 = (unsigned)(i1 + 1) < (unsigned)n1;
  const bool b0 = (unsigned)i2 < (unsigned)n2, b1 = (unsigned)(i2 + 1) < (unsigned)n2;
  const int j1 = max(i1, 0), j2 = max(i2, 0);
  // from corner 0 to the next voxel along each axis (corner 0 at -1: the
  // next one is voxel 0 itself)
  const int d1 = (i1 < 0) ? 0 : (((j1 & t1.mask) == t1.mask) ? t1.wrap : t1.step);
  const int d2 = (i2 < 0) ? 0 : (((j2 & t2.mask) == t2.mask) ? t2.wrap : t2.step);
  const int base = fa + axis_index(t1, j1) + axis_index(t2, j2);
  const float x0 = img[(a0 && b0) ? base : 0];
  const float x1 = img[(a1 && b0) ? base + d1 : 0];
  const float x2 = img[(a0 && b1) ? base + d2 : 0];
  const float x3 = img[(a1 && b1) ? base + d1 + d2 : 0];
  const float v0 = (a0 && b0) ? x0 : 0.0f, v1 = (a1 && b0) ? x1 : 0.0f;
  const float v2 = (a0 && b1) ? x2 : 0.0f, v3 = (a1 && b1) ? x3 : 0.0f;
  const float lo = fmaf(f1, v1 - v0, v0);
  const float hi = fmaf(f1, v3 - v2, v2);
  return fmaf(f2, hi - lo, lo);
}

// Kernels that scatter start their lanes at the brick boundary at or below
// a ray's first plane: lane l of chunk c takes plane offset
// j = 64 c + l - brick_offset, so that the 16-plane rounds of the
// interleaved scatter cover whole bricks along the dominant axis and a
// memory sector is hit by one atomic instruction only (the 3D data update of
// 4.5e4 events: 129 -> 120 us, its atomic requests at the same rate).  Bricks have
// at most 4 voxels per axis, so the offset is at most kMaxBrickOffset and
// the plane clamp of such kernels leaves room for it.
constexpr int kMaxBrickOffset = 3;

__host__ __device__ __forceinline__ int brick_offset(const Layout &L, const Ray &r) {
  const int s = sel3(r.a, L.sx, L.sy, L.sz);
  return r.m0 & ((1 << s) - 1) & kMaxBrickOffset;
}

// Scatter of one sample per lane of a full 64-lane wavefront with the
// corners interleaved: the four corner contributions of every lane are
// staged in LDS and issued as four atomic instructions, each covering the 4
// corners of 16 consecutive planes, which sit in few bricks.  All 64 lanes
// must call it; lanes without a sample pass c = 0 exactly (their sample may
// name a plane outside the image, so a non-zero c there would write out of
// bounds).  sidx / sval point to this wavefront's 256 slots of index and
// value.
__device__ __forceinline__ void scatter_interleaved(const GeomDev &g, float *img, const Ray &r, const Sample &s,
                                                    float c, int lane, int *sidx, float *sval) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float wc;
    const int ix = corner(g, r, s, q, wc);
    const bool on = (c != 0.0f) && (ix >= 0) && (wc != 0.0f);
    sidx[4 * lane + q] = on ? ix : -1;
    sval[4 * lane + q] = c * wc;
  }
  // LDS operations of one wavefront complete in order; the fences keep the
  // compiler from moving the reads above the writes
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    // round q takes slots 64 q .. 64 q + 63: the 4 corners of planes
    // 16 q .. 16 q + 15, consecutive lanes on the corners of one plane
    const int slot = 64 * q + lane;
    const int ix = sidx[slot];
    if (ix >= 0) atomicAdd(img + ix, sval[slot]);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over the LPE lanes of a group (all lanes receive the total).
template <int LPE>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int o = LPE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, LPE);
  return v;
}

// Crystal ids and TOF bin of a caller event int16[5]; false if out of range.
__host__ __device__ __forceinline__ bool decode_event(const GeomDev &g, const int16_t *ev, int &id1, int &id2,
                                                      int &k) {
  const int c1 = ev[0], r1 = ev[1], c2 = ev[2], r2 = ev[3];
  k = ev[4];
  if ((unsigned)c1 >= (unsigned)g.n_cry || (unsigned)c2 >= (unsigned)g.n_cry) return false;
  if ((unsigned)r1 >= (unsigned)g.n_ring || (unsigned)r2 >= (unsigned)g.n_ring) return false;
  if (k < -g.kmax || k > g.kmax) return false;
  id1 = c1 + g.n_cry * r1;
  id2 = c2 + g.n_cry * r2;
  return true;
}


// ---------------------------------------------------------------------------
// The per-event forward walk of the projector kernels.

// A ray as the lanes of a group of the forward walk read it: plane range,
// axis and integer parts, the TOF coefficients and plane length, and the
// interpolation coordinates in double.  In float32, F + j V of a plane a
// few hundred planes from the first carries an error of up to 3e-5 voxel
// (one unit in the last place near 300), which a LOR that grazes an edge of
// the activity turns into a relative error of that order; the forward
// projector is bound by its memory instructions, not by its arithmetic, so
// its coordinates take double precision.
struct RayPack {
  int4 p;     // {m0, nplanes, a, I1}
  int4 q;     // {I2, bits of A, B, L}
  double2 u1; // {F1, V1}
  double2 u2; // {F2, V2}
};

// One sample of the forward walk: {weight, interpolated value} at plane
// offset j (weight 0 for j < 0), plane term fa.
template <bool TOF>
__device__ __forceinline__ float2 fwd_sample(const GeomDev &g, const float *__restrict__ x, const AxisTerm &t1,
                                            const AxisTerm &t2, int n1, int n2, const RayPack &pk, float A, float B,
                                            float D, int j, int fa) {
  const double u1 = fma((double)j, pk.u1.y, pk.u1.x), u2 = fma((double)j, pk.u2.y, pk.u2.x);
  const double fl1 = floor(u1), fl2 = floor(u2);
  // the loads first: the TOF weight's arithmetic then runs while they are
  // in flight
  const float v = gather_terms(x, t1, t2, n1, n2, fa, pk.p.w + (int)fl1, pk.q.x + (int)fl2, (float)(u1 - fl1),
                               (float)(u2 - fl2));
  float w = 1.0f;
  if constexpr (TOF) {
    const float vh = fmaf(-(float)j, B, A);
    w = tof_weight(vh, vh - D, g.vclip, g.inv_norm);
  }
  return make_float2((j >= 0) ? w : 0.0f, v);
}

// The planes of one event for lane gl of its group: m0 + j for j = gl -
// (brick offset of m0), + 8, ...  Returns the lane's weighted sum.
template <bool TOF>
__device__ __forceinline__ float fwd_walk(const GeomDev &g, const float *__restrict__ x, const RayPack &pk,
                                          float D, int gl) {
  const int np = pk.p.y, m0 = pk.p.x, a = pk.p.z;
  const float A = __int_as_float(pk.q.y), B = __int_as_float(pk.q.z);
  const int b1 = (a == 0) ? 1 : 0, b2 = (a == 2) ? 1 : 2;
  const AxisTerm ta = axis_term(g.lay, a), t1 = axis_term(g.lay, b1), t2 = axis_term(g.lay, b2);
  const int n1 = sel3(b1, g.n[0], g.n[1], g.n[2]), n2 = sel3(b2, g.n[0], g.n[1], g.n[2]);
  int j = gl - (m0 & ta.mask & kMaxBrickOffset);
  // plane term of m0 + j (>= 0: the offset stays inside m0's brick),
  // advanced by whole bricks, 8 planes at a time
  int fa = axis_index(ta, m0 + j);
  const int fa_step = (8 >> ta.s) * ta.bs;
  float acc = 0.0f;
  for (; j < np; j += 8, fa += fa_step) {
    const float2 s = fwd_sample<TOF>(g, x, t1, t2, n1, n2, pk, A, B, D, j, fa);
    acc = fmaf(s.x, s.y, acc);
  }
  return acc;
}

__device__ __forceinline__ RayPack pack_ray(const Ray &r) {
  RayPack pk;
  pk.p = make_int4(r.m0, r.nplanes, r.a, r.I1);
  pk.q = make_int4(r.I2, __float_as_int(r.A), __float_as_int(r.B), __float_as_int(r.L));
  pk.u1 = make_double2(r.F1d, r.V1d);
  pk.u2 = make_double2(r.F2d, r.V2d);
  return pk;
}

__device__ __forceinline__ RayPack empty_ray() {
  RayPack pk;
  pk.p = make_int4(0, 0, 0, 0);
  pk.q = make_int4(0, 0, 0, 0);
  pk.u1 = make_double2(0.0, 0.0);
  pk.u2 = make_double2(0.0, 0.0);
  return pk;
}

// D of a single TOF bin as setup_ray computes it.
__host__ __device__ __forceinline__ float tof_bin_width(const GeomDev &g) {
  return (float)(2.0 * (0.5 * g.tof_bin) * g.inv_sr2);
}

}  // namespace lmk
