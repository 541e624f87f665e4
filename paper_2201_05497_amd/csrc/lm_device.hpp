// Device core of the listmode TOF Joseph projector (gfx950).
//
// One event is handled by a group of LPE lanes (LPE = 16, 32 or 64) of a
// 64-wide wavefront; the lanes of a group walk the image planes of the
// event's line of response, lane l taking planes m0 + l, m0 + l + LPE, ...
// For a LOR whose dominant axis is x, consecutive lanes then read
// consecutive x addresses, so the gathers of a group are coalesced along the
// fastest image axis.
//
// The per-event set-up (dominant axis, plane range, interpolation and TOF
// coefficients) is done in double precision, once per event.  The
// per-sample arithmetic is float32 and works on small numbers only: the
// interpolation coordinate of a sample is written as an integer part fixed
// per event plus F + j*V with j the plane offset inside the event's range,
// and the TOF argument as A - j*B, so float32 rounding stays at the 1e-6
// level of a voxel or a TOF sigma.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lmk {

// The functions below except scatter and group_sum are __host__ __device__
// so that the projector can also be exercised by a CPU build.

// Geometry in the form the kernels use (built on the host from lm_geom).
struct GeomDev {
  const float *det;  // [n_det][3]
  int n_cry, n_ring, n_det;
  int n[3];          // nx, ny, nz
  int stride[3];     // 1, nx, nx*ny
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
  int sa, s1, s2;    // voxel strides of the dominant axis and the two others
  int n1, n2;        // image size along the two other axes
  int I1, I2;        // integer parts of the interpolation coordinates at m0
  float F1, V1, F2, V2;  // u_b(m0 + j) = I_b + F_b + j V_b
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
  r.m0 = r.sa = r.s1 = r.s2 = r.n1 = r.n2 = r.I1 = r.I2 = 0;
  r.F1 = r.V1 = r.F2 = r.V2 = r.A = r.B = r.D = r.L = 0.0f;
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
  if (np > max_planes) np = max_planes;  // never reached for a valid plan bound
  r.nplanes = np;
  r.m0 = m0;
  r.sa = sel3(a, g.stride[0], g.stride[1], g.stride[2]);
  r.s1 = sel3(b1, g.stride[0], g.stride[1], g.stride[2]);
  r.s2 = sel3(b2, g.stride[0], g.stride[1], g.stride[2]);
  r.n1 = nb1;
  r.n2 = nb2;
  const double u1 = U1 + m0 * V1, u2 = U2 + m0 * V2;
  const double i1 = floor(u1), i2 = floor(u2);
  r.I1 = (int)i1;
  r.I2 = (int)i2;
  r.F1 = (float)(u1 - i1);
  r.F2 = (float)(u2 - i2);
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

// Integral of the truncated, renormalised Gaussian between the bin edges
// vl < vh (in units of sigma sqrt 2): (erf(vh) - erf(vl)) / (2 erf(vclip))
// after clipping both to [-vclip, vclip], written with erfc of |v| so that
// tails do not cancel.
__host__ __device__ __forceinline__ float tof_weight(float vh, float vl, float vclip, float inv_norm) {
  vh = fminf(fmaxf(vh, -vclip), vclip);
  vl = fminf(fmaxf(vl, -vclip), vclip);
  const float eh = erfcf(fabsf(vh));
  const float el = erfcf(fabsf(vl));
  float w;
  if (vl >= 0.0f)
    w = el - eh;
  else if (vh <= 0.0f)
    w = eh - el;
  else
    w = 2.0f - el - eh;
  return w * inv_norm;
}

// One sample of a ray: voxel index of the lower corner and the weights.
struct Sample {
  int base;     // index of corner (i1, i2) in plane m (may be out of range)
  int i1, i2;   // corner indices along the two other axes
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
  s.base = (r.m0 + j) * r.sa + s.i1 * r.s1 + s.i2 * r.s2;
  if (tof_on) {
    const float vh = fmaf(-(float)j, r.B, r.A);
    s.w = tof_weight(vh, vh - r.D, g.vclip, g.inv_norm);
  } else {
    s.w = 1.0f;
  }
  return s;
}

// Bilinear gather of a sample (corners outside the image read as zero).
__host__ __device__ __forceinline__ float gather(const float *__restrict__ img, const Ray &r, const Sample &s) {
  const bool a0 = (unsigned)s.i1 < (unsigned)r.n1;
  const bool a1 = (unsigned)(s.i1 + 1) < (unsigned)r.n1;
  const bool b0 = (unsigned)s.i2 < (unsigned)r.n2;
  const bool b1 = (unsigned)(s.i2 + 1) < (unsigned)r.n2;
  float v00 = (a0 && b0) ? img[s.base] : 0.0f;
  float v10 = (a1 && b0) ? img[s.base + r.s1] : 0.0f;
  float v01 = (a0 && b1) ? img[s.base + r.s2] : 0.0f;
  float v11 = (a1 && b1) ? img[s.base + r.s1 + r.s2] : 0.0f;
  const float lo = fmaf(s.f1, v10 - v00, v00);
  const float hi = fmaf(s.f1, v11 - v01, v01);
  return fmaf(s.f2, hi - lo, lo);
}

// Bilinear scatter-add of c into the four corners.
__device__ __forceinline__ void scatter(float *img, const Ray &r, const Sample &s, float c) {
  const bool a0 = (unsigned)s.i1 < (unsigned)r.n1;
  const bool a1 = (unsigned)(s.i1 + 1) < (unsigned)r.n1;
  const bool b0 = (unsigned)s.i2 < (unsigned)r.n2;
  const bool b1 = (unsigned)(s.i2 + 1) < (unsigned)r.n2;
  const float g1 = 1.0f - s.f1, g2 = 1.0f - s.f2;
  if (a0 && b0) atomicAdd(img + s.base, c * g1 * g2);
  if (a1 && b0) atomicAdd(img + s.base + r.s1, c * s.f1 * g2);
  if (a0 && b1 && s.f2 != 0.0f) atomicAdd(img + s.base + r.s2, c * g1 * s.f2);
  if (a1 && b1 && s.f2 != 0.0f) atomicAdd(img + s.base + r.s1 + r.s2, c * s.f1 * s.f2);
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

}  // namespace lmk
