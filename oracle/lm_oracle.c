/*
 * FP64 reference implementation ("oracle") of the listmode time-of-flight
 * Joseph projector pair and the sensitivity image.
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU
 * baseline of the benchmark are the only users of this file.  It shares no
 * code, header or table with the HIP library, and nothing in the library
 * calls it.  Everything is plain single-threaded double precision.
 *
 * What is computed (paper: listmode operator, Eq. (lmop): the listmode
 * forward operator evaluates row i_e of P for every event e; the system
 * model is a Joseph ray tracer with a Gaussian TOF kernel, Section 2,
 * "Listmode SPDHG", the paragraph on the GPU Joseph projectors).  The paper
 * fixes neither the ray tracer's details nor the TOF kernel; the readings
 * taken here are:
 *
 *  - Scanner: a float32 table det[id][3] of crystal centres (id = c +
 *    n_cry*r) is the scanner description; values are promoted to double.
 *  - Event e = (c1, r1, c2, r2, k).  The LOR is q(lam) = p1 + lam*d with
 *    p1 = det[id1], p2 = det[id2], d = p2 - p1 (exact in double), lam in
 *    [0, 1].
 *  - Joseph: dominant axis a = argmax_b |d_b|, decided on the float32
 *    round-to-nearest differences fl(p2_b - p1_b) with ties going to the
 *    lower axis (x < y < z).  This integer decision is taken in float32 so
 *    that a float32 implementation takes exactly the same one; fl(-v) =
 *    -fl(v) keeps it invariant under swapping the crystals.  For every
 *    image plane m = 0..N_a-1 perpendicular to a with centre coordinate
 *    c_a(m), lam_m = (c_a(m) - p1_a)/d_a; planes with lam
 *    outside [0, 1] are skipped.  In the plane, the image is interpolated
 *    bilinearly over the two other axes at q(lam_m); a corner outside the
 *    image contributes zero.  Every sample is weighted by the plane length
 *    L = h_a |d| / |d_a|.
 *  - TOF: t_m = (lam_m - 1/2)|d| is the signed distance from the LOR centre,
 *    positive towards crystal 2.  Bin k has centre k*Delta and width Delta.
 *    The kernel is a Gaussian of the given FWHM truncated at nsig*sigma and
 *    renormalised to unit mass; w_k(t) is its integral over bin k:
 *        w_k(t) = max(0, erf(min(u_hi, nsig)/sqrt2) - erf(max(u_lo, -nsig)/sqrt2))
 *                 / (2 erf(nsig/sqrt2)),
 *        u_hi = (k*Delta + Delta/2 - t)/sigma, u_lo = (k*Delta - Delta/2 - t)/sigma.
 *    With TOF switched off w == 1.
 *  - (P x)_e = L * sum_m w_k(t_m) * bilinear(x, q(lam_m)).
 *  - Sensitivity g = P^T 1 over every unordered crystal pair and every TOF
 *    bin (Section 2, the remarks on the initialisation of z and the step
 *    sizes T: g is one back projection of a sinogram of ones).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  const float *det; /* [n_cry*n_ring][3] crystal centres, mm */
  int32_t n_cry, n_ring;
  int32_t n[3];     /* image size nx, ny, nz (x fastest in memory) */
  double h[3];      /* voxel size, mm */
  int32_t n_tof;    /* odd number of TOF bins */
  double tof_bin;   /* Delta, mm */
  double tof_fwhm;  /* mm */
  double tof_nsig;  /* truncation, in sigma */
  int32_t tof_on;
} orc_geom;

static double tof_sigma(const orc_geom *g) {
  return g->tof_fwhm / (2.0 * sqrt(2.0 * log(2.0)));
}

/* Weight of TOF bin k for a point at signed distance t from the LOR centre. */
double orc_tof_weight(const orc_geom *g, int k, double t) {
  const double sig = tof_sigma(g), ns = g->tof_nsig, r2 = sqrt(2.0);
  const double ck = k * g->tof_bin;
  double u_hi = (ck + 0.5 * g->tof_bin - t) / sig;
  double u_lo = (ck - 0.5 * g->tof_bin - t) / sig;
  double hi = erf(fmin(u_hi, ns) / r2);
  double lo = erf(fmax(u_lo, -ns) / r2);
  double w = hi - lo;
  if (w < 0.0) w = 0.0;
  return w / (2.0 * erf(ns / r2));
}

/* mode for the per-sample weight */
enum { W_BIN = 0, W_ALL_BINS = 1 };

/*
 * Trace one LOR.  If x != NULL the forward value is returned; if img != NULL,
 * v * (row of P) is added into img.
 */
static double trace(const orc_geom *g, int id1, int id2, int k, int wmode,
                    const double *x, double v, double *img) {
  const float *f1 = g->det + 3 * (int64_t)id1;
  const float *f2 = g->det + 3 * (int64_t)id2;
  double p1[3], d[3];
  float df[3];
  for (int b = 0; b < 3; ++b) {
    volatile float diff = f2[b] - f1[b]; /* float32 subtraction, RN */
    df[b] = diff;
    p1[b] = (double)f1[b];
    d[b] = (double)f2[b] - (double)f1[b];
  }
  int a = 0;
  if (fabsf(df[1]) > fabsf(df[a])) a = 1;
  if (fabsf(df[2]) > fabsf(df[a])) a = 2;
  if (df[a] == 0.0f || d[a] == 0.0) return 0.0; /* degenerate LOR */
  const int b1 = (a == 0) ? 1 : 0;
  const int b2 = (a == 2) ? 1 : 2;
  const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double L = g->h[a] * dn / fabs(d[a]);
  const int na = g->n[a], n1 = g->n[b1], n2 = g->n[b2];
  const double c01 = -0.5 * (n1 - 1) * g->h[b1];
  const double c02 = -0.5 * (n2 - 1) * g->h[b2];
  const int kmax = (g->n_tof - 1) / 2;
  double acc = 0.0;
  for (int m = 0; m < na; ++m) {
    const double ca = (m - 0.5 * (na - 1)) * g->h[a];
    const double lam = (ca - p1[a]) / d[a];
    if (lam < 0.0 || lam > 1.0) continue;
    const double t = (lam - 0.5) * dn;
    double w;
    if (!g->tof_on) {
      w = 1.0;
    } else if (wmode == W_BIN) {
      w = orc_tof_weight(g, k, t);
    } else {
      w = 0.0;
      for (int kk = -kmax; kk <= kmax; ++kk) w += orc_tof_weight(g, kk, t);
    }
    if (w == 0.0) continue;
    const double u1 = (p1[b1] + lam * d[b1] - c01) / g->h[b1];
    const double u2 = (p1[b2] + lam * d[b2] - c02) / g->h[b2];
    const double i1f = floor(u1), i2f = floor(u2);
    const double f1w = u1 - i1f, f2w = u2 - i2f;
    const long i1 = (long)i1f, i2 = (long)i2f;
    for (int s2 = 0; s2 < 2; ++s2) {
      const long j2 = i2 + s2;
      if (j2 < 0 || j2 >= n2) continue;
      const double w2 = s2 ? f2w : 1.0 - f2w;
      for (int s1 = 0; s1 < 2; ++s1) {
        const long j1 = i1 + s1;
        if (j1 < 0 || j1 >= n1) continue;
        const double w1 = s1 ? f1w : 1.0 - f1w;
        long ix[3];
        ix[a] = m;
        ix[b1] = j1;
        ix[b2] = j2;
        const long vox = ix[0] + (long)g->n[0] * (ix[1] + (long)g->n[1] * ix[2]);
        const double cw = w * w1 * w2;
        if (x) acc += cw * x[vox];
        if (img) img[vox] += L * cw * v;
      }
    }
  }
  return L * acc;
}

static void ids(const orc_geom *g, const int16_t *ev, int *id1, int *id2, int *k) {
  *id1 = ev[0] + g->n_cry * ev[1];
  *id2 = ev[2] + g->n_cry * ev[3];
  *k = ev[4];
}

/* out[e] = (P^LM x)_e for n events. */
void orc_fwd(const orc_geom *g, const double *x, const int16_t *ev, int64_t n, double *out) {
  for (int64_t e = 0; e < n; ++e) {
    int id1, id2, k;
    ids(g, ev + 5 * e, &id1, &id2, &k);
    out[e] = trace(g, id1, id2, k, W_BIN, x, 0.0, NULL);
  }
}

/* img += (P^LM)^T v for n events. */
void orc_back(const orc_geom *g, const double *v, const int16_t *ev, int64_t n, double *img) {
  for (int64_t e = 0; e < n; ++e) {
    int id1, id2, k;
    ids(g, ev + 5 * e, &id1, &id2, &k);
    trace(g, id1, id2, k, W_BIN, NULL, v[e], img);
  }
}

/* g += P^T 1 summed over every unordered crystal pair id1 < id2 and every
 * TOF bin (for each sample the weights of all bins are summed). */
void orc_sens(const orc_geom *g, double *img) {
  const int nd = g->n_cry * g->n_ring;
  for (int i1 = 0; i1 < nd; ++i1)
    for (int i2 = i1 + 1; i2 < nd; ++i2)
      trace(g, i1, i2, 0, W_ALL_BINS, NULL, 1.0, img);
}
