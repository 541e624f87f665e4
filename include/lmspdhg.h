/*
 * lmspdhg.h -- C ABI of the MI355X (gfx950) listmode SPDHG library.
 *
 * The library solves the Poisson problem of the paper's Eq. (1),
 *     argmin_{x >= 0}  sum_i (Px+s)_i - d_i log (Px+s)_i  +  beta ||Kx||_{2,1},
 * event by event (listmode), with the stochastic primal-dual algorithm
 * LM-SPDHG (Algorithm 2).  P is a time-of-flight Joseph projector, K the
 * forward-difference gradient (Section 3, the TV prior).
 *
 * Conventions for every call:
 *  - Array arguments are DEVICE pointers owned by the caller unless marked
 *    "host".  The library never frees caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls only enqueue work on it unless marked "synchronous".
 *  - Every call returns LM_OK (0) or a negative error code; a thread-local
 *    message is available from lm_last_error().  No C++ exception crosses
 *    the ABI.  On an error return nothing has been enqueued.
 *  - Images are float32, C-order [z][y][x] (x fastest), voxel (i, j, k)
 *    centred at ((i-(nx-1)/2) hx, (j-(ny-1)/2) hy, (k-(nz-1)/2) hz) mm.
 *  - An event is int16[5] = (c1, r1, c2, r2, k): crystal c1 of ring r1,
 *    crystal c2 of ring r2, signed TOF bin k with |k| <= (n_tof-1)/2 (the
 *    paper's 10-byte event, Table 1).  The crystal id is c + n_cry * r.
 *    Events with an out-of-range id or TOF bin contribute nothing to any
 *    projection (their forward value is 0); lm_validate_events reports them
 *    and lm_plan_create rejects them.
 *
 * The projector (the paper specifies only "Joseph" and a Gaussian TOF
 * kernel; Section 2, "Listmode SPDHG", and Section 3):
 *  - the LOR of an event runs from p1 = det[id1] to p2 = det[id2];
 *  - Joseph: dominant axis a = argmax_b |fl32(p2_b - p1_b)| (ties to the
 *    lower axis x < y < z); one sample per image plane perpendicular to a
 *    with the LOR parameter lam in [0, 1]; bilinear interpolation over the
 *    two other axes (corners outside the image count as zero); each sample
 *    weighted by the plane length h_a |p2-p1| / |p2_a - p1_a|;
 *  - TOF: t = signed distance of the sample from the LOR centre, positive
 *    towards p2; bin k is centred at k*tof_bin with width tof_bin; the
 *    kernel is a Gaussian of FWHM tof_fwhm truncated at tof_nsigma sigmas,
 *    renormalised to unit mass, integrated over the bin.  tof_on = 0 gives
 *    the non-TOF projector (weight 1).
 */
#ifndef LMSPDHG_H
#define LMSPDHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LM_OK = 0,
  LM_EINVAL = -1, /* bad shape, size or parameter */
  LM_ERANGE = -2, /* crystal, ring or TOF index out of range; an event factor <= 0 */
  LM_ENOMEM = -3, /* device allocation failed */
  LM_EHIP = -4,   /* a HIP runtime call failed (message has the HIP text) */
  LM_ESTATE = -5  /* plan used before lm_spdhg_init, or inconsistent state */
};

/* Scanner, image grid and TOF model.  `det` is a DEVICE pointer to
 * float[n_cry * n_ring][3] crystal centres in mm (id = c + n_cry * r); it
 * must stay valid while calls that use this geometry run.  The scalars are
 * double: the per-event set-up of the projector runs in double precision,
 * and a float voxel size (2.6f != 2.6) would shift the grid by ~1e-5 mm at
 * the image edge. */
typedef struct lm_geom {
  const float *det;
  int32_t n_cry, n_ring;
  int32_t n[3];      /* image size nx, ny, nz (each 1..512) */
  double h[3];       /* voxel size in mm */
  int32_t n_tof;     /* odd number of TOF bins (>= 1) */
  double tof_bin;    /* TOF bin width, mm */
  double tof_fwhm;   /* Gaussian FWHM, mm */
  double tof_nsigma; /* truncation in sigmas (> 0) */
  int32_t tof_on;    /* 0: non-TOF projector */
} lm_geom;

/* Thread-local text of the last error of this thread ("" if none). */
const char *lm_last_error(void);

/* ---------------------------------------------------------------- projector */

/* Images passed to the projector calls are row-major float[nz][ny][nx]
 * device arrays.  Each call copies the image into a temporary in the
 * library's 4x4x4-voxel brick layout (stream-ordered hipMallocAsync on
 * `stream`, freed stream-ordered before the call returns; LM_ENOMEM if it
 * cannot be allocated), runs on the copy, and for lm_back / lm_sens writes
 * the result back.  All work is queued on `stream` (NULL: the default
 * stream); the calls do not synchronise. */

/* Listmode forward projection (Eq. lmop): out[e] = (P^LM x)_e for the n
 * events ev[n][5] in the caller's order.  x: image; out: float[n].  Events
 * that are out of range get out[e] = 0.  On a cylindrical scanner (as for
 * lm_back, decided on the device) a list of at least 64 events per
 * transaxial crystal pair and fewer than 2^31 events is projected by
 * transaxial line after a counting sort on the device: 24 more bytes per
 * event of stream-ordered temporary memory (without room for it the events
 * are projected in their own order).  The result is the same up to float32
 * rounding in either order.  The call never synchronises the stream. */
int lm_fwd(const lm_geom *G, const float *x, const int16_t *ev, int64_t n, float *out,
           void *stream);

/* lm_fwd for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result as lm_fwd, but the bricked copy of x goes to a scratch
 * array that the library holds in every device's memory from the moment
 * its code is loaded there until the process ends (64 MiB per device), so
 * the call allocates nothing.  LM_EINVAL when the image needs more than
 * 2^24 floats in the 4x4x4 brick layout (e.g. beyond 512 x 512 x 64 voxels),
 * when `stream` belongs to a device other than the current one, or for the
 * arguments lm_fwd rejects.  Every call on a device shares its scratch:
 * calls that overlap on one device (other streams, other host threads)
 * race, and the caller must order them. */
int lm_fwd_noalloc(const lm_geom *G, const float *x, const int16_t *ev, int64_t n, float *out,
                   void *stream);

/* Listmode back projection, the adjoint of lm_fwd: img += (P^LM)^T v.  It
 * ACCUMULATES (FP32 atomics, so the summation order is not fixed); the
 * caller zeroes img.  v: float[n].  Events that are out of range or have
 * v = 0 contribute nothing.  On a cylindrical scanner (crystal c of ring r
 * at (x_c, y_c, z_r), z increasing with r) a list of at least 64 events per
 * transaxial crystal pair is back projected by transaxial line after a
 * counting sort on the device; the list then needs 32 more bytes per event
 * of stream-ordered temporary memory (without room for it the per-event
 * path runs).  Whether the scanner is cylindrical is decided by a kernel
 * that reads the crystal table: the call never synchronises the stream. */
int lm_back(const lm_geom *G, const float *v, const int16_t *ev, int64_t n, float *img,
            void *stream);

/* Sensitivity image g += P^T 1 over every unordered crystal pair and every
 * TOF bin (the back projection of a sinogram of ones that Algorithm 2's
 * initialisation and the step sizes T need; Section 2, after Eq.
 * lm_stepsizes).  Accumulates into g; the caller zeroes it.  On a
 * cylindrical 3D scanner (as for lm_back, decided on the device) the pairs
 * are taken by transaxial line.  Asynchronous. */
int lm_sens(const lm_geom *G, float *g, void *stream);

/* Synchronous: count events whose crystal, ring or TOF index is out of
 * range.  *n_bad (host) receives the count. */
int lm_validate_events(const lm_geom *G, const int16_t *ev, int64_t n, int64_t *n_bad,
                       void *stream);

/* ---------------------------------------------------------------- prior */

/* gx = K x: forward differences along x, y, z (Section 3, TV prior), zero
 * in the last layer of each axis; gx is float[3][nz][ny][nx] (component 0 =
 * x).  n = {nx, ny, nz} (host array). */
int tv_grad(const int32_t n[3], const float *x, float *gx, void *stream);

/* out = div w = -K^T w (the negative adjoint of tv_grad); w is
 * float[3][nz][ny][nx]. */
int tv_div(const int32_t n[3], const float *w, float *out, void *stream);

/* ---------------------------------------------------------------- cost */

/* Synchronous.  The objective of Eq. (1) in listmode form, for monitoring
 * (the relative cost c_rel(x) = (c(x) - c(x*)) / (c(x0) - c(x*)) of
 * Section 3, Numerical Experiments):
 *   c(x) = <g, x> - sum_e log((P^LM x)_e + s_e) + beta ||K x||_{2,1},
 * where g = P^T 1 (sum_i (Px)_i over all bins is <g, x>) and each event
 * gives the log term of its bin once; the constant sum of s over all bins
 * is left out.  K is the forward-difference gradient of tv_grad.  x, g:
 * row-major float images; ev: int16[n][5]; s: float[n] (> 0 keeps the
 * logarithms finite).  Outputs (host, either may be NULL but not both):
 * *cost, and terms[3] = {<g, x>, sum_e log((P^LM x)_e + s_e), ||K x||_{2,1}}.
 * The projections are float32 (lm_fwd); the sums are accumulated in
 * double.  Temporaries (4 B per event, a bricked copy of x) are allocated
 * stream-ordered. */
int lm_cost(const lm_geom *G, const float *x, const int16_t *ev, const float *s, int64_t n, const float *g,
            double beta, double *cost, double *terms, void *stream);

/* ---------------------------------------------------------------- LM-SPDHG */

typedef struct lm_plan lm_plan;

/* Device bytes a plan for n_ev events and n_sub subsets will allocate,
 * including the temporary memory of lm_plan_create; host output *bytes.
 * Used to admit reconstructions against an HBM budget.  lm_plan_bytes
 * counts the base plan; lm_plan_bytes_ex adds the optional parts named in
 * `parts` (an OR of the LM_PART_* flags): the directional TV prior
 * (lm_plan_set_prior_image), per-event factors (lm_plan_set_event_factors)
 * and the resolution model (lm_plan_set_resolution).  LM_EINVAL for an
 * unknown flag. */
enum { LM_PART_DTV = 1, LM_PART_FACTORS = 2, LM_PART_RESOLUTION = 4 };
int lm_plan_bytes(const lm_geom *G, int64_t n_ev, int32_t n_sub, size_t *bytes);
int lm_plan_bytes_ex(const lm_geom *G, int64_t n_ev, int32_t n_sub, int32_t parts, size_t *bytes);

/* Synchronous.  Builds a plan: copies and validates the events (LM_ERANGE
 * on any out-of-range index, nothing allocated), computes the event counts
 * mu_e (Algorithm 2 and its footnote: the number of events in the list in
 * the same sinogram bin, i.e. the same unordered crystal pair and TOF bin
 * with the sign of k flipped when the pair is swapped), splits the list
 * into n_sub interleaved subsets (event e goes to subset e mod n_sub, the
 * text after Algorithm 2), and the step sizes of Eq. lm_stepsizes with
 * p_k = 1/(2 n_sub) and p_prior = 1/2 (Section 3):
 *   S_e = gamma rho / (P^LM 1)_e  (0 where the LOR misses the image:
 *         (P^LM 1)_e <= 1e-6 of the smallest voxel side, which also
 *         covers a LOR that meets the image only within rounding),
 *   S_prior = gamma rho / knorm,
 *   T_j = rho / (2 gamma max(g_j, knorm)).
 * ev: int16[n][5]; s: float[n] contamination per event (> 0); g: the
 * sensitivity image or NULL (then lm_sens is run); knorm <= 0 selects the
 * exact norm of K, sqrt(sum_a 4 sin^2(pi (N_a-1) / (2 N_a))).  The plan
 * keeps a copy of G (det must stay valid) and owns all its device memory
 * until lm_plan_destroy; it allocates stream-ordered (hipMallocAsync on
 * `stream`, from the device's default memory pool), so creating or
 * destroying a plan never waits for work on other streams.  Work runs on
 * `stream`; the call returns after it finished. */
int lm_plan_create(const lm_geom *G, const int16_t *ev, const float *s, int64_t n, int32_t n_sub,
                   const float *g, double gamma, double rho, double beta, double knorm, void *stream,
                   lm_plan **out);

/* Initialisation (Algorithm 2): y_e = 1 - mu_e / ((P^LM x0)_e + s_e),
 * w = 0, z = zbar = g + (P^LM)^T((y - 1)/mu) + K^T w.  (The printed
 * initialisation of z has "-" before the back projection; "+" is the sign
 * under which z is the back projection of the sinogram dual of Eq. yinit,
 * as the text after the algorithm states.)  Resets the update counter to
 * 0. */
int lm_spdhg_init(lm_plan *p, const float *x0, void *stream);

/* Runs n_updates updates of Algorithm 2.  seq_host (host) lists
 * the random choices: entry u is a data subset 0..n_sub-1 or n_sub for the
 * prior update; the caller draws them with p_k = 1/(2 n_sub), p_prior = 1/2.
 * x (in/out, float image) enters as the x returned by the previous call (x0
 * after init) and leaves as the x of the last update's primal step (the
 * value Algorithm 2 returns).  Calls on one plan must be ordered (one
 * stream).  LM_EINVAL if an entry of seq is out of range (nothing run). */
int lm_spdhg_epoch(lm_plan *p, float *x, const int32_t *seq_host, int32_t n_updates, void *stream);

/* Per-event multiplicative factors of the forward model (Section 1: P
 * includes attenuation and normalisation; m_e is that factor for the LOR of
 * event e), so that the plan's operator becomes P' = diag(m) P^LM.  The g
 * given to lm_plan_create must then be the sensitivity of P' (the sum over
 * all LORs of m P^T 1).  The factors fold into the stored lists exactly.
 * With S' = gamma rho / (m P^LM 1):
 *   S' (m P x + s) = S (P x + s/m),
 *   the prox term 4 S' mu = 4 S (mu/m),
 *   P'^T (dy / mu) = P^T (dy / (mu/m)).
 * So the plan stores s/m and mu/m, and keeps m (4 B per event) so that
 * lm_plan_get_lists still returns the integer counts.  P^LM 1 as read back
 * stays the geometric one.  m: float[n], device, caller event order.
 * Synchronous.  Call once, after lm_plan_create and before lm_spdhg_init or
 * lm_plan_set_state (LM_ESTATE otherwise).  LM_ESTATE as well when the plan
 * computed g itself (lm_plan_create with g = NULL): the sensitivity of P'
 * sums m over every LOR, which the event list cannot give.  LM_ERANGE if a
 * factor is not positive and finite (nothing changed). */
int lm_plan_set_event_factors(lm_plan *p, const float *m, void *stream);

/* Image-space resolution model (Section 1: P includes limited spatial
 * resolution): the plan's operator becomes G B, G the projector, B a
 * separable Gaussian convolution with FWHM fwhm_vox[a] voxels along x, y, z
 * (host array; 0 leaves an axis alone, all 0 removes the model).  Taps are
 * truncated at ceil(3 sigma) voxels (at most 16) and normalised to sum 1;
 * outside the image counts as zero, so B is symmetric and the back
 * projection is B G^T.  Each data update then blurs x before its
 * projections and blurs its back projection before the z step: four more
 * images of plan memory and two passes per blurred axis.  P^LM 1 and S_e are
 * recomputed for G B; the g given to lm_plan_create must be the sensitivity
 * of the whole operator.  When the plan computed g = G^T 1 itself (g = NULL
 * at creation) it replaces it by B G^T 1, the sensitivity of G B, and
 * recomputes T (one more image of plan memory).  Synchronous.  Before lm_spdhg_init or
 * lm_plan_set_state (LM_ESTATE otherwise); LM_EINVAL for a negative FWHM or
 * one beyond 16 taps of radius. */
int lm_plan_set_resolution(lm_plan *p, const double fwhm_vox[3], void *stream);

/* Directional TV prior (Section 3, DTV; Ehrhardt & Betcke 2016) in place of
 * TV: K = D grad with D_j = I - xi_j xi_j^T, which removes from each
 * voxel's finite-difference vector its component along the normalised
 * gradient xi = grad v / sqrt(|grad v|^2 + eta^2) of the structural prior
 * image v (row-major float[nz][ny][nx], device; the paper's experiments use
 * the image itself with flipped contrast).  The prior updates of later
 * lm_spdhg_epoch calls use it: w <- proj_beta(w + S_prior K x), z gains
 * K^T of the change of w.  The step sizes keep ||grad|| (|D_j| <= 1).
 * v = NULL returns to TV.  The first call allocates two more images of
 * ncomp components (stream-ordered); work is enqueued on stream.  LM_EINVAL
 * for eta <= 0. */
int lm_plan_set_prior_image(lm_plan *p, const float *v, double eta, void *stream);

/* Number of events, subsets and the image size of a plan (host outputs,
 * any may be NULL). */
int lm_plan_info(const lm_plan *p, int64_t *n_ev, int32_t *n_sub, int64_t *nvox);

/* Read back per-event lists in the caller's event order: y (dual variable,
 * float[n], rounded from the stored complement 1 - y, see below), mu (event
 * counts, int32[n]), subset (subset index, int32[n]), p1 (P^LM 1, float[n]);
 * any output may be NULL.  Enqueued on stream. */
int lm_plan_get_lists(const lm_plan *p, float *y, int32_t *mu, int32_t *subset, float *p1,
                      void *stream);

/* Internal processing order: perm[j] = caller index of the j-th stored
 * event (int32[n]); offsets[i] = first stored position of subset i
 * (int32[n_sub + 1]).  Either may be NULL. */
int lm_plan_get_layout(const lm_plan *p, int32_t *perm, int32_t *offsets, void *stream);

/* Device images of the plan state: sensitivity g and primal step T
 * (float[nvox]); either may be NULL. */
int lm_plan_get_images(const lm_plan *p, float *g, float *T, void *stream);

/* Checkpoint.  The state is x (held by the caller), and z, zbar,
 * w (float[3][nvox]), c = 1 - y (float[n], caller event order) plus the
 * update counter.  The plan stores the dual as its complement c, which
 * stays accurate where y tends to 1; checkpoints carry c so that a resumed
 * run continues from exactly the stored state.  get copies the state out
 * into caller buffers (any may be NULL); set copies it in and marks the
 * plan initialised.  *u (host) is the update counter. */
int lm_plan_get_state(const lm_plan *p, float *z, float *zbar, float *w, float *c, int64_t *u,
                      void *stream);
int lm_plan_set_state(lm_plan *p, const float *z, const float *zbar, const float *w,
                      const float *c, int64_t u, void *stream);

/* Kernel classes of lm_spdhg_epoch, for lm_plan_get_timing. */
enum {
  LM_K_PRIMAL = 0,      /* primal step at the start of a call, layout conversions of x */
  LM_K_DATA = 1,        /* fused forward / dual prox / back projection of a subset */
  LM_K_DUAL_IMAGE = 2,  /* z, zbar (and fused primal) after a data update */
  LM_K_TV = 3,          /* prior update: w, K^T(w_new - w), z, zbar (and fused primal) */
  LM_K_COUNT = 4
};

/* Per-kernel timing of lm_spdhg_epoch.  lm_plan_timing(p, every) resets the
 * counters and, for every > 0, brackets every every-th launch of each kernel
 * class of the plan's update loop (the 1st, (every+1)-th, ... since the
 * reset) by a pair of HIP events on the stream it runs on; every = 0 turns
 * timing off.  Sampling keeps the cost of the events (a few microseconds per
 * bracketed launch) small against the update loop.  lm_plan_get_timing
 * (synchronous) adds the elapsed times of the bracketed launches to
 * ms[LM_K_COUNT] and their number to launches[LM_K_COUNT] (host arrays,
 * accumulated since the reset).  LM_EINVAL for a negative stride. */
int lm_plan_timing(lm_plan *p, int every);
int lm_plan_get_timing(lm_plan *p, double *ms, int64_t *launches);

/* Tracing of lm_spdhg_epoch.  With on != 0 every later epoch call pushes a
 * roctx range "lm_spdhg_epoch" for the call and, inside it, one range per
 * update of Algorithm 2 ("data update, subset i" or "prior update") around
 * the launches that update enqueues; the ranges are host-side (they mark
 * when the launches were enqueued), so that a trace taken with rocprofv3
 * --marker-trace --kernel-trace ties every kernel to its update.  on = 0
 * (the default) turns tracing off; the iterates are the same either way.
 * LM_EINVAL for a NULL plan. */
int lm_plan_set_tracing(lm_plan *p, int on);

/* Synchronises the plan's last stream, then frees its device memory
 * stream-ordered on that stream (hipFreeAsync: no device-wide wait).  That
 * stream (the one of the plan's last call) must still exist.  A plan is not
 * safe for concurrent use from several host threads. */
int lm_plan_destroy(lm_plan *p);

/* ---------------------------------------------------------------- warm start */

/* Listmode EM-TV (Algorithm 3), the warm start of LM-SPDHG: Section 2
 * (after Eq. yinit) proposes it for x0, and Section 3 runs one iteration
 * with 28 subsets before every reconstruction, y0 then following from
 * Eq. yinit (lm_spdhg_init).  n_iter passes over the n_subsets interleaved
 * subsets (event e in subset e mod n_subsets), visited in the order 0, 1,
 * ..., n_subsets - 1.  Each subset update computes
 *   z = x n_subsets / g * P_i^LM^T (1 / (P_i^LM x + s_i))   (EM step; an
 *       event with P x + s <= 0 adds nothing; z = 0 where g = 0),
 *   w = g / (beta x)                                        (inf where x = 0),
 *   x <- argmin_{u >= 0} sum_j w_j / 2 (u_j - z_j)^2 + ||K u||_{2,1},
 * the last by denoise_iter steps of the accelerated primal-dual algorithm
 * of Chambolle & Pock (J. Math. Imaging Vis. 40, 2011, Algorithm 2; 20 in
 * Section 3) from u = z and a zero dual, with tau_0 = sigma_0 = 1/||K||,
 * the convexity constant equal to the smallest finite w, and u held at z
 * where w is infinite.  beta = 0 skips the denoising (OSEM).
 * ev: int16[n][5]; s: float[n] contamination per event; g: sensitivity
 * image (row-major float[nz][ny][nx], e.g. from lm_sens); x: row-major
 * float image, x0 >= 0 on entry, the result on return.  All device
 * pointers, caller-owned.  Asynchronous on stream: temporaries (14 B per
 * event, 4 B per event of the largest subset, ten images) are allocated
 * and freed stream-ordered.  LM_EINVAL for bad arguments (nothing run),
 * LM_ENOMEM when a temporary does not fit. */
int lm_emtv(const lm_geom *G, const int16_t *ev, const float *s, int64_t n, int32_t n_subsets,
            int32_t n_iter, const float *g, float beta, int32_t denoise_iter, float *x, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LMSPDHG_H */
