// Host-side helpers shared by the translation units of the library: error
// reporting through the C ABI, conversion of lm_geom into the kernel form,
// and the launch shape of the projector kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "lm_device.hpp"
#include "lmspdhg.h"

namespace lmh {

// thread-local message of the last error (defined in lm_plan.hip)
void set_error(const char *fmt, ...);
void clear_error();

#define LM_TRY_HIP(expr)                                                                  \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) {                                                               \
      lmh::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
      return LM_EHIP;                                                                     \
    }                                                                                     \
  } while (0)

#define LM_REQUIRE(cond, code, ...)   \
  do {                                \
    if (!(cond)) {                    \
      lmh::set_error(__VA_ARGS__);    \
      return (code);                  \
    }                                 \
  } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

constexpr int kMaxDim = 512;

// Checks lm_geom and converts it; returns LM_OK or LM_EINVAL.
int make_geom(const lm_geom *G, lmk::GeomDev *out);

// Largest number of planes a single event can visit (bound used to size
// the per-lane sample cache of the projector kernels).
int max_planes(const lmk::GeomDev &g, int mode);


// Voxel count with overflow check.
inline long long nvox_of(const int n[3]) { return (long long)n[0] * n[1] * n[2]; }

// Row-major layout of an n[0] x n[1] x n[2] image (the caller's layout).
inline lmk::Layout row_major(const int n[3]) {
  lmk::Layout L;
  L.nbx = n[0];
  L.nby = n[1];
  L.nbz = n[2];
  L.sx = L.sy = L.sz = 0;
  return L;
}

// Brick layout of the plans: 4 x 4 x 4 voxels per brick (4 x 4 x 1 for a
// single slice), the grid padded up to whole bricks.
inline lmk::Layout brick_layout(const int n[3]) {
  lmk::Layout L;
  L.sx = 2;
  L.sy = 2;
  L.sz = n[2] > 1 ? 2 : 0;
  L.nbx = (n[0] + 3) >> 2;
  L.nby = (n[1] + 3) >> 2;
  L.nbz = (n[2] + (1 << L.sz) - 1) >> L.sz;
  return L;
}

}  // namespace lmh

// Kernel launchers defined in lm_project.hip, used by the plan code.
namespace lmk {
int launch_fwd(const GeomDev &g, const float *x, const int16_t *ev, long long n, float *out,
               hipStream_t st);
int launch_back(const GeomDev &g, const float *v, const int16_t *ev, long long n, float *img,
                hipStream_t st);
int launch_sens(const GeomDev &g, float *img, hipStream_t st);
// Paths by transaxial line (lm_lines.hip) for cylindrical 3D scanners.
// lines_possible: the host-side part of the test (at least two rings and
// crystals); launch_cylindrical writes the rest of it to a device flag
// (1: crystal c of ring r at (x_c, y_c, z_r), z increasing with r), which
// the line kernels and the per-event fallback read, so that choosing the
// path never synchronises the stream.
bool lines_possible(const GeomDev &g);
int launch_cylindrical(const GeomDev &g, int *flag, hipStream_t st);
// Sensitivity by line: nothing happens unless *cyl.
int launch_sens_lines(const GeomDev &g, const int *cyl, float *img, hipStream_t st);
// Back projection of a long event list by line, guarded by *cyl; `queued`
// is false (nothing enqueued) when the list is too short or the
// temporaries of the sort do not fit.
int launch_back_lines(const GeomDev &g, const int *cyl, const float *v, const int16_t *ev, long long n, float *img,
                      hipStream_t st, bool &queued);
// For a long list (at least 64 events per transaxial crystal pair): the
// events' indices in the order of a counting sort by transaxial crystal
// pair (any scanner), in a stream-ordered allocation *order (nullptr: the
// list is short or the temporaries do not fit), and, when offsets is not
// NULL, the first sorted position of every pair and of the last bucket
// (events of one crystal or out of range) plus the list's end, nlines + 2
// entries; the caller frees both stream-ordered.
int sort_events_by_line(const GeomDev &g, const int16_t *ev, long long n, unsigned **order, unsigned **offsets,
                        hipStream_t st);
// Forward projection of a sorted list by line (lm_lines.hip): queued is set
// when the kernel was launched (a scanner with at least two rings and two
// crystals, and an LDS sheet of the image's planes that fits one block);
// it writes every out[e] when *cyl is set at run time and nothing
// otherwise.  x in the brick layout of g.
int launch_fwd_lines(const GeomDev &g, const int *cyl, const float *x, const int16_t *ev, const unsigned *order,
                     const unsigned *off, long long n, float *out, hipStream_t st, bool &queued);
// The tabulated TOF weights of a geometry with TOF (see TofTab): *tab is a
// stream-ordered allocation of tof_tab_size(t) intervals that the caller
// frees, or nullptr (no TOF, a table too large, or no memory for it: the
// kernels then evaluate erfc).
int build_tof_table(const GeomDev &g, TofTab &t, float4 **tab, hipStream_t st);
// Plan-internal event records: int4 {id1, id2, k, s bits}.
int launch_fwd_rec(const GeomDev &g, const float *x, const int4 *rec, long long n, float *out,
                   hipStream_t st);
int launch_back_rec(const GeomDev &g, const float *v, const int4 *rec, long long n, float *img,
                    hipStream_t st);
// Fused data update of one subset (Algorithm 2, data branch); cdual holds
// the complement 1 - y of the dual variable.
int launch_data_update(const GeomDev &g, const float *x, const int4 *rec, const float *S,
                       const float *mu, float *cdual, float *dz, long long n, hipStream_t st);
}  // namespace lmk

namespace lmh {

// The plain projector calls run on a bricked copy of the caller's row-major
// image (the layout of the plans, 4x4x4 voxels per brick): gathers and the
// interleaved scatter then touch few cache lines per instruction.  The copy
// is a stream-ordered temporary freed (stream-ordered) when the call
// returns; its padding voxels are never read or written, since every
// corner is checked against the image size.
struct BrickImage {
  float *p = nullptr;
  hipStream_t st = nullptr;
  int alloc(lmk::GeomDev &g, hipStream_t s) {
    g.lay = lmh::brick_layout(g.n);
    st = s;
    const hipError_t e = hipMallocAsync((void **)&p, (size_t)lmk::layout_size(g.lay) * sizeof(float), s);
    if (e != hipSuccess) {
      p = nullptr;
      lmh::set_error("image temporary: %s", hipGetErrorString(e));
      return LM_ENOMEM;
    }
    return LM_OK;
  }
  ~BrickImage() {
    if (p) (void)hipFreeAsync(p, st);  // a release error has no caller to go to
  }
};

}  // namespace lmh
