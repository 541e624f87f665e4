// The data update of LM-SPDHG by image tile (lm_tiles.hip): the back
// projection of a subset's dual increments is binned by 8x8x8-voxel tile
// once, at plan creation, so that each update accumulates every tile in LDS
// without global atomics and applies the z / zbar / primal step to the
// tile's voxels in the same kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "lm_device.hpp"

namespace lmk {

// Tiles of 8 x 8 x 8 voxels (2 x 2 x 2 bricks of the plan's layout) over an
// image with 4x4x4-voxel bricks.
struct TileGeom {
  int ntx, nty, ntz, ntiles;
};

// One segment as phase 2 reads it (64 bytes, one memory sector; written by
// phase 1, the records of an event in a row): the in-plane coordinates of
// the event's samples on the tile's 8 planes along its dominant axis are
// u_p = G + p V (p = 0..7; G the coordinate at the tile's first plane), and
// for each plane p the sample's value v[p] = cf w_j (cf = L dy / mu; 0
// outside the ray) and meta[p] = 0 when no corner of the sample adds to the
// tile, else (tile-local index of corner 0 + 128) | (corner mask << 10) |
// (dominant axis << 14), the mask having bit c set for each bilinear corner
// c inside both the tile and the image.
struct __align__(64) TileRec {
  float4 h;  // {G1, V1, G2, V2}
  float v[8];
  unsigned short meta[8];
};

// Per-plan state of the tile path; `on` false: the per-event path runs.
struct TilePlan {
  bool on = false;
  TileGeom tg{};
  int maxp = 0;                  // plane bound of every event (setup_ray's clamp)
  long long nseg = 0;            // segments of all subsets
  long long rec_max = 0;         // segments of the largest subset
  long long *seg_off = nullptr;  // [nsub * ntiles + 1] first entry of seg of (subset, tile), all subsets in a row
  unsigned long long *eoff = nullptr;  // [N + 1] first record of each stored event (records of an event in a row)
  unsigned *seg = nullptr;       // record numbers (relative to the subset's first) of every tile, by subset and tile
  int *order = nullptr;          // tiles by decreasing load (launch order of phase 2)
  TileRec *rec = nullptr;        // [rec_max] segments of the subset being updated
  TofTab tt{};                   // layout of the tabulated TOF weights
  float4 *tab = nullptr;         // the table (nullptr: phase 1 evaluates erfc)
};

bool tiles_supported(const GeomDev &g);
TileGeom tile_geom(const int n[3]);

// Upper bound of the device bytes the tile path of a plan of n events in
// nsub subsets holds (segments, offsets, launch order, the phase-1 records
// of the largest subset) plus its temporaries at creation; 0 when the
// geometry does not qualify.  Each event has at most one segment per tile
// that its corners reach on 8 consecutive planes.
size_t tile_bytes_bound(const GeomDev &g, long long n, int nsub);

// Builds the segment lists of every subset of the plan's stored events
// (subset i at rec[off[i] .. off[i+1])).  Device memory that the plan keeps
// is allocated stream-ordered and appended to `owned` (the plan frees it);
// temporaries are freed before returning.  Returns LM_OK with tp.on ==
// false when the geometry does not qualify or the segments do not fit (the
// per-event path then runs), an error code for a failed HIP call.
// Synchronous.
int build_tiles(const GeomDev &g, const int4 *rec, const std::vector<int> &off, TilePlan &tp,
                std::vector<void *> &owned, hipStream_t st);

// Phase 1 of a data update of the subset stored at positions [o, o + n):
// forward projection, dual prox, and the subset's segment records.
int launch_tile_fwd(const GeomDev &g, const TilePlan &tp, const float *x, const int4 *rec, const float *S,
                    const float *mu, float *cdual, long long o, long long n, hipStream_t st);
// Phase 2: back projection by tile; dz_out != NULL writes dz (every voxel of
// the layout) instead of the z / zbar / primal step.
int launch_tile_back(const GeomDev &g, const TilePlan &tp, int subset, float *z, float *x, const float *T,
                     float *zbar, float *dz_out, float inv_p, bool fuse, hipStream_t st);

}  // namespace lmk
