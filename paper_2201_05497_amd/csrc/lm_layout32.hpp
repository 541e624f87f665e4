// Decoding of a position of the brick layout in 32-bit arithmetic, for the
// element-wise passes over plan images (they hold fewer than 2^31
// elements; the 64-bit division of vpos would dominate such a pass).
#pragma once

#include <hip/hip_runtime.h>

#include "lm_device.hpp"

namespace lmk {

// Position p of layout L -> voxel (i, j, k) (padding positions decode to
// coordinates beyond the image size).
__device__ __forceinline__ void vpos32(const Layout &L, unsigned p, int &i, int &j, int &k) {
  const int sh = L.sx + L.sy + L.sz;
  const unsigned b = p >> sh, loc = p & ((1u << sh) - 1u);
  const unsigned row = b / (unsigned)L.nbx, bi = b - row * (unsigned)L.nbx;
  const unsigned bk = row / (unsigned)L.nby, bj = row - bk * (unsigned)L.nby;
  i = (int)((bi << L.sx) | (loc & ((1u << L.sx) - 1u)));
  j = (int)((bj << L.sy) | ((loc >> L.sx) & ((1u << L.sy) - 1u)));
  k = (int)((bk << L.sz) | (loc >> (L.sx + L.sy)));
}

}  // namespace lmk
