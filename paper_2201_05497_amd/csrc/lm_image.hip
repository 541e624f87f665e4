// Image-space kernels of LM-SPDHG on gfx950: the primal step with the
// non-negativity prox, the z / zbar updates, the TV dual update with its
// adjoint stencil, and the tv_grad / tv_div entry points.
//
// All of these stream whole images and are bound by memory bandwidth; each
// thread handles one voxel, loads are coalesced along x (the fastest axis)
// and every pass that can be fused with the next primal step is.
#include <hip/hip_runtime.h>

#include "lm_host.hpp"
#include "lm_image.hpp"

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Primal step of Algorithm 2: x <- max(0, x - T zbar).
__global__ __launch_bounds__(kBlock) void k_primal(float *__restrict__ x, const float *__restrict__ T,
                                                   const float *__restrict__ zbar, long long nv) {
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v < nv) x[v] = fmaxf(0.0f, fmaf(-T[v], zbar[v], x[v]));
}

// The z / zbar step of Algorithm 2 after a data update, fused with the
// primal step of the next update when `fuse` is set:
//   z += dz;  zbar = z + dz / p;  (fuse ? x = max(0, x - T zbar) : store zbar);
//   dz = 0 (ready for the next subset's atomics).
__global__ __launch_bounds__(kBlock) void k_dual_image(float *__restrict__ z, float *__restrict__ dz,
                                                       float *__restrict__ x, const float *__restrict__ T,
                                                       float *__restrict__ zbar, float inv_p, int fuse,
                                                       long long nv) {
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nv) return;
  const float d = dz[v];
  const float zn = z[v] + d;
  const float zb = fmaf(d, inv_p, zn);
  z[v] = zn;
  dz[v] = 0.0f;
  if (fuse)
    x[v] = fmaxf(0.0f, fmaf(-T[v], zb, x[v]));
  else
    zbar[v] = zb;
}

// w+ - w at voxel (i, j, k): the dual prior step evaluated from x and w
// (three components; the z-component is zero when ncomp == 2).
__device__ __forceinline__ void tv_step_at(const float *__restrict__ x, const float *__restrict__ w,
                                           const lmk::Layout &L, int nx, int ny, int nz, long long ne, int ncomp,
                                           float Sp, float beta, int i, int j, int k, float &q0, float &q1,
                                           float &q2) {
  const int p = lmk::vidx(L, i, j, k);
  const float xv = x[p];
  const float gx = (i < nx - 1) ? x[lmk::vidx(L, i + 1, j, k)] - xv : 0.0f;
  const float gy = (j < ny - 1) ? x[lmk::vidx(L, i, j + 1, k)] - xv : 0.0f;
  const float gz = (ncomp == 3 && k < nz - 1) ? x[lmk::vidx(L, i, j, k + 1)] - xv : 0.0f;
  const float w0 = w[p], w1 = w[ne + p], w2 = (ncomp == 3) ? w[2 * ne + p] : 0.0f;
  const float v0 = fmaf(Sp, gx, w0), v1 = fmaf(Sp, gy, w1), v2 = fmaf(Sp, gz, w2);
  const float nrm = sqrtf(fmaf(v0, v0, fmaf(v1, v1, v2 * v2)));
  const float sc = 1.0f / fmaxf(1.0f, nrm / beta);
  q0 = v0 * sc - w0;
  q1 = v1 * sc - w1;
  q2 = v2 * sc - w2;
}

// The whole prior update in one pass (the dual prior step, its
// back-projection through K^T and the z / zbar step of Algorithm 2, fused
// with the next primal step when `fuse` is set):
//   q = proj_beta(w + S_prior K x) - w;  w_out = w + q;  dz = K^T q;
//   z += dz;  zbar = z + dz / p;  fuse ? x_out = max(0, x - T zbar) : store zbar.
// K^T q at a voxel needs q at the voxel and at its three lower neighbours;
// each is recomputed here from x and w (the projection couples the three
// components), so x and w are read-only and the results go to separate
// buffers (x_out, w_out).
__global__ __launch_bounds__(kBlock) void k_tv_fused(const float *__restrict__ x, const float *__restrict__ w,
                                                     float *__restrict__ w_out, float *__restrict__ z,
                                                     float *__restrict__ x_out, const float *__restrict__ T,
                                                     float *__restrict__ zbar, lmk::Layout L, int nx, int ny,
                                                     int nz, long long ne, int ncomp, float Sp, float beta,
                                                     float inv_p, int fuse) {
  const long long p = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (p >= ne) return;
  int i, j, k;
  lmk::vpos(L, p, i, j, k);
  if (i >= nx || j >= ny || k >= nz) return;
  float q0, q1, q2;
  tv_step_at(x, w, L, nx, ny, nz, ne, ncomp, Sp, beta, i, j, k, q0, q1, q2);
  w_out[p] = w[p] + q0;
  w_out[ne + p] = w[ne + p] + q1;
  if (ncomp == 3) w_out[2 * ne + p] = w[2 * ne + p] + q2;
  float d = 0.0f;
  if (i < nx - 1) d -= q0;
  if (j < ny - 1) d -= q1;
  if (ncomp == 3 && k < nz - 1) d -= q2;
  float a0, a1, a2;
  if (i > 0) {
    tv_step_at(x, w, L, nx, ny, nz, ne, ncomp, Sp, beta, i - 1, j, k, a0, a1, a2);
    d += a0;
  }
  if (j > 0) {
    tv_step_at(x, w, L, nx, ny, nz, ne, ncomp, Sp, beta, i, j - 1, k, a0, a1, a2);
    d += a1;
  }
  if (ncomp == 3 && k > 0) {
    tv_step_at(x, w, L, nx, ny, nz, ne, ncomp, Sp, beta, i, j, k - 1, a0, a1, a2);
    d += a2;
  }
  const float zn = z[p] + d;
  const float zb = fmaf(d, inv_p, zn);
  z[p] = zn;
  if (fuse)
    x_out[p] = fmaxf(0.0f, fmaf(-T[p], zb, x[p]));
  else
    zbar[p] = zb;
}

// The whole prior update, tiled through LDS.  A block owns a tile of
// TBX x TBY x 1 bricks (2 x 2 bricks of 4x4x4 voxels, or 4 x 4 bricks of
// 4x4x1 for a single slice: 256 voxels); wavefront w reads brick w of the
// tile, so those loads are whole 256-byte bricks.  The tile stages x with a
// one-voxel halo and computes q = proj_beta(w + S K x) - w once for the tile
// and its lower halo (K^T q at a voxel needs q at the voxel and at its three
// lower neighbours), then forms dz = K^T q, z, zbar and the fused primal
// step.  Every global load of the block is issued before the first barrier.
// Tiles are numbered so that each XCD (blocks are dealt to the 8 XCDs round
// robin) works on one contiguous run of tiles, which keeps the halo reads of
// neighbouring tiles in that XCD's L2.  x and w are read-only; results go to
// x_out and w_out.
template <int BX, int BY, int BZ, int TBX, int TBY>
__global__ __launch_bounds__(kBlock) void k_tv_tiled(const float *__restrict__ x, const float *__restrict__ w,
                                                     float *__restrict__ w_out, float *__restrict__ z,
                                                     float *__restrict__ x_out, const float *__restrict__ T,
                                                     float *__restrict__ zbar, lmk::Layout L, int nx, int ny,
                                                     int nz, long long ne, int ncomp, float Sp, float beta,
                                                     float inv_p, int fuse, int ntiles) {
  constexpr int TX = TBX * BX, TY = TBY * BY, TZ = BZ;                  // tile in voxels
  constexpr int XX = TX + 2, XY = TY + 2, XZ = (TZ > 1) ? TZ + 2 : 1;  // x with halo -1 .. +1
  constexpr int QX = TX + 1, QY = TY + 1, QZ = (TZ > 1) ? TZ + 1 : 1;  // q with halo -1
  constexpr int ZOFF = (TZ > 1) ? 1 : 0;
  constexpr int NXS = XX * XY * XZ, NQ = QX * QY * QZ;
  constexpr int RX = (NXS + kBlock - 1) / kBlock, RQ = (NQ + kBlock - 1) / kBlock;
  constexpr int BV = BX * BY * BZ;
  static_assert(TBX * TBY * BV == kBlock, "one voxel of the tile per thread");
  __shared__ float xs[NXS];
  __shared__ float qs[3][NQ];
  int tile = blockIdx.x;
  const int full = ntiles & ~7;
  if (tile < full) tile = (tile & 7) * (full >> 3) + (tile >> 3);
  const int ntx = (L.nbx + TBX - 1) / TBX, nty = (L.nby + TBY - 1) / TBY;
  const int tbx = tile % ntx, tby = (tile / ntx) % nty, tbz = tile / (ntx * nty);
  const int x0 = tbx * TX, y0 = tby * TY, z0 = tbz * TZ;
  const int t = threadIdx.x;
  // this thread's voxel: brick t / BV of the tile, voxel t % BV of the brick
  const int b = t / BV, l = t % BV;
  const int tx = (b % TBX) * BX + l % BX, ty = (b / TBX) * BY + (l / BX) % BY, tz = l / (BX * BY);
  const int i = x0 + tx, j = y0 + ty, k = z0 + tz;
  const bool mine = i < nx && j < ny && k < nz;
  const int p = mine ? lmk::vidx(L, i, j, k) : 0;
  // all global loads: x with halo, w on the q positions, z and T
  float xr[RX], wr[RQ][3];
#pragma unroll
  for (int r = 0; r < RX; ++r) {
    const int e = t + kBlock * r;
    xr[r] = 0.0f;
    if (e < NXS) {
      const int ix = e % XX, iy = (e / XX) % XY, iz = e / (XX * XY);
      const int a = x0 - 1 + ix, c = y0 - 1 + iy, d = z0 - ZOFF + iz;
      if (a >= 0 && a < nx && c >= 0 && c < ny && d >= 0 && d < nz) xr[r] = x[lmk::vidx(L, a, c, d)];
    }
  }
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
    const int e = t + kBlock * r;
    wr[r][0] = wr[r][1] = wr[r][2] = 0.0f;
    if (e < NQ) {
      const int ix = e % QX, iy = (e / QX) % QY, iz = e / (QX * QY);
      const int a = x0 - 1 + ix, c = y0 - 1 + iy, d = z0 - ZOFF + iz;
      if (a >= 0 && a < nx && c >= 0 && c < ny && d >= 0 && d < nz) {
        const int q = lmk::vidx(L, a, c, d);
        wr[r][0] = w[q];
        wr[r][1] = w[ne + q];
        if (ncomp == 3) wr[r][2] = w[2 * ne + q];
      }
    }
  }
  const float zv = mine ? z[p] : 0.0f;
  const float Tv = (mine && fuse) ? T[p] : 0.0f;
#pragma unroll
  for (int r = 0; r < RX; ++r)
    if (t + kBlock * r < NXS) xs[t + kBlock * r] = xr[r];
  __syncthreads();
  // q on the tile and its lower halo
#pragma unroll
  for (int r = 0; r < RQ; ++r) {
    const int e = t + kBlock * r;
    if (e >= NQ) break;
    const int ix = e % QX, iy = (e / QX) % QY, iz = e / (QX * QY);
    const int a = x0 - 1 + ix, c = y0 - 1 + iy, d = z0 - ZOFF + iz;
    float q0 = 0.0f, q1 = 0.0f, q2 = 0.0f;
    if (a >= 0 && a < nx && c >= 0 && c < ny && d >= 0 && d < nz) {
      const int sx = ix + XX * (iy + XY * iz);  // xs and q both start at the tile origin minus one
      const float xv = xs[sx];
      const float gx = (a < nx - 1) ? xs[sx + 1] - xv : 0.0f;
      const float gy = (c < ny - 1) ? xs[sx + XX] - xv : 0.0f;
      const float gz = (ncomp == 3 && d < nz - 1) ? xs[sx + XX * XY] - xv : 0.0f;
      const float w0 = wr[r][0], w1 = wr[r][1], w2 = wr[r][2];
      const float v0 = fmaf(Sp, gx, w0), v1 = fmaf(Sp, gy, w1), v2 = fmaf(Sp, gz, w2);
      const float nrm = sqrtf(fmaf(v0, v0, fmaf(v1, v1, v2 * v2)));
      const float sc = 1.0f / fmaxf(1.0f, nrm / beta);
      q0 = v0 * sc - w0;
      q1 = v1 * sc - w1;
      q2 = v2 * sc - w2;
      if (ix >= 1 && iy >= 1 && iz >= ZOFF) {  // a voxel of the tile: store w+
        const int q = lmk::vidx(L, a, c, d);
        w_out[q] = w0 + q0;
        w_out[ne + q] = w1 + q1;
        if (ncomp == 3) w_out[2 * ne + q] = w2 + q2;
      }
    }
    qs[0][e] = q0;
    qs[1][e] = q1;
    qs[2][e] = q2;
  }
  __syncthreads();
  if (!mine) return;
  const int qi = (tx + 1) + QX * ((ty + 1) + QY * (tz + ZOFF));
  float dz = 0.0f;
  if (i < nx - 1) dz -= qs[0][qi];
  if (i > 0) dz += qs[0][qi - 1];
  if (j < ny - 1) dz -= qs[1][qi];
  if (j > 0) dz += qs[1][qi - QX];
  if (ncomp == 3) {
    if (k < nz - 1) dz -= qs[2][qi];
    if (k > 0) dz += qs[2][qi - QX * QY];
  }
  const float zn = zv + dz;
  const float zb = fmaf(dz, inv_p, zn);
  z[p] = zn;
  if (fuse)
    x_out[p] = fmaxf(0.0f, fmaf(-Tv, zb, xs[(tx + 1) + XX * ((ty + 1) + XY * (tz + ZOFF))]));
  else
    zbar[p] = zb;
}

// Index of voxel (i, j, k) in the 4x4x4 brick layout with nbx x nby bricks
// per brick layer, split into a part that depends on (i, j) and one that
// depends on k only.
__device__ __forceinline__ int brick_ij(int nbx, int i, int j) {
  return (((j >> 2) * nbx + (i >> 2)) << 6) | ((j & 3) << 2) | (i & 3);
}
__device__ __forceinline__ int brick_k(int nbx, int nby, int k) { return (((k >> 2) * nby * nbx) << 6) | ((k & 3) << 4); }

// The whole prior update for a 3D image in the 4x4x4 brick layout, marching
// along z.  A block owns a column of 16 x 16 voxels and a run of CZ planes
// (plus one plane below it, whose dual step only feeds the z-difference of
// the first plane).  Per plane k it holds x of planes k and k+1 with a
// one-voxel ring in LDS (two 18 x 18 buffers) and x of plane k+2 in
// registers, computes
// q = proj_beta(w + S K x) - w for its 256 voxels and for the 32 voxels of
// the lower x- and y-faces of the ring (K^T q needs q at the three lower
// neighbours; the z one is the same thread's q of plane k-1), writes w+,
// then dz = K^T q, z, zbar and the fused primal step.  The loads of later
// planes (x three planes ahead, w, z and T one plane ahead) are issued
// before the current plane is computed.  Thread t owns
// voxel (t & 3) + 4 (t >> 4 & 3), ((t >> 2) & 3) + 4 (t >> 6) of the column,
// so a wavefront reads four 64-byte brick slabs per plane.  Columns are
// dealt so that each XCD works on a contiguous run (halo reads stay in its
// L2).  x and w are read-only; results go to x_out and w_out.
template <int CZ>
__global__ __launch_bounds__(kBlock) void k_tv_march(const float *__restrict__ x, const float *__restrict__ w,
                                                     float *__restrict__ w_out, float *__restrict__ z,
                                                     float *__restrict__ x_out, const float *__restrict__ T,
                                                     float *__restrict__ zbar, int nbx, int nby, int nx, int ny,
                                                     int nz, long long ne, float Sp, float beta, float inv_p,
                                                     int fuse, int nblocks) {
  constexpr int B = 18;   // x box: x0-1 .. x0+16
  constexpr int Q = 17;   // q box: x0-1 .. x0+15
  __shared__ float xb[2][B * B];
  __shared__ float q0s[Q * Q], q1s[Q * Q];
  int blk = blockIdx.x;
  const int full = nblocks & ~7;
  if (blk < full) blk = (blk & 7) * (full >> 3) + (blk >> 3);
  const int ntx = (nx + 15) >> 4, nty = (ny + 15) >> 4;
  const int cx = blk % ntx, cy = (blk / ntx) % nty, cz = blk / (ntx * nty);
  const int x0 = cx * 16, y0 = cy * 16;
  const int kz0 = cz * CZ, kz1 = min(nz, kz0 + CZ);
  const int ks = kz0 > 0 ? kz0 - 1 : 0;
  const int t = threadIdx.x;
  // own voxel
  const int ti = (t & 3) + 4 * ((t >> 4) & 3), tj = ((t >> 2) & 3) + 4 * (t >> 6);
  const int i = x0 + ti, j = y0 + tj;
  const bool own = i < nx && j < ny;
  const int own_b = (ti + 1) + B * (tj + 1), own_q = (ti + 1) + Q * (tj + 1);
  const int own_ij = own ? brick_ij(nbx, i, j) : 0;
  // ring of the x box (68 positions): rows by = 0 and 17, columns bx = 0 and 17
  int rb = -1, r_ij = 0;
  bool r_ok = false;
  if (t < 68) {
    int bx, by;
    if (t < 18) { bx = t; by = 0; }
    else if (t < 36) { bx = t - 18; by = 17; }
    else if (t < 52) { bx = 0; by = t - 35; }
    else { bx = 17; by = t - 51; }
    rb = bx + B * by;
    const int gi = x0 - 1 + bx, gj = y0 - 1 + by;
    r_ok = gi >= 0 && gi < nx && gj >= 0 && gj < ny;
    r_ij = r_ok ? brick_ij(nbx, gi, gj) : 0;
  }
  // q on the lower faces: t < 16: (x0-1, y0+t); 16 <= t < 32: (x0+t-16, y0-1)
  int hb = 0, hq = 0, h_ij = 0, hgi = 0, hgj = 0;
  bool h_ok = false;
  if (t < 32) {
    const int bx = t < 16 ? 0 : t - 15, by = t < 16 ? t + 1 : 0;
    hb = bx + B * by;
    hq = bx + Q * by;
    hgi = x0 - 1 + bx;
    hgj = y0 - 1 + by;
    h_ok = hgi >= 0 && hgi < nx && hgj >= 0 && hgj < ny;
    h_ij = h_ok ? brick_ij(nbx, hgi, hgj) : 0;
  }
  auto load_x = [&](int k, float &xo, float &xr) {
    xo = 0.0f;
    xr = 0.0f;
    if (k < nz) {
      const int off = brick_k(nbx, nby, k);
      if (own) xo = x[own_ij + off];
      if (r_ok) xr = x[r_ij + off];
    }
  };
  auto load_w = [&](int k, float (&wo)[3], float (&wh)[3], float &zo, float &to) {
    const int off = brick_k(nbx, nby, k);
    wo[0] = wo[1] = wo[2] = wh[0] = wh[1] = wh[2] = zo = to = 0.0f;
    if (own) {
      wo[0] = w[own_ij + off];
      wo[1] = w[ne + own_ij + off];
      wo[2] = w[2 * ne + own_ij + off];
      if (k >= kz0) {
        zo = z[own_ij + off];
        if (fuse) to = T[own_ij + off];
      }
    }
    if (h_ok && k >= kz0) {
      wh[0] = w[h_ij + off];
      wh[1] = w[ne + h_ij + off];
      wh[2] = w[2 * ne + h_ij + off];
    }
  };
  auto prox = [&](float gx, float gy, float gz, const float (&wv)[3], float (&q)[3]) {
    const float v0 = fmaf(Sp, gx, wv[0]), v1 = fmaf(Sp, gy, wv[1]), v2 = fmaf(Sp, gz, wv[2]);
    const float nrm = sqrtf(fmaf(v0, v0, fmaf(v1, v1, v2 * v2)));
    const float sc = 1.0f / fmaxf(1.0f, nrm / beta);
    q[0] = v0 * sc - wv[0];
    q[1] = v1 * sc - wv[1];
    q[2] = v2 * sc - wv[2];
  };
  // planes ks and ks+1 into LDS, plane ks+2 into registers (x is read two
  // planes ahead, so a load has a whole plane step to arrive); w, z, T of
  // plane ks into registers
  float pxo, pxr;
  {
    float a, b, c, d;
    load_x(ks, a, b);
    load_x(ks + 1, c, d);
    load_x(ks + 2, pxo, pxr);
    xb[0][own_b] = a;
    xb[1][own_b] = c;
    if (rb >= 0) {
      xb[0][rb] = b;
      xb[1][rb] = d;
    }
  }
  float wo[3], wh[3], zo, to;
  load_w(ks, wo, wh, zo, to);
  float q2prev = 0.0f;
  int cur = 0;
  __syncthreads();
  for (int k = ks; k < kz1; ++k) {
    // next loads: x of plane k+3, w / z / T of plane k+1
    float nxo, nxr, nwo[3], nwh[3], nzo, nto;
    load_x(k + 3, nxo, nxr);
    if (k + 1 < kz1) load_w(k + 1, nwo, nwh, nzo, nto);
    const float *xc = xb[cur], *xn = xb[cur ^ 1];
    const bool out = k >= kz0;
    // q of the own voxel
    const float xv = xc[own_b];
    float q[3];
    {
      const float gx = (i < nx - 1) ? xc[own_b + 1] - xv : 0.0f;
      const float gy = (j < ny - 1) ? xc[own_b + B] - xv : 0.0f;
      const float gz = (k < nz - 1) ? xn[own_b] - xv : 0.0f;
      prox(gx, gy, gz, wo, q);
    }
    if (out && own) {
      const int p = own_ij + brick_k(nbx, nby, k);
      w_out[p] = wo[0] + q[0];
      w_out[ne + p] = wo[1] + q[1];
      w_out[2 * ne + p] = wo[2] + q[2];
    }
    q0s[own_q] = q[0];
    q1s[own_q] = q[1];
    // q on the lower faces (only the component the own voxels need)
    if (t < 32 && out) {
      float hqv[3] = {0.0f, 0.0f, 0.0f};
      if (h_ok) {
        const float hv = xc[hb];
        const float gx = (hgi < nx - 1) ? xc[hb + 1] - hv : 0.0f;
        const float gy = (hgj < ny - 1) ? xc[hb + B] - hv : 0.0f;
        const float gz = (k < nz - 1) ? xn[hb] - hv : 0.0f;
        prox(gx, gy, gz, wh, hqv);
      }
      if (t < 16)
        q0s[hq] = hqv[0];
      else
        q1s[hq] = hqv[1];
    }
    __syncthreads();
    // plane k+2 (loaded one step ago) replaces plane k in LDS (nobody reads
    // plane k any more)
    xb[cur][own_b] = pxo;
    if (rb >= 0) xb[cur][rb] = pxr;
    pxo = nxo;
    pxr = nxr;
    if (out && own) {
      float dz = 0.0f;
      if (i < nx - 1) dz -= q0s[own_q];
      if (i > 0) dz += q0s[own_q - 1];
      if (j < ny - 1) dz -= q1s[own_q];
      if (j > 0) dz += q1s[own_q - Q];
      if (k < nz - 1) dz -= q[2];
      if (k > 0) dz += q2prev;
      const int p = own_ij + brick_k(nbx, nby, k);
      const float zn = zo + dz;
      const float zb = fmaf(dz, inv_p, zn);
      z[p] = zn;
      if (fuse)
        x_out[p] = fmaxf(0.0f, fmaf(-to, zb, xv));
      else
        zbar[p] = zb;
    }
    q2prev = q[2];
    if (k + 1 < kz1) {
      for (int c = 0; c < 3; ++c) {
        wo[c] = nwo[c];
        wh[c] = nwh[c];
      }
      zo = nzo;
      to = nto;
    }
    cur ^= 1;
    __syncthreads();
  }
}

// Row-major image (caller layout) -> layout L, ncomp components; padding is
// left untouched (zero).
__global__ __launch_bounds__(kBlock) void k_to_layout(const float *__restrict__ src, float *__restrict__ dst,
                                                      lmk::Layout L, int nx, int ny, int nz, long long ne,
                                                      int ncomp) {
  const long long nv = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nv) return;
  const int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((long long)nx * ny));
  const int q = lmk::vidx(L, i, j, k);
  for (int c = 0; c < ncomp; ++c) dst[c * ne + q] = src[c * nv + v];
}

// Layout L -> row-major image, ncomp components.
__global__ __launch_bounds__(kBlock) void k_from_layout(const float *__restrict__ src, float *__restrict__ dst,
                                                        lmk::Layout L, int nx, int ny, int nz, long long ne,
                                                        int ncomp) {
  const long long nv = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nv) return;
  const int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((long long)nx * ny));
  const int q = lmk::vidx(L, i, j, k);
  for (int c = 0; c < ncomp; ++c) dst[c * nv + v] = src[c * ne + q];
}

// gx = K x (three components).
__global__ __launch_bounds__(kBlock) void k_grad(const float *__restrict__ x, float *__restrict__ gx, int nx,
                                                 int ny, int nz) {
  const long long nv = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nv) return;
  const int i = (int)(v % nx);
  const int j = (int)((v / nx) % ny);
  const int k = (int)(v / ((long long)nx * ny));
  const float xv = x[v];
  gx[v] = (i < nx - 1) ? x[v + 1] - xv : 0.0f;
  gx[nv + v] = (j < ny - 1) ? x[v + nx] - xv : 0.0f;
  gx[2 * nv + v] = (k < nz - 1) ? x[v + (long long)nx * ny] - xv : 0.0f;
}

// out = -K^T w (the divergence).
__global__ __launch_bounds__(kBlock) void k_div(const float *__restrict__ w, float *__restrict__ out, int nx,
                                                int ny, int nz) {
  const long long nv = (long long)nx * ny * nz;
  const long long v = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (v >= nv) return;
  const int i = (int)(v % nx);
  const int j = (int)((v / nx) % ny);
  const int k = (int)(v / ((long long)nx * ny));
  const long long sxy = (long long)nx * ny;
  float d = 0.0f;
  if (i < nx - 1) d += w[v];
  if (i > 0) d -= w[v - 1];
  if (j < ny - 1) d += w[nv + v];
  if (j > 0) d -= w[nv + v - nx];
  if (k < nz - 1) d += w[2 * nv + v];
  if (k > 0) d -= w[2 * nv + v - sxy];
  out[v] = d;
}

}  // namespace

namespace lmk {

using lmk::Layout;

int launch_primal(float *x, const float *T, const float *zbar, long long nv, hipStream_t st) {
  hipLaunchKernelGGL(k_primal, dim3(grid_for(nv)), dim3(kBlock), 0, st, x, T, zbar, nv);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_dual_image(float *z, float *dz, float *x, const float *T, float *zbar, float inv_p, bool fuse,
                      long long nv, hipStream_t st) {
  hipLaunchKernelGGL(k_dual_image, dim3(grid_for(nv)), dim3(kBlock), 0, st, z, dz, x, T, zbar, inv_p,
                     fuse ? 1 : 0, nv);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_tv_fused(const int n[3], const Layout &L, int ncomp, const float *x, const float *w, float *w_out,
                    float *z, float *x_out, const float *T, float *zbar, float Sp, float beta, float inv_p, bool fuse,
                    hipStream_t st) {
  const long long ne = layout_size(L);
  if (L.sx == 2 && L.sy == 2 && L.sz == 2 && ncomp == 3) {
    constexpr int CZ = 4;
    const int nblocks = ((n[0] + 15) / 16) * ((n[1] + 15) / 16) * ((n[2] + CZ - 1) / CZ);
    hipLaunchKernelGGL((k_tv_march<CZ>), dim3(nblocks), dim3(kBlock), 0, st, x, w, w_out, z, x_out, T, zbar, L.nbx,
                       L.nby, n[0], n[1], n[2], ne, Sp, beta, inv_p, fuse ? 1 : 0, nblocks);
  } else if (L.sx == 2 && L.sy == 2 && L.sz == 2) {
    const int ntiles = ((L.nbx + 1) / 2) * ((L.nby + 1) / 2) * L.nbz;
    hipLaunchKernelGGL((k_tv_tiled<4, 4, 4, 2, 2>), dim3(ntiles), dim3(kBlock), 0, st, x, w, w_out, z, x_out, T, zbar,
                       L, n[0], n[1], n[2], ne, ncomp, Sp, beta, inv_p, fuse ? 1 : 0, ntiles);
  } else if (L.sx == 2 && L.sy == 2 && L.sz == 0 && n[2] == 1) {
    const int ntiles = ((L.nbx + 3) / 4) * ((L.nby + 3) / 4);
    hipLaunchKernelGGL((k_tv_tiled<4, 4, 1, 4, 4>), dim3(ntiles), dim3(kBlock), 0, st, x, w, w_out, z, x_out, T,
                       zbar, L, n[0], n[1], n[2], ne, ncomp, Sp, beta, inv_p, fuse ? 1 : 0, ntiles);
  } else {
    hipLaunchKernelGGL(k_tv_fused, dim3(grid_for(ne)), dim3(kBlock), 0, st, x, w, w_out, z, x_out, T, zbar, L, n[0],
                       n[1], n[2], ne, ncomp, Sp, beta, inv_p, fuse ? 1 : 0);
  }
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_to_layout(const int n[3], const Layout &L, int ncomp, const float *src, float *dst, hipStream_t st) {
  const long long nv = (long long)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_to_layout, dim3(grid_for(nv)), dim3(kBlock), 0, st, src, dst, L, n[0], n[1], n[2],
                     layout_size(L), ncomp);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_from_layout(const int n[3], const Layout &L, int ncomp, const float *src, float *dst, hipStream_t st) {
  const long long nv = (long long)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_from_layout, dim3(grid_for(nv)), dim3(kBlock), 0, st, src, dst, L, n[0], n[1], n[2],
                     layout_size(L), ncomp);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_grad(const int n[3], const float *x, float *gx, hipStream_t st) {
  const long long nv = (long long)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_grad, dim3(grid_for(nv)), dim3(kBlock), 0, st, x, gx, n[0], n[1], n[2]);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

int launch_div(const int n[3], const float *w, float *out, hipStream_t st) {
  const long long nv = (long long)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_div, dim3(grid_for(nv)), dim3(kBlock), 0, st, w, out, n[0], n[1], n[2]);
  LM_TRY_HIP(hipGetLastError());
  return LM_OK;
}

}  // namespace lmk

extern "C" {

static int check_dims(const int32_t n[3]) {
  LM_REQUIRE(n != nullptr, LM_EINVAL, "NULL size");
  for (int a = 0; a < 3; ++a)
    LM_REQUIRE(n[a] >= 1 && n[a] <= (1 << 20), LM_EINVAL, "image size n[%d]=%d invalid", a, n[a]);
  LM_REQUIRE((long long)n[0] * n[1] * n[2] < (1LL << 40), LM_EINVAL, "image too large");
  return LM_OK;
}

int tv_grad(const int32_t n[3], const float *x, float *gx, void *stream) {
  lmh::clear_error();
  if (int rc = check_dims(n)) return rc;
  LM_REQUIRE(x && gx, LM_EINVAL, "NULL array");
  const int nn[3] = {n[0], n[1], n[2]};
  return lmk::launch_grad(nn, x, gx, lmh::as_stream(stream));
}

int tv_div(const int32_t n[3], const float *w, float *out, void *stream) {
  lmh::clear_error();
  if (int rc = check_dims(n)) return rc;
  LM_REQUIRE(w && out, LM_EINVAL, "NULL array");
  const int nn[3] = {n[0], n[1], n[2]};
  return lmk::launch_div(nn, w, out, lmh::as_stream(stream));
}

}  // extern "C"
