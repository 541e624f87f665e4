// Image-space kernels of LM-SPDHG on gfx950: the primal step with the
// non-negativity prox, the z / zbar updates, the TV dual update with its
// adjoint stencil, the layout conversions, and the tv_grad / tv_div entry
// points.
//
// All of these stream whole images and are bound by memory bandwidth.  Plan
// images are in 4x4x4-voxel bricks (4x4x1 for one slice); the element-wise
// passes take one voxel per thread in layout order, the prior update stages
// x through LDS (a tile for one slice, a column marching along z in 3D), and
// every pass that can be fused with the next primal step is.  The
// conversions and tv_grad / tv_div address the caller's row-major images.
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

// The whole prior update, tiled through LDS (used for single-slice images;
// 3D images take the z-marching kernel below).  A block owns a tile of
// TBX x TBY x 1 bricks (4 x 4 bricks of 4x4x1 voxels: 256 voxels);
// wavefront w reads brick w of the tile, so those loads are whole bricks.
// The tile stages x with a one-voxel halo and computes
// q = proj_beta(w + S K x) - w once for the tile and its lower halo (K^T q at
// a voxel needs q at the voxel and at its lower neighbours), then forms
// dz = K^T q, z, zbar and the fused primal step.  Every global load of the
// block is issued before the first barrier.  Tiles are numbered so that
// each XCD (blocks are dealt to the 8 XCDs round robin) works on one
// contiguous run of tiles, which keeps the halo reads of neighbouring tiles
// in that XCD's L2.  x and w are read-only; results go to x_out and w_out.
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

// The part of the index of voxel (i, j, k) in the 4x4x4 brick layout (nbx
// bricks along x) that depends on (i, j); the k part is added per plane.
__device__ __forceinline__ int brick_ij(int nbx, int i, int j) {
  return (((j >> 2) * nbx + (i >> 2)) << 6) | ((j & 3) << 2) | (i & 3);
}

// The whole prior update for a 3D image in the 4x4x4 brick layout, marching
// along z two planes per step: TV, or with DTV = true the directional TV of
// Section 3 (K = D grad, D = I - xi xi^T per voxel: the dual step takes D g
// and K^T takes D (w+ - w); xi is read next to w, 56 instead of 44 bytes
// per voxel).  A block owns a 16 x 16 column and a run of
// CZ planes (CZ even, so a step covers planes k and k+1 of one brick layer
// and writes whole 128-byte lines of every brick).  Thread t owns voxel
// (t & 3) + 4 (t >> 4 & 3), ((t >> 2) & 3) + 4 (t >> 6) of the column in
// every plane, so a wavefront reads four 64-byte brick slabs per plane; K^T q
// needs q at the three lower neighbours, which are the thread's own q of the
// plane below (z), LDS (x, y) or the lower faces of the column's ring.
// Columns are dealt so that each XCD works on a contiguous run (halo reads
// stay in its L2).  x and w are read-only; results go to x_out and w_out.  The
// dual step of the plane below the run is computed first (own voxels only);
// it feeds the z-difference of the run's first plane.  Per step the block
// holds x of planes k, k+1, k+2 with a one-voxel ring in LDS (three 18 x 18
// buffers, used as a ring) and x of planes k+3, k+4 in registers (loaded one
// step ahead); w, z and T of the next two planes are loaded one step ahead.
// Threads 0..31 compute the lower-face dual steps of plane k, threads
// 32..63 those of plane k+1; threads 0..135 load the x ring of two planes.
template <int CZ, bool DTV>
__global__ __launch_bounds__(kBlock) void k_tv_march(const float *__restrict__ x, const float *__restrict__ w,
                                                      const float *__restrict__ xi, float *__restrict__ w_out,
                                                      float *__restrict__ z,
                                                      float *__restrict__ x_out, const float *__restrict__ T,
                                                      float *__restrict__ zbar, int nbx, int nby, int nx, int ny,
                                                      int nz, long long ne, float Sp, float beta, float inv_p,
                                                      int fuse, int nblocks) {
  static_assert(CZ % 2 == 0, "two planes per step");
  constexpr int B = 18;  // x box: x0-1 .. x0+16
  constexpr int Q = 17;  // q box: x0-1 .. x0+15
  __shared__ float xb[3][B * B];
  __shared__ float q0s[2][Q * Q], q1s[2][Q * Q];
  int blk = blockIdx.x;
  const int full = nblocks & ~7;
  if (blk < full) blk = (blk & 7) * (full >> 3) + (blk >> 3);
  const int ntx = (nx + 15) >> 4, nty = (ny + 15) >> 4;
  const int cx = blk % ntx, cy = (blk / ntx) % nty, cz = blk / (ntx * nty);
  const int x0 = cx * 16, y0 = cy * 16;
  const int kz0 = cz * CZ, kz1 = min(nz, kz0 + CZ);
  const int t = threadIdx.x;
  // own voxel (one per thread in every plane)
  const int ti = (t & 3) + 4 * ((t >> 4) & 3), tj = ((t >> 2) & 3) + 4 * (t >> 6);
  const int i = x0 + ti, j = y0 + tj;
  const bool own = i < nx && j < ny;
  const int own_b = (ti + 1) + B * (tj + 1), own_q = (ti + 1) + Q * (tj + 1);
  const int own_ij = own ? brick_ij(nbx, i, j) : 0;
  // ring of the x box: threads 0..67 plane a, 68..135 plane a+1 of a pair
  int rb = -1, r_ij = 0, rpl = 0;
  bool r_ok = false;
  if (t < 136) {
    const int r = t < 68 ? t : t - 68;
    rpl = t < 68 ? 0 : 1;
    int bx, by;
    if (r < 18) { bx = r; by = 0; }
    else if (r < 36) { bx = r - 18; by = 17; }
    else if (r < 52) { bx = 0; by = r - 35; }
    else { bx = 17; by = r - 51; }
    rb = bx + B * by;
    const int gi = x0 - 1 + bx, gj = y0 - 1 + by;
    r_ok = gi >= 0 && gi < nx && gj >= 0 && gj < ny;
    r_ij = r_ok ? brick_ij(nbx, gi, gj) : 0;
  }
  // lower-face dual steps: threads 0..31 plane k, 32..63 plane k+1
  int hb = 0, hq = 0, h_ij = 0, hgi = 0, hgj = 0, hpl = 0;
  bool h_ok = false;
  if (t < 64) {
    const int u = t & 31;
    hpl = t >> 5;
    const int bx = u < 16 ? 0 : u - 15, by = u < 16 ? u + 1 : 0;
    hb = bx + B * by;
    hq = bx + Q * by;
    hgi = x0 - 1 + bx;
    hgj = y0 - 1 + by;
    h_ok = hgi >= 0 && hgi < nx && hgj >= 0 && hgj < ny;
    h_ij = h_ok ? brick_ij(nbx, hgi, hgj) : 0;
  }
  const int koff_layer = (nby * nbx) << 6;
  auto koff = [&](int k) { return (k >> 2) * koff_layer + ((k & 3) << 4); };
  // x of the own voxel of plane k and of this thread's ring position of
  // plane k + rpl (0 where outside the image)
  auto load_own = [&](int k) { return (own && k < nz) ? x[own_ij + koff(k)] : 0.0f; };
  auto load_ring = [&](int k) { return (r_ok && k + rpl < nz) ? x[r_ij + koff(k + rpl)] : 0.0f; };
  // dual step at a voxel with forward differences g and dual w: q = the
  // increment K^T needs, wn = the new dual.  TV: q = wn - w.  DTV (K = D
  // grad, D = I - e e^T with e the voxel's xi): the step takes D g, and q =
  // D (wn - w).
  auto prox = [&](float gx, float gy, float gz, const float (&wv)[3], const float (&e)[3], float (&q)[3],
                  float (&wn)[3]) {
    if constexpr (DTV) {
      const float eg = fmaf(e[2], gz, fmaf(e[1], gy, e[0] * gx));
      gx = fmaf(-e[0], eg, gx);
      gy = fmaf(-e[1], eg, gy);
      gz = fmaf(-e[2], eg, gz);
    }
    const float v0 = fmaf(Sp, gx, wv[0]), v1 = fmaf(Sp, gy, wv[1]), v2 = fmaf(Sp, gz, wv[2]);
    const float nrm = sqrtf(fmaf(v0, v0, fmaf(v1, v1, v2 * v2)));
    const float sc = 1.0f / fmaxf(1.0f, nrm / beta);
    if constexpr (DTV) {
      wn[0] = v0 * sc;
      wn[1] = v1 * sc;
      wn[2] = v2 * sc;
      const float d0 = wn[0] - wv[0], d1 = wn[1] - wv[1], d2 = wn[2] - wv[2];
      const float ed = fmaf(e[2], d2, fmaf(e[1], d1, e[0] * d0));
      q[0] = fmaf(-e[0], ed, d0);
      q[1] = fmaf(-e[1], ed, d1);
      q[2] = fmaf(-e[2], ed, d2);
    } else {
      q[0] = v0 * sc - wv[0];
      q[1] = v1 * sc - wv[1];
      q[2] = v2 * sc - wv[2];
      wn[0] = wv[0] + q[0];
      wn[1] = wv[1] + q[1];
      wn[2] = wv[2] + q[2];
    }
  };
  // xi of layout position p (DTV), else zeros
  auto load_e = [&](int p, float (&e)[3]) {
    if constexpr (DTV) {
      e[0] = xi[p];
      e[1] = xi[ne + p];
      e[2] = xi[2 * ne + p];
    } else {
      e[0] = e[1] = e[2] = 0.0f;
    }
  };
  // dual step of the plane below the run, own voxels only (its z-component
  // feeds the first plane's z-difference)
  float q2prev = 0.0f;
  if (kz0 > 0) {
    const int kb = kz0 - 1;
    // planes kb (own + ring) and kz0 (own) through LDS buffers 0 and 1
    xb[0][own_b] = load_own(kb);
    if (rb >= 0 && rpl == 0) xb[0][rb] = load_ring(kb);
    const float xup = load_own(kz0);
    float wb[3] = {0.0f, 0.0f, 0.0f}, eb[3] = {0.0f, 0.0f, 0.0f};
    if (own) {
      const int p = own_ij + koff(kb);
      wb[0] = w[p];
      wb[1] = w[ne + p];
      wb[2] = w[2 * ne + p];
      load_e(p, eb);
    }
    __syncthreads();
    const float xv = xb[0][own_b];
    const float gx = (i < nx - 1) ? xb[0][own_b + 1] - xv : 0.0f;
    const float gy = (j < ny - 1) ? xb[0][own_b + B] - xv : 0.0f;
    const float gz = xup - xv;  // kb < nz - 1
    float qb[3], wnb[3];
    prox(gx, gy, gz, wb, eb, qb, wnb);
    q2prev = qb[2];
    __syncthreads();
  }
  // planes kz0, kz0+1, kz0+2 into LDS; kz0+3, kz0+4 into registers
  int bk0 = 0, bk1 = 1, bk2 = 2;  // LDS buffers of planes k, k+1, k+2
  xb[0][own_b] = load_own(kz0);
  xb[1][own_b] = load_own(kz0 + 1);
  xb[2][own_b] = load_own(kz0 + 2);
  if (rb >= 0) {
    // ring threads of plane a load planes a = kz0 and kz0+2; those of
    // plane a+1 load kz0+1
    if (rpl == 0) {
      xb[0][rb] = load_ring(kz0);
      xb[2][rb] = load_ring(kz0 + 2);
    } else {
      xb[1][rb] = load_ring(kz0);
    }
  }
  float pxo0 = load_own(kz0 + 3), pxo1 = load_own(kz0 + 4), pxr = load_ring(kz0 + 3);
  // w, z, T (and xi) of the own voxel for planes k, k+1; w (and xi) of the
  // face voxel
  float wo[2][3], zo[2], to[2], wh[3], eo[2][3], eh[3];
  auto load_w = [&](int k, float (&wv)[2][3], float (&zv)[2], float (&tv)[2], float (&whv)[3], float (&ev)[2][3],
                    float (&ehv)[3]) {
    for (int s = 0; s < 2; ++s) {
      wv[s][0] = wv[s][1] = wv[s][2] = zv[s] = tv[s] = 0.0f;
      ev[s][0] = ev[s][1] = ev[s][2] = 0.0f;
      if (own && k + s < kz1) {
        const int p = own_ij + koff(k + s);
        wv[s][0] = w[p];
        wv[s][1] = w[ne + p];
        wv[s][2] = w[2 * ne + p];
        zv[s] = z[p];
        if (fuse) tv[s] = T[p];
        load_e(p, ev[s]);
      }
    }
    whv[0] = whv[1] = whv[2] = 0.0f;
    ehv[0] = ehv[1] = ehv[2] = 0.0f;
    if (h_ok && k + hpl < kz1) {
      const int p = h_ij + koff(k + hpl);
      whv[0] = w[p];
      whv[1] = w[ne + p];
      whv[2] = w[2 * ne + p];
      load_e(p, ehv);
    }
  };
  load_w(kz0, wo, zo, to, wh, eo, eh);
  __syncthreads();
  for (int k = kz0; k < kz1; k += 2) {
    // loads for the next step: x of planes k+5, k+6; w, z, T of k+2, k+3
    const float nxo0 = load_own(k + 5), nxo1 = load_own(k + 6), nxr = load_ring(k + 5);
    float nwo[2][3], nzo[2], nto[2], nwh[3], neo[2][3], neh[3];
    load_w(k + 2, nwo, nzo, nto, nwh, neo, neh);
    const float *xa = xb[bk0], *xc = xb[bk1], *xd = xb[bk2];
    // own dual steps of planes k (s = 0) and k+1 (s = 1)
    float q[2][3], xv[2];
    for (int s = 0; s < 2; ++s) {
      const float *xs = s ? xc : xa, *xu = s ? xd : xc;
      const int kk = k + s;
      xv[s] = xs[own_b];
      const float gx = (i < nx - 1) ? xs[own_b + 1] - xv[s] : 0.0f;
      const float gy = (j < ny - 1) ? xs[own_b + B] - xv[s] : 0.0f;
      const float gz = (kk < nz - 1) ? xu[own_b] - xv[s] : 0.0f;
      float wn[3];
      prox(gx, gy, gz, wo[s], eo[s], q[s], wn);
      q0s[s][own_q] = q[s][0];
      q1s[s][own_q] = q[s][1];
      if (own && kk < kz1) {
        const int p = own_ij + koff(kk);
        w_out[p] = wn[0];
        w_out[ne + p] = wn[1];
        w_out[2 * ne + p] = wn[2];
      }
    }
    // lower-face dual steps (the component the own voxels need)
    if (t < 64) {
      float hq3[3] = {0.0f, 0.0f, 0.0f};
      const int kk = k + hpl;
      if (h_ok && kk < kz1) {
        const float *xs = hpl ? xc : xa, *xu = hpl ? xd : xc;
        const float hv = xs[hb];
        const float gx = (hgi < nx - 1) ? xs[hb + 1] - hv : 0.0f;
        const float gy = (hgj < ny - 1) ? xs[hb + B] - hv : 0.0f;
        const float gz = (kk < nz - 1) ? xu[hb] - hv : 0.0f;
        float hwn[3];
        prox(gx, gy, gz, wh, eh, hq3, hwn);
      }
      if ((t & 31) < 16)
        q0s[hpl][hq] = hq3[0];
      else
        q1s[hpl][hq] = hq3[1];
    }
    __syncthreads();
    // planes k+3, k+4 (loaded one step ago) replace k and k+1 in LDS
    xb[bk0][own_b] = pxo0;
    xb[bk1][own_b] = pxo1;
    if (rb >= 0) xb[rpl ? bk1 : bk0][rb] = pxr;
    pxo0 = nxo0;
    pxo1 = nxo1;
    pxr = nxr;
    if (own) {
      for (int s = 0; s < 2; ++s) {
        const int kk = k + s;
        if (kk >= kz1) break;
        float dz = 0.0f;
        if (i < nx - 1) dz -= q0s[s][own_q];
        if (i > 0) dz += q0s[s][own_q - 1];
        if (j < ny - 1) dz -= q1s[s][own_q];
        if (j > 0) dz += q1s[s][own_q - Q];
        if (kk < nz - 1) dz -= q[s][2];
        if (kk > 0) dz += s ? q[0][2] : q2prev;
        const int p = own_ij + koff(kk);
        const float zn = zo[s] + dz;
        const float zb = fmaf(dz, inv_p, zn);
        z[p] = zn;
        if (fuse)
          x_out[p] = fmaxf(0.0f, fmaf(-to[s], zb, xv[s]));
        else
          zbar[p] = zb;
      }
    }
    q2prev = q[1][2];
    for (int s = 0; s < 2; ++s) {
      zo[s] = nzo[s];
      to[s] = nto[s];
      for (int c = 0; c < 3; ++c) {
        wo[s][c] = nwo[s][c];
        eo[s][c] = neo[s][c];
      }
    }
    for (int c = 0; c < 3; ++c) {
      wh[c] = nwh[c];
      eh[c] = neh[c];
    }
    // the buffer of plane k+2 becomes plane k of the next step
    const int b0 = bk0, b1 = bk1;
    bk0 = bk2;
    bk1 = b0;
    bk2 = b1;
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

bool prior_march_ok(const Layout &L, int ncomp) { return L.sx == 2 && L.sy == 2 && L.sz == 2 && ncomp == 3; }

int launch_tv_fused(const int n[3], const Layout &L, int ncomp, const float *x, const float *w, const float *xi,
                    float *w_out, float *z, float *x_out, const float *T, float *zbar, float Sp, float beta,
                    float inv_p, bool fuse, hipStream_t st) {
  const long long ne = layout_size(L);
  if (prior_march_ok(L, ncomp)) {
    constexpr int CZ = 16;
    const int nblocks = ((n[0] + 15) / 16) * ((n[1] + 15) / 16) * ((n[2] + CZ - 1) / CZ);
    if (xi)
      hipLaunchKernelGGL((k_tv_march<CZ, true>), dim3(nblocks), dim3(kBlock), 0, st, x, w, xi, w_out, z, x_out, T,
                         zbar, L.nbx, L.nby, n[0], n[1], n[2], ne, Sp, beta, inv_p, fuse ? 1 : 0, nblocks);
    else
      hipLaunchKernelGGL((k_tv_march<CZ, false>), dim3(nblocks), dim3(kBlock), 0, st, x, w, xi, w_out, z, x_out, T,
                         zbar, L.nbx, L.nby, n[0], n[1], n[2], ne, Sp, beta, inv_p, fuse ? 1 : 0, nblocks);
  } else if (xi) {
    lmh::set_error("prior update by column march: the image layout must be 4x4x4 bricks with 3 components");
    return LM_EINVAL;
  } else if (L.sx == 2 && L.sy == 2 && L.sz == 0 && n[2] == 1) {
    const int ntiles = ((L.nbx + 3) / 4) * ((L.nby + 3) / 4);
    hipLaunchKernelGGL((k_tv_tiled<4, 4, 1, 4, 4>), dim3(ntiles), dim3(kBlock), 0, st, x, w, w_out, z, x_out, T,
                       zbar, L, n[0], n[1], n[2], ne, ncomp, Sp, beta, inv_p, fuse ? 1 : 0, ntiles);
  } else {
    lmh::set_error("prior update: the image layout must be 4x4x4 bricks (or 4x4x1 for one slice)");
    return LM_EINVAL;
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
