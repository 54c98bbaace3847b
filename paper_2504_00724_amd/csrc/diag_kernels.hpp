// Device kernel of the on-demand residual diagnostics (gfx950): maximum and
// sum of squares of the residual of a caller's iterate over the non-empty
// level-0 cells.  Not part of a solve.  The host side is ccgmg.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "vcycle_kernels.hpp"

// Partial maximum and sum of squares of r - bterm - L u (zero_u: of
// r - bterm) per workgroup, in the layout of the residual-norm launch:
// workgroups [0, nrb) take BLOCK explicit rows each, the others one TX x TY
// tile of stencil cells.  partial[2 * (z * gridDim.x + b)] is the maximum,
// the next entry the sum of squares (both reduced in a fixed order).
template <bool CROSS>
__global__ __launch_bounds__(BLOCK) void k_res_norms(const double* __restrict__ u, const double* __restrict__ r,
                                                     const uint8_t* __restrict__ kind, int nx, int ny, int nbx,
                                                     int ntiles, CoefT<double> c, int zero_u,
                                                     const double* __restrict__ bterm,
                                                     const int32_t* __restrict__ cell, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ cols,
                                                     const double* __restrict__ vals,
                                                     const double* __restrict__ rowsum, int nrows,
                                                     double* __restrict__ partial) {
  __shared__ double tile[LH][LW];
  __shared__ double red[2][BLOCK / 64];
  const int z = blockIdx.z;
  const size_t plane = (size_t)nx * ny;
  const double* uz = u + z * plane;
  const double* rz = r + z * plane;
  const int nrb = (int)gridDim.x - ntiles;
  const int l = blockIdx.x;
  double mx = 0.0, sq = 0.0;
  if (l >= nrb) {
    const int t = l - nrb;
    const int tyi = t / nbx;
    const int bx = (t - tyi * nbx) * TX, by = tyi * TY;
    const int tx = threadIdx.x & (TX - 1), w = threadIdx.x >> 6;
    load_tile(tile, uz, nx, ny, bx, by);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TY / 4; ++k) {
      const int gx = bx + tx, gy = by + w + 4 * k;
      if (gx < nx && gy < ny && (kind[(size_t)gy * nx + gx] & F_REG)) {
        double v = rz[(size_t)gy * nx + gx];
        if (!zero_u) v -= apply_regular<double, CROSS>(tile, w + 4 * k + HALO, tx + HALO, c);
        mx = nanmax(mx, fabs(v));
        sq += v * v;
      }
    }
  } else {
    const int k = l * BLOCK + threadIdx.x;
    if (k < nrows) {
      const int q = cell[k];
      double v = rz[q];
      if (bterm) v -= bterm[(size_t)z * nrows + k];
      if (!zero_u) v = row_residual(uz, v, q, cols + rp[k], vals + rp[k], rp[k + 1] - rp[k], rowsum[k]);
      mx = fabs(v);
      sq = v * v;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    mx = nanmax(mx, __shfl_xor(mx, off, 64));
    sq += __shfl_xor(sq, off, 64);
  }
  if ((threadIdx.x & 63) == 0) red[0][threadIdx.x >> 6] = mx, red[1][threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0][0], s = red[1][0];
    for (int i = 1; i < BLOCK / 64; ++i) m = nanmax(m, red[0][i]), s += red[1][i];
    const size_t o = 2 * ((size_t)z * gridDim.x + blockIdx.x);
    partial[o] = m;
    partial[o + 1] = s;
  }
}

// Totals of the partials written by k_res_norms: workgroup (k, z) reduces
// the np (maximum, sum of squares) pairs of plane z of launch k (0: the
// reference r - bterm, 1: the residual r - bterm - L u), stored at
// part + k * per, into out[4 z + 2 k] (maximum) and out[4 z + 2 k + 1] (sum
// of squares).  Fixed order (strided per thread, then a tree), so repeated
// calls give identical totals.
__global__ __launch_bounds__(BLOCK) void k_norm_finish(const double* __restrict__ part, size_t per, int np,
                                                       double* __restrict__ out) {
  __shared__ double red[2][BLOCK];
  const int k = blockIdx.x, z = blockIdx.y;
  const double* p = part + k * per + 2 * (size_t)z * np;
  double mx = 0.0, sq = 0.0;
  for (int b = threadIdx.x; b < np; b += BLOCK) {
    mx = nanmax(mx, p[2 * b]);
    sq += p[2 * b + 1];
  }
  red[0][threadIdx.x] = mx;
  red[1][threadIdx.x] = sq;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] = nanmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[4 * (size_t)z + 2 * k] = red[0][0];
    out[4 * (size_t)z + 2 * k + 1] = red[1][0];
  }
}
