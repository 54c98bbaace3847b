// Device kernels of the cut-cell multigrid V-cycle (gfx950): SMO-1 sweeps,
// SMO-2 block updates, the fused smoothing step, residual + restriction,
// prolongation, residual norms, the coarsest solve and the mixed-precision
// helpers.  The host driver that launches them is ccgmg.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "kernels.hpp"

// private header of ccgmg.hip (included once); kernels keep global names
using namespace ccgk;

// cell flag bits of kind[]
constexpr uint8_t F_REG = 1;      // regular row of L
constexpr uint8_t F_NONEMPTY = 2;
constexpr uint8_t F_REG_T = 4;    // regular row of L^T
constexpr uint8_t F_JAC = 8;      // smoothed by SMO-1 (L)
constexpr uint8_t F_JAC_T = 16;   // smoothed by SMO-1 (L^T)
constexpr uint8_t F_S2 = 32;      // row of an SMO-2 block (L)
constexpr uint8_t F_S2_T = 64;    // row of an SMO-2 block (L^T)

// ===========================================================================
// Kernels
// ===========================================================================

// SMO-1 on one tile: u_out = u + omega/D (r - L u) on cells flagged `regbit`,
// u_out = u elsewhere except on cells flagged `skipbit` (left to the SMO-2
// blocks of a fused step).  Jacobi: reads u, writes a second buffer.  Tiles
// of TX x TYS cells (TYS = 8, 16 or 32, picked per level by measurement);
// t is the tile index, nbx the number of tiles per grid row.
// LDS of one tile: the (TYS + 4) x (TX + 4) neighbourhood of u, and with the
// cross-derivative term (CROSS) a TYS x (TX + 4) tile of y-differences.
template <typename T, int TYS, bool CROSS = false>
constexpr int sweep_lds_doubles() {
  return ((TYS + 2 * HALO + (CROSS ? TYS : 0)) * LW * (int)sizeof(T) + 7) / 8;
}

// NORM: also returns the thread's norm accumulators of r - L u over the
// cells it updates (the residual of the old iterate the update uses).
template <typename T, bool CROSS, int TYS, bool PRO = false, bool NORM = false>
__device__ __forceinline__ NormAcc sweep_tile(double* smem, int t, const T* __restrict__ u, const T* __restrict__ r,
                                             const uint8_t* __restrict__ kind, T* __restrict__ out, int nx, int ny,
                                             int nbx, const CoefT<T>& c, uint8_t regbit, uint8_t skipbit,
                                             const T* __restrict__ e = nullptr, int ncx = 0, uint8_t probit = 0) {
  NormAcc m;
  constexpr int RPW = TYS / 4;            // rows per wave
  constexpr int ROWS = TYS + 2 * HALO;
  T (*tile)[LW] = reinterpret_cast<T (*)[LW]>(smem);
  const int tyi = t / nbx;
  const int bx = (t - tyi * nbx) * TX, by = tyi * TYS;
  const int tx = threadIdx.x & (TX - 1), w = threadIdx.x >> 6;
  // row of the k-th cell of this thread: interleaved over the 4 waves, or
  // (cross-derivative stencil) RPW contiguous rows per wave, swept with a
  // register window
  auto row_of = [&](int k) { return CROSS ? w * RPW + k : w + 4 * k; };
  // the plane through buffer views (planes stay below 2^31 bytes): a cell
  // outside the grid reads flags 0 and value 0, and a store there (or to a
  // cell left to the SMO-2 blocks, given offset BUF_OUT) is dropped
  const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
  const bufrsrc br = make_buf(r, plane * (uint32_t)sizeof(T)), bk = make_buf(kind, plane),
                bo = make_buf(out, plane * (uint32_t)sizeof(T));
  const int gx = bx + tx;
  const int g0 = (unsigned)gx < (unsigned)nx ? by * nx + gx : BUF_OUT;   // this thread's column, tile row 0
  auto gcell = [&](int k) { return g0 == BUF_OUT ? BUF_OUT : g0 + row_of(k) * nx; };
  // issue the kind and right-hand-side loads before the tile barrier
  uint8_t kd[RPW];
  T rr[RPW];
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int g = gcell(k);
    kd[k] = buf_ld<uint8_t>(bk, g);
    rr[k] = buf_ld<T>(br, g == BUF_OUT ? BUF_OUT : g * (int)sizeof(T));
  }
  if (PRO) {
    // tile of u + P e: the pending coarse-grid correction (piecewise
    // constant, cells flagged probit only) is added while staging.  A level
    // with a coarser one has even sides, so the parent (gy/2, gx/2) of an
    // in-grid cell is a coarse cell: its value is loaded alongside u and
    // kind (no load waits for the flag) and selected by the flag
    // (the loads of 5 entries per thread first, then their combination:
    // no load waits behind another)
    constexpr int N = ROWS * LW, NIT = (N + BLOCK - 1) / BLOCK, CH = 5;
#pragma unroll
    for (int i0 = 0; i0 < NIT; i0 += CH) {
      T uv[CH], ev[CH];
      uint8_t kb[CH];
      bool inn[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        if (i0 + i < NIT) {
          const int k = (int)threadIdx.x + (i0 + i) * BLOCK;
          const int kk = k < N ? k : 0;
          const int ly = kk / LW, lx = kk - ly * LW;
          const int gx = bx + lx - HALO, gy = by + ly - HALO;
          inn[i] = k < N && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
          const size_t g = inn[i] ? (size_t)gy * nx + gx : 0;
          uv[i] = u[g];
          kb[i] = kind[g];
          ev[i] = e[inn[i] ? (size_t)(gy >> 1) * ncx + (gx >> 1) : 0];
        }
      }
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int k = (int)threadIdx.x + (i0 + i) * BLOCK;
        if (i0 + i < NIT && k < N) {
          const int ly = k / LW, lx = k - ly * LW;
          const T w = (kb[i] & probit) ? uv[i] + ev[i] : uv[i];
          tile[ly][lx] = inn[i] ? w : (T)0;
        }
      }
    }
  } else {
    stage_cols<T, ROWS, HALO>(tile, make_buf(u, plane * (uint32_t)sizeof(T)), nx, ny, bx, by);
  }
  __syncthreads();
  if (CROSS) {
    // the cross-derivative term is a difference in x of the y-differences
    // Dy(y, x) = 8 (u(y+1) - u(y-1)) - (u(y+2) - u(y-2)): they are formed
    // once per tile column into a second LDS tile (each wave's own columns
    // from a vertical window of 5 values, then the 4 halo columns), so a
    // cell reads 4 of them instead of the 16 values they come from
    T (*dyt)[LW] = tile + ROWS;
    const int r0 = w * RPW;   // tile row of the wave's first cell (before HALO offset)
    {
      T c0 = tile[r0][tx + HALO], c1 = tile[r0 + 1][tx + HALO], c2 = tile[r0 + 2][tx + HALO],
        c3 = tile[r0 + 3][tx + HALO];
#pragma unroll
      for (int k = 0; k < RPW; ++k) {
        const T c4 = tile[r0 + k + 4][tx + HALO];
        dyt[r0 + k][tx + HALO] = (T)8 * (c3 - c1) - (c4 - c0);
        c0 = c1, c1 = c2, c2 = c3, c3 = c4;
      }
      for (int h = threadIdx.x; h < TYS * 2 * HALO; h += BLOCK) {
        const int y = h / (2 * HALO), q = h - y * (2 * HALO);
        const int lx = q < HALO ? q : TX + q;
        dyt[y][lx] = (T)8 * (tile[y + 3][lx] - tile[y + 1][lx]) - (tile[y + 4][lx] - tile[y][lx]);
      }
    }
    __syncthreads();
    T c0 = tile[r0][tx + HALO], c1 = tile[r0 + 1][tx + HALO], c2 = tile[r0 + 2][tx + HALO],
      c3 = tile[r0 + 3][tx + HALO];
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const T c4 = tile[r0 + k + 4][tx + HALO];
      const int g = gcell(k);
      T v = c2;
      if ((kd[k] & regbit) && !(kd[k] & skipbit)) {
        const T* row = tile[r0 + k + HALO] + tx + HALO;
        const T* dyr = dyt[r0 + k] + tx + HALO;
        const T d = rr[k] - regular_row_dy<T>(
                                c2, row[1], row[-1], row[2], row[-2], c3, c1, c4, c0,
                                [&](int dx) { return dyr[dx]; }, c);
        if (NORM) m.add((double)d);
        v += c.omega_invD * d;
      }
      buf_st(bo, (kd[k] & skipbit) || g == BUF_OUT ? BUF_OUT : g * (int)sizeof(T), v);
      c0 = c1, c1 = c2, c2 = c3, c3 = c4;
    }
    return m;
  }
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int ry = w + 4 * k;
    const int g = gcell(k);
    T v = tile[ry + HALO][tx + HALO];
    if ((kd[k] & regbit) && !(kd[k] & skipbit)) {
      const T d = rr[k] - apply_regular<T, CROSS>(tile, ry + HALO, tx + HALO, c);
      if (NORM) m.add((double)d);
      v += c.omega_invD * d;
    }
    buf_st(bo, (kd[k] & skipbit) || g == BUF_OUT ? BUF_OUT : g * (int)sizeof(T), v);
  }
  return m;
}

// SMO-1 sweep launch: one workgroup per tile on a 1-D grid remapped by
// xcd_tile.  FINEST only selects a separate instantiation for the finest
// level so that kernel traces separate it from the coarse levels.
template <typename T, bool CROSS, bool FINEST, int TYS>
__global__ __launch_bounds__(BLOCK) void k_sweep(const T* __restrict__ u, const T* __restrict__ r,
                                                 const uint8_t* __restrict__ kind, T* __restrict__ out, int nx,
                                                 int ny, int nbx, CoefT<T> c, uint8_t regbit) {
  __shared__ double smem[sweep_lds_doubles<T, TYS, CROSS>()];
  const size_t zoff = (size_t)blockIdx.z * nx * ny;
  sweep_tile<T, CROSS, TYS>(smem, xcd_tile(blockIdx.x, gridDim.x), u + zoff, r + zoff, kind, out + zoff, nx, ny,
                            nbx, c, regbit, 0);
}

// Two SMO-1 sweeps in one launch: two consecutive plain sweeps (no SMO-2
// between them, so the block rows keep their values) by temporal blocking.
// A workgroup stages u on its tile plus a halo of 4, sweeps the tile plus a
// halo of 2 into a second LDS tile, then sweeps its tile from that into
// out: the same operations per cell as two k_sweep launches, but u', the
// intermediate iterate, never leaves LDS (25 instead of 50 bytes per cell
// for the pair, one launch instead of two).  With the cross-derivative term
// (CROSS) each sweep first forms the y-differences of its input in LDS (as
// sweep_tile does), the second sweep's in the first one's space.
template <typename T, int TYS, bool CROSS>
constexpr int sweep2_lds_doubles() {
  constexpr int W0 = TX + 4 * HALO, R0 = TYS + 4 * HALO, R1 = TYS + 2 * HALO;
  return ((R0 * W0 + R1 * LW + (CROSS ? R1 * W0 : 0)) * (int)sizeof(T) + 7) / 8;
}

// One tile t of one plane (pointers already offset to the plane); smem
// holds sweep2_lds_doubles<T, TYS, CROSS>() doubles.
template <typename T, bool CROSS, int TYS>
__device__ __forceinline__ void sweep2_tile(double* smem, int t, const T* __restrict__ u, const T* __restrict__ r,
                                            const uint8_t* __restrict__ kind, T* __restrict__ out, int nx, int ny,
                                            int nbx, const CoefT<T>& c, uint8_t regbit) {
  constexpr int H2 = 2 * HALO;
  constexpr int W0 = TX + 2 * H2, R0 = TYS + 2 * H2;    // u on the tile plus 4
  constexpr int R1 = TYS + 2 * HALO;                    // u' on the tile plus 2 (LW columns)
  constexpr int RPW = TYS / 4, M0 = R0 / 4, M1 = R1 / 4;
  T (*t0)[W0] = reinterpret_cast<T (*)[W0]>(smem);
  T (*t1)[LW] = reinterpret_cast<T (*)[LW]>(smem + (R0 * W0 * (int)sizeof(T) + 7) / 8);
  T (*dy)[W0] = reinterpret_cast<T (*)[W0]>(smem + ((R0 * W0 + R1 * LW) * (int)sizeof(T) + 7) / 8);
  const int tyi = t / nbx;
  const int bx = (t - tyi * nbx) * TX, by = tyi * TYS;
  const int tx = threadIdx.x & (TX - 1), w = threadIdx.x >> 6, q = threadIdx.x;
  const unsigned unx = nx, uny = ny;
  // Work split: thread (w, tx) owns tile column tx (grid column gx) and the
  // rows w, w + 4, ... of each region; the columns left and right of the
  // tile's 64 are taken by threads q = 0, 1, ... in a pass of their own.
  // Loads and stores go through buffer views of the plane (the launcher
  // keeps planes below 2^31 bytes): an offset outside the plane reads 0 and
  // writes nothing, so a cell outside the grid (a row above or below it, or
  // the whole column when gx >= nx) stages value 0 and flags 0 with no select.
  const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
  const bufrsrc bu = make_buf(u, plane * (uint32_t)sizeof(T)), br = make_buf(r, plane * (uint32_t)sizeof(T)),
                bk = make_buf(kind, plane), bo = make_buf(out, plane * (uint32_t)sizeof(T));
  constexpr int SZ = (int)sizeof(T);
  const int gx = bx + tx;
  const bool xin = (unsigned)gx < unx;
  // cell index of row gyy of this thread's column (BUF_OUT off the grid's
  // columns; rows above the grid give negative, rows below it too large
  // indices, both outside the plane)
  auto col_idx = [&](int gyy) { return xin ? gyy * nx + gx : BUF_OUT; };
  auto col_off = [&](int gyy) { return xin ? (gyy * nx + gx) * SZ : BUF_OUT; };
  // index of cell (gyy, gxx), BUF_OUT outside the grid
  auto cell_idx = [&](int gyy, int gxx) {
    return (unsigned)gxx < unx && (unsigned)gyy < uny ? gyy * nx + gxx : BUF_OUT;
  };
  // (1) every load before the barrier.  u on t0: main columns, rows w + 4 i
  T v0[M0];
  {
    const int o0 = col_off(by - H2 + w);
#pragma unroll
    for (int i = 0; i < M0; ++i) v0[i] = buf_ld<T>(bu, o0 + 4 * i * nx * SZ);
  }
  // u on t0: the 2 x H2 side columns (8 R0 entries)
  constexpr int NS0 = 2 * H2 * R0, NIS0 = (NS0 + BLOCK - 1) / BLOCK;
  T vs[NIS0];
#pragma unroll
  for (int i = 0; i < NIS0; ++i) {
    const int qq = q + i * BLOCK, cc = qq & (2 * H2 - 1), ly = qq / (2 * H2);
    const int lx = cc < H2 ? cc : TX + cc;
    const int g = qq < NS0 ? cell_idx(by - H2 + ly, bx - H2 + lx) : BUF_OUT;
    vs[i] = buf_ld<T>(bu, g == BUF_OUT ? BUF_OUT : g * SZ);
  }
  // flags and right-hand side of the first sweep's cells.  (A) the tile's
  // own cells, rows w + 4 k (the same cell in the second sweep: one load
  // serves both); (B) the two rows above and below the tile, wave w taking
  // row {0, 1, R1 - 2, R1 - 1}[w]; (C) the 2 x HALO side columns, all R1
  // rows (4 R1 entries)
  uint8_t ka[RPW], kb1, kc1;
  T ra[RPW], rb1, rc1;
  const int ia = col_idx(by + w), oa = col_off(by + w);
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    ka[k] = buf_ld<uint8_t>(bk, ia + 4 * k * nx);
    ra[k] = buf_ld<T>(br, oa + 4 * k * nx * SZ);
  }
  const int lyb = w < 2 ? w : R1 - 4 + w;
  kb1 = buf_ld<uint8_t>(bk, col_idx(by - HALO + lyb));
  rb1 = buf_ld<T>(br, col_off(by - HALO + lyb));
  constexpr int NC = 2 * HALO * R1;
  const int cc1 = q & (2 * HALO - 1), lyc = q / (2 * HALO);
  const int lxc = cc1 < HALO ? cc1 : TX + cc1;     // t1 column 0, 1, 66, 67
  {
    const int g = q < NC ? cell_idx(by - HALO + lyc, bx - HALO + lxc) : BUF_OUT;
    kc1 = buf_ld<uint8_t>(bk, g);
    rc1 = buf_ld<T>(br, g == BUF_OUT ? BUF_OUT : g * SZ);
  }
#pragma unroll
  for (int i = 0; i < M0; ++i) t0[w + 4 * i][tx + H2] = v0[i];
#pragma unroll
  for (int i = 0; i < NIS0; ++i) {
    const int qq = q + i * BLOCK, cc = qq & (2 * H2 - 1), ly = qq / (2 * H2);
    if (qq < NS0) t0[ly][cc < H2 ? cc : TX + cc] = vs[i];
  }
  __syncthreads();
  if (CROSS) {
    // y-differences of u on the first sweep's rows, every staged column
    auto dyu = [&](int y, int x) {
      dy[y][x] = (T)8 * (t0[y + HALO + 1][x] - t0[y + HALO - 1][x]) - (t0[y + HALO + 2][x] - t0[y + HALO - 2][x]);
    };
#pragma unroll
    for (int i = 0; i < M1; ++i) dyu(w + 4 * i, tx + H2);
    for (int qq = q; qq < 2 * H2 * R1; qq += BLOCK) {
      const int cc = qq & (2 * H2 - 1);
      dyu(qq / (2 * H2), cc < H2 ? cc : TX + cc);
    }
    __syncthreads();
  }
  // (2) first sweep: u' on the tile plus 2 (cells outside the grid copy
  // their staged value; no regular cell reads it)
  auto sweep1 = [&](int ly, int lx, uint8_t kf, T rv) {
    const int cy = ly + HALO, cx = lx + HALO;   // in t0
    T v = t0[cy][cx];
    if (kf & regbit) {
      T lu;
      if (CROSS) {
        const T* dr = dy[ly] + cx;
        lu = regular_row_dy<T>(t0[cy][cx], t0[cy][cx + 1], t0[cy][cx - 1], t0[cy][cx + 2], t0[cy][cx - 2],
                               t0[cy + 1][cx], t0[cy - 1][cx], t0[cy + 2][cx], t0[cy - 2][cx],
                               [&](int dx) { return dr[dx]; }, c);
      } else {
        lu = regular_row<T, false>([&](int ddy, int ddx) { return t0[cy + ddy][cx + ddx]; }, c);
      }
      v += c.omega_invD * (rv - lu);
    }
    t1[ly][lx] = v;
  };
#pragma unroll
  for (int k = 0; k < RPW; ++k) sweep1(HALO + w + 4 * k, tx + HALO, ka[k], ra[k]);
  sweep1(lyb, tx + HALO, kb1, rb1);
  if (q < NC) sweep1(lyc, lxc, kc1, rc1);
  __syncthreads();
  if (CROSS) {
    // y-differences of u' on the tile rows (in the first ones' space)
    auto dyu1 = [&](int y, int x) {
      dy[y][x] = (T)8 * (t1[y + HALO + 1][x] - t1[y + HALO - 1][x]) - (t1[y + HALO + 2][x] - t1[y + HALO - 2][x]);
    };
#pragma unroll
    for (int k = 0; k < RPW; ++k) dyu1(w + 4 * k, tx + HALO);
    for (int qq = q; qq < 2 * HALO * TYS; qq += BLOCK) {
      const int cc = qq & (2 * HALO - 1);
      dyu1(qq / (2 * HALO), cc < HALO ? cc : TX + cc);
    }
    __syncthreads();
  }
  // (3) second sweep on the tile (a store outside the grid is dropped)
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int ry = w + 4 * k;
    {
      const int cy = ry + HALO, cx = tx + HALO;
      T v = t1[cy][cx];
      if (ka[k] & regbit) {
        T lu;
        if (CROSS) {
          const T* dr = dy[ry] + cx;
          lu = regular_row_dy<T>(t1[cy][cx], t1[cy][cx + 1], t1[cy][cx - 1], t1[cy][cx + 2], t1[cy][cx - 2],
                                 t1[cy + 1][cx], t1[cy - 1][cx], t1[cy + 2][cx], t1[cy - 2][cx],
                                 [&](int dx) { return dr[dx]; }, c);
        } else {
          lu = apply_regular<T, false>(t1, cy, cx, c);
        }
        v += c.omega_invD * (ra[k] - lu);
      }
      buf_st(bo, oa + 4 * k * nx * SZ, v);
    }
  }
}

template <typename T, bool CROSS, bool FINEST, int TYS>
__global__ __launch_bounds__(BLOCK) void k_sweep2(const T* __restrict__ u, const T* __restrict__ r,
                                                  const uint8_t* __restrict__ kind, T* __restrict__ out, int nx,
                                                  int ny, int nbx, CoefT<T> c, uint8_t regbit) {
  __shared__ double smem[sweep2_lds_doubles<T, TYS, CROSS>()];
  const size_t zoff = (size_t)blockIdx.z * nx * ny;
  sweep2_tile<T, CROSS, TYS>(smem, xcd_tile(blockIdx.x, gridDim.x), u + zoff, r + zoff, kind, out + zoff, nx, ny,
                             nbx, c, regbit);
}

// Residual of the regular cells restricted to the coarse grid:
// rc_I = 1/4 sum over regular children c of (r - L u)_c  (Section 4.1).
// The same launch sets the coarse iterate uc to the recursion's zero guess
// (Alg. 2) and zeroes the compact copy cc of its block rows.  With ckind
// set it writes instead the result of one plain SMO-1 sweep of the coarse
// level from that zero guess: uc_I = cw * rc_I where ckind_I has cregbit
// (cw = omega / D of the coarse level), 0 elsewhere -- the value the sweep
// itself computes there (0 + cw * (rc - L 0)), so that sweep can be left
// out.
// One tile t of one plane (pointers already offset to the plane); l is the
// workgroup's index within the plane, which zeroes entries [l * BLOCK,
// (l + 1) * BLOCK) of the plane's compact copy cc.
template <typename T, typename TC, bool CROSS>
__device__ __forceinline__ void restrict_tile(int t, int l, const T* __restrict__ u, const T* __restrict__ r,
                                              const uint8_t* __restrict__ kind, TC* __restrict__ rc,
                                              TC* __restrict__ uc, double* __restrict__ cc, int ncc, int nx, int ny,
                                              int nbx, int ncx, int ncy, const CoefT<T>& c, uint8_t regbit,
                                              const uint8_t* __restrict__ ckind = nullptr, TC cw = (TC)0,
                                              uint8_t cregbit = 0) {
  __shared__ T tile[LH][LW];
  __shared__ T dyt[CROSS ? TY : 1][LW];   // y-differences of the cross term
  {
    const int flat = l * BLOCK + threadIdx.x;
    if (flat < ncc) cc[flat] = 0.0;
  }
  const int tyi = t / nbx, txi = t - tyi * nbx;
  const int bx = txi * TX, by = tyi * TY;
  const int cx = threadIdx.x & 31, cy = threadIdx.x >> 5;  // 32 x 8 coarse cells
  // fine cells through buffer views of the plane (cells outside the grid
  // read value 0 and flags 0; planes stay below 2^31 bytes)
  const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
  const bufrsrc bu = make_buf(u, plane * (uint32_t)sizeof(T)), br = make_buf(r, plane * (uint32_t)sizeof(T)),
                bk = make_buf(kind, plane);
  uint8_t kd[4];
  T rr[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int gx = bx + 2 * cx + (d & 1), gy = by + 2 * cy + (d >> 1);
    const int g = (unsigned)gx < (unsigned)nx ? gy * nx + gx : BUF_OUT;   // gy >= 0; gy >= ny is outside the plane
    kd[d] = buf_ld<uint8_t>(bk, g);
    rr[d] = buf_ld<T>(br, g == BUF_OUT ? BUF_OUT : g * (int)sizeof(T));
  }
  stage_cols<T, LH, HALO>(tile, bu, nx, ny, bx, by);
  __syncthreads();
  if (CROSS) {
    fill_dy<T, TY>(dyt, tile);
    __syncthreads();
  }
  const int I = txi * (TX / 2) + cx, J = tyi * (TY / 2) + cy;
  if (I >= ncx || J >= ncy) return;
  const size_t gc = (size_t)J * ncx + I;
  const uint8_t ck = ckind ? ckind[gc] : (uint8_t)0;
  T s = (T)0;
#pragma unroll
  for (int d = 0; d < 4; ++d)
    if (kd[d] & regbit) {
      const int ly = 2 * cy + (d >> 1) + HALO, lx = 2 * cx + (d & 1) + HALO;
      s += rr[d] - (CROSS ? apply_regular_dy<T>(tile, dyt, ly, lx, c) : apply_regular<T, false>(tile, ly, lx, c));
    }
  const TC rv = (TC)((T)0.25 * s);
  rc[gc] = rv;
  uc[gc] = (ck & cregbit) ? cw * rv : (TC)0;
}

template <typename T, typename TC, bool CROSS, bool FINEST>
__global__ __launch_bounds__(BLOCK) void k_restrict(const T* __restrict__ u, const T* __restrict__ r,
                                                    const uint8_t* __restrict__ kind, TC* __restrict__ rc,
                                                    TC* __restrict__ uc, double* __restrict__ cc, int ncc, int nx,
                                                    int ny, int nbx, int ncx, int ncy, CoefT<T> c, uint8_t regbit,
                                                    const uint8_t* __restrict__ ckind, TC cw, uint8_t cregbit) {
  const size_t z = blockIdx.z;
  restrict_tile<T, TC, CROSS>(xcd_tile(blockIdx.x, gridDim.x), blockIdx.x, u + z * nx * ny, r + z * nx * ny, kind,
                              rc + z * ncx * ncy, uc + z * ncx * ncy, cc + z * ncc, ncc, nx, ny, nbx, ncx, ncy, c,
                              regbit, ckind, cw, cregbit);
}

// Correction u_c += P e on regular fine cells: piecewise constant
// (Section 4.1) or bilinear with the 9/16, 3/16, 3/16, 1/16 cell-centred
// weights where all four coarse cells are non-empty.
template <typename T>
__device__ __forceinline__ T prolong_value(const T* __restrict__ e, const uint8_t* __restrict__ ckind, int i, int j,
                                           int ncx, int ncy, int bilinear) {
  const int I = i >> 1, J = j >> 1;
  T v = e[(size_t)J * ncx + I];
  if (bilinear) {
    const int I2 = I + ((i & 1) ? 1 : -1), J2 = J + ((j & 1) ? 1 : -1);
    if (I2 >= 0 && I2 < ncx && J2 >= 0 && J2 < ncy && (ckind[(size_t)J * ncx + I2] & F_NONEMPTY) &&
        (ckind[(size_t)J2 * ncx + I] & F_NONEMPTY) && (ckind[(size_t)J2 * ncx + I2] & F_NONEMPTY))
      v = ((T)9 * v + (T)3 * e[(size_t)J * ncx + I2] + (T)3 * e[(size_t)J2 * ncx + I] + e[(size_t)J2 * ncx + I2]) *
          (T)0.0625;
  }
  return v;
}

// Grid rows 0..ny-1 update u; the extra rows apply the same correction to
// the compact copy c of the block rows (SMO-2), computed from the same
// inputs so that c stays equal to u on those cells.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_prolong(T* __restrict__ u, const T* __restrict__ e,
                                                   const uint8_t* __restrict__ kind,
                                                   const uint8_t* __restrict__ ckind, int nx, int ny, int ncx,
                                                   int ncy, int bilinear, uint8_t regbit,
                                                   const int32_t* __restrict__ scell, double* __restrict__ c, int ns) {
  const int z = blockIdx.z;
  e += (size_t)z * ncx * ncy;
  if ((int)blockIdx.y < ny) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= nx) return;
    const size_t g = (size_t)j * nx + i;
    if (!(kind[g] & regbit)) return;
    u[(size_t)z * nx * ny + g] += prolong_value(e, ckind, i, j, ncx, ncy, bilinear);
    return;
  }
  const int k = ((blockIdx.y - ny) * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= ns) return;
  const int q = scell[k];
  if (!(kind[q] & regbit)) return;
  const T v = (T)(c[(size_t)z * ns + k]) + prolong_value(e, ckind, q % nx, q / nx, ncx, ncy, bilinear);
  c[(size_t)z * ns + k] = (double)v;
}

// Residual of one explicit row (FP64, difference form):
//   r_q - bterm - sum_s beta_s (u_s - u_q) - S u_q,  S = sum_s beta_s.
// The entries are taken 8 at a time: their columns and weights, then the 8
// gathers, each group of loads issued together (two accumulators, even and
// odd entries).
template <typename T>
__device__ __forceinline__ double row_residual(const T* __restrict__ u, double rhs, int q, const int32_t* cols,
                                               const double* vals, int len, double rowsum) {
  const double uq = (double)u[q];
  double a0 = 0.0, a1 = 0.0;
  for (int s = 0; s < len; s += 8) {
    int c[8];
    double w[8], x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool in = s + k < len;
      c[k] = cols[in ? s + k : 0];
      w[k] = in ? vals[s + k] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = (double)u[c[k]];
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
      a0 += w[k] * (x[k] - uq);
      a1 += w[k + 1] * (x[k + 1] - uq);
    }
  }
  return rhs - (a0 + a1) - rowsum * uq;
}

// Arguments of an SMO-2 pass (see k_smo2).
struct Smo2Args {
  const double* bterm;
  const int32_t *ecell, *ecols;   // ecols, evals, epar: ELL, row e at e * ew
  const double *evals, *ersum;
  const int32_t *eidx, *ebt, *ext_ptr, *own_cnt;
  const int64_t* inv_off;
  const float* inv;              // dense block inverses stored in FP32 (or, if inv64, in FP64);
  const double* inv64;           // applied in FP64 either way
  const double* c_in;
  double* c_out;
  int ns, nbt, ew;
  const int32_t* epar;    // per CSR entry: coarse parent of the column cell if it takes the correction, else -1
  const int32_t* eqpar;   // per overlapped row: the same for the row's own cell
};

// One RAS block b of plane z: reads uin (non-block columns) and c_in, writes
// its own rows to uout and c_out.  With a pending coarse-grid correction
// (PRO, coarse values ecor), every value read is taken as value +
// ecor[parent] where the cell takes the correction (a.epar / a.eqpar >= 0),
// i.e. the block works on u + P e.
constexpr int SMO2_LDS_DOUBLES = 1024 + 4 * 64 + 64;

// NORM: also returns the thread's norm accumulators of res over the
// block's own rows (their residual at the old iterate).
template <typename T, bool PRO = false, bool NORM = false>
__device__ __forceinline__ NormAcc smo2_block(double* smem, int b, int z, const T* uin, T* uout,
                                              const T* __restrict__ r, const Smo2Args& a,
                                              const T* __restrict__ ecor = nullptr) {
  NormAcc m;
  double* res = smem;                                              // [1024]
  double (*part)[64] = reinterpret_cast<double (*)[64]>(smem + 1024);   // [4][64]
  double* uown = smem + 1024 + 4 * 64;                             // [64]
  const double* c_in = a.c_in + (size_t)z * a.ns;
  double* c_out = a.c_out + (size_t)z * a.ns;
  const int e0 = a.ext_ptr[b], ne = a.ext_ptr[b + 1] - e0, nown = a.own_cnt[b];
  // grp (the wavefront) is uniform across a wavefront: taken through
  // readfirstlane, the product's column offsets (grp + 4 k) * nown stay in
  // scalar registers and only the row varies per lane
  const int row = threadIdx.x & 63, grp = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t iblk = a.inv_off[b];   // the block's inverse (column-major, nown rows)
  // G lanes per overlapped row (4, 2 or 1: as many as the block's rows
  // leave), each summing a contiguous slice of the row's ELL entries in
  // rounds of 8 loads; the slices' sums are added by lane shuffles (every
  // lane of the group gets the same sum: fp addition commutes)
  const int G = ne <= BLOCK / 4 ? 4 : (ne <= BLOCK / 2 ? 2 : 1);
  const int sub = threadIdx.x & (G - 1);
  const int per = (a.ew + G - 1) / G;
  for (int t0 = 0; t0 < ne; t0 += BLOCK / G) {
    const int t = t0 + (int)threadIdx.x / G;
    const bool live = t < ne;
    const int e = e0 + (live ? t : 0);
    // every conditional value below is loaded from a valid address and
    // selected afterwards (no load sits behind a branch that waits for it)
    double uq = c_in[a.eidx[e]];
    if (PRO) {
      const int pq = a.eqpar[e];
      uq += keep_or_zero((double)ecor[pq >= 0 ? pq : 0], pq >= 0);
    }
    // boundary term: loaded from a valid address either way (the row sums
    // stand in when there is none) and masked
    const int bi = a.ebt[e];
    const bool hasbt = a.bterm != nullptr && bi >= 0;
    const double* btp = a.bterm ? a.bterm + (size_t)z * a.nbt : a.ersum;
    const double rhs = (double)r[a.ecell[e]] - keep_or_zero(btp[hasbt ? bi : 0], hasbt);
    const int p0 = e * a.ew + sub * per, p1 = min(p0 + per, (e + 1) * a.ew);
    double acc = 0.0;
    for (int p = p0; p < p1; p += 8) {
      int cc[8], pp[8];
      double vv[8], uu[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const bool in = p + k < p1;
        cc[k] = in ? a.ecols[p + k] : 0;
        vv[k] = in ? a.evals[p + k] : 0.0;
        pp[k] = (PRO && in) ? a.epar[p + k] : -1;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const bool blk = cc[k] < 0;   // a block row: its value is in the compact copy
        if constexpr (std::is_same<T, double>::value) {
          uu[k] = *(blk ? c_in + (-cc[k] - 1) : uin + cc[k]);
        } else {
          const double xc = c_in[blk ? -cc[k] - 1 : 0];
          const double xu = (double)uin[blk ? 0 : cc[k]];
          uu[k] = blk ? xc : xu;
        }
        if (PRO) uu[k] += keep_or_zero((double)ecor[pp[k] >= 0 ? pp[k] : 0], pp[k] >= 0);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) acc += vv[k] * (uu[k] - uq);
    }
    if (G >= 2) acc += __shfl_xor(acc, 1, 64);
    if (G >= 4) acc += __shfl_xor(acc, 2, 64);
    if (live && sub == 0) {
      if (t < 64) uown[t] = uq;
      const double rt = rhs - acc - a.ersum[e] * uq;
      res[t] = rt;
      if (NORM && t < nown) m.add(rt);
    }
  }
  __syncthreads();
  // indices of this thread's own row for the final write, loaded ahead
  const int wr = grp == 0 && row < nown ? e0 + row : e0;
  const int widx = a.eidx[wr], wcell = a.ecell[wr];
  double s = 0.0;
  // the own rows' inverse (column-major) times the residual; the storage
  // precision is uniform per launch
  // (rounds of 8 loads; in the last round the columns past ne reload the
  // first one and add +0, so the sum keeps its column order).  A is the
  // block's inverse; entry (row, col) at col * nown + row.
  auto matvec = [&](const auto* A) {
    int c0 = grp;
    for (; c0 + 28 < ne; c0 += 32) {
      double v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = (double)A[(c0 + 4 * k) * nown + row];
#pragma unroll
      for (int k = 0; k < 8; ++k) s += v[k] * res[c0 + 4 * k];
    }
    if (c0 < ne) {
      double v[7];
#pragma unroll
      for (int k = 0; k < 7; ++k) v[k] = (double)A[(c0 + 4 * k < ne ? c0 + 4 * k : grp) * nown + row];
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const bool in = c0 + 4 * k < ne;
        s += keep_or_zero(v[k] * res[in ? c0 + 4 * k : grp], in);
      }
    }
  };
  if (row < nown) {
    if (a.inv64)
      matvec(a.inv64 + iblk);
    else
      matvec(a.inv + iblk);
  }
  part[grp][row] = s;
  __syncthreads();
  if (grp == 0 && row < nown) {
    const T v = (T)(uown[row] + (part[0][row] + part[1][row] + part[2][row] + part[3][row]));
    uout[wcell] = v;
    c_out[widx] = (double)v;
  }
  return m;
}

// SMO-2 by restricted additive Schwarz.  Workgroup = one block of <= 64
// consecutive rows of the block numbering plus its overlap.  The rows of
// the overlapped set are stored per block (cell, CSR columns and weights,
// row sum); a column that is itself a block row is encoded as -(row + 1)
// and read from the compact copy c_in of the block rows' values, all other
// columns are read from u.  Every block therefore reads only cells that no
// block writes, and writes its own rows straight into u (and c_out):
//   res_t = r_q - bterm - sum_s beta_s (u_s - u_q) - S_t u_q   (FP64),
//   u_own = c_in_own + (A_ext^{-1})_{own,:} res_ext.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_smo2(T* u, const T* __restrict__ r, Smo2Args a, size_t plane) {
  __shared__ double smem[SMO2_LDS_DOUBLES];
  const size_t zoff = (size_t)blockIdx.y * plane;
  smo2_block<T>(smem, blockIdx.x, blockIdx.y, u + zoff, u + zoff, r + zoff, a);
}

// Fused smoothing step: SMO-1 on the regular cells and SMO-2 on the blocks
// in one launch, both from the same old iterate u (additive instead of
// SMO-1 followed by SMO-2).  The first nblk workgroups are SMO-2 blocks
// (dispatched first, so that their chains of dependent loads overlap the
// streaming tiles), the rest SMO-1 tiles remapped by xcd_tile; u_out
// receives every cell.  PRO: the
// first step after the coarse-grid correction, which it applies on the fly
// (the iterate is u + P e, P piecewise constant onto the cells flagged
// probit; the coarse grid is ncx x ncy).  NORM: every workgroup also
// stores the maximum of |r - bterm - L u| (the old iterate's residual, FP64)
// over the cells it updates in partial[z * gridDim.x + blockIdx.x]; the
// SMO-1 cells and the block rows together are every non-empty cell, so the
// partials carry the residual norm of the incoming iterate.  With the
// maximum goes the sum of squares: partial[2 q], partial[2 q + 1] for
// q = z * gridDim.x + blockIdx.x.
// Occupancy floor of the fused step's variants (waves per SIMD the
// register allocation must allow): the norm-taking variant needs a few
// registers more than the plain one and would drop from 7 to 6 waves (it
// fits in 70 without spills).  The correction-applying one is left alone
// (held at 6 waves it spills).
constexpr int fused_min_waves(bool pro, bool norm) { return norm && !pro ? 7 : 1; }

template <typename T, bool CROSS, bool FINEST, int TYS, bool PRO, bool NORM = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(fused_min_waves(PRO, NORM)))) void k_smooth_fused(const T* __restrict__ u, const T* __restrict__ r,
                                                        const uint8_t* __restrict__ kind, T* __restrict__ out,
                                                        int nx, int ny, int nbx, int nblk, CoefT<T> c,
                                                        uint8_t regbit, uint8_t s2bit, Smo2Args a,
                                                        const T* __restrict__ e, int ncx, int ncy, uint8_t probit,
                                                        double* __restrict__ partial = nullptr) {
  // one LDS buffer shared by the two kinds of workgroup
  constexpr int NS = sweep_lds_doubles<T, TYS, CROSS>();
  __shared__ double smem[NS > SMO2_LDS_DOUBLES ? NS : SMO2_LDS_DOUBLES];
  const size_t zoff = (size_t)blockIdx.z * nx * ny;
  const T* ez = PRO ? e + (size_t)blockIdx.z * ncx * ncy : nullptr;
  NormAcc m;
  if ((int)blockIdx.x < nblk)
    m = smo2_block<T, PRO, NORM>(smem, blockIdx.x, blockIdx.z, u + zoff, out + zoff, r + zoff, a, ez);
  else
    m = sweep_tile<T, CROSS, TYS, PRO, NORM>(smem, xcd_tile(blockIdx.x - nblk, gridDim.x - nblk), u + zoff,
                                             r + zoff, kind, out + zoff, nx, ny, nbx, c, regbit, s2bit, ez, ncx,
                                             probit);
  if constexpr (NORM) {
    __shared__ double red[2 * BLOCK / 64];
    const NormAcc o = block_norm(m, red);
    if (threadIdx.x == 0) {
      const size_t q = 2 * ((size_t)blockIdx.z * gridDim.x + blockIdx.x);
      partial[q] = o.m, partial[q + 1] = o.s;
    }
  }
}

// c[k] = u[cell[k]] for every block row (start of a solve on level 0).
template <typename T>
__global__ void k_gather_rows(const T* __restrict__ u, const int32_t* __restrict__ cell, double* __restrict__ c,
                              int ns, size_t plane) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ns) return;
  const int z = blockIdx.y;
  c[(size_t)z * ns + k] = (double)u[(size_t)z * plane + cell[k]];
}

// (A u) for explicit rows (plain sum).
__global__ void k_rows_apply(const double* __restrict__ u, double* __restrict__ Lu, const int32_t* __restrict__ cell,
                             const int32_t* __restrict__ rp, const int32_t* __restrict__ cols,
                             const double* __restrict__ vals, int nrows) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nrows) return;
  double acc = 0.0;
  for (int s = rp[k]; s < rp[k + 1]; ++s) acc += vals[s] * u[cols[s]];
  Lu[cell[k]] = acc;
}

// (L u) on cells flagged `regbit`; zero elsewhere.
template <bool CROSS>
__global__ __launch_bounds__(BLOCK) void k_apply(const double* __restrict__ u, const uint8_t* __restrict__ kind,
                                                 double* __restrict__ Lu, int nx, int ny, CoefT<double> c,
                                                 uint8_t regbit) {
  __shared__ double tile[LH][LW];
  const int bx = blockIdx.x * TX, by = blockIdx.y * TY;
  load_tile(tile, u, nx, ny, bx, by);
  __syncthreads();
  const int tx = threadIdx.x & (TX - 1), w = threadIdx.x >> 6;
  for (int k = 0; k < TY / 4; ++k) {
    const int ry = w + 4 * k, gx = bx + tx, gy = by + ry;
    if (gx < nx && gy < ny) {
      const size_t g = (size_t)gy * nx + gx;
      Lu[g] = (kind[g] & regbit) ? apply_regular<double, CROSS>(tile, ry + HALO, tx + HALO, c) : 0.0;
    }
  }
}

// max over non-empty cells of |r - bterm - L u| (difference form), or of
// |r - bterm| when zero_u is set, in one launch: the first workgroups take
// BLOCK explicit rows each (FP64), the last ntiles the stencil cells of one
// TX x TY tile each (remapped by xcd_tile).  With res_out, the residual of every
// cell is also stored there as FP32 (0 on empty cells) for the refinement
// loop: stencil cells by the tile workgroups, explicit rows by the row
// workgroups, so no cell is written twice.  Every workgroup stores its
// partial maximum and sum of squares in partial[2 q], partial[2 q + 1],
// q = z * gridDim.x + b; the host, which reads the norms back anyway,
// reduces the partials (no second launch and no device-wide fence).
// Workgroup l of one plane (pointers offset to the plane; bterm and res_out
// too): workgroups [0, nrb) take BLOCK explicit rows each, the others one
// tile (remapped by xcd_tile over ntiles).  Returns the workgroup's
// accumulators (valid in thread 0).
template <typename T, bool CROSS>
__device__ __forceinline__ NormAcc resnorm_block(int l, int nrb, int ntiles, const T* __restrict__ u,
                                                const T* __restrict__ r, const uint8_t* __restrict__ kind, int nx,
                                                int ny, int nbx, const CoefT<T>& c, int zero_u, uint8_t regbit,
                                                const double* __restrict__ bterm, const int32_t* __restrict__ cell,
                                                const int32_t* __restrict__ rp, const int32_t* __restrict__ cols,
                                                const double* __restrict__ vals, const double* __restrict__ rowsum,
                                                int nrows, float* __restrict__ res_out) {
  __shared__ T tile[LH][LW];
  __shared__ T dyt[CROSS ? TY : 1][LW];   // y-differences of the cross term
  __shared__ double red[2 * BLOCK / 64];
  NormAcc m;
  if (l >= nrb) {
    const int t = xcd_tile(l - nrb, ntiles);
    const int tyi = t / nbx;
    const int bx = (t - tyi * nbx) * TX, by = tyi * TY;
    const int tx = threadIdx.x & (TX - 1), w = threadIdx.x >> 6;
    // the plane through buffer views (planes stay below 2^31 bytes): cells
    // outside the grid read flags 0 and value 0, stores there are dropped
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const bufrsrc bk = make_buf(kind, plane), br = make_buf(r, plane * (uint32_t)sizeof(T)),
                  bro = make_buf(res_out, plane * (uint32_t)sizeof(float));
    const int gx = bx + tx;
    const int g0 = (unsigned)gx < (unsigned)nx ? by * nx + gx : BUF_OUT;
    auto gcell = [&](int k) { return g0 == BUF_OUT ? BUF_OUT : g0 + (w + 4 * k) * nx; };
    uint8_t kd[TY / 4];
    T rr[TY / 4];
#pragma unroll
    for (int k = 0; k < TY / 4; ++k) {
      const int g = gcell(k);
      kd[k] = buf_ld<uint8_t>(bk, g);
      rr[k] = buf_ld<T>(br, g == BUF_OUT ? BUF_OUT : g * (int)sizeof(T));
    }
    stage_cols<T, LH, HALO>(tile, make_buf(u, plane * (uint32_t)sizeof(T)), nx, ny, bx, by);
    __syncthreads();
    if (CROSS && !zero_u) {
      fill_dy<T, TY>(dyt, tile);
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < TY / 4; ++k) {
      const int g = gcell(k);
      T v = rr[k];
      if (kd[k] & regbit) {
        if (!zero_u)
          v -= CROSS ? apply_regular_dy<T>(tile, dyt, w + 4 * k + HALO, tx + HALO, c)
                     : apply_regular<T, false>(tile, w + 4 * k + HALO, tx + HALO, c);
        m.add((double)v);
      }
      // the FP32 residual: regular cells and empty ones (0); the explicit
      // rows are written by the row workgroups
      if (res_out) {
        const bool reg = kd[k] & regbit, wr = reg || !(kd[k] & F_NONEMPTY);
        buf_st(bro, wr && g != BUF_OUT ? g * (int)sizeof(float) : BUF_OUT, reg ? (float)v : 0.0f);
      }
    }
  } else {
    const int k = l * BLOCK + threadIdx.x;
    if (k < nrows) {
      const int q = cell[k];
      double rhs = (double)r[q];
      if (bterm) rhs -= bterm[k];
      if (!zero_u) rhs = row_residual(u, rhs, q, cols + rp[k], vals + rp[k], rp[k + 1] - rp[k], rowsum[k]);
      if (res_out) res_out[q] = (float)rhs;
      m.add(rhs);
    }
  }
  return block_norm(m, red);
}

template <typename T, bool CROSS>
__global__ __launch_bounds__(BLOCK) void k_resnorm(const T* __restrict__ u, const T* __restrict__ r,
                                                   const uint8_t* __restrict__ kind, int nx, int ny, int nbx,
                                                   int ntiles, CoefT<T> c, int zero_u, uint8_t regbit,
                                                   const double* __restrict__ bterm, const int32_t* __restrict__ cell,
                                                   const int32_t* __restrict__ rp, const int32_t* __restrict__ cols,
                                                   const double* __restrict__ vals,
                                                   const double* __restrict__ rowsum, int nrows,
                                                   float* __restrict__ res_out, double* __restrict__ partial) {
  const int z = blockIdx.z;
  const size_t plane = (size_t)nx * ny;
  // the row workgroups (chains of dependent loads) come first in the grid so
  // that their latency overlaps the streaming tiles
  const NormAcc m = resnorm_block<T, CROSS>(blockIdx.x, (int)gridDim.x - ntiles, ntiles, u + z * plane,
                                            r + z * plane, kind, nx, ny, nbx, c, zero_u, regbit,
                                            bterm ? bterm + (size_t)z * nrows : nullptr, cell, rp, cols, vals,
                                            rowsum, nrows, res_out ? res_out + z * plane : nullptr);
  if (threadIdx.x == 0) {
    const size_t q = 2 * ((size_t)z * gridDim.x + blockIdx.x);
    partial[q] = m.m, partial[q + 1] = m.s;
  }
}

// Coarsest level: u[cell_k] = sum_j Inv[k, j] r[cell_j] (FP64), one wavefront
// per row (WAVES rows per workgroup), the gathered right-hand side staged in
// LDS once per workgroup.
template <typename T, int WAVES = BLOCK / 64>
__device__ __forceinline__ void coarse_rows(double* rv, int wg, T* __restrict__ u, const T* __restrict__ r,
                                            const int32_t* __restrict__ cell, const float* __restrict__ inv,
                                            const double* __restrict__ inv64, int nm) {
  // gathered in chunks of 4 entries per thread: the cell indices of a
  // chunk, then their values, are each loaded together
  for (int k0 = threadIdx.x; k0 < nm; k0 += 4 * WAVES * 64) {
    int ci[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ci[i] = cell[min(k0 + i * WAVES * 64, nm - 1)];
    double x[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = (double)r[ci[i]];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (k0 + i * WAVES * 64 < nm) rv[k0 + i * WAVES * 64] = x[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int row = wg * WAVES + (threadIdx.x >> 6);
  if (row >= nm) return;
  double s0 = 0.0, s1 = 0.0;
  if (inv64) {
    const double* A = inv64 + (size_t)row * nm;
    int k = lane;
    for (; k + 64 < nm; k += 128) s0 += A[k] * rv[k], s1 += A[k + 64] * rv[k + 64];
    if (k < nm) s0 += A[k] * rv[k];
  } else {
    // FP32 row read as 16-byte vectors (the stream is latency-bound with
    // 4-byte loads): the 0-3 entries before the first 16-byte boundary, the
    // aligned body (8 vectors per lane in flight), then the remaining 0-3
    // entries
    const float* A = inv + (size_t)row * nm;
    const int head = min((int)(((16 - (reinterpret_cast<uintptr_t>(A) & 15)) & 15) >> 2), nm);
    if (lane < head) s0 += (double)A[lane] * rv[lane];
    const int nb = (nm - head) >> 2;
    const float4* A4 = reinterpret_cast<const float4*>(A + head);
    const double* rb = rv + head;
    const int nq = lane < nb ? (nb - lane + 63) / 64 : 0;
    // full chunks of 8 vectors per lane, all 8 loaded before any is used,
    // then the remaining vectors one at a time
    int it = 0;
    for (; it + 8 <= nq; it += 8) {
      float4 a[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = A4[lane + 64 * (it + i)];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const double* x = rb + 4 * (lane + 64 * (it + i));
        const double t = (double)a[i].x * x[0] + (double)a[i].y * x[1] + (double)a[i].z * x[2] + (double)a[i].w * x[3];
        if (i & 1)
          s1 += t;
        else
          s0 += t;
      }
    }
#pragma unroll 8
    for (; it < nq; ++it) {
      const int q = lane + 64 * it;
      const float4 a = A4[q];
      const double* x = rb + 4 * q;
      const double t = (double)a.x * x[0] + (double)a.y * x[1] + (double)a.z * x[2] + (double)a.w * x[3];
      if (it & 1)
        s1 += t;
      else
        s0 += t;
    }
    const int k = head + 4 * nb + lane;
    if (k < nm) s1 += (double)A[k] * rv[k];
  }
  double s = s0 + s1;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) u[cell[row]] = (T)s;
}

// the one-right-hand-side coarsest solve: 16 rows per workgroup
constexpr int COARSE_WAVES = 16;

template <typename T>
__global__ __launch_bounds__(64 * COARSE_WAVES) void k_coarse(T* __restrict__ u, const T* __restrict__ r,
                                                              const int32_t* __restrict__ cell,
                                                              const float* __restrict__ inv,
                                                              const double* __restrict__ inv64, int nm,
                                                              size_t plane) {
  extern __shared__ double rv[];
  const size_t z = blockIdx.y;
  coarse_rows<T, COARSE_WAVES>(rv, blockIdx.x, u + z * plane, r + z * plane, cell, inv, inv64, nm);
}

template <typename T>
__global__ void k_coarse_gather(const T* __restrict__ r, const int32_t* __restrict__ cell, double* __restrict__ rg,
                                int nm, int nrhs, size_t plane) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nm) return;
  const int z = blockIdx.y;
  rg[(size_t)k * nrhs + z] = (double)r[z * plane + cell[k]];
}

// Step 2: U = Inv * Rg on the matrix cores (FP64 16x16x4 products).
// Workgroup = 16 rows x 64 right-hand sides and CMW waves; wave w takes the
// w-th slice of the k range (a multiple of 16 long) and keeps 4 16x16 tiles
// of partial sums; the slices are added in LDS in the order w = 0..CMW-1.
// Within a group of 16 k values, lane group g = lane / 16 feeds k = k0 +
// 4 g + s to product s (the same k on the A and the B side), so each lane
// reads 4 consecutive entries of its row of the inverse.
constexpr int CMW = 8;                  // waves per workgroup (k slices)
constexpr int CM_ROWS = 16, CM_RHS = 64;
typedef double dbl4 __attribute__((ext_vector_type(4)));
template <typename T>
__global__ __launch_bounds__(64 * CMW) void k_coarse_multi(T* __restrict__ u, const double* __restrict__ rg,
                                                           const int32_t* __restrict__ cell,
                                                           const float* __restrict__ inv,
                                                           const double* __restrict__ inv64, int nm, int nrhs,
                                                           size_t plane) {
  __shared__ double red[CMW][CM_ROWS][CM_RHS];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int row0 = blockIdx.x * CM_ROWS, z0 = blockIdx.y * CM_RHS;
  const int kc = (nm + CMW * 16 - 1) / (CMW * 16) * 16;
  const int kb = w * kc, ke = min(nm, kb + kc);
  const int arow = row0 + i;
  const size_t aoff = (size_t)min(arow, nm - 1) * nm;
  dbl4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    double a[4], b[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * g + s;
      const bool ok = k < ke;
      a[s] = ok && arow < nm ? (inv64 ? inv64[aoff + k] : (double)inv[aoff + k]) : 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int z = z0 + 16 * c + i;
        b[s][c] = ok && z < nrhs ? rg[(size_t)k * nrhs + z] : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s][c], acc[c], 0, 0, 0);
  }
  // tile c, register j of lane (i, g): row g + 4 j, right-hand side 16 c + i
  // (the FP64 16x16 result layout, checked on the device)
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int j = 0; j < 4; ++j) red[w][g + 4 * j][16 * c + i] = acc[c][j];
  __syncthreads();
  for (int t = threadIdx.x; t < CM_ROWS * CM_RHS; t += 64 * CMW) {
    const int r = t / CM_RHS, zc = t - r * CM_RHS;
    double sum = 0.0;
#pragma unroll
    for (int v = 0; v < CMW; ++v) sum += red[v][r][zc];
    const int row = row0 + r, z = z0 + zc;
    if (row < nm && z < nrhs) u[(size_t)z * plane + cell[row]] = (T)sum;
  }
}

// Set-up of the coarsest solve: dense inverse by Gauss-Jordan elimination
// with partial pivoting on [A | B], B = I initially (row-major n x n, FP64),
// one pivot per pair of launches.  status != 0 (singular) makes every later
// launch a no-op.
//
// Pivot step (one workgroup): pivot row = argmax_{r >= k} |A[r][k]| (ties:
// the smaller r); swap rows k and pivot in A and B; scale row k by
// 1 / A[k][k]; copy column k into colk (the multipliers of the elimination).
__global__ __launch_bounds__(1024) void k_gj_pivot(double* __restrict__ A, double* __restrict__ B, int n, int k,
                                                   double* __restrict__ colk, int* __restrict__ status,
                                                   double tiny) {
  __shared__ double bv[1024];
  __shared__ int bi[1024];
  if (*status) return;
  const int t = threadIdx.x;
  double best = -1.0;
  int bidx = n;
  for (int r = k + t; r < n; r += 1024) {
    const double v = fabs(A[(size_t)r * n + k]);
    if (v > best) best = v, bidx = r;
  }
  bv[t] = best;
  bi[t] = bidx;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if (t < st) {
      const double v2 = bv[t + st];
      const int i2 = bi[t + st];
      if (v2 > bv[t] || (v2 == bv[t] && i2 < bi[t])) bv[t] = v2, bi[t] = i2;
    }
    __syncthreads();
  }
  const int piv = bi[0];
  const double pv = bv[0];
  // a pivot at rounding level of the matrix (tiny = 1e-12 max |A_ij|) means
  // the matrix is singular (a constant null vector, all-Neumann data)
  if (!(pv > tiny) || !isfinite(pv) || piv >= n) {
    if (t == 0) *status = 1;
    return;
  }
  if (piv != k)
    for (int c = t; c < n; c += 1024) {
      const double a = A[(size_t)k * n + c], b = B[(size_t)k * n + c];
      A[(size_t)k * n + c] = A[(size_t)piv * n + c];
      B[(size_t)k * n + c] = B[(size_t)piv * n + c];
      A[(size_t)piv * n + c] = a;
      B[(size_t)piv * n + c] = b;
    }
  __syncthreads();
  const double inv = 1.0 / A[(size_t)k * n + k];
  __syncthreads();
  for (int c = t; c < n; c += 1024) {
    A[(size_t)k * n + c] *= inv;
    B[(size_t)k * n + c] *= inv;
  }
  __syncthreads();
  for (int r = t; r < n; r += 1024) colk[r] = A[(size_t)r * n + k];
}

// Elimination step: every row r != k subtracts colk[r] times the pivot row,
// on the columns c >= k of A (columns < k are already unit vectors with a 0
// in the pivot row) and on all columns of B.  grid.y = rows; grid.x covers
// 2n columns (A then B) four per thread.
__global__ __launch_bounds__(256) void k_gj_elim(double* __restrict__ A, double* __restrict__ B, int n, int k,
                                                 const double* __restrict__ colk, const int* __restrict__ status) {
  if (*status) return;
  const int r = blockIdx.y;
  if (r == k) return;
  const double f = colk[r];
  if (f == 0.0) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = (blockIdx.x * 256 + threadIdx.x) * 4 + j;
    if (c < n) {
      if (c >= k) A[(size_t)r * n + c] -= f * A[(size_t)k * n + c];
    } else if (c < 2 * n) {
      const int cb = c - n;
      B[(size_t)r * n + cb] -= f * B[(size_t)k * n + cb];
    }
  }
}

// out = in^T (n x n); the inverse of A^T is the transpose of the inverse of A.
// out = in rounded to FP32 (the stored coarsest inverse)
__global__ void k_to_f32(const double* __restrict__ in, float* __restrict__ out, size_t n) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    out[k] = (float)in[k];
}

// out = in^T (the stored inverse of the transpose, FP32 or FP64)
template <typename TO>
__global__ void k_transpose(const double* __restrict__ in, TO* __restrict__ out, int n) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int j = threadIdx.y; j < 32; j += 8) {
    const int r = by + j, c = bx + threadIdx.x;
    if (r < n && c < n) tile[j][threadIdx.x] = in[(size_t)r * n + c];
  }
  __syncthreads();
  for (int j = threadIdx.y; j < 32; j += 8) {
    const int r = bx + j, c = by + threadIdx.x;
    if (r < n && c < n) out[(size_t)r * n + c] = (TO)tile[threadIdx.x][j];
  }
}

__global__ void k_set_identity(double* __restrict__ B, int n) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < (size_t)n * n) B[k] = (k / n == k % n) ? 1.0 : 0.0;
}

// Boundary term of the irregular rows: bterm_k = sum over k's faces of N g.
__global__ void k_bterm(const double* __restrict__ g, const int32_t* __restrict__ fptr,
                        const int32_t* __restrict__ fface, const double* __restrict__ fval, double* __restrict__ bterm,
                        int nirr, int nfaces) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nirr) return;
  const int z = blockIdx.y;
  double s = 0.0;
  for (int t = fptr[k]; t < fptr[k + 1]; ++t) s += fval[t] * g[(size_t)z * nfaces + fface[t]];
  bterm[(size_t)z * nirr + k] = s;
}

// out = N^T lambda: out[face] = nweight[face] * lambda[cell[face]].
__global__ void k_apply_NT(const double* __restrict__ lam, const int32_t* __restrict__ fcell,
                           const double* __restrict__ fw, double* __restrict__ out, int nfaces, size_t plane) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int z = blockIdx.y;
  if (k < nfaces) out[(size_t)z * nfaces + k] = fw[k] * lam[(size_t)z * plane + fcell[k]];
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, size_t n, T v) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = v;
}

// Plain FP64 copy, 16 bytes per element: the calibration kernel for HBM
// byte counters.
__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, size_t n) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    dst[k] = src[k];
}

__global__ void k_axpy_f32(double* __restrict__ u, const float* __restrict__ e, const uint8_t* __restrict__ kind,
                           size_t plane, size_t n) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    if (kind[k % plane] & F_NONEMPTY) u[k] += (double)e[k];
}

__global__ void k_mask_empty(double* __restrict__ u, const uint8_t* __restrict__ kind, size_t plane, size_t n) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    if (!(kind[k % plane] & F_NONEMPTY)) u[k] = 0.0;
}

// ===========================================================================
// Lockstep batches: one launch performs one V-cycle step for every geometry
// of a batch.  Each launch has a table of per-geometry descriptors in device
// memory; geometry d owns workgroups [st.start[d], st.start[d + 1]) of the
// 1-D grid (the prefix offsets travel in the kernel arguments, so finding
// the descriptor costs no memory access).  A geometry whose flag in `active`
// is 0 has converged: its workgroups return at once.
// ===========================================================================
constexpr int BMAX = 64;   // geometries per batched launch
struct BStarts {
  int n;
  int start[BMAX + 1];
};

__device__ __forceinline__ int bfind(const BStarts& st, int b) {
  int d = 0;
  while (d + 1 < st.n && b >= st.start[d + 1]) ++d;
  return d;
}

struct BFused {                    // fused smoothing step of one geometry on one level
  const void *u, *r;
  void* out;
  const uint8_t* kind;
  Coef c;
  size_t plane, cplane;            // cells of a plane on this level / on the coarser level
  int nx, ny, nbx, ntiles, nblk;   // workgroups per plane: nblk + ntiles
  int ncx, ncy;
  const void* e;                   // pending coarse correction (PRO)
  uint8_t regbit, s2bit, probit;
  int geo;
  Smo2Args a;
};

template <typename T, bool CROSS, bool PRO, int TYS>
__global__ __launch_bounds__(BLOCK) void k_fused_batched(const BFused* __restrict__ descs, BStarts st,
                                                         const int* __restrict__ active) {
  constexpr int NS = sweep_lds_doubles<T, TYS, CROSS>();
  __shared__ double smem[NS > SMO2_LDS_DOUBLES ? NS : SMO2_LDS_DOUBLES];
  const int di = bfind(st, blockIdx.x);
  const BFused& d = descs[di];
  if (!active[d.geo]) return;
  const int local = blockIdx.x - st.start[di];
  const int per = d.nblk + d.ntiles;
  const int z = local / per, l = local - z * per;
  const T* u = (const T*)d.u + z * d.plane;
  const T* r = (const T*)d.r + z * d.plane;
  T* out = (T*)d.out + z * d.plane;
  const T* e = PRO ? (const T*)d.e + z * d.cplane : nullptr;
  if (l < d.nblk) {
    smo2_block<T, PRO>(smem, l, z, u, out, r, d.a, e);
  } else {
    const CoefT<T> c(d.c);
    sweep_tile<T, CROSS, TYS, PRO>(smem, xcd_tile(l - d.nblk, d.ntiles), u, r, d.kind, out, d.nx, d.ny, d.nbx, c,
                                   d.regbit, d.s2bit, e, d.ncx, d.probit);
  }
}

// Two plain SMO-1 sweeps of one geometry on one level per descriptor (the
// fused step's descriptor, nblk = 0): sweep2_tile on tiles of TYS rows.
template <typename T, bool CROSS, int TYS>
__global__ __launch_bounds__(BLOCK) void k_sweep2_batched(const BFused* __restrict__ descs, BStarts st,
                                                          const int* __restrict__ active) {
  __shared__ double smem[sweep2_lds_doubles<T, TYS, CROSS>()];
  const int di = bfind(st, blockIdx.x);
  const BFused& d = descs[di];
  if (!active[d.geo]) return;
  const int local = blockIdx.x - st.start[di];
  const int z = local / d.ntiles, l = local - z * d.ntiles;
  const CoefT<T> c(d.c);
  sweep2_tile<T, CROSS, TYS>(smem, xcd_tile(l, d.ntiles), (const T*)d.u + z * d.plane, (const T*)d.r + z * d.plane,
                             d.kind, (T*)d.out + z * d.plane, d.nx, d.ny, d.nbx, c, d.regbit);
}

struct BRestrict {                 // residual + restriction of one geometry from one level
  const void *u, *r;
  const uint8_t* kind;
  void *rc, *uc;
  double* cc;
  Coef c;
  size_t plane, cplane;
  int ncc, nx, ny, nbx, ncx, ncy, ntiles;
  uint8_t regbit;
  int geo;
};

template <typename T, bool CROSS>
__global__ __launch_bounds__(BLOCK) void k_restrict_batched(const BRestrict* __restrict__ descs, BStarts st,
                                                            const int* __restrict__ active) {
  const int di = bfind(st, blockIdx.x);
  const BRestrict& d = descs[di];
  if (!active[d.geo]) return;
  const int local = blockIdx.x - st.start[di];
  const int z = local / d.ntiles, l = local - z * d.ntiles;
  const CoefT<T> c(d.c);
  restrict_tile<T, T, CROSS>(xcd_tile(l, d.ntiles), l, (const T*)d.u + z * d.plane, (const T*)d.r + z * d.plane,
                             d.kind, (T*)d.rc + z * d.cplane, (T*)d.uc + z * d.cplane, d.cc + (size_t)z * d.ncc,
                             d.ncc, d.nx, d.ny, d.nbx, d.ncx, d.ncy, c, d.regbit);
}

struct BCoarse {                   // coarsest solve (dense inverse) of one geometry
  void* u;
  const void* r;
  const int32_t* cell;
  const float* inv;
  const double* inv64;             // set: the inverse is stored in FP64
  size_t plane;
  int nm, nwg;                     // workgroups per plane
  int geo;
};

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_coarse_batched(const BCoarse* __restrict__ descs, BStarts st,
                                                          const int* __restrict__ active) {
  extern __shared__ double rv[];
  const int di = bfind(st, blockIdx.x);
  const BCoarse& d = descs[di];
  if (!active[d.geo]) return;
  const int local = blockIdx.x - st.start[di];
  const int z = local / d.nwg, l = local - z * d.nwg;
  coarse_rows<T>(rv, l, (T*)d.u + z * d.plane, (const T*)d.r + z * d.plane, d.cell, d.inv, d.inv64, d.nm);
}

struct BNorm {                     // residual check of one geometry (level 0, FP64)
  const double *u, *r;
  const uint8_t* kind;
  Coef c;
  size_t plane;
  int nx, ny, nbx, ntiles, nrb;    // workgroups per plane: nrb + ntiles
  const double* bterm;
  const int32_t *cell, *rp, *cols;
  const double *vals, *rowsum;
  int nrows;
  float* res_out;
  double* partial;                 // [plane][nrb + ntiles][max, sum of squares]
  uint8_t regbit;
  int geo;
};

template <bool CROSS>
__global__ __launch_bounds__(BLOCK) void k_resnorm_batched(const BNorm* __restrict__ descs, BStarts st,
                                                           const int* __restrict__ active) {
  const int di = bfind(st, blockIdx.x);
  const BNorm& d = descs[di];
  if (!active[d.geo]) return;
  const int local = blockIdx.x - st.start[di];
  const int per = d.nrb + d.ntiles;
  const int z = local / per, l = local - z * per;
  const CoefT<double> c(d.c);
  const NormAcc m = resnorm_block<double, CROSS>(l, d.nrb, d.ntiles, d.u + z * d.plane, d.r + z * d.plane,
                                                 d.kind, d.nx, d.ny, d.nbx, c, 0, d.regbit,
                                                 d.bterm ? d.bterm + (size_t)z * d.nrows : nullptr, d.cell, d.rp,
                                                 d.cols, d.vals, d.rowsum, d.nrows,
                                                 d.res_out ? d.res_out + z * d.plane : nullptr);
  if (threadIdx.x == 0) d.partial[2 * local] = m.m, d.partial[2 * local + 1] = m.s;
}

struct BAux {                      // mixed precision, level 0: zero start / correction
  float* u32;                      // zeroed (start) or read (u += u32)
  double* cc;                      // compact copies zeroed at the start
  double* u;                       // FP64 iterate
  const uint8_t* kind;
  size_t plane, n, ncc;            // n = plane * planes
  int geo;
};

// mode 0: u32 = 0 and cc = 0 (zero guess of the correction); mode 1:
// u += u32 on non-empty cells.  BAUX_WG workgroups per geometry.
constexpr int BAUX_WG = 256;
__global__ __launch_bounds__(BLOCK) void k_aux_batched(const BAux* __restrict__ descs, BStarts st,
                                                       const int* __restrict__ active, int mode) {
  const int di = bfind(st, blockIdx.x);
  const BAux& d = descs[di];
  if (!active[d.geo]) return;
  const size_t l = blockIdx.x - st.start[di];
  const size_t stride = (size_t)BAUX_WG * BLOCK;
  if (mode == 0) {
    for (size_t k = l * BLOCK + threadIdx.x; k < d.n; k += stride) d.u32[k] = 0.0f;
    for (size_t k = l * BLOCK + threadIdx.x; k < d.ncc; k += stride) d.cc[k] = 0.0;
  } else {
    for (size_t k = l * BLOCK + threadIdx.x; k < d.n; k += stride)
      if (d.kind[k % d.plane] & F_NONEMPTY) d.u[k] += (double)d.u32[k];
  }
}
