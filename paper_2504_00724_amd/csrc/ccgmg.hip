// MI355X cut-cell multigrid: device kernels, V-cycle driver and the C
// interface declared in ccgmg.h.
//
// The V-cycle is Alg. 2: on each level nu1 smoothing steps, residual and
// restriction, recursion with a zero guess, prolongation and correction,
// nu2 smoothing steps; the coarsest level is solved exactly.  A smoothing
// step is SMO-1 (omega-weighted Jacobi on the regular cells, Section 4.1)
// followed by SMO-2 (the block update of the irregular cells, eq.
// updateByBlock).  SMO-2 is carried out by restricted additive Schwarz over
// consecutive runs of the Alg. 3 numbering with precomputed FP64 block
// inverses, instead of the paper's banded LU of the whole block: a banded
// triangular solve is a chain of dependent steps, while the blocks are
// independent and map onto one workgroup each.  The converged solution does
// not depend on the smoother.
//
// The adjoint solve runs the same V-cycle on L^T (and its coarse-level
// counterparts): cells whose 5x5 box is regular and that no irregular row
// references keep the symmetric regular stencil, all other rows of L^T are
// explicit (setup.hpp: transposed_rows).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "ccgmg.h"
#include "kernels.hpp"
#include "setup.hpp"

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
template <typename T, int TYS>
constexpr int sweep_lds_doubles() { return ((TYS + 2 * HALO) * LW * (int)sizeof(T) + 7) / 8; }

template <typename T, bool CROSS, int TYS, bool PRO = false>
__device__ __forceinline__ void sweep_tile(double* smem, int t, const T* __restrict__ u, const T* __restrict__ r,
                                           const uint8_t* __restrict__ kind, T* __restrict__ out, int nx, int ny,
                                           int nbx, const CoefT<T>& c, uint8_t regbit, uint8_t skipbit,
                                           const T* __restrict__ e = nullptr, int ncx = 0, uint8_t probit = 0) {
  constexpr int RPW = TYS / 4;            // rows per wave
  constexpr int ROWS = TYS + 2 * HALO;
  T (*tile)[LW] = reinterpret_cast<T (*)[LW]>(smem);
  const int tyi = t / nbx;
  const int bx = (t - tyi * nbx) * TX, by = tyi * TYS;
  const int tx = threadIdx.x & (TX - 1), w = threadIdx.x >> 6;
  // issue the kind and right-hand-side loads before the tile barrier
  uint8_t kd[RPW];
  T rr[RPW];
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int gx = bx + tx, gy = by + w + 4 * k;
    const bool in = gx < nx && gy < ny;
    kd[k] = in ? kind[(size_t)gy * nx + gx] : (uint8_t)0;
    rr[k] = in ? r[(size_t)gy * nx + gx] : (T)0;
  }
  if (PRO) {
    // tile of u + P e: the pending coarse-grid correction (piecewise
    // constant, cells flagged probit only) is added while staging
    for (int k = threadIdx.x; k < ROWS * LW; k += BLOCK) {
      const int ly = k / LW, lx = k - ly * LW;
      const int gx = bx + lx - HALO, gy = by + ly - HALO;
      T v = (T)0;
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
        const size_t g = (size_t)gy * nx + gx;
        v = u[g];
        if (kind[g] & probit) v += e[(size_t)(gy >> 1) * ncx + (gx >> 1)];
      }
      tile[ly][lx] = v;
    }
  } else {
    load_tile<T, ROWS>(tile, u, nx, ny, bx, by);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RPW; ++k) {
    const int ry = w + 4 * k;
    const int gx = bx + tx, gy = by + ry;
    if (gx < nx && gy < ny && !(kd[k] & skipbit)) {
      T v = tile[ry + HALO][tx + HALO];
      if (kd[k] & regbit) v += c.omega_invD * (rr[k] - apply_regular<T, CROSS>(tile, ry + HALO, tx + HALO, c));
      out[(size_t)gy * nx + gx] = v;
    }
  }
}

// SMO-1 sweep launch: one workgroup per tile on a 1-D grid remapped by
// xcd_tile.  FINEST only selects a separate instantiation for the finest
// level so that kernel traces separate it from the coarse levels.
template <typename T, bool CROSS, bool FINEST, int TYS>
__global__ __launch_bounds__(BLOCK) void k_sweep(const T* __restrict__ u, const T* __restrict__ r,
                                                 const uint8_t* __restrict__ kind, T* __restrict__ out, int nx,
                                                 int ny, int nbx, CoefT<T> c, uint8_t regbit) {
  __shared__ double smem[sweep_lds_doubles<T, TYS>()];
  const size_t zoff = (size_t)blockIdx.z * nx * ny;
  sweep_tile<T, CROSS, TYS>(smem, xcd_tile(blockIdx.x, gridDim.x), u + zoff, r + zoff, kind, out + zoff, nx, ny,
                            nbx, c, regbit, 0);
}

// Residual of the regular cells restricted to the coarse grid:
// rc_I = 1/4 sum over regular children c of (r - L u)_c  (Section 4.1).
// The same launch zeroes the coarse iterate uc (the recursion starts from a
// zero guess, Alg. 2) and the compact copy cc of its block rows.
template <typename T, typename TC, bool CROSS, bool FINEST>
__global__ __launch_bounds__(BLOCK) void k_restrict(const T* __restrict__ u, const T* __restrict__ r,
                                                    const uint8_t* __restrict__ kind, TC* __restrict__ rc,
                                                    TC* __restrict__ uc, double* __restrict__ cc, int ncc, int nx,
                                                    int ny, int nbx, int ncx, int ncy, CoefT<T> c, uint8_t regbit) {
  __shared__ T tile[LH][LW];
  const size_t zoff = (size_t)blockIdx.z * nx * ny;
  u += zoff, r += zoff;
  rc += (size_t)blockIdx.z * ncx * ncy;
  uc += (size_t)blockIdx.z * ncx * ncy;
  {
    const int flat = blockIdx.x * BLOCK + threadIdx.x;
    if (flat < ncc) cc[(size_t)blockIdx.z * ncc + flat] = 0.0;
  }
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int tyi = t / nbx, txi = t - tyi * nbx;
  const int bx = txi * TX, by = tyi * TY;
  const int cx = threadIdx.x & 31, cy = threadIdx.x >> 5;  // 32 x 8 coarse cells
  uint8_t kd[4];
  T rr[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int gx = bx + 2 * cx + (d & 1), gy = by + 2 * cy + (d >> 1);
    const bool in = gx < nx && gy < ny;
    kd[d] = in ? kind[(size_t)gy * nx + gx] : (uint8_t)0;
    rr[d] = in ? r[(size_t)gy * nx + gx] : (T)0;
  }
  load_tile(tile, u, nx, ny, bx, by);
  __syncthreads();
  const int I = txi * (TX / 2) + cx, J = tyi * (TY / 2) + cy;
  if (I >= ncx || J >= ncy) return;
  T s = (T)0;
#pragma unroll
  for (int d = 0; d < 4; ++d)
    if (kd[d] & regbit)
      s += rr[d] - apply_regular<T, CROSS>(tile, 2 * cy + (d >> 1) + HALO, 2 * cx + (d & 1) + HALO, c);
  rc[(size_t)J * ncx + I] = (TC)((T)0.25 * s);
  uc[(size_t)J * ncx + I] = (TC)0;
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
template <typename T>
__device__ __forceinline__ double row_residual(const T* __restrict__ u, double rhs, int q, const int32_t* cols,
                                               const double* vals, int len, double rowsum) {
  const double uq = (double)u[q];
  double a0 = 0.0, a1 = 0.0;
  int s = 0;
  for (; s + 1 < len; s += 2) {
    a0 += vals[s] * ((double)u[cols[s]] - uq);
    a1 += vals[s + 1] * ((double)u[cols[s + 1]] - uq);
  }
  if (s < len) a0 += vals[s] * ((double)u[cols[s]] - uq);
  return rhs - (a0 + a1) - rowsum * uq;
}

// Arguments of an SMO-2 pass (see k_smo2).
struct Smo2Args {
  const double* bterm;
  const int32_t *ecell, *erp, *ecols;
  const double *evals, *ersum;
  const int32_t *eidx, *ebt, *ext_ptr, *own_cnt;
  const int64_t* inv_off;
  const double* inv;
  const double* c_in;
  double* c_out;
  int ns, nbt;
  const int32_t* epar;    // per CSR entry: coarse parent of the column cell if it takes the correction, else -1
  const int32_t* eqpar;   // per overlapped row: the same for the row's own cell
};

// One RAS block b of plane z: reads uin (non-block columns) and c_in, writes
// its own rows to uout and c_out.  With a pending coarse-grid correction
// (PRO, coarse values ecor), every value read is taken as value +
// ecor[parent] where the cell takes the correction (a.epar / a.eqpar >= 0),
// i.e. the block works on u + P e.
constexpr int SMO2_LDS_DOUBLES = 1024 + 4 * 64 + 64;

template <typename T, bool PRO = false>
__device__ __forceinline__ void smo2_block(double* smem, int b, int z, const T* uin, T* uout,
                                           const T* __restrict__ r, const Smo2Args& a,
                                           const T* __restrict__ ecor = nullptr) {
  double* res = smem;                                              // [1024]
  double (*part)[64] = reinterpret_cast<double (*)[64]>(smem + 1024);   // [4][64]
  double* uown = smem + 1024 + 4 * 64;                             // [64]
  const double* c_in = a.c_in + (size_t)z * a.ns;
  double* c_out = a.c_out + (size_t)z * a.ns;
  const int e0 = a.ext_ptr[b], ne = a.ext_ptr[b + 1] - e0, nown = a.own_cnt[b];
  for (int t = threadIdx.x; t < ne; t += BLOCK) {
    const int e = e0 + t;
    double uq = c_in[a.eidx[e]];
    if (PRO) {
      const int pq = a.eqpar[e];
      if (pq >= 0) uq += (double)ecor[pq];
    }
    if (t < 64) uown[t] = uq;
    double rhs = (double)r[a.ecell[e]];
    if (a.bterm && a.ebt[e] >= 0) rhs -= a.bterm[(size_t)z * a.nbt + a.ebt[e]];
    const int p1 = a.erp[e + 1];
    double acc = 0.0;
    for (int p = a.erp[e]; p < p1; p += 8) {
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
        uu[k] = cc[k] >= 0 ? (double)uin[cc[k]] : c_in[-cc[k] - 1];
        if (PRO && pp[k] >= 0) uu[k] += (double)ecor[pp[k]];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) acc += vv[k] * (uu[k] - uq);
    }
    res[t] = rhs - acc - a.ersum[e] * uq;
  }
  __syncthreads();
  const int row = threadIdx.x & 63, grp = threadIdx.x >> 6;
  double s = 0.0;
  if (row < nown) {
    const double* A = a.inv + a.inv_off[b] + row;
    int col = grp;
    for (; col + 28 < ne; col += 32) {
      double v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = A[(size_t)(col + 4 * k) * nown];
#pragma unroll
      for (int k = 0; k < 8; ++k) s += v[k] * res[col + 4 * k];
    }
    for (; col < ne; col += 4) s += A[(size_t)col * nown] * res[col];
  }
  part[grp][row] = s;
  __syncthreads();
  if (grp == 0 && row < nown) {
    const int k = a.eidx[e0 + row];
    const T v = (T)(uown[row] + (part[0][row] + part[1][row] + part[2][row] + part[3][row]));
    uout[a.ecell[e0 + row]] = v;
    c_out[k] = (double)v;
  }
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
// probit; the coarse grid is ncx x ncy).
template <typename T, bool CROSS, bool FINEST, int TYS, bool PRO>
__global__ __launch_bounds__(BLOCK) void k_smooth_fused(const T* __restrict__ u, const T* __restrict__ r,
                                                        const uint8_t* __restrict__ kind, T* __restrict__ out,
                                                        int nx, int ny, int nbx, int nblk, CoefT<T> c,
                                                        uint8_t regbit, uint8_t s2bit, Smo2Args a,
                                                        const T* __restrict__ e, int ncx, int ncy, uint8_t probit) {
  // one LDS buffer shared by the two kinds of workgroup
  constexpr int NS = sweep_lds_doubles<T, TYS>();
  __shared__ double smem[NS > SMO2_LDS_DOUBLES ? NS : SMO2_LDS_DOUBLES];
  const size_t zoff = (size_t)blockIdx.z * nx * ny;
  const T* ez = PRO ? e + (size_t)blockIdx.z * ncx * ncy : nullptr;
  if ((int)blockIdx.x < nblk)
    smo2_block<T, PRO>(smem, blockIdx.x, blockIdx.z, u + zoff, out + zoff, r + zoff, a, ez);
  else
    sweep_tile<T, CROSS, TYS, PRO>(smem, xcd_tile(blockIdx.x - nblk, gridDim.x - nblk), u + zoff, r + zoff, kind,
                                   out + zoff, nx, ny, nbx, c, regbit, s2bit, ez, ncx, probit);
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
// |r - bterm| when zero_u is set, in one launch: workgroups [0, ntiles) take
// the stencil cells of one TX x TY tile each (remapped by xcd_tile), the
// rest BLOCK explicit rows each (FP64; optionally writing the row residual
// into res_out as FP32 for the refinement loop).  Every workgroup stores its
// partial maximum in partial[z * gridDim.x + b]; the host, which reads the
// norm back anyway, takes the maximum of the partials (no second launch and
// no device-wide fence).
template <typename T, bool CROSS>
__global__ __launch_bounds__(BLOCK) void k_resnorm(const T* __restrict__ u, const T* __restrict__ r,
                                                   const uint8_t* __restrict__ kind, int nx, int ny, int nbx,
                                                   int ntiles, CoefT<T> c, int zero_u, uint8_t regbit,
                                                   const double* __restrict__ bterm, const int32_t* __restrict__ cell,
                                                   const int32_t* __restrict__ rp, const int32_t* __restrict__ cols,
                                                   const double* __restrict__ vals,
                                                   const double* __restrict__ rowsum, int nrows,
                                                   float* __restrict__ res_out, double* __restrict__ partial) {
  __shared__ T tile[LH][LW];
  __shared__ double red[BLOCK];
  const int z = blockIdx.z;
  const size_t plane = (size_t)nx * ny;
  u += z * plane, r += z * plane;
  double m = 0.0;
  if ((int)blockIdx.x < ntiles) {
    const int t = xcd_tile(blockIdx.x, ntiles);
    const int tyi = t / nbx;
    const int bx = (t - tyi * nbx) * TX, by = tyi * TY;
    const int tx = threadIdx.x & (TX - 1), w = threadIdx.x >> 6;
    uint8_t kd[TY / 4];
    T rr[TY / 4];
#pragma unroll
    for (int k = 0; k < TY / 4; ++k) {
      const int gx = bx + tx, gy = by + w + 4 * k;
      const bool in = gx < nx && gy < ny;
      kd[k] = in ? kind[(size_t)gy * nx + gx] : (uint8_t)0;
      rr[k] = in ? r[(size_t)gy * nx + gx] : (T)0;
    }
    load_tile(tile, u, nx, ny, bx, by);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TY / 4; ++k) {
      if (kd[k] & regbit) {
        T v = rr[k];
        if (!zero_u) v -= apply_regular<T, CROSS>(tile, w + 4 * k + HALO, tx + HALO, c);
        m = fmax(m, fabs((double)v));
      }
    }
  } else {
    const int k = (blockIdx.x - ntiles) * BLOCK + threadIdx.x;
    if (k < nrows) {
      const int q = cell[k];
      double rhs = (double)r[q];
      if (bterm) rhs -= bterm[(size_t)z * nrows + k];
      if (!zero_u) rhs = row_residual(u, rhs, q, cols + rp[k], vals + rp[k], rp[k + 1] - rp[k], rowsum[k]);
      if (res_out) res_out[z * plane + q] = (float)rhs;
      m = fabs(rhs);
    }
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int st = BLOCK / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)z * gridDim.x + blockIdx.x] = red[0];
}

// FP64 refinement residual on stencil cells, written as FP32 (MP mode).
template <bool CROSS>
__global__ __launch_bounds__(BLOCK) void k_residual_f32(const double* __restrict__ u, const double* __restrict__ r,
                                                        const uint8_t* __restrict__ kind, float* __restrict__ out,
                                                        int nx, int ny, int nbx, CoefT<double> c, uint8_t regbit) {
  __shared__ double tile[LH][LW];
  const size_t zoff = (size_t)blockIdx.z * nx * ny;
  u += zoff, r += zoff, out += zoff;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  const int tyi = t / nbx;
  const int bx = (t - tyi * nbx) * TX, by = tyi * TY;
  const int tx = threadIdx.x & (TX - 1), w = threadIdx.x >> 6;
  uint8_t kd[TY / 4];
  double rr[TY / 4];
#pragma unroll
  for (int k = 0; k < TY / 4; ++k) {
    const int gx = bx + tx, gy = by + w + 4 * k;
    const bool in = gx < nx && gy < ny;
    kd[k] = in ? kind[(size_t)gy * nx + gx] : (uint8_t)0;
    rr[k] = in ? r[(size_t)gy * nx + gx] : 0.0;
  }
  load_tile(tile, u, nx, ny, bx, by);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < TY / 4; ++k) {
    const int ry = w + 4 * k, gx = bx + tx, gy = by + ry;
    if (gx < nx && gy < ny)
      out[(size_t)gy * nx + gx] =
          (kd[k] & regbit) ? (float)(rr[k] - apply_regular<double, CROSS>(tile, ry + HALO, tx + HALO, c)) : 0.0f;
  }
}

// Coarsest level: u[cell_k] = sum_j Inv[k, j] r[cell_j] (FP64), one wavefront
// per row (4 rows per workgroup), the gathered right-hand side staged in LDS.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_coarse(T* __restrict__ u, const T* __restrict__ r,
                                                  const int32_t* __restrict__ cell, const double* __restrict__ inv,
                                                  int nm, size_t plane) {
  extern __shared__ double rv[];
  const int z = blockIdx.y;
  u += (size_t)z * plane, r += (size_t)z * plane;
  for (int k = threadIdx.x; k < nm; k += BLOCK) rv[k] = (double)r[cell[k]];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= nm) return;
  const double* A = inv + (size_t)row * nm;
  double s0 = 0.0, s1 = 0.0;
  int k = lane;
  for (; k + 64 < nm; k += 128) s0 += A[k] * rv[k], s1 += A[k + 64] * rv[k + 64];
  if (k < nm) s0 += A[k] * rv[k];
  double s = s0 + s1;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) u[cell[row]] = (T)s;
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
// Host side
// ===========================================================================
namespace {

thread_local std::string g_create_error;

#define HIP_OK(x)                                                                                          \
  do {                                                                                                     \
    hipError_t e_ = (x);                                                                                   \
    if (e_ != hipSuccess) throw ccg::Error(CCGMG_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
T* dalloc(size_t n, std::vector<void*>& owned) {
  void* p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw ccg::Error(CCGMG_ENOMEM, "hipMalloc failed");
  owned.push_back(p);
  return (T*)p;
}

template <typename T>
T* upload(const std::vector<T>& v, std::vector<void*>& owned) {
  T* p = dalloc<T>(v.size(), owned);
  if (!v.empty()) HIP_OK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}

struct Smo2Data {                 // RAS blocks of one row set
  int nblk = 0;
  int32_t *ext_ptr = nullptr, *ext_idx = nullptr, *own_cnt = nullptr;
  int32_t *ecell = nullptr, *erp = nullptr, *ecols = nullptr;   // overlapped rows, CSR
  int32_t* ebt = nullptr;         // boundary-term index of each overlapped row (-1: none)
  int32_t* scell = nullptr;       // cell of every block row
  int32_t *epar = nullptr, *eqpar = nullptr;   // coarse parents (fused prolongation), -1: none
  int ns = 0;                     // block rows
  double* cbuf[2] = {nullptr, nullptr};   // compact copies of the block rows' values
  int cur = 0;                    // which copy is current while a cycle is recorded
  double *evals = nullptr, *ersum = nullptr;
  int64_t* inv_off = nullptr;
  double* inv = nullptr;
  size_t inv_bytes = 0;
  int max_ext = 0;
  long n_ext = 0, n_ext_nnz = 0;   // overlapped rows and their CSR entries, all blocks
};

struct DevRows {                  // explicit rows of L (or L^T) on one level
  int n = 0;
  int32_t *cell = nullptr, *rp = nullptr, *cols = nullptr;
  double *vals = nullptr, *rowsum = nullptr;
  Smo2Data smo2;
};

struct DevLevel {
  int nx = 0, ny = 0;
  size_t n = 0;
  double h = 0;
  Coef coef;
  bool cross = false;
  uint8_t* kind = nullptr;
  DevRows fwd, adj;
  // work arrays (max_nrhs planes)
  double *u = nullptr, *v = nullptr, *r = nullptr;
  float *u32 = nullptr, *v32 = nullptr, *r32 = nullptr;
  double* du = nullptr;
  double* part = nullptr;         // reduction partials
  int sweep_ty[2] = {16, 16};     // SMO-1 tile height (FP64, FP32), tuned at set-up
  int npart_reg = 0, npart_irr = 0;
};

}  // namespace

struct ccgmg_ctx {
  ccgmg_options opt;
  double a = 1, b = 0, c = 1;
  ccg::Hierarchy H;
  std::vector<DevLevel> lv;
  std::vector<void*> owned;
  hipStream_t stream = nullptr;
  int M = 0;                        // coarsest level index in use
  int nm = 0;                       // coarsest unknowns
  int32_t* mcell = nullptr;
  double* minv = nullptr;           // inverse of the coarsest operator
  double* mtinv = nullptr;          // inverse of its transpose
  struct Coarse {
    int nm;
    int32_t* cell;
    double *inv, *tinv;
  };
  std::map<int, Coarse> coarse_cache;   // per coarsest level index
  std::vector<double> tune_ms;          // autotune: solve time per depth (index = M)
  int nfaces = 0;                   // level-0 boundary data
  int32_t *fptr = nullptr, *fface = nullptr, *fcell = nullptr;
  double *fval = nullptr, *fweight = nullptr;
  double* g = nullptr;              // [max_nrhs][nfaces]
  double* bterm = nullptr;          // [max_nrhs][nirr0]
  int g_nrhs = 0;
  double* norm_host = nullptr;      // pinned: partial maxima of the residual norm (level 0)
  double setup_seconds = 0;
  double plg_max_cond = 0;
  std::string err;
  bool host_only = false;
  // solves run on a private stream (ordered after the caller's stream by
  // events) so that each V-cycle can be captured into a hipGraph
  hipStream_t ws = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  struct GraphEntry {
    const void *u, *f, *bterm;
    int nrhs, precision, M;
    bool adjoint;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  void clear_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }
};

namespace {

// 1-D grid of TX x ty tiles (remapped per XCD in the kernels), nrhs planes
int tiles_x(int nx) { return (nx + TX - 1) / TX; }
dim3 tiles1d(int nx, int ny, int nrhs, int ty = TY) {
  return dim3(tiles_x(nx) * ((ny + ty - 1) / ty), 1, nrhs);
}
dim3 tiles(int nx, int ny, int nrhs) { return dim3((nx + TX - 1) / TX, (ny + TY - 1) / TY, nrhs); }

// RAS block data for a row set: blocks of `bsize` consecutive rows of the
// numbering `order`, each extended by `overlap` layers of its matrix-graph
// neighbourhood (restricted to the row set); the dense inverse of the
// extended block is kept for the block's own rows (column-major).
void build_smo2(const ccg::RowSet& R, const std::vector<int32_t>& bt, const std::vector<int32_t>& parent,
                size_t ncells, int bsize, int overlap, int threads, Smo2Data& out, std::vector<void*>& owned) {
  const int ni = (int)R.cell.size();
  if (ni == 0) return;
  std::vector<int32_t> pos(ncells, -1);
  for (int k = 0; k < ni; ++k) pos[R.cell[k]] = k;
  std::vector<std::vector<int>> nb(ni);
  for (int k = 0; k < ni; ++k)
    for (int s = R.rp[k]; s < R.rp[k + 1]; ++s) {
      int p = pos[R.cols[s]];
      if (p >= 0 && p != k) nb[k].push_back(p), nb[p].push_back(k);
    }
  for (auto& v : nb) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  const int nblk = (ni + bsize - 1) / bsize;
  std::vector<std::vector<int>> ext(nblk);
  std::vector<int> own(nblk);
  std::vector<std::vector<double>> inv(nblk);
  std::vector<int> fail(nblk, 0);
  ccg::parallel_for(nblk, threads, [&](int b0, int b1) {
    for (int b = b0; b < b1; ++b) {
      int s = b * bsize, e = std::min(ni, s + bsize);
      std::vector<int> cur;
      for (int p = s; p < e; ++p) cur.push_back(R.order[p]);
      own[b] = (int)cur.size();
      std::set<int> in(cur.begin(), cur.end());
      std::vector<int> frontier = cur;
      for (int l = 0; l < overlap; ++l) {
        std::vector<int> nxt;
        for (int k : frontier)
          for (int m : nb[k])
            if (in.insert(m).second) nxt.push_back(m);
        std::sort(nxt.begin(), nxt.end());
        for (int m : nxt) {
          if ((int)cur.size() >= 1024) break;
          cur.push_back(m);
        }
        frontier = nxt;
        if ((int)cur.size() >= 1024) break;
      }
      const int ne = (int)cur.size();
      std::map<int, int> where;
      for (int t = 0; t < ne; ++t) where[cur[t]] = t;
      std::vector<double> A((size_t)ne * ne, 0.0);
      for (int t = 0; t < ne; ++t) {
        const int k = cur[t];
        for (int q = R.rp[k]; q < R.rp[k + 1]; ++q) {
          int p = pos[R.cols[q]];
          if (p < 0) continue;
          auto it = where.find(p);
          if (it != where.end()) A[(size_t)t * ne + it->second] += R.vals[q];
        }
      }
      if (!ccg::dense_inverse(A, ne, 1)) {
        fail[b] = 1;
        continue;
      }
      std::vector<double> keep((size_t)ne * own[b]);
      for (int col = 0; col < ne; ++col)
        for (int row = 0; row < own[b]; ++row) keep[(size_t)col * own[b] + row] = A[(size_t)row * ne + col];
      inv[b].swap(keep);
      ext[b] = cur;
    }
  });
  for (int b = 0; b < nblk; ++b)
    if (fail[b]) throw ccg::Error(CCGMG_ESINGULAR, "singular SMO-2 block");
  std::vector<int32_t> eptr(nblk + 1, 0), eidx, ocnt(nblk);
  std::vector<int64_t> ioff(nblk);
  std::vector<double> all;
  for (int b = 0; b < nblk; ++b) {
    eptr[b + 1] = eptr[b] + (int)ext[b].size();
    eidx.insert(eidx.end(), ext[b].begin(), ext[b].end());
    ocnt[b] = own[b];
    ioff[b] = (int64_t)all.size();
    all.insert(all.end(), inv[b].begin(), inv[b].end());
    out.max_ext = std::max(out.max_ext, (int)ext[b].size());
  }
  std::vector<int32_t> ecell(eidx.size()), erp(eidx.size() + 1, 0), ecols, ebt(eidx.size()), epar,
      eqpar(eidx.size());
  std::vector<double> evals, ersum(eidx.size());
  for (size_t e = 0; e < eidx.size(); ++e) {
    const int k = eidx[e];
    ecell[e] = R.cell[k];
    ebt[e] = bt[k];
    eqpar[e] = parent[R.cell[k]];
    double rs = 0;
    for (int t = R.rp[k]; t < R.rp[k + 1]; ++t) {
      const int p = pos[R.cols[t]];
      ecols.push_back(p >= 0 ? -(p + 1) : R.cols[t]);
      epar.push_back(parent[R.cols[t]]);
      evals.push_back(R.vals[t]);
      rs += R.vals[t];
    }
    erp[e + 1] = (int32_t)ecols.size();
    ersum[e] = rs;
  }
  out.ecell = upload(ecell, owned);
  out.ebt = upload(ebt, owned);
  out.scell = upload(R.cell, owned);
  out.ns = ni;
  out.erp = upload(erp, owned);
  out.ecols = upload(ecols, owned);
  out.epar = upload(epar, owned);
  out.eqpar = upload(eqpar, owned);
  out.evals = upload(evals, owned);
  out.ersum = upload(ersum, owned);
  out.nblk = nblk;
  out.ext_ptr = upload(eptr, owned);
  out.ext_idx = upload(eidx, owned);
  out.own_cnt = upload(ocnt, owned);
  out.inv_off = upload(ioff, owned);
  out.inv = upload(all, owned);
  out.inv_bytes = all.size() * sizeof(double);
  out.n_ext = (long)eidx.size();
  out.n_ext_nnz = (long)ecols.size();
}

void upload_rows(const ccg::RowSet& R, const ccg::RowSet& S, const std::vector<int32_t>& bt,
                 const std::vector<int32_t>& parent, size_t ncells, const ccgmg_options& opt, DevRows& D,
                 std::vector<void*>& owned) {
  D.n = (int)R.cell.size();
  std::vector<double> rs(D.n);
  for (int k = 0; k < D.n; ++k) {
    double s = 0;
    for (int t = R.rp[k]; t < R.rp[k + 1]; ++t) s += R.vals[t];
    rs[k] = s;
  }
  D.cell = upload(R.cell, owned);
  D.rp = upload(R.rp, owned);
  D.cols = upload(R.cols, owned);
  D.vals = upload(R.vals, owned);
  D.rowsum = upload(rs, owned);
  build_smo2(S, bt, parent, ncells, opt.smo2_block, opt.smo2_overlap, opt.num_threads, D.smo2, owned);
}

}  // namespace

// ---------------------------------------------------------------------------
// V-cycle driver
// ---------------------------------------------------------------------------
namespace {

template <typename T>
struct Buf {
  T *u, *v, *r;
};

template <typename T>
Buf<T> bufs(DevLevel& L) {
  if constexpr (sizeof(T) == 8)
    return {(T*)L.u, (T*)L.v, (T*)L.r};
  else
    return {(T*)L.u32, (T*)L.v32, (T*)L.r32};
}

struct Driver {
  ccgmg_ctx* X;
  hipStream_t s;
  int nrhs;
  bool adjoint;

  uint8_t regbit() const { return adjoint ? F_REG_T : F_REG; }
  uint8_t jacbit() const { return adjoint ? F_JAC_T : F_JAC; }
  DevRows& rows(DevLevel& L) const { return adjoint ? L.adj : L.fwd; }

  template <typename T, bool CROSS, bool FIN>
  void sweep_t(DevLevel& L, const T* u, const T* r, T* out, int ty) {
    CoefT<T> c(L.coef);
    const dim3 g = tiles1d(L.nx, L.ny, nrhs, ty);
    const int nbx = tiles_x(L.nx);
    const uint8_t rb = jacbit();
    switch (ty) {
      case 8: hipLaunchKernelGGL((k_sweep<T, CROSS, FIN, 8>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, c, rb); break;
      case 32: hipLaunchKernelGGL((k_sweep<T, CROSS, FIN, 32>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, c, rb); break;
      default: hipLaunchKernelGGL((k_sweep<T, CROSS, FIN, 16>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, c, rb); break;
    }
  }

  template <typename T>
  void sweep(DevLevel& L, const T* u, const T* r, T* out, int ty = 0) {
    if (ty == 0) ty = L.sweep_ty[sizeof(T) == 8 ? 0 : 1];
    const bool fin = &L == &X->lv[0];
    if (L.cross) {
      if (fin) sweep_t<T, true, true>(L, u, r, out, ty);
      else sweep_t<T, true, false>(L, u, r, out, ty);
    } else {
      if (fin) sweep_t<T, false, true>(L, u, r, out, ty);
      else sweep_t<T, false, false>(L, u, r, out, ty);
    }
  }

  // restriction into rc; also zeroes the coarse iterate uc and the coarse
  // block rows' compact copy (which becomes the current one)
  template <typename T>
  void restrict_(DevLevel& L, DevLevel& C, const T* u, const T* r, T* rc, T* uc) {
    CoefT<T> c(L.coef);
    const dim3 g = tiles1d(L.nx, L.ny, nrhs);
    const int nbx = tiles_x(L.nx);
    const bool fin = &L == &X->lv[0];
    const uint8_t rb = regbit();
    Smo2Data& CS = rows(C).smo2;
    CS.cur = 0;
    double* cc = CS.cbuf[0];
    const int ncc = CS.ns;
    if (L.cross) {
      if (fin) hipLaunchKernelGGL((k_restrict<T, T, true, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, rc, uc, cc, ncc, L.nx, L.ny, nbx, C.nx, C.ny, c, rb);
      else hipLaunchKernelGGL((k_restrict<T, T, true, false>), g, dim3(BLOCK), 0, s, u, r, L.kind, rc, uc, cc, ncc, L.nx, L.ny, nbx, C.nx, C.ny, c, rb);
    } else {
      if (fin) hipLaunchKernelGGL((k_restrict<T, T, false, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, rc, uc, cc, ncc, L.nx, L.ny, nbx, C.nx, C.ny, c, rb);
      else hipLaunchKernelGGL((k_restrict<T, T, false, false>), g, dim3(BLOCK), 0, s, u, r, L.kind, rc, uc, cc, ncc, L.nx, L.ny, nbx, C.nx, C.ny, c, rb);
    }
  }

  template <typename T>
  void prolong(DevLevel& L, DevLevel& C, T* u, const T* e) {
    Smo2Data& S = rows(L).smo2;
    const int gx = (L.nx + 255) / 256;
    const int extra = S.ns > 0 ? (S.ns + 256 * gx - 1) / (256 * gx) : 0;
    hipLaunchKernelGGL((k_prolong<T>), dim3(gx, L.ny + extra, nrhs), dim3(256), 0, s, u, e, L.kind, C.kind, L.nx,
                       L.ny, C.nx, C.ny, X->opt.prolongation, regbit(), S.scell, S.cbuf[S.cur], S.ns);
  }

  // kernel arguments of one SMO-2 pass (reads the current compact copy,
  // writes the other one)
  Smo2Args smo2_args(DevLevel& L, const double* bterm) {
    DevRows& R = rows(L);
    Smo2Data& S = R.smo2;
    Smo2Args a;
    a.bterm = bterm;
    a.ecell = S.ecell, a.erp = S.erp, a.ecols = S.ecols;
    a.evals = S.evals, a.ersum = S.ersum;
    a.eidx = S.ext_idx, a.ebt = S.ebt, a.ext_ptr = S.ext_ptr, a.own_cnt = S.own_cnt;
    a.inv_off = S.inv_off, a.inv = S.inv;
    a.c_in = S.cbuf[S.cur], a.c_out = S.cbuf[1 - S.cur];
    a.ns = S.ns, a.nbt = R.n;
    a.epar = S.epar, a.eqpar = S.eqpar;
    return a;
  }

  template <typename T>
  void smo2_pass(DevLevel& L, T* u, const T* r, const double* bterm) {
    Smo2Data& S = rows(L).smo2;
    hipLaunchKernelGGL((k_smo2<T>), dim3(S.nblk, nrhs), dim3(BLOCK), 0, s, u, r, smo2_args(L, bterm), L.n);
    S.cur = 1 - S.cur;
  }

  // one fused smoothing step (SMO-1 and SMO-2 from the same iterate u)
  template <typename T, bool CROSS, bool FIN, bool PRO>
  void fused_t(DevLevel& L, const T* u, const T* r, T* out, const double* bterm, int ty, const T* e,
               const DevLevel* C) {
    Smo2Data& S = rows(L).smo2;
    CoefT<T> c(L.coef);
    const int nbx = tiles_x(L.nx);
    const int ntiles = nbx * ((L.ny + ty - 1) / ty);
    const dim3 g(ntiles + S.nblk, 1, nrhs);
    const uint8_t rb = jacbit(), sb = adjoint ? F_S2_T : F_S2;
    const Smo2Args a = smo2_args(L, bterm);
    const int ncx = C ? C->nx : 0, ncy = C ? C->ny : 0;
    const uint8_t pb = regbit();
    switch (ty) {
      case 8: hipLaunchKernelGGL((k_smooth_fused<T, CROSS, FIN, 8, PRO>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, S.nblk, c, rb, sb, a, e, ncx, ncy, pb); break;
      case 32: hipLaunchKernelGGL((k_smooth_fused<T, CROSS, FIN, 32, PRO>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, S.nblk, c, rb, sb, a, e, ncx, ncy, pb); break;
      default: hipLaunchKernelGGL((k_smooth_fused<T, CROSS, FIN, 16, PRO>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, S.nblk, c, rb, sb, a, e, ncx, ncy, pb); break;
    }
    S.cur = 1 - S.cur;
  }

  template <typename T, bool CROSS, bool FIN>
  void fused_p(DevLevel& L, const T* u, const T* r, T* out, const double* bterm, int ty, const T* e,
               const DevLevel* C) {
    if (e) fused_t<T, CROSS, FIN, true>(L, u, r, out, bterm, ty, e, C);
    else fused_t<T, CROSS, FIN, false>(L, u, r, out, bterm, ty, nullptr, nullptr);
  }

  // one fused step; with e, the pending coarse-grid correction P e (coarse
  // level C) is applied on the fly
  template <typename T>
  void fused_step(DevLevel& L, const T* u, const T* r, T* out, const double* bterm, const T* e = nullptr,
                  const DevLevel* C = nullptr) {
    const int ty = L.sweep_ty[sizeof(T) == 8 ? 0 : 1];
    const bool fin = &L == &X->lv[0];
    if (L.cross) {
      if (fin) fused_p<T, true, true>(L, u, r, out, bterm, ty, e, C);
      else fused_p<T, true, false>(L, u, r, out, bterm, ty, e, C);
    } else {
      if (fin) fused_p<T, false, true>(L, u, r, out, bterm, ty, e, C);
      else fused_p<T, false, false>(L, u, r, out, bterm, ty, e, C);
    }
  }

  template <typename T>
  void smo2(DevLevel& L, T* u, const T* r, const double* bterm) {
    if (rows(L).smo2.ns == 0) return;
    for (int it = 0; it < X->opt.smo2_iters; ++it) smo2_pass<T>(L, u, r, bterm);
  }

  // copy of the block rows' values, from an iterate (start of a solve)
  template <typename T>
  void gather_rows(DevLevel& L, const T* u) {
    Smo2Data& S = rows(L).smo2;
    S.cur = 0;
    if (S.ns > 0)
      hipLaunchKernelGGL((k_gather_rows<T>), dim3((S.ns + 255) / 256, nrhs), dim3(256), 0, s, u, S.scell,
                         S.cbuf[0], S.ns, L.n);
  }

  // a recorded cycle must leave the current copy where it found it
  void settle_rows(DevLevel& L) {
    Smo2Data& S = rows(L).smo2;
    if (S.cur != 0 && S.ns > 0) {
      HIP_OK(hipMemcpyAsync(S.cbuf[0], S.cbuf[1], sizeof(double) * S.ns * nrhs, hipMemcpyDeviceToDevice, s));
      S.cur = 0;
    }
  }

  bool fused(DevLevel& L) const { return X->opt.smoother_fused && rows(L).smo2.ns > 0; }

  // smooth nsteps times; returns pointer to the buffer holding the result.
  // Fused mode: e (if given) is the pending coarse-grid correction from
  // level C, applied by the first step.
  template <typename T>
  T* smooth(DevLevel& L, T* cur, T* other, const T* r, const double* bterm, int nsteps, const T* e = nullptr,
            const DevLevel* C = nullptr) {
    if (fused(L)) {
      for (int k = 0; k < nsteps; ++k) {
        fused_step<T>(L, cur, r, other, bterm, k == 0 ? e : nullptr, C);
        std::swap(cur, other);
      }
      return cur;
    }
    for (int k = 0; k < nsteps; ++k) {
      sweep<T>(L, cur, r, other);
      std::swap(cur, other);
      if (X->opt.smo2_every_sweep || k == nsteps - 1) smo2<T>(L, cur, r, bterm);
    }
    return cur;
  }

  template <typename T>
  void fill(T* p, size_t n, T v) {
    hipLaunchKernelGGL((k_fill<T>), dim3(std::min<size_t>(4096, (n + 255) / 256)), dim3(256), 0, s, p, n, v);
  }

  template <typename T>
  void coarse(DevLevel& L, T* u, const T* r) {
    const double* inv = adjoint ? X->mtinv : X->minv;
    const int nm = X->nm;
    hipLaunchKernelGGL((k_coarse<T>), dim3((nm + 3) / 4, nrhs), dim3(BLOCK), nm * sizeof(double), s, u, r,
                       X->mcell, inv, nm, L.n);
  }

  // Alg. 2 on level m with iterate in (u, spare v) and rhs r.
  template <typename T>
  T* vcycle(int m, T* u, T* v, const T* r, const double* bterm) {
    DevLevel& L = X->lv[m];
    if (m == X->M) {
      coarse<T>(L, u, r);
      return u;
    }
    T* cur = smooth<T>(L, u, v, r, bterm, X->opt.nu1);
    T* oth = cur == u ? v : u;
    DevLevel& C = X->lv[m + 1];
    Buf<T> cb = bufs<T>(C);
    restrict_<T>(L, C, cur, r, cb.r, cb.u);
    T* e = vcycle<T>(m + 1, cb.u, cb.v, cb.r, nullptr);
    T* out;
    if (fused(L) && X->opt.prolongation == 0 && X->opt.nu2 > 0) {
      out = smooth<T>(L, cur, oth, r, bterm, X->opt.nu2, e, &C);   // correction applied by the first step
    } else {
      prolong<T>(L, C, cur, e);
      out = smooth<T>(L, cur, oth, r, bterm, X->opt.nu2);
    }
    settle_rows(L);
    return out;
  }

  // partial maxima over non-empty cells of |r - bterm - A u| (zero_u: of
  // |r - bterm|), one launch, into L.part[z * norm_parts(L) + b]
  int norm_parts(DevLevel& L) {
    return tiles_x(L.nx) * ((L.ny + TY - 1) / TY) + (rows(L).n + BLOCK - 1) / BLOCK;
  }

  template <typename T>
  void resmax(DevLevel& L, const T* u, const T* r, const double* bterm, int zero_u, float* res_out) {
    const int nbx = tiles_x(L.nx);
    const int ntiles = nbx * ((L.ny + TY - 1) / TY);
    DevRows& R = rows(L);
    const int nrb = (R.n + BLOCK - 1) / BLOCK;
    const dim3 g(ntiles + nrb, 1, nrhs);
    CoefT<T> c(L.coef);
    const uint8_t rb = regbit();
    if (L.cross)
      hipLaunchKernelGGL((k_resnorm<T, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, L.nx, L.ny, nbx, ntiles, c, zero_u,
                         rb, bterm, R.cell, R.rp, R.cols, R.vals, R.rowsum, R.n, res_out, L.part);
    else
      hipLaunchKernelGGL((k_resnorm<T, false>), g, dim3(BLOCK), 0, s, u, r, L.kind, L.nx, L.ny, nbx, ntiles, c,
                         zero_u, rb, bterm, R.cell, R.rp, R.cols, R.vals, R.rowsum, R.n, res_out, L.part);
  }
};

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// Device data
// ---------------------------------------------------------------------------
constexpr long MAX_COARSE_UNKNOWNS = 8000;   // gathered rhs must fit in LDS

void upload_level(ccgmg_ctx* X, int m, int maxr) {
  ccg::Discretization& D = X->H.disc[m];
  DevLevel& L = X->lv[m];
  L.nx = D.nx, L.ny = D.ny, L.n = (size_t)D.nx * D.ny, L.h = D.h;
  const double h2 = D.h * D.h;
  L.coef.ax1 = 16.0 * X->a / (12.0 * h2);
  L.coef.ax2 = -1.0 * X->a / (12.0 * h2);
  L.coef.cy1 = 16.0 * X->c / (12.0 * h2);
  L.coef.cy2 = -1.0 * X->c / (12.0 * h2);
  L.coef.bxy = X->b / (144.0 * h2);
  L.coef.omega_invD = X->opt.omega / (-30.0 * (X->a + X->c) / (12.0 * h2));
  L.cross = X->b != 0.0;
  ccg::RowSet F, T, SF, ST;
  std::vector<uint8_t> treg, jf, jt;
  std::vector<int32_t> btf, btt;
  ccg::forward_rows(D, F);
  ccg::transposed_rows(D, T, treg);
  ccg::smoother_rows(D, F, D.regular, X->opt.smo2_widen, SF, btf, jf);
  ccg::smoother_rows(D, T, treg, X->opt.smo2_widen, ST, btt, jt);
  for (int32_t& v : btt) v = -1;   // the adjoint has no boundary term
  std::vector<uint8_t> kind(L.n);
  for (size_t k = 0; k < L.n; ++k)
    kind[k] = (D.regular[k] ? F_REG : 0) | (D.nonempty[k] ? F_NONEMPTY : 0) | (treg[k] ? F_REG_T : 0) |
              (jf[k] ? F_JAC : 0) | (jt[k] ? F_JAC_T : 0);
  for (int32_t q : SF.cell) kind[q] |= F_S2;
  for (int32_t q : ST.cell) kind[q] |= F_S2_T;
  L.kind = upload(kind, X->owned);
  // coarse parent of every cell that takes the piecewise-constant correction
  // (regular rows of L, resp. of L^T); -1 elsewhere and on the coarsest level
  std::vector<int32_t> parf(L.n, -1), part(L.n, -1);
  if (m + 1 < (int)X->H.disc.size()) {
    const int ncx = X->H.disc[m + 1].nx, ncy = X->H.disc[m + 1].ny;
    for (int j = 0; j < L.ny; ++j)
      for (int i = 0; i < L.nx; ++i) {
        const size_t q = (size_t)j * L.nx + i;
        if ((i >> 1) >= ncx || (j >> 1) >= ncy) continue;
        const int32_t pc = (int32_t)((j >> 1) * ncx + (i >> 1));
        if (kind[q] & F_REG) parf[q] = pc;
        if (kind[q] & F_REG_T) part[q] = pc;
      }
  }
  upload_rows(F, SF, btf, parf, L.n, X->opt, L.fwd, X->owned);
  upload_rows(T, ST, btt, part, L.n, X->opt, L.adj, X->owned);
  L.u = dalloc<double>(L.n * maxr, X->owned);
  L.r = dalloc<double>(L.n * maxr, X->owned);
  L.v = dalloc<double>(L.n * maxr, X->owned);
  L.u32 = dalloc<float>(L.n * maxr, X->owned);
  L.v32 = dalloc<float>(L.n * maxr, X->owned);
  L.r32 = dalloc<float>(L.n * maxr, X->owned);
  for (DevRows* R : {&L.fwd, &L.adj})
    for (int k = 0; k < 2; ++k) R->smo2.cbuf[k] = dalloc<double>((size_t)std::max(1, R->smo2.ns) * maxr, X->owned);
  const int nrows = std::max(1, std::max(std::max(L.fwd.n, L.adj.n), std::max(L.fwd.smo2.ns, L.adj.smo2.ns)));
  L.du = dalloc<double>((size_t)nrows * maxr, X->owned);
  L.npart_reg = (int)(((L.nx + TX - 1) / TX) * ((L.ny + TY - 1) / TY));
  L.npart_irr = std::max(1, (nrows + BLOCK - 1) / BLOCK);
  L.part = dalloc<double>((size_t)(L.npart_reg + L.npart_irr) * maxr, X->owned);
}

void upload_coarsest(ccgmg_ctx* X) {
  auto hit = X->coarse_cache.find(X->M);
  if (hit != X->coarse_cache.end()) {
    X->nm = hit->second.nm, X->mcell = hit->second.cell, X->minv = hit->second.inv, X->mtinv = hit->second.tinv;
    return;
  }
  ccg::Discretization& D = X->H.disc[X->M];
  std::vector<int32_t> cells;
  std::vector<int32_t> pos(D.nonempty.size(), -1);
  for (size_t k = 0; k < D.nonempty.size(); ++k)
    if (D.nonempty[k]) pos[k] = (int32_t)cells.size(), cells.push_back((int32_t)k);
  const int n = (int)cells.size();
  if (n > MAX_COARSE_UNKNOWNS) throw ccg::Error(CCGMG_EINVAL, "coarsest level has too many unknowns");
  std::vector<double> A((size_t)n * n, 0.0);
  for (int r = 0; r < n; ++r) {
    int q = cells[r];
    if (D.regular[q]) {
      int i = q % D.nx, j = q / D.nx;
      for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
          double w = D.coef[dy + 2][dx + 2];
          if (w != 0.0) A[(size_t)r * n + pos[(j + dy) * D.nx + i + dx]] += w;
        }
    } else {
      int k = D.irr_pos[q];
      for (int t = 0; t < 15; ++t) A[(size_t)r * n + pos[D.sten[15 * k + t]]] += D.wts[15 * k + t];
    }
  }
  std::vector<double> AT((size_t)n * n);
  for (int r = 0; r < n; ++r)
    for (int cc = 0; cc < n; ++cc) AT[(size_t)cc * n + r] = A[(size_t)r * n + cc];
  if (!ccg::dense_inverse(A, n, X->opt.num_threads)) throw ccg::Error(CCGMG_ESINGULAR, "singular coarsest operator");
  if (!ccg::dense_inverse(AT, n, X->opt.num_threads)) throw ccg::Error(CCGMG_ESINGULAR, "singular coarsest operator");
  X->nm = n;
  X->mcell = upload(cells, X->owned);
  X->minv = upload(A, X->owned);
  X->mtinv = upload(AT, X->owned);
  X->coarse_cache[X->M] = {n, X->mcell, X->minv, X->mtinv};
}

// Tile-height autotuning of the SMO-1 sweep: on every level and in both
// precisions, time each admissible tile height (HIP events, private stream,
// work buffers of that level) and keep the fastest.
void tune_tiles(ccgmg_ctx* X) {
  static const int cand[] = {8, 16, 32};
  Driver Dr{X, X->ws, 1, false};
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  const int reps = 10;
  for (DevLevel& L : X->lv) {
    Dr.fill<double>(L.u, L.n, 1.0);
    Dr.fill<double>(L.r, L.n, 0.5);
    Dr.fill<float>(L.u32, L.n, 1.0f);
    Dr.fill<float>(L.r32, L.n, 0.5f);
    for (int prec = 0; prec < 2; ++prec) {
      float best = 1e30f;
      for (int ty : cand) {
        auto launch = [&]() {
          if (prec == 0) Dr.sweep<double>(L, L.u, L.r, L.v, ty);
          else Dr.sweep<float>(L, L.u32, L.r32, L.v32, ty);
        };
        launch();
        launch();
        HIP_OK(hipEventRecord(e0, X->ws));
        for (int k = 0; k < reps; ++k) launch();
        HIP_OK(hipEventRecord(e1, X->ws));
        HIP_OK(hipEventSynchronize(e1));
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) best = ms, L.sweep_ty[prec] = ty;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

int guard(ccgmg_ctx* X, const std::function<void()>& body) {
  if (!X) return CCGMG_EINVAL;
  try {
    if (X->host_only) throw ccg::Error(CCGMG_EINVAL, "context was created with host_only");
    body();
  } catch (const ccg::Error& e) {
    X->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    X->err = e.what();
    return CCGMG_EINVAL;
  }
  return CCGMG_OK;
}

// One FP64 V-cycle on level 0 (u = caller's iterate, v = spare buffer).
void fp64_cycle(Driver& Dr, double* u, const double* f, const double* bterm) {
  DevLevel& L0 = Dr.X->lv[0];
  double* res = Dr.vcycle<double>(0, u, L0.v, f, bterm);
  if (res != u) HIP_OK(hipMemcpyAsync(u, res, sizeof(double) * L0.n * Dr.nrhs, hipMemcpyDeviceToDevice, Dr.s));
}

// One refinement step of the mixed-precision solve: r32 = f - N g - A u
// (FP64, difference form) stored as FP32, one FP32 V-cycle on A e = r32 with
// zero guess (explicit rows and coarsest solve in FP64 arithmetic), u += e.
void mp_cycle(Driver& Dr, double* u, const double* f, const double* bterm) {
  ccgmg_ctx* X = Dr.X;
  DevLevel& L0 = X->lv[0];
  const int nr = Dr.nrhs;
  CoefT<double> c(L0.coef);
  const uint8_t rb = Dr.regbit();
  if (L0.cross)
    hipLaunchKernelGGL((k_residual_f32<true>), tiles1d(L0.nx, L0.ny, nr), dim3(BLOCK), 0, Dr.s, u, f, L0.kind, L0.r32, L0.nx, L0.ny, tiles_x(L0.nx), c, rb);
  else
    hipLaunchKernelGGL((k_residual_f32<false>), tiles1d(L0.nx, L0.ny, nr), dim3(BLOCK), 0, Dr.s, u, f, L0.kind, L0.r32, L0.nx, L0.ny, tiles_x(L0.nx), c, rb);
  Dr.resmax<double>(L0, u, f, bterm, 0, L0.r32);
  Dr.fill<float>(L0.u32, L0.n * nr, 0.0f);
  Dr.gather_rows<float>(L0, L0.u32);
  float* e = Dr.vcycle<float>(0, L0.u32, L0.v32, L0.r32, nullptr);
  const size_t n = L0.n * nr;
  hipLaunchKernelGGL(k_axpy_f32, dim3(std::min<size_t>(4096, (n + 255) / 256)), dim3(256), 0, Dr.s, u, e, L0.kind, L0.n, n);
}

int solve_impl(ccgmg_ctx* X, const double* f, double* u, int nrhs, ccgmg_report* rep, bool adjoint) {
  return guard(X, [&]() {
    if (!f || !u || nrhs < 1 || nrhs > X->opt.max_nrhs) throw ccg::Error(CCGMG_EINVAL, "bad solve arguments");
    hipStream_t ws = X->ws;
    Driver Dr{X, ws, nrhs, adjoint};
    DevLevel& L0 = X->lv[0];
    const size_t n = L0.n * nrhs;
    HIP_OK(hipEventRecord(X->ev_in, X->stream));
    HIP_OK(hipStreamWaitEvent(ws, X->ev_in, 0));
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    HIP_OK(hipEventRecord(e0, ws));
    const double* bterm = nullptr;
    if (!adjoint && X->nfaces > 0 && X->g_nrhs >= nrhs && L0.fwd.n > 0) {
      hipLaunchKernelGGL(k_bterm, dim3((L0.fwd.n + 255) / 256, nrhs), dim3(256), 0, ws, X->g, X->fptr, X->fface,
                         X->fval, X->bterm, L0.fwd.n, X->nfaces);
      bterm = X->bterm;
    }
    if (!X->opt.use_initial_guess) Dr.fill<double>(u, n, 0.0);
    hipLaunchKernelGGL(k_mask_empty, dim3(std::min<size_t>(4096, (n + 255) / 256)), dim3(256), 0, ws, u, L0.kind, L0.n, n);
    if (X->opt.precision != 1) Dr.gather_rows<double>(L0, u);
    // residual norms: per-workgroup partial maxima read back and reduced here
    const int nparts = Dr.norm_parts(L0);
    const size_t part_bytes = sizeof(double) * nparts * nrhs;
    auto norm_of = [&](int z) {
      double m = 0.0;
      for (int k = 0; k < nparts; ++k) m = std::max(m, X->norm_host[(size_t)z * nparts + k]);
      return m;
    };
    Dr.resmax<double>(L0, u, f, bterm, 1, nullptr);
    std::vector<double> rn(nrhs);
    HIP_OK(hipMemcpyAsync(X->norm_host, L0.part, part_bytes, hipMemcpyDeviceToHost, ws));
    HIP_OK(hipStreamSynchronize(ws));
    for (int z = 0; z < nrhs; ++z) {
      const double m = norm_of(z);
      rn[z] = m > 0 ? m : 1.0;
    }
    // one V-cycle (FP64, or FP32 inside one FP64 refinement step), the FP64
    // residual check and its read-back, replayed from a graph when allowed
    auto cycle = [&]() {
      if (X->opt.precision == 1)
        mp_cycle(Dr, u, f, bterm);
      else
        fp64_cycle(Dr, u, f, bterm);
      Dr.resmax<double>(L0, u, f, bterm, 0, nullptr);
      HIP_OK(hipMemcpyAsync(X->norm_host, L0.part, part_bytes, hipMemcpyDeviceToHost, ws));
    };
    hipGraphExec_t exec = nullptr;
    if (X->opt.use_graph) {
      for (auto& g : X->graphs)
        if (g.u == u && g.f == f && g.bterm == bterm && g.nrhs == nrhs && g.precision == X->opt.precision &&
            g.M == X->M && g.adjoint == adjoint)
          exec = g.exec;
      if (!exec) {
        hipGraph_t graph;
        HIP_OK(hipStreamBeginCapture(ws, hipStreamCaptureModeThreadLocal));
        cycle();
        HIP_OK(hipStreamEndCapture(ws, &graph));
        HIP_OK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        (void)hipGraphDestroy(graph);
        if (X->graphs.size() >= 8) {
          (void)hipGraphExecDestroy(X->graphs.front().exec);
          X->graphs.erase(X->graphs.begin());
        }
        X->graphs.push_back({u, f, bterm, nrhs, X->opt.precision, X->M, adjoint, exec});
      }
    }
    int cycles = 0, hist = 0, slow = 0;
    double prev = 1e300, rel = 1.0;
    if (rep) std::memset(rep, 0, sizeof(*rep));
    bool converged = false;
    for (int it = 0; it < X->opt.max_cycles; ++it) {
      if (exec)
        HIP_OK(hipGraphLaunch(exec, ws));
      else
        cycle();
      ++cycles;
      HIP_OK(hipStreamSynchronize(ws));
      rel = 0;
      for (int z = 0; z < nrhs; ++z) rel = std::max(rel, norm_of(z) / rn[z]);
      if (rep && hist < 64) rep->history[hist++] = rel;
      if (!std::isfinite(rel)) break;
      if (rel <= X->opt.tol) {
        converged = true;
        break;
      }
      if (rel > 0.95 * prev) {
        if (++slow >= 3) break;
      } else {
        slow = 0;
      }
      prev = rel;
    }
    HIP_OK(hipEventRecord(e1, ws));
    HIP_OK(hipEventRecord(X->ev_out, ws));
    HIP_OK(hipStreamWaitEvent(X->stream, X->ev_out, 0));
    HIP_OK(hipEventSynchronize(e1));
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rep) {
      rep->cycles = cycles;
      rep->outer_iters = X->opt.precision == 1 ? cycles : 0;
      rep->rel_res_inf = rel;
      rep->seconds = ms * 1e-3;
    }
    if (!converged) throw ccg::Error(CCGMG_ENOCONV, "tolerance not reached");
  });
}

// V-cycles on a seeded random right-hand side with the current depth; the
// geometric-mean contraction of the residual over 6 cycles.
double depth_test_rate(ccgmg_ctx* X, double tol = 0.0, int max_cycles = 6, double* seconds = nullptr,
                       bool keep_graphs = false, double* score = nullptr) {
  DevLevel& L0 = X->lv[0];
  std::vector<double> r(L0.n, 0.0);
  std::mt19937_64 gen(12345);
  std::normal_distribution<double> nd(0.0, 1.0);
  const ccg::Discretization& D = X->H.disc[0];
  for (size_t k = 0; k < L0.n; ++k) r[k] = D.nonempty[k] ? nd(gen) : 0.0;
  double* rd = L0.r;   // level-0 scratch buffers
  double* ud = L0.u;
  HIP_OK(hipMemcpy(rd, r.data(), sizeof(double) * L0.n, hipMemcpyHostToDevice));
  ccgmg_options saved = X->opt;
  X->opt.max_cycles = max_cycles;
  X->opt.tol = tol;
  X->opt.use_initial_guess = 0;
  X->opt.precision = 0;
  X->opt.use_graph = 1;   // timed as the solves will run: graph replays
  int g_saved = X->g_nrhs;
  X->g_nrhs = 0;
  ccgmg_report rep;
  solve_impl(X, rd, ud, 1, &rep, false);
  X->opt = saved;
  X->g_nrhs = g_saved;
  if (!keep_graphs) X->clear_graphs();
  if (seconds) *seconds = rep.seconds;
  double last = rep.cycles > 0 ? rep.history[std::min(rep.cycles, 64) - 1] : 1.0;
  if (score) {
    // estimated time to reduce the residual by 1e10 at the asymptotic rate
    // (geometric mean over the cycles after the first two): time per cycle
    // times cycles needed; less sensitive to whole-cycle rounding than the
    // solve time itself
    const int nc = std::min(rep.cycles, 64);
    double tail = 1.0;
    if (nc >= 4) tail = std::pow(rep.history[nc - 1] / rep.history[1], 1.0 / (nc - 2));
    *score = (tail > 0.0 && tail < 1.0) ? rep.seconds / rep.cycles * std::log(1e-10) / std::log(tail) : 1e300;
  }
  // with a tolerance, a depth whose solve stops short of it (stagnation or
  // the cycle limit) is not admissible
  if (tol > 0.0 && !(rep.rel_res_inf <= tol)) return 1e300;
  return (std::isfinite(last) && rep.cycles > 0) ? std::pow(last, 1.0 / rep.cycles) : 1e300;
}

}  // namespace

// ===========================================================================
// C interface
// ===========================================================================
extern "C" {

void ccgmg_default_options(ccgmg_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->theta = 0.3;
  o->w_min = 0.5;
  o->omega = 0.5;
  o->nu1 = 3;
  o->nu2 = 3;
  o->coarsest_min_n = 16;
  o->max_levels = 16;
  o->auto_depth = 2;
  o->depth_max_rate = 0.5;
  o->precision = 0;
  o->prolongation = 0;
  o->smo2_every_sweep = 1;
  o->smo2_iters = 1;
  o->smo2_block = 64;
  o->smo2_overlap = 1;
  o->smo2_widen = 1;
  o->tol = 1e-10;
  o->max_cycles = 100;
  o->max_nrhs = 1;
  o->use_initial_guess = 0;
  o->num_threads = 0;
  o->use_graph = 1;
  o->tune_tiles = 1;
  o->smoother_fused = 0;
  o->tune_schedule = 1;
  o->host_only = 0;
  o->hip_stream = nullptr;
}

const char* ccgmg_create_error(void) { return g_create_error.c_str(); }

const char* ccgmg_last_error(const ccgmg_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

int ccgmg_create(const ccgmg_grid* grid, const ccgmg_curve* curves, int ncurves, double a, double b, double c,
                 const ccgmg_options* opts, ccgmg_ctx** out) {
  if (!out) return CCGMG_EINVAL;
  *out = nullptr;
  g_create_error.clear();
  std::unique_ptr<ccgmg_ctx> X(new ccgmg_ctx());
  try {
    if (!grid || !curves || ncurves <= 0 || grid->nx <= 0 || grid->ny <= 0 || !(grid->h > 0))
      throw ccg::Error(CCGMG_EINVAL, "invalid grid or curves");
    if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(c))
      throw ccg::Error(CCGMG_EINVAL, "non-finite coefficient");
    if (b * b - 4.0 * a * c >= 0.0) throw ccg::Error(CCGMG_ENOTELLIPTIC, "b^2 - 4ac >= 0");
    if (opts)
      X->opt = *opts;
    else
      ccgmg_default_options(&X->opt);
    if (X->opt.max_nrhs < 1) X->opt.max_nrhs = 1;
    if (X->opt.smo2_block < 1 || X->opt.smo2_block > 64) throw ccg::Error(CCGMG_EINVAL, "smo2_block must be in 1..64");
    if (X->opt.nu1 < 0 || X->opt.nu2 < 0 || X->opt.smo2_iters < 1 || X->opt.smo2_overlap < 0 ||
        X->opt.smo2_widen < 0 || X->opt.smo2_widen > 4)
      throw ccg::Error(CCGMG_EINVAL, "bad smoothing parameters");
    X->a = a, X->b = b, X->c = c;
    X->host_only = X->opt.host_only != 0;
    std::vector<ccg::Curve> cs(ncurves);
    for (int k = 0; k < ncurves; ++k) {
      cs[k].kind = curves[k].kind;
      for (int t = 0; t < 8; ++t) {
        cs[k].p[t] = curves[k].p[t];
        if (!std::isfinite(cs[k].p[t])) throw ccg::Error(CCGMG_EINVAL, "non-finite curve parameter");
      }
      cs[k].inside = curves[k].domain_inside;
      cs[k].bc = curves[k].bc;
      cs[k].index = k;
    }
    double t0 = now();
    ccg::Options so;
    so.theta = X->opt.theta;
    so.w_min = X->opt.w_min;
    so.coarsest_min_n = std::max(2, X->opt.coarsest_min_n);
    so.max_levels = std::max(1, X->opt.max_levels);
    so.threads = X->opt.num_threads;
    X->H.build(cs, grid->nx, grid->ny, grid->x0, grid->y0, grid->h, a, b, c, so);
    for (double v : X->H.disc[0].cond) X->plg_max_cond = std::max(X->plg_max_cond, v);
    X->M = (int)X->H.disc.size() - 1;
    if (!X->host_only) {
      X->stream = (hipStream_t)X->opt.hip_stream;
      HIP_OK(hipStreamCreateWithFlags(&X->ws, hipStreamNonBlocking));
      HIP_OK(hipEventCreateWithFlags(&X->ev_in, hipEventDisableTiming));
      HIP_OK(hipEventCreateWithFlags(&X->ev_out, hipEventDisableTiming));
      const int maxr = X->opt.max_nrhs;
      X->lv.resize(X->H.disc.size());
      for (size_t m = 0; m < X->H.disc.size(); ++m) upload_level(X.get(), (int)m, maxr);
      ccg::Discretization& D0 = X->H.disc[0];
      X->nfaces = (int)D0.faces.size();
      X->fptr = upload(D0.fw_ptr, X->owned);
      X->fface = upload(D0.fw_face, X->owned);
      X->fval = upload(D0.fw_val, X->owned);
      std::vector<int32_t> fc(X->nfaces);
      std::vector<double> fw(X->nfaces, 0.0);
      for (int k = 0; k < X->nfaces; ++k) fc[k] = D0.faces[k].first;
      for (size_t k = 0; k < D0.irr.size(); ++k)
        for (int t = D0.fw_ptr[k]; t < D0.fw_ptr[k + 1]; ++t) fw[D0.fw_face[t]] = D0.fw_val[t];
      X->fcell = upload(fc, X->owned);
      X->fweight = upload(fw, X->owned);
      X->g = dalloc<double>((size_t)std::max(1, X->nfaces) * maxr, X->owned);
      X->bterm = dalloc<double>((size_t)std::max(1, (int)D0.irr.size()) * maxr, X->owned);

      HIP_OK(hipHostMalloc((void**)&X->norm_host,
                           sizeof(double) * (X->lv[0].npart_reg + X->lv[0].npart_irr) * maxr,
                           hipHostMallocDefault));
      // the coarsest level must be small enough for the dense inverse
      while (X->M > 0) {
        long nu = 0;
        for (uint8_t v : X->H.disc[X->M].nonempty) nu += v;
        if (nu <= MAX_COARSE_UNKNOWNS) break;
        throw ccg::Error(CCGMG_EINVAL, "coarsest level has too many unknowns; allow more levels");
      }
      upload_coarsest(X.get());
      if (X->opt.tune_tiles) tune_tiles(X.get());
      if (X->opt.auto_depth == 2 && X->M > 1) {
        // measured: time a full solve (seeded right-hand side, 1e-10) for
        // every admissible coarsest level and, with tune_schedule, every
        // candidate smoothing schedule; among those that converge keep the
        // one with the smallest estimated time to a 1e10 reduction
        struct Sched {
          int fused, nu1, nu2;
        };
        std::vector<Sched> cands;
        if (X->opt.tune_schedule)
          cands = {{0, 3, 3}, {1, 3, 3}, {1, 4, 4}, {1, 5, 5}};
        else
          cands = {{X->opt.smoother_fused, X->opt.nu1, X->opt.nu2}};
        const int Mmax = X->M;
        X->tune_ms.assign(Mmax + 1, -1.0);
        double best = 1e300;
        int bestM = Mmax;
        Sched bestS = cands[0];
        for (const Sched& sc : cands) {
          X->opt.smoother_fused = sc.fused, X->opt.nu1 = sc.nu1, X->opt.nu2 = sc.nu2;
          for (int Mc = Mmax; Mc >= 1; --Mc) {
            long nu = 0;
            for (uint8_t v : X->H.disc[Mc].nonempty) nu += v;
            if (nu > MAX_COARSE_UNKNOWNS) break;
            X->M = Mc;
            upload_coarsest(X.get());
            double sec = 0, score = 0;
            depth_test_rate(X.get(), 1e-10, 60, &sec, true);   // captures the graph
            const double rate = depth_test_rate(X.get(), 1e-10, 60, &sec, false, &score);
            const bool ok = rate <= X->opt.depth_max_rate;
            if (ok && (X->tune_ms[Mc] < 0 || 1e3 * score < X->tune_ms[Mc])) X->tune_ms[Mc] = 1e3 * score;
            if (ok && score < best) best = score, bestM = Mc, bestS = sc;
          }
        }
        X->opt.smoother_fused = bestS.fused, X->opt.nu1 = bestS.nu1, X->opt.nu2 = bestS.nu2;
        X->M = bestM;
        upload_coarsest(X.get());
        X->clear_graphs();
      } else if (X->opt.auto_depth == 1 && X->M > 1) {
        for (;;) {
          const double rate = depth_test_rate(X.get());
          if (rate <= X->opt.depth_max_rate || X->M <= 1) break;
          long next = 0;
          for (uint8_t v : X->H.disc[X->M - 1].nonempty) next += v;
          if (next > MAX_COARSE_UNKNOWNS) break;
          X->M -= 1;
          upload_coarsest(X.get());
        }
        X->clear_graphs();
      }
    }
    X->setup_seconds = now() - t0;
  } catch (const ccg::Error& e) {
    g_create_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_create_error = "out of host memory";
    return CCGMG_ENOMEM;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return CCGMG_EINVAL;
  }
  *out = X.release();
  return CCGMG_OK;
}

int ccgmg_query(const ccgmg_ctx* X, ccgmg_info* info) {
  if (!X || !info) return CCGMG_EINVAL;
  std::memset(info, 0, sizeof(*info));
  const ccg::Discretization& D = X->H.disc[0];
  info->n_cells = (long)D.nx * D.ny;
  long nu = 0;
  for (uint8_t v : D.nonempty) nu += v;
  info->n_unknowns = nu;
  info->n_irregular = (long)D.irr.size();
  info->n_bdry_faces = (long)D.faces.size();
  const int M = X->host_only ? (int)X->H.disc.size() - 1 : X->M;
  info->n_levels = M + 1;
  info->nx_coarsest = X->H.disc[M].nx;
  info->ny_coarsest = X->H.disc[M].ny;
  long cu = 0;
  for (uint8_t v : X->H.disc[M].nonempty) cu += v;
  info->coarse_unknowns = cu;
  info->setup_seconds = X->setup_seconds;
  info->plg_max_cond = X->plg_max_cond;
  info->smoother_fused = X->opt.smoother_fused;
  info->nu1 = X->opt.nu1;
  info->nu2 = X->opt.nu2;
  return CCGMG_OK;
}

int ccgmg_get_level_shape(const ccgmg_ctx* X, int level, int* nx, int* ny) {
  if (!X || level < 0 || level >= (int)X->H.disc.size()) return CCGMG_EINVAL;
  if (nx) *nx = X->H.disc[level].nx;
  if (ny) *ny = X->H.disc[level].ny;
  return CCGMG_OK;
}

int ccgmg_get_cell_kinds(const ccgmg_ctx* X, int level, int8_t* kinds, int32_t* hosts) {
  if (!X || level < 0 || level >= (int)X->H.disc.size()) return CCGMG_EINVAL;
  const ccg::Discretization& D = X->H.disc[level];
  if (kinds) std::memcpy(kinds, D.kind.data(), D.kind.size());
  if (hosts) std::memcpy(hosts, X->H.geo[level].host.data(), sizeof(int32_t) * D.kind.size());
  return CCGMG_OK;
}

int ccgmg_get_volumes(const ccgmg_ctx* X, int level, double* vol) {
  if (!X || !vol || level < 0 || level >= (int)X->H.disc.size()) return CCGMG_EINVAL;
  const auto& v = X->H.geo[level].vol;
  std::memcpy(vol, v.data(), sizeof(double) * v.size());
  return CCGMG_OK;
}

int ccgmg_get_tuning(const ccgmg_ctx* X, int level, int* sweep_ty_fp64, int* sweep_ty_fp32) {
  if (!X || X->host_only || level < 0 || level >= (int)X->lv.size()) return CCGMG_EINVAL;
  if (sweep_ty_fp64) *sweep_ty_fp64 = X->lv[level].sweep_ty[0];
  if (sweep_ty_fp32) *sweep_ty_fp32 = X->lv[level].sweep_ty[1];
  return CCGMG_OK;
}

int ccgmg_get_smo2_stats(const ccgmg_ctx* X, int level, int adjoint, long* stats) {
  if (!X || X->host_only || !stats || level < 0 || level >= (int)X->lv.size()) return CCGMG_EINVAL;
  const Smo2Data& S = adjoint ? X->lv[level].adj.smo2 : X->lv[level].fwd.smo2;
  stats[0] = S.nblk;
  stats[1] = S.ns;
  stats[2] = S.n_ext;
  stats[3] = S.n_ext_nnz;
  stats[4] = (long)S.inv_bytes;
  return CCGMG_OK;
}

int ccgmg_get_counts(const ccgmg_ctx* X, int level, long* n_irregular, long* n_faces) {
  if (!X || level < 0 || level >= (int)X->H.disc.size()) return CCGMG_EINVAL;
  if (n_irregular) *n_irregular = (long)X->H.disc[level].irr.size();
  if (n_faces) *n_faces = (long)X->H.disc[level].faces.size();
  return CCGMG_OK;
}

int ccgmg_get_irregular(const ccgmg_ctx* X, int level, int32_t* rows, int32_t* cols, double* vals, double* cond) {
  if (!X || level < 0 || level >= (int)X->H.disc.size()) return CCGMG_EINVAL;
  const ccg::Discretization& D = X->H.disc[level];
  if (rows) std::memcpy(rows, D.irr.data(), sizeof(int32_t) * D.irr.size());
  if (cols) std::memcpy(cols, D.sten.data(), sizeof(int32_t) * D.sten.size());
  if (vals) std::memcpy(vals, D.wts.data(), sizeof(double) * D.wts.size());
  if (cond) std::memcpy(cond, D.cond.data(), sizeof(double) * D.cond.size());
  return CCGMG_OK;
}

int ccgmg_get_boundary_faces(const ccgmg_ctx* X, int32_t* cell, int32_t* curve, double* nweight) {
  if (!X) return CCGMG_EINVAL;
  const ccg::Discretization& D = X->H.disc[0];
  for (size_t k = 0; k < D.faces.size(); ++k) {
    if (cell) cell[k] = D.faces[k].first;
    if (curve) curve[k] = D.faces[k].second;
  }
  if (nweight)
    for (size_t k = 0; k < D.irr.size(); ++k)
      for (int t = D.fw_ptr[k]; t < D.fw_ptr[k + 1]; ++t) nweight[D.fw_face[t]] = D.fw_val[t];
  return CCGMG_OK;
}

int ccgmg_get_alg3_order(const ccgmg_ctx* X, int level, int32_t* perm) {
  if (!X || !perm || level < 0 || level >= (int)X->H.disc.size()) return CCGMG_EINVAL;
  const auto& o = X->H.disc[level].order;
  std::memcpy(perm, o.data(), sizeof(int32_t) * o.size());
  return CCGMG_OK;
}

int ccgmg_cell_quadrature(const ccgmg_ctx* X, long* count, int32_t* cell_of, double* x, double* y, double* w) {
  if (!X || !count) return CCGMG_EINVAL;
  return ccg::cell_quadrature(X->H.geo[0], count, cell_of, x, y, w) == 0 ? CCGMG_OK : CCGMG_EINVAL;
}

int ccgmg_face_quadrature(const ccgmg_ctx* X, long* count, int32_t* face_of, double* x, double* y, double* w,
                          double* nxo, double* nyo) {
  if (!X || !count) return CCGMG_EINVAL;
  return ccg::face_quadrature(X->H.geo[0], X->H.disc[0], count, face_of, x, y, w, nxo, nyo) == 0 ? CCGMG_OK
                                                                                                  : CCGMG_EINVAL;
}

static int apply_impl(ccgmg_ctx* X, const double* u, double* Lu, bool adjoint) {
  return guard(X, [&]() {
    if (!u || !Lu || u == Lu) throw ccg::Error(CCGMG_EINVAL, "bad apply arguments");
    DevLevel& L = X->lv[0];
    CoefT<double> c(L.coef);
    const uint8_t rb = adjoint ? F_REG_T : F_REG;
    if (L.cross)
      hipLaunchKernelGGL((k_apply<true>), tiles(L.nx, L.ny, 1), dim3(BLOCK), 0, X->stream, u, L.kind, Lu, L.nx, L.ny, c, rb);
    else
      hipLaunchKernelGGL((k_apply<false>), tiles(L.nx, L.ny, 1), dim3(BLOCK), 0, X->stream, u, L.kind, Lu, L.nx, L.ny, c, rb);
    const DevRows& R = adjoint ? L.adj : L.fwd;
    if (R.n > 0)
      hipLaunchKernelGGL(k_rows_apply, dim3((R.n + 255) / 256), dim3(256), 0, X->stream, u, Lu, R.cell, R.rp, R.cols,
                         R.vals, R.n);
    HIP_OK(hipGetLastError());
  });
}

int ccgmg_apply(ccgmg_ctx* X, const double* u, double* Lu) { return apply_impl(X, u, Lu, false); }

int ccgmg_apply_adjoint(ccgmg_ctx* X, const double* lam, double* out) { return apply_impl(X, lam, out, true); }

int ccgmg_set_boundary(ccgmg_ctx* X, const double* g, int nrhs) {
  return guard(X, [&]() {
    if (nrhs < 0 || nrhs > X->opt.max_nrhs) throw ccg::Error(CCGMG_EINVAL, "bad nrhs");
    if (X->nfaces > 0 && nrhs > 0) {
      if (!g) throw ccg::Error(CCGMG_EINVAL, "null boundary data");
      HIP_OK(hipMemcpyAsync(X->g, g, sizeof(double) * X->nfaces * nrhs, hipMemcpyDeviceToDevice, X->stream));
    }
    X->g_nrhs = nrhs;
  });
}

int ccgmg_solve(ccgmg_ctx* X, const double* f, double* u, int nrhs, ccgmg_report* rep) {
  return solve_impl(X, f, u, nrhs, rep, false);
}

int ccgmg_solve_adjoint(ccgmg_ctx* X, const double* rhs, double* lam, int nrhs, ccgmg_report* rep) {
  return solve_impl(X, rhs, lam, nrhs, rep, true);
}

int ccgmg_apply_NT(ccgmg_ctx* X, const double* lam, double* out, int nrhs) {
  return guard(X, [&]() {
    if (!lam || !out || nrhs < 1) throw ccg::Error(CCGMG_EINVAL, "bad arguments");
    if (X->nfaces > 0)
      hipLaunchKernelGGL(k_apply_NT, dim3((X->nfaces + 255) / 256, nrhs), dim3(256), 0, X->stream, lam, X->fcell,
                         X->fweight, out, X->nfaces, X->lv[0].n);
  });
}

int ccgmg_profile_kernel(ccgmg_ctx* X, int kernel, int level, int reps, double* avg_us) {
  return guard(X, [&]() {
    if (!avg_us || reps < 1 || level < 0 || level > X->M || kernel < 0 || kernel > 7)
      throw ccg::Error(CCGMG_EINVAL, "bad profile arguments");
    Driver Dr{X, X->stream, 1, false};
    DevLevel& L = X->lv[level];
    Dr.fill<double>(L.u, L.n, 1.0);
    Dr.fill<double>(L.r, L.n, 0.5);
    Dr.fill<double>(L.v, L.n, 0.0);
    Dr.fill<float>(L.u32, L.n, 1.0f);
    Dr.fill<float>(L.r32, L.n, 0.5f);
    DevLevel* C = level < X->M ? &X->lv[level + 1] : nullptr;
    if ((kernel == 1 || kernel == 2) && !C) throw ccg::Error(CCGMG_EINVAL, "no coarser level");
    if (kernel == 4 && level != X->M) throw ccg::Error(CCGMG_EINVAL, "coarsest solve only on the coarsest level");
    auto launch = [&]() {
      switch (kernel) {
        case 0: Dr.sweep<double>(L, L.u, L.r, L.v); break;
        case 1: Dr.restrict_<double>(L, *C, L.u, L.r, C->r, C->u); break;
        case 2: Dr.prolong<double>(L, *C, L.u, C->u); break;
        case 3:
          if (L.fwd.smo2.ns > 0) Dr.smo2_pass<double>(L, L.u, L.r, nullptr);
          Dr.settle_rows(L);
          break;
        case 4: Dr.coarse<double>(L, L.u, L.r); break;
        case 7:
          Dr.fused_step<double>(L, L.u, L.r, L.v, nullptr);
          Dr.settle_rows(L);
          break;
        case 6:
          hipLaunchKernelGGL(k_copy, dim3(std::min<size_t>(8192, (L.n + 255) / 256)), dim3(256), 0, X->stream, L.v,
                             L.u, L.n);
          break;
        default: Dr.sweep<float>(L, L.u32, L.r32, L.v32); break;
      }
    };
    launch();
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    HIP_OK(hipEventRecord(e0, X->stream));
    for (int k = 0; k < reps; ++k) launch();
    HIP_OK(hipEventRecord(e1, X->stream));
    HIP_OK(hipEventSynchronize(e1));
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_us = 1e3 * ms / reps;
  });
}

void ccgmg_destroy(ccgmg_ctx* X) {
  if (!X) return;
  if (!X->host_only) {
    if (X->stream) (void)hipStreamSynchronize(X->stream);
    if (X->ws) (void)hipStreamSynchronize(X->ws);
    X->clear_graphs();
    if (X->ws) (void)hipStreamDestroy(X->ws);
    if (X->ev_in) (void)hipEventDestroy(X->ev_in);
    if (X->ev_out) (void)hipEventDestroy(X->ev_out);
    for (void* p : X->owned) (void)hipFree(p);
    if (X->norm_host) (void)hipHostFree(X->norm_host);
  }
  delete X;
}

}  // extern "C"
