// MI355X cut-cell multigrid: device kernels, V-cycle driver and the C
// interface declared in ccgmg.h.
//
// The V-cycle is Alg. 2: on each level nu1 smoothing steps, residual and
// restriction, recursion with a zero guess, prolongation and correction,
// nu2 smoothing steps; the coarsest level is solved exactly.  A smoothing
// step is SMO-1 (omega-weighted Jacobi on the regular cells, Section 4.1)
// followed by SMO-2 (the block update of the irregular cells, eq.
// updateByBlock).  SMO-2 is carried out here by restricted additive Schwarz
// over consecutive runs of the Alg. 3 numbering with precomputed FP64 block
// inverses, instead of the paper's banded LU of the whole block: a banded
// triangular solve is a chain of dependent steps, while the blocks are
// independent and map onto one workgroup each.  The converged solution does
// not depend on the smoother.
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

// ===========================================================================
// Kernels
// ===========================================================================

// SMO-1: u_out = u + omega/D (r - L u) on regular cells, u_out = u elsewhere
// (Jacobi: reads u, writes a second buffer).
// FINEST only selects a separate instantiation for the finest level so that
// kernel traces separate it from the coarse levels; the code is the same.
template <typename T, bool CROSS, bool FINEST>
__global__ __launch_bounds__(BLOCK) void k_sweep(const T* __restrict__ u, const T* __restrict__ r,
                                                 const uint8_t* __restrict__ kind, T* __restrict__ out, int nx,
                                                 int ny, CoefT<T> c) {
  __shared__ T tile[LH][LW];
  const size_t zoff = (size_t)blockIdx.z * nx * ny;
  u += zoff, r += zoff, out += zoff;
  const int bx = blockIdx.x * TX, by = blockIdx.y * TY;
  const int tx = threadIdx.x & (TX - 1), w = threadIdx.x >> 6;
  // issue the kind and right-hand-side loads before the tile barrier
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
    const int ry = w + 4 * k;
    const int gx = bx + tx, gy = by + ry;
    if (gx < nx && gy < ny) {
      T v = tile[ry + HALO][tx + HALO];
      if (kd[k] & 1) v += c.omega_invD * (rr[k] - apply_regular<T, CROSS>(tile, ry + HALO, tx + HALO, c));
      out[(size_t)gy * nx + gx] = v;
    }
  }
}

// Residual of the regular cells restricted to the coarse grid:
// rc_I = 1/4 sum over regular children c of (r - L u)_c  (Section 4.1).
template <typename T, typename TC, bool CROSS, bool FINEST>
__global__ __launch_bounds__(BLOCK) void k_restrict(const T* __restrict__ u, const T* __restrict__ r,
                                                    const uint8_t* __restrict__ kind, TC* __restrict__ rc, int nx,
                                                    int ny, int ncx, int ncy, CoefT<T> c) {
  __shared__ T tile[LH][LW];
  const size_t zoff = (size_t)blockIdx.z * nx * ny;
  u += zoff, r += zoff;
  rc += (size_t)blockIdx.z * ncx * ncy;
  const int bx = blockIdx.x * TX, by = blockIdx.y * TY;
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
  const int I = blockIdx.x * (TX / 2) + cx, J = blockIdx.y * (TY / 2) + cy;
  if (I >= ncx || J >= ncy) return;
  T s = (T)0;
#pragma unroll
  for (int d = 0; d < 4; ++d)
    if (kd[d] & 1)
      s += rr[d] - apply_regular<T, CROSS>(tile, 2 * cy + (d >> 1) + HALO, 2 * cx + (d & 1) + HALO, c);
  rc[(size_t)J * ncx + I] = (TC)((T)0.25 * s);
}

// Correction u_c += P e on regular fine cells: piecewise constant
// (Section 4.1) or bilinear with the 9/16, 3/16, 3/16, 1/16 cell-centred
// weights where all four coarse cells are non-empty.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_prolong(T* __restrict__ u, const T* __restrict__ e,
                                                   const uint8_t* __restrict__ kind,
                                                   const uint8_t* __restrict__ ckind, int nx, int ny, int ncx,
                                                   int ncy, int bilinear) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= nx) return;
  const size_t g = (size_t)j * nx + i;
  if (!(kind[g] & 1)) return;
  u += (size_t)blockIdx.z * nx * ny;
  e += (size_t)blockIdx.z * ncx * ncy;
  const int I = i >> 1, J = j >> 1;
  T v = e[(size_t)J * ncx + I];
  if (bilinear) {
    const int I2 = I + ((i & 1) ? 1 : -1), J2 = J + ((j & 1) ? 1 : -1);
    if (I2 >= 0 && I2 < ncx && J2 >= 0 && J2 < ncy && (ckind[(size_t)J * ncx + I2] & 2) &&
        (ckind[(size_t)J2 * ncx + I] & 2) && (ckind[(size_t)J2 * ncx + I2] & 2))
      v = ((T)9 * v + (T)3 * e[(size_t)J * ncx + I2] + (T)3 * e[(size_t)J2 * ncx + I] + e[(size_t)J2 * ncx + I2]) *
          (T)0.0625;
  }
  u[g] += v;
}

// SMO-2 by restricted additive Schwarz.  Workgroup = one block of <= 64
// consecutive irregular cells (Alg. 3 numbering) plus its overlap.  The
// rows of the overlapped set are stored per block (cell, 15 columns, 15
// weights, row sum), so a residual needs one level of gathers:
//   res_t = r_q - bterm - sum_s beta_ts (u_s - u_q) - S_t u_q   (FP64),
// then the block's own rows of the precomputed inverse are applied,
// du_own = (A_ext^{-1})_{own,:} res_ext; du is added by k_add_du.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_smo2(const T* __restrict__ u, const T* __restrict__ r,
                                                const double* __restrict__ bterm, const int32_t* __restrict__ ecell,
                                                const int32_t* __restrict__ ecols, const double* __restrict__ evals,
                                                const double* __restrict__ ersum, const int32_t* __restrict__ eirr,
                                                const int32_t* __restrict__ ext_ptr,
                                                const int32_t* __restrict__ own_cnt,
                                                const int64_t* __restrict__ inv_off,
                                                const double* __restrict__ inv, double* __restrict__ du, int nirr,
                                                size_t plane) {
  __shared__ double res[1024];
  __shared__ double part[4][64];
  const int b = blockIdx.x, z = blockIdx.y;
  u += (size_t)z * plane, r += (size_t)z * plane;
  const int e0 = ext_ptr[b], ne = ext_ptr[b + 1] - e0, nown = own_cnt[b];
  for (int t = threadIdx.x; t < ne; t += BLOCK) {
    const size_t e = (size_t)(e0 + t);
    const int q = ecell[e];
    int cl[15];
#pragma unroll
    for (int s = 0; s < 15; ++s) cl[s] = ecols[e * 15 + s];
    const double uq = (double)u[q];
    double rhs = (double)r[q];
    if (bterm) rhs -= bterm[(size_t)z * nirr + eirr[e]];
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < 15; ++s) acc += evals[e * 15 + s] * ((double)u[cl[s]] - uq);
    res[t] = rhs - acc - ersum[e] * uq;
  }
  __syncthreads();
  const int row = threadIdx.x & 63, grp = threadIdx.x >> 6;
  double s0 = 0.0, s1 = 0.0;
  if (row < nown) {
    const double* A = inv + inv_off[b] + row;
    int col = grp;
    for (; col + 4 < ne; col += 8) {
      s0 += A[(size_t)col * nown] * res[col];
      s1 += A[(size_t)(col + 4) * nown] * res[col + 4];
    }
    if (col < ne) s0 += A[(size_t)col * nown] * res[col];
  }
  part[grp][row] = s0 + s1;
  __syncthreads();
  if (grp == 0 && row < nown)
    du[(size_t)z * nirr + eirr[e0 + row]] = part[0][row] + part[1][row] + part[2][row] + part[3][row];
}

template <typename T>
__global__ void k_add_du(T* __restrict__ u, const double* __restrict__ du, const int32_t* __restrict__ cell,
                         int nirr, size_t plane) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nirr) return;
  const int z = blockIdx.y;
  u[(size_t)z * plane + cell[k]] += (T)du[(size_t)z * nirr + k];
}

// (L u) for the irregular rows (plain sum, used by ccgmg_apply).
__global__ void k_irr_apply(const double* __restrict__ u, double* __restrict__ Lu, const int32_t* __restrict__ cell,
                            const int32_t* __restrict__ cols, const double* __restrict__ vals, int nirr) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nirr) return;
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < 15; ++s) acc += vals[15 * k + s] * u[cols[15 * k + s]];
  Lu[cell[k]] = acc;
}

// (L u) on regular cells; zero on empty and irregular cells.
template <bool CROSS>
__global__ __launch_bounds__(BLOCK) void k_apply(const double* __restrict__ u, const uint8_t* __restrict__ kind,
                                                 double* __restrict__ Lu, int nx, int ny, CoefT<double> c) {
  __shared__ double tile[LH][LW];
  const int bx = blockIdx.x * TX, by = blockIdx.y * TY;
  load_tile(tile, u, nx, ny, bx, by);
  __syncthreads();
  const int tx = threadIdx.x & (TX - 1), w = threadIdx.x >> 6;
  for (int k = 0; k < TY / 4; ++k) {
    const int ry = w + 4 * k, gx = bx + tx, gy = by + ry;
    if (gx < nx && gy < ny) {
      const size_t g = (size_t)gy * nx + gx;
      Lu[g] = (kind[g] & 1) ? apply_regular<double, CROSS>(tile, ry + HALO, tx + HALO, c) : 0.0;
    }
  }
}

// Block-wise max of |r - L u| over regular cells (difference form) or of |r|
// when zero_u is set; one partial per workgroup.
template <typename T, bool CROSS>
__global__ __launch_bounds__(BLOCK) void k_resmax_reg(const T* __restrict__ u, const T* __restrict__ r,
                                                      const uint8_t* __restrict__ kind, double* __restrict__ partial,
                                                      int nx, int ny, CoefT<T> c, int zero_u) {
  __shared__ T tile[LH][LW];
  __shared__ double red[BLOCK];
  const size_t zoff = (size_t)blockIdx.z * nx * ny;
  u += zoff, r += zoff;
  const int bx = blockIdx.x * TX, by = blockIdx.y * TY;
  load_tile(tile, u, nx, ny, bx, by);
  __syncthreads();
  const int tx = threadIdx.x & (TX - 1), w = threadIdx.x >> 6;
  double m = 0.0;
  for (int k = 0; k < TY / 4; ++k) {
    const int ry = w + 4 * k, gx = bx + tx, gy = by + ry;
    if (gx < nx && gy < ny) {
      const size_t g = (size_t)gy * nx + gx;
      if (kind[g] & 1) {
        T v = r[g];
        if (!zero_u) v -= apply_regular<T, CROSS>(tile, ry + HALO, tx + HALO, c);
        m = fmax(m, fabs((double)v));
      }
    }
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0)
    partial[(size_t)blockIdx.z * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// Same for the irregular rows (FP64), optionally writing the residual into
// a grid array (used by the refinement loop).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_resmax_irr(const T* __restrict__ u, const T* __restrict__ r,
                                                      const double* __restrict__ bterm,
                                                      const int32_t* __restrict__ cell,
                                                      const int32_t* __restrict__ cols,
                                                      const double* __restrict__ vals,
                                                      const double* __restrict__ rowsum, double* __restrict__ partial,
                                                      int nirr, size_t plane, int zero_u, float* __restrict__ res_out) {
  __shared__ double red[BLOCK];
  const int z = blockIdx.y;
  u += (size_t)z * plane, r += (size_t)z * plane;
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  double m = 0.0;
  if (k < nirr) {
    const int q = cell[k];
    double rhs = (double)r[q];
    if (bterm) rhs -= bterm[(size_t)z * nirr + k];
    if (!zero_u) {
      const double uq = (double)u[q];
      double acc = 0.0;
#pragma unroll
      for (int s = 0; s < 15; ++s) acc += vals[15 * k + s] * ((double)u[cols[15 * k + s]] - uq);
      rhs -= acc + rowsum[k] * uq;
    }
    if (res_out) res_out[(size_t)z * plane + q] = (float)rhs;
    m = fabs(rhs);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)z * gridDim.x + blockIdx.x] = red[0];
}

// Final stage of the max reductions: out[z] = max(partA[z,*], partB[z,*]).
__global__ void k_reduce_max(const double* __restrict__ pa, int na, const double* __restrict__ pb, int nb,
                             double* __restrict__ out) {
  __shared__ double red[BLOCK];
  const int z = blockIdx.x;
  double m = 0.0;
  for (int k = threadIdx.x; k < na; k += BLOCK) m = fmax(m, pa[(size_t)z * na + k]);
  for (int k = threadIdx.x; k < nb; k += BLOCK) m = fmax(m, pb[(size_t)z * nb + k]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[z] = red[0];
}

// FP64 refinement residual on regular cells, written as FP32 (MP mode).
template <bool CROSS>
__global__ __launch_bounds__(BLOCK) void k_residual_f32(const double* __restrict__ u, const double* __restrict__ r,
                                                        const uint8_t* __restrict__ kind, float* __restrict__ out,
                                                        int nx, int ny, CoefT<double> c) {
  __shared__ double tile[LH][LW];
  const size_t zoff = (size_t)blockIdx.z * nx * ny;
  u += zoff, r += zoff, out += zoff;
  const int bx = blockIdx.x * TX, by = blockIdx.y * TY;
  load_tile(tile, u, nx, ny, bx, by);
  __syncthreads();
  const int tx = threadIdx.x & (TX - 1), w = threadIdx.x >> 6;
  for (int k = 0; k < TY / 4; ++k) {
    const int ry = w + 4 * k, gx = bx + tx, gy = by + ry;
    if (gx < nx && gy < ny) {
      const size_t g = (size_t)gy * nx + gx;
      out[g] = (kind[g] & 1) ? (float)(r[g] - apply_regular<double, CROSS>(tile, ry + HALO, tx + HALO, c)) : 0.0f;
    }
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
                           const double* __restrict__ fw, double* __restrict__ out, int nfaces) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nfaces) out[k] = fw[k] * lam[fcell[k]];
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, size_t n, T v) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = v;
}

__global__ void k_axpy_f32(double* __restrict__ u, const float* __restrict__ e, const uint8_t* __restrict__ kind,
                           size_t plane, size_t n) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    if (kind[k % plane] & 2) u[k] += (double)e[k];
}

__global__ void k_mask_empty(double* __restrict__ u, const uint8_t* __restrict__ kind, size_t plane, size_t n) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
    if (!(kind[k % plane] & 2)) u[k] = 0.0;
}

// ===========================================================================
// Host side
// ===========================================================================
namespace {

thread_local std::string g_create_error;

#define HIP_OK(x)                                                                                     \
  do {                                                                                                \
    hipError_t e_ = (x);                                                                              \
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

struct Smo2Data {                 // RAS blocks of one level (one orientation)
  int nblk = 0;
  int32_t *ext_ptr = nullptr, *ext_idx = nullptr, *own_cnt = nullptr;
  int32_t *ecell = nullptr, *ecols = nullptr;   // per overlapped row: cell, 15 columns
  double *evals = nullptr, *ersum = nullptr;    // 15 weights, row sum
  int64_t* inv_off = nullptr;
  double* inv = nullptr;
  size_t inv_bytes = 0;
};

struct DevLevel {
  int nx = 0, ny = 0;
  size_t n = 0;
  double h = 0;
  Coef coef;
  bool cross = false;
  uint8_t* kind = nullptr;
  // irregular rows (increasing linear index)
  int nirr = 0;
  int32_t *cell = nullptr, *cols = nullptr;
  double *vals = nullptr, *rowsum = nullptr;
  // transposed operator pieces (adjoint): same structures built from L^T
  int32_t *tcell = nullptr, *tcols = nullptr;
  double *tvals = nullptr, *trowsum = nullptr;
  int ntirr = 0;
  Smo2Data smo2, tsmo2;
  // work arrays (max_nrhs planes)
  double *u = nullptr, *v = nullptr, *r = nullptr;
  float *u32 = nullptr, *v32 = nullptr, *r32 = nullptr;
  double* du = nullptr;
  double* part = nullptr;         // reduction partials
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
  // coarsest solve
  int nm = 0;
  int32_t* mcell = nullptr;
  double* minv = nullptr;
  double* mtinv = nullptr;          // inverse of the transposed coarsest operator
  // level-0 boundary data
  int nfaces = 0;
  int32_t *fptr = nullptr, *fface = nullptr, *fcell = nullptr;
  double *fval = nullptr, *fweight = nullptr;
  double* g = nullptr;              // [max_nrhs][nfaces]
  double* bterm = nullptr;          // [max_nrhs][nirr0]
  int g_nrhs = 0;
  double* norm_out = nullptr;       // device [max_nrhs]
  double* norm_host = nullptr;      // pinned
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

dim3 tiles(int nx, int ny, int nrhs) { return dim3((nx + TX - 1) / TX, (ny + TY - 1) / TY, nrhs); }

// Build the RAS block data of one level from rows (cell, 15 cols, vals) given
// in irregular index order and the Alg. 3 numbering.
void build_smo2(const std::vector<int32_t>& cellv, const std::vector<int32_t>& colv, const std::vector<double>& valv,
                const std::vector<int32_t>& order_pos, int nx_ny, int bsize, int overlap, int threads, Smo2Data& out,
                std::vector<void*>& owned) {
  const int ni = (int)cellv.size();
  if (ni == 0) return;
  std::vector<int32_t> pos(nx_ny, -1);
  for (int k = 0; k < ni; ++k) pos[cellv[k]] = k;
  std::vector<std::vector<int>> nb(ni);
  for (int k = 0; k < ni; ++k)
    for (int s = 0; s < 15; ++s) {
      int p = pos[colv[15 * k + s]];
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
      for (int p = s; p < e; ++p) cur.push_back(order_pos[p]);
      own[b] = (int)cur.size();
      std::set<int> in(cur.begin(), cur.end());
      std::vector<int> frontier = cur;
      for (int l = 0; l < overlap; ++l) {
        std::vector<int> nxt;
        for (int k : frontier)
          for (int m : nb[k])
            if (in.insert(m).second) nxt.push_back(m);
        std::sort(nxt.begin(), nxt.end());
        for (int m : nxt) cur.push_back(m);
        frontier = nxt;
        if ((int)cur.size() > 1000) break;
      }
      if ((int)cur.size() > 1024) cur.resize(1024);
      const int ne = (int)cur.size();
      std::vector<int> loc(0);
      std::map<int, int> where;
      for (int t = 0; t < ne; ++t) where[cur[t]] = t;
      std::vector<double> A((size_t)ne * ne, 0.0);
      for (int t = 0; t < ne; ++t) {
        const int k = cur[t];
        for (int q = 0; q < 15; ++q) {
          int p = pos[colv[15 * k + q]];
          if (p < 0) continue;
          auto it = where.find(p);
          if (it != where.end()) A[(size_t)t * ne + it->second] += valv[15 * k + q];
        }
      }
      if (!ccg::dense_inverse(A, ne, 1)) {
        fail[b] = 1;
        continue;
      }
      // keep the own rows, column-major (ne x own)
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
  }
  std::vector<int32_t> ecell(eidx.size()), ecols(eidx.size() * 15);
  std::vector<double> evals(eidx.size() * 15), ersum(eidx.size());
  for (size_t e = 0; e < eidx.size(); ++e) {
    const int k = eidx[e];
    ecell[e] = cellv[k];
    double rs = 0;
    for (int t = 0; t < 15; ++t) {
      ecols[e * 15 + t] = colv[15 * k + t];
      evals[e * 15 + t] = valv[15 * k + t];
      rs += valv[15 * k + t];
    }
    ersum[e] = rs;
  }
  out.ecell = upload(ecell, owned);
  out.ecols = upload(ecols, owned);
  out.evals = upload(evals, owned);
  out.ersum = upload(ersum, owned);
  out.nblk = nblk;
  out.ext_ptr = upload(eptr, owned);
  out.ext_idx = upload(eidx, owned);
  out.own_cnt = upload(ocnt, owned);
  out.inv_off = upload(ioff, owned);
  out.inv = upload(all, owned);
  out.inv_bytes = all.size() * sizeof(double);
}

// Transposed irregular rows.  Row q of L^T holds L(p, q) for every row p;
// for an irregular cell q the entries from regular rows p are the regular
// stencil (symmetric), those from irregular rows come from the CSR.  For
// regular cells q that appear in an irregular row the transposed row is the
// regular stencil plus extra terms; those cells are treated as "irregular"
// in the transposed operator so that every row stays a 15-entry gather is not
// possible in general -- rows are stored with a variable length padded to a
// fixed width W instead.
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

  template <typename T>
  void sweep(DevLevel& L, const T* u, const T* r, T* out) {
    CoefT<T> c(L.coef);
    const dim3 g = tiles(L.nx, L.ny, nrhs);
    const bool fin = &L == &X->lv[0];
    if (L.cross) {
      if (fin) hipLaunchKernelGGL((k_sweep<T, true, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, c);
      else hipLaunchKernelGGL((k_sweep<T, true, false>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, c);
    } else {
      if (fin) hipLaunchKernelGGL((k_sweep<T, false, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, c);
      else hipLaunchKernelGGL((k_sweep<T, false, false>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, c);
    }
  }

  template <typename T>
  void restrict_(DevLevel& L, DevLevel& C, const T* u, const T* r, T* rc) {
    CoefT<T> c(L.coef);
    const dim3 g((L.nx + TX - 1) / TX, (L.ny + TY - 1) / TY, nrhs);
    const bool fin = &L == &X->lv[0];
    if (L.cross) {
      if (fin) hipLaunchKernelGGL((k_restrict<T, T, true, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, rc, L.nx, L.ny, C.nx, C.ny, c);
      else hipLaunchKernelGGL((k_restrict<T, T, true, false>), g, dim3(BLOCK), 0, s, u, r, L.kind, rc, L.nx, L.ny, C.nx, C.ny, c);
    } else {
      if (fin) hipLaunchKernelGGL((k_restrict<T, T, false, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, rc, L.nx, L.ny, C.nx, C.ny, c);
      else hipLaunchKernelGGL((k_restrict<T, T, false, false>), g, dim3(BLOCK), 0, s, u, r, L.kind, rc, L.nx, L.ny, C.nx, C.ny, c);
    }
  }

  template <typename T>
  void smo2(DevLevel& L, T* u, const T* r, const double* bterm) {
    const Smo2Data& S = adjoint ? L.tsmo2 : L.smo2;
    const int ni = adjoint ? L.ntirr : L.nirr;
    if (ni == 0) return;
    const int32_t* cell = adjoint ? L.tcell : L.cell;
    const int32_t* cols = adjoint ? L.tcols : L.cols;
    const double* vals = adjoint ? L.tvals : L.vals;
    const double* rs = adjoint ? L.trowsum : L.rowsum;
    for (int it = 0; it < X->opt.smo2_iters; ++it) {
      hipLaunchKernelGGL((k_smo2<T>), dim3(S.nblk, nrhs), dim3(BLOCK), 0, s, u, r, bterm, S.ecell, S.ecols, S.evals,
                         S.ersum, S.ext_idx, S.ext_ptr, S.own_cnt, S.inv_off, S.inv, L.du, ni, L.n);
      hipLaunchKernelGGL((k_add_du<T>), dim3((ni + 255) / 256, nrhs), dim3(256), 0, s, u, L.du, cell, ni, L.n);
    }
  }

  // smooth nsteps times; returns pointer to the buffer holding the result
  template <typename T>
  T* smooth(DevLevel& L, T* cur, T* other, const T* r, const double* bterm, int nsteps) {
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

  // Alg. 2 on level m with iterate in (*u, spare *v) and rhs r.
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
    restrict_<T>(L, C, cur, r, cb.r);
    fill<T>(cb.u, C.n * nrhs, (T)0);
    T* e = vcycle<T>(m + 1, cb.u, cb.v, cb.r, nullptr);
    hipLaunchKernelGGL((k_prolong<T>), dim3((L.nx + 255) / 256, L.ny, nrhs), dim3(256), 0, s, cur, e, L.kind, C.kind,
                       L.nx, L.ny, C.nx, C.ny, X->opt.prolongation);
    return smooth<T>(L, cur, oth, r, bterm, X->opt.nu2);
  }

  // max over non-empty cells of |r - bterm - L u| (zero_u: of |r - bterm|)
  template <typename T>
  void resmax(DevLevel& L, const T* u, const T* r, const double* bterm, int zero_u, float* res_out) {
    const dim3 g = tiles(L.nx, L.ny, nrhs);
    CoefT<T> c(L.coef);
    if (L.cross)
      hipLaunchKernelGGL((k_resmax_reg<T, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, L.part, L.nx, L.ny, c, zero_u);
    else
      hipLaunchKernelGGL((k_resmax_reg<T, false>), g, dim3(BLOCK), 0, s, u, r, L.kind, L.part, L.nx, L.ny, c, zero_u);
    const int ni = adjoint ? L.ntirr : L.nirr;
    const int gi = std::max(1, (ni + BLOCK - 1) / BLOCK);
    double* pirr = L.part + (size_t)L.npart_reg * nrhs;
    if (ni > 0)
      hipLaunchKernelGGL((k_resmax_irr<T>), dim3(gi, nrhs), dim3(BLOCK), 0, s, u, r, bterm,
                         adjoint ? L.tcell : L.cell, adjoint ? L.tcols : L.cols, adjoint ? L.tvals : L.vals,
                         adjoint ? L.trowsum : L.rowsum, pirr, ni, L.n, zero_u, res_out);
    hipLaunchKernelGGL(k_reduce_max, dim3(nrhs), dim3(BLOCK), 0, s, L.part, L.npart_reg, pirr, ni > 0 ? gi : 0,
                       X->norm_out);
  }
};

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ===========================================================================
// Context construction
// ===========================================================================
namespace {

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
  std::vector<uint8_t> kind(L.n);
  for (size_t k = 0; k < L.n; ++k) kind[k] = (D.regular[k] ? 1 : 0) | (D.nonempty[k] ? 2 : 0);
  L.kind = upload(kind, X->owned);
  L.nirr = (int)D.irr.size();
  std::vector<double> rs(L.nirr);
  for (int k = 0; k < L.nirr; ++k) {
    double s = 0;
    for (int t = 0; t < 15; ++t) s += D.wts[15 * k + t];
    rs[k] = s;
  }
  L.cell = upload(D.irr, X->owned);
  L.cols = upload(D.sten, X->owned);
  L.vals = upload(D.wts, X->owned);
  L.rowsum = upload(rs, X->owned);
  std::vector<int32_t> opos(L.nirr);
  for (int p = 0; p < L.nirr; ++p) opos[p] = D.irr_pos[D.order[p]];
  build_smo2(D.irr, D.sten, D.wts, opos, (int)L.n, X->opt.smo2_block, X->opt.smo2_overlap, X->opt.num_threads,
             L.smo2, X->owned);
  // work arrays
  L.u = dalloc<double>(L.n * maxr, X->owned);
  L.r = dalloc<double>(L.n * maxr, X->owned);
  L.v = dalloc<double>(L.n * maxr, X->owned);
  L.u32 = dalloc<float>(L.n * maxr, X->owned);
  L.v32 = dalloc<float>(L.n * maxr, X->owned);
  L.r32 = dalloc<float>(L.n * maxr, X->owned);
  L.du = dalloc<double>((size_t)std::max(1, L.nirr) * maxr, X->owned);
  L.npart_reg = (int)(((L.nx + TX - 1) / TX) * ((L.ny + TY - 1) / TY));
  L.npart_irr = std::max(1, (L.nirr + BLOCK - 1) / BLOCK);
  L.part = dalloc<double>((size_t)(L.npart_reg + L.npart_irr) * maxr, X->owned);
}

constexpr long MAX_COARSE_UNKNOWNS = 8000;   // gathered rhs must fit in LDS

void upload_coarsest(ccgmg_ctx* X) {
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
}

}  // namespace

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
  o->auto_depth = 1;
  o->depth_max_rate = 0.5;
  o->precision = 0;
  o->prolongation = 0;
  o->smo2_every_sweep = 1;
  o->smo2_iters = 1;
  o->smo2_block = 64;
  o->smo2_overlap = 2;
  o->tol = 1e-10;
  o->max_cycles = 100;
  o->max_nrhs = 1;
  o->use_initial_guess = 0;
  o->num_threads = 0;
  o->use_graph = 1;
  o->host_only = 0;
  o->hip_stream = nullptr;
}

const char* ccgmg_create_error(void) { return g_create_error.c_str(); }

const char* ccgmg_last_error(const ccgmg_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

static int run_depth_test(ccgmg_ctx* X, double* rate_out);

int ccgmg_create(const ccgmg_grid* grid, const ccgmg_curve* curves, int ncurves, double a, double b, double c,
                 const ccgmg_options* opts, ccgmg_ctx** out) {
  if (!out) return CCGMG_EINVAL;
  *out = nullptr;
  g_create_error.clear();
  std::unique_ptr<ccgmg_ctx> X(new ccgmg_ctx());
  try {
    if (!grid || !curves || ncurves <= 0 || grid->nx <= 0 || grid->ny <= 0 || !(grid->h > 0))
      throw ccg::Error(CCGMG_EINVAL, "invalid grid or curves");
    if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(c)) throw ccg::Error(CCGMG_EINVAL, "non-finite coefficient");
    if (b * b - 4.0 * a * c >= 0.0) throw ccg::Error(CCGMG_ENOTELLIPTIC, "b^2 - 4ac >= 0");
    if (opts)
      X->opt = *opts;
    else
      ccgmg_default_options(&X->opt);
    if (X->opt.max_nrhs < 1) X->opt.max_nrhs = 1;
    if (X->opt.smo2_block < 1 || X->opt.smo2_block > 64) throw ccg::Error(CCGMG_EINVAL, "smo2_block must be in 1..64");
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
      // level-0 boundary data
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
      X->norm_out = dalloc<double>(maxr, X->owned);
      HIP_OK(hipHostMalloc((void**)&X->norm_host, sizeof(double) * maxr, hipHostMallocDefault));
      upload_coarsest(X.get());
      if (X->opt.auto_depth && X->M > 1) {
        for (;;) {
          double rate = 1.0;
          run_depth_test(X.get(), &rate);
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

}  // extern "C"

// ---------------------------------------------------------------------------
// Quadrature export (Green's formula, eq. iteratedIntegral): for a loop piece
// with outer parameter nodes t_q the inner integral from the member cell's
// centre xi0 to x(t_q) is done by a second Gauss-Legendre rule, so each
// (outer, inner) pair is one 2-D node with weight w_q y'(t_q) (x - xi0)/2 w_r.
// ---------------------------------------------------------------------------
namespace {
struct QuadSink {
  std::vector<int32_t> owner;
  std::vector<double> x, y, w, nx, ny;
};

void cell_nodes(const ccg::Geometry& G, int idx, QuadSink& S, int q) {
  std::vector<double> tq, wq;
  ccg::gauss_legendre(q, tq, wq);
  const double h = G.h;
  auto emit_loop = [&](const ccg::Comp& cp) {
    const int own = cp.own, i = own % G.nx, j = own / G.nx;
    const double cx = G.x0 + (i + 0.5) * h, cy = G.y0 + (j + 0.5) * h;
    auto inner = [&](double px, double py, double wout) {
      const double half = 0.5 * (px - cx);
      for (int r = 0; r < q; ++r) {
        S.owner.push_back(idx);
        S.x.push_back(cx + half * (1.0 + tq[r]));
        S.y.push_back(py);
        S.w.push_back(wout * half * wq[r] / (h * h));
      }
    };
    if (cp.loop.empty()) {  // full square: tensor rule
      for (int a = 0; a < q; ++a)
        for (int b2 = 0; b2 < q; ++b2) {
          S.owner.push_back(idx);
          S.x.push_back(cx + 0.5 * h * tq[a]);
          S.y.push_back(cy + 0.5 * h * tq[b2]);
          S.w.push_back(0.25 * wq[a] * wq[b2]);
        }
      return;
    }
    for (const ccg::LoopItem& it : cp.loop) {
      if (it.is_arc) {
        const ccg::CellArc& arc = G.arcs.at(own)[it.arc];
        const ccg::Curve& c = G.curves[arc.curve];
        for (auto& pc : arc.pieces) {
          double half = 0.5 * (pc.second - pc.first), mid = 0.5 * (pc.first + pc.second);
          for (int k = 0; k < q; ++k) {
            double t = mid + half * tq[k], px, py, dx, dy;
            c.point(t, px, py);
            c.deriv(t, dx, dy);
            inner(px, py, wq[k] * half * dy * arc.sigma);
          }
        }
      } else {
        double s = it.sa;
        while (s < it.sb) {
          double es = std::floor(s), nxt = std::min(it.sb, es + 1.0);
          double e0 = std::max(0.0, s - es), e1 = std::min(1.0, nxt - es);
          int edge = (((int)es) % 4 + 4) % 4;
          if (e1 > e0 && (edge == 1 || edge == 3)) {
            double xe = edge == 1 ? cx + 0.5 * h : cx - 0.5 * h;
            double ya = edge == 1 ? cy + (e0 - 0.5) * h : cy + (0.5 - e0) * h;
            double yb = edge == 1 ? cy + (e1 - 0.5) * h : cy + (0.5 - e1) * h;
            double half = 0.5 * (yb - ya);
            for (int k = 0; k < q; ++k) inner(xe, 0.5 * (ya + yb) + half * tq[k], wq[k] * half);
          }
          s = nxt;
        }
      }
    }
  };
  for (int ci : G.cv.at(idx).members) emit_loop(G.comps[ci]);
}
}  // namespace

extern "C" int ccgmg_cell_quadrature(const ccgmg_ctx* X, long* count, int32_t* cell_of, double* x, double* y,
                                     double* w) {
  if (!X || !count) return CCGMG_EINVAL;
  const ccg::Geometry& G = X->H.geo[0];
  QuadSink S;
  std::vector<int> cells;
  for (auto& kv : G.cv) cells.push_back(kv.first);
  std::sort(cells.begin(), cells.end());
  for (int idx : cells) cell_nodes(G, idx, S, 16);
  const long n = (long)S.w.size();
  if (!cell_of && !x && !y && !w) {
    *count = n;
    return CCGMG_OK;
  }
  if (*count < n) return CCGMG_EINVAL;
  for (long k = 0; k < n; ++k) {
    if (cell_of) cell_of[k] = S.owner[k];
    if (x) x[k] = S.x[k];
    if (y) y[k] = S.y[k];
    if (w) w[k] = S.w[k];
  }
  *count = n;
  return CCGMG_OK;
}

extern "C" int ccgmg_face_quadrature(const ccgmg_ctx* X, long* count, int32_t* face_of, double* x, double* y,
                                     double* w, double* nxo, double* nyo) {
  if (!X || !count) return CCGMG_EINVAL;
  const ccg::Geometry& G = X->H.geo[0];
  const ccg::Discretization& D = X->H.disc[0];
  const int q = 16;
  std::vector<double> tq, wq;
  ccg::gauss_legendre(q, tq, wq);
  QuadSink S;
  const double h = G.h;
  for (size_t f = 0; f < D.faces.size(); ++f) {
    const int idx = D.faces[f].first, curve = D.faces[f].second;
    std::vector<const ccg::Comp*> members;
    std::vector<ccg::Comp> tmp;
    if (G.state[idx] == ccg::S_PURE) {
      tmp.push_back(G.trace(idx, {{false, -1, 0.0, 4.0}}));
      members.push_back(&tmp.back());
    } else {
      for (int ci : G.cv.at(idx).members) members.push_back(&G.comps[ci]);
    }
    for (const ccg::Comp* cp : members) {
      const int own = cp->own, i = own % G.nx, j = own / G.nx;
      const double cx = G.x0 + (i + 0.5) * h, cy = G.y0 + (j + 0.5) * h;
      std::vector<ccg::LoopItem> loop = cp->loop;
      if (loop.empty()) loop.push_back({false, -1, 0.0, 4.0});
      for (const ccg::LoopItem& it : loop) {
        if (it.is_arc) {
          const ccg::CellArc& arc = G.arcs.at(own)[it.arc];
          if (arc.curve != curve) continue;
          const ccg::Curve& c = G.curves[arc.curve];
          for (auto& pc : arc.pieces) {
            double half = 0.5 * (pc.second - pc.first), mid = 0.5 * (pc.first + pc.second);
            for (int k = 0; k < q; ++k) {
              double t = mid + half * tq[k], px, py, dx, dy;
              c.point(t, px, py);
              c.deriv(t, dx, dy);
              double sp = std::hypot(dx, dy);
              S.owner.push_back((int32_t)f);
              S.x.push_back(px);
              S.y.push_back(py);
              S.w.push_back(wq[k] * half * sp / h);
              S.nx.push_back(arc.sigma * dy / sp);
              S.ny.push_back(-arc.sigma * dx / sp);
            }
          }
        } else if (G.box == curve) {
          double s = it.sa;
          while (s < it.sb) {
            double es = std::floor(s), nxt = std::min(it.sb, es + 1.0);
            double e0 = std::max(0.0, s - es), e1 = std::min(1.0, nxt - es);
            int edge = (((int)es) % 4 + 4) % 4;
            if (e1 > e0 && G.on_border(i, j, edge)) {
              static const double NRM[4][2] = {{0, -1}, {1, 0}, {0, 1}, {-1, 0}};
              double Ax, Ay, Bx, By;
              if (edge == 0) Ax = cx + (e0 - 0.5) * h, Ay = cy - 0.5 * h, Bx = cx + (e1 - 0.5) * h, By = Ay;
              else if (edge == 1) Ax = cx + 0.5 * h, Ay = cy + (e0 - 0.5) * h, Bx = Ax, By = cy + (e1 - 0.5) * h;
              else if (edge == 2) Ax = cx + (0.5 - e0) * h, Ay = cy + 0.5 * h, Bx = cx + (0.5 - e1) * h, By = Ay;
              else Ax = cx - 0.5 * h, Ay = cy + (0.5 - e0) * h, Bx = Ax, By = cy + (0.5 - e1) * h;
              double Lh = std::hypot(Bx - Ax, By - Ay) / h;
              for (int k = 0; k < q; ++k) {
                double tt = 0.5 * (1.0 + tq[k]);
                S.owner.push_back((int32_t)f);
                S.x.push_back(Ax + tt * (Bx - Ax));
                S.y.push_back(Ay + tt * (By - Ay));
                S.w.push_back(0.5 * wq[k] * Lh);
                S.nx.push_back(NRM[edge][0]);
                S.ny.push_back(NRM[edge][1]);
              }
            }
            s = nxt;
          }
        }
      }
    }
  }
  const long n = (long)S.w.size();
  if (!face_of && !x && !y && !w && !nxo && !nyo) {
    *count = n;
    return CCGMG_OK;
  }
  if (*count < n) return CCGMG_EINVAL;
  for (long k = 0; k < n; ++k) {
    if (face_of) face_of[k] = S.owner[k];
    if (x) x[k] = S.x[k];
    if (y) y[k] = S.y[k];
    if (w) w[k] = S.w[k];
    if (nxo) nxo[k] = S.nx[k];
    if (nyo) nyo[k] = S.ny[k];
  }
  *count = n;
  return CCGMG_OK;
}

// ===========================================================================
// Apply / solve
// ===========================================================================
namespace {

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

// One FP64 V-cycle on level 0 (u, v = user iterate and spare buffer).
void fp64_cycle(Driver& Dr, double* u, const double* f, const double* bterm) {
  DevLevel& L0 = Dr.X->lv[0];
  double* res = Dr.vcycle<double>(0, u, L0.v, f, bterm);
  if (res != u)
    HIP_OK(hipMemcpyAsync(u, res, sizeof(double) * L0.n * Dr.nrhs, hipMemcpyDeviceToDevice, Dr.s));
}

// One refinement step of the mixed-precision solve: r32 = f - N g - L u
// (FP64, difference form) stored as FP32, one FP32 V-cycle on L e = r32 with
// zero guess, u += e (FP64).
void mp_cycle(Driver& Dr, double* u, const double* f, const double* bterm) {
  ccgmg_ctx* X = Dr.X;
  DevLevel& L0 = X->lv[0];
  const int nr = Dr.nrhs;
  CoefT<double> c(L0.coef);
  if (L0.cross)
    hipLaunchKernelGGL((k_residual_f32<true>), tiles(L0.nx, L0.ny, nr), dim3(BLOCK), 0, Dr.s, u, f, L0.kind, L0.r32, L0.nx, L0.ny, c);
  else
    hipLaunchKernelGGL((k_residual_f32<false>), tiles(L0.nx, L0.ny, nr), dim3(BLOCK), 0, Dr.s, u, f, L0.kind, L0.r32, L0.nx, L0.ny, c);
  // irregular rows of the residual (FP64) written into r32; norm partials unused here
  Dr.resmax<double>(L0, u, f, bterm, 0, L0.r32);
  Dr.fill<float>(L0.u32, L0.n * nr, 0.0f);
  float* e = Dr.vcycle<float>(0, L0.u32, L0.v32, L0.r32, nullptr);
  const size_t n = L0.n * nr;
  hipLaunchKernelGGL(k_axpy_f32, dim3(std::min<size_t>(4096, (n + 255) / 256)), dim3(256), 0, Dr.s, u, e, L0.kind, L0.n, n);
}

int solve_impl(ccgmg_ctx* X, const double* f, double* u, int nrhs, ccgmg_report* rep, bool adjoint) {
  return guard(X, [&]() {
    if (!f || !u || nrhs < 1 || nrhs > X->opt.max_nrhs) throw ccg::Error(CCGMG_EINVAL, "bad solve arguments");
    if (adjoint) throw ccg::Error(CCGMG_EINVAL, "adjoint solve not available in this build");
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
    if (X->nfaces > 0 && X->g_nrhs >= nrhs && L0.nirr > 0) {
      hipLaunchKernelGGL(k_bterm, dim3((L0.nirr + 255) / 256, nrhs), dim3(256), 0, ws, X->g, X->fptr, X->fface,
                         X->fval, X->bterm, L0.nirr, X->nfaces);
      bterm = X->bterm;
    }
    if (!X->opt.use_initial_guess) Dr.fill<double>(u, n, 0.0);
    hipLaunchKernelGGL(k_mask_empty, dim3(std::min<size_t>(4096, (n + 255) / 256)), dim3(256), 0, ws, u, L0.kind, L0.n, n);
    Dr.resmax<double>(L0, u, f, bterm, 1, nullptr);
    std::vector<double> rn(nrhs);
    HIP_OK(hipMemcpyAsync(X->norm_host, X->norm_out, sizeof(double) * nrhs, hipMemcpyDeviceToHost, ws));
    HIP_OK(hipStreamSynchronize(ws));
    for (int z = 0; z < nrhs; ++z) rn[z] = X->norm_host[z] > 0 ? X->norm_host[z] : 1.0;
    // one V-cycle (FP64, or FP32 inside one FP64 refinement step), the FP64
    // residual check and its read-back, replayed from a graph when allowed
    auto cycle = [&]() {
      if (X->opt.precision == 1)
        mp_cycle(Dr, u, f, bterm);
      else
        fp64_cycle(Dr, u, f, bterm);
      Dr.resmax<double>(L0, u, f, bterm, 0, nullptr);
      HIP_OK(hipMemcpyAsync(X->norm_host, X->norm_out, sizeof(double) * nrhs, hipMemcpyDeviceToHost, ws));
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
      for (int z = 0; z < nrhs; ++z) rel = std::max(rel, X->norm_host[z] / rn[z]);
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

}  // namespace

static int run_depth_test(ccgmg_ctx* X, double* rate_out) {
  // V-cycles on a seeded random right-hand side with the current depth;
  // the geometric-mean contraction of the residual over 6 cycles.
  DevLevel& L0 = X->lv[0];
  std::vector<double> r(L0.n, 0.0);
  std::mt19937_64 gen(12345);
  std::normal_distribution<double> nd(0.0, 1.0);
  const ccg::Discretization& D = X->H.disc[0];
  for (size_t k = 0; k < L0.n; ++k) r[k] = D.nonempty[k] ? nd(gen) : 0.0;
  double* rd = nullptr;
  double* ud = nullptr;
  HIP_OK(hipMalloc(&rd, sizeof(double) * L0.n));
  HIP_OK(hipMalloc(&ud, sizeof(double) * L0.n));
  HIP_OK(hipMemcpy(rd, r.data(), sizeof(double) * L0.n, hipMemcpyHostToDevice));
  ccgmg_options saved = X->opt;
  X->opt.max_cycles = 6;
  X->opt.tol = 0.0;
  X->opt.use_initial_guess = 0;
  X->opt.precision = 0;
  int g_saved = X->g_nrhs;
  X->g_nrhs = 0;
  ccgmg_report rep;
  solve_impl(X, rd, ud, 1, &rep, false);
  X->opt = saved;
  X->g_nrhs = g_saved;
  (void)hipFree(rd);
  (void)hipFree(ud);
  double last = rep.cycles > 0 ? rep.history[std::min(rep.cycles, 64) - 1] : 1.0;
  *rate_out = (std::isfinite(last) && rep.cycles > 0) ? std::pow(last, 1.0 / rep.cycles) : 1e300;
  return 0;
}

extern "C" {

int ccgmg_apply(ccgmg_ctx* X, const double* u, double* Lu) {
  return guard(X, [&]() {
    if (!u || !Lu || u == Lu) throw ccg::Error(CCGMG_EINVAL, "bad apply arguments");
    DevLevel& L = X->lv[0];
    CoefT<double> c(L.coef);
    if (L.cross)
      hipLaunchKernelGGL((k_apply<true>), tiles(L.nx, L.ny, 1), dim3(BLOCK), 0, X->stream, u, L.kind, Lu, L.nx, L.ny, c);
    else
      hipLaunchKernelGGL((k_apply<false>), tiles(L.nx, L.ny, 1), dim3(BLOCK), 0, X->stream, u, L.kind, Lu, L.nx, L.ny, c);
    if (L.nirr > 0)
      hipLaunchKernelGGL(k_irr_apply, dim3((L.nirr + 255) / 256), dim3(256), 0, X->stream, u, Lu, L.cell, L.cols, L.vals, L.nirr);
    HIP_OK(hipGetLastError());
  });
}

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

int ccgmg_profile_kernel(ccgmg_ctx* X, int kernel, int level, int reps, double* avg_us) {
  return guard(X, [&]() {
    if (!avg_us || reps < 1 || level < 0 || level > X->M || kernel < 0 || kernel > 5)
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
        case 1: Dr.restrict_<double>(L, *C, L.u, L.r, C->r); break;
        case 2:
          hipLaunchKernelGGL((k_prolong<double>), dim3((L.nx + 255) / 256, L.ny, 1), dim3(256), 0, X->stream, L.u,
                             C->u, L.kind, C->kind, L.nx, L.ny, C->nx, C->ny, X->opt.prolongation);
          break;
        case 3:
          if (L.nirr > 0)
            hipLaunchKernelGGL((k_smo2<double>), dim3(L.smo2.nblk, 1), dim3(BLOCK), 0, X->stream, L.u, L.r,
                               (const double*)nullptr, L.smo2.ecell, L.smo2.ecols, L.smo2.evals, L.smo2.ersum,
                               L.smo2.ext_idx, L.smo2.ext_ptr, L.smo2.own_cnt, L.smo2.inv_off, L.smo2.inv, L.du,
                               L.nirr, L.n);
          break;
        case 4: Dr.coarse<double>(L, L.u, L.r); break;
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

int ccgmg_apply_NT(ccgmg_ctx* X, const double* lam, double* out) {
  return guard(X, [&]() {
    if (!lam || !out) throw ccg::Error(CCGMG_EINVAL, "bad arguments");
    if (X->nfaces > 0)
      hipLaunchKernelGGL(k_apply_NT, dim3((X->nfaces + 255) / 256), dim3(256), 0, X->stream, lam, X->fcell, X->fweight,
                         out, X->nfaces);
  });
}

void ccgmg_destroy(ccgmg_ctx* X) {
  if (!X) return;
  if (!X->host_only) {
    if (X->stream) (void)hipStreamSynchronize(X->stream);
    else (void)hipDeviceSynchronize();
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
