// HIP kernels of the cut-cell multigrid V-cycle for gfx950.
//
// Layout: every level stores cell averages row-major [nrhs][ny][nx] (x
// fastest); blockIdx.z selects the right-hand side.  kind[] holds one byte
// per cell: bit 0 = regular (Section 3.2), bit 1 = non-empty.
//
// Regular rows use the fourth-order formulas eq. stdLap (u_xx, u_yy) and the
// twice-applied eq. stdGrad (u_xy) in difference form,
//   (L u)_i = sum_{m != 0} c_m (u_{i+m} - u_i),
// an exact rewrite because the stencil coefficients sum to zero; it keeps
// the FP64 rounding floor of the residual near eps * h |grad u| / h^2
// instead of eps * |u| / h^2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccgk {

constexpr int TX = 64;        // tile width (one wavefront per row)
constexpr int TY = 16;        // tile height; 4 waves x 4 rows each
constexpr int HALO = 2;       // half width of the 5x5 stencil
constexpr int LW = TX + 2 * HALO;
constexpr int LH = TY + 2 * HALO;
constexpr int BLOCK = 256;

struct Coef {                 // regular stencil, units 1/h^2
  double ax1, ax2;            // 16a/12h^2, -a/12h^2
  double cy1, cy2;            // 16c/12h^2, -c/12h^2
  double bxy;                 // b/144h^2
  double omega_invD;          // omega / D, D = -30(a+c)/12h^2
};

template <typename T>
struct CoefT {
  T ax1, ax2, cy1, cy2, bxy, omega_invD;
  __host__ __device__ CoefT() {}
  __host__ __device__ CoefT(const Coef& c)
      : ax1((T)c.ax1), ax2((T)c.ax2), cy1((T)c.cy1), cy2((T)c.cy2), bxy((T)c.bxy), omega_invD((T)c.omega_invD) {}
};

// Fill a ROWS x W LDS tile (W = TX + 4 by default): entry k (row-major) is ld(ly, lx),
// computed by thread k mod BLOCK.  The loads of CH of a thread's entries
// are issued together, with no wait between them, and only then written
// to LDS: a loop that waits for each load before issuing the next one
// serializes the memory latency (6-10 round trips per workgroup).
template <typename T, int ROWS, int W = LW, int CH = 5, typename Ld>
__device__ __forceinline__ void stage_tile(T (*tile)[W], const Ld& ld) {
  constexpr int N = ROWS * W, NIT = (N + BLOCK - 1) / BLOCK;
#pragma unroll
  for (int i0 = 0; i0 < NIT; i0 += CH) {
    T v[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      if (i0 + i < NIT) {
        const int k = (int)threadIdx.x + (i0 + i) * BLOCK;
        const int kk = k < N ? k : 0;
        const int ly = kk / W, lx = kk - ly * W;
        v[i] = ld(ly, lx);
      }
    }
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int k = (int)threadIdx.x + (i0 + i) * BLOCK;
      if (i0 + i < NIT && k < N) {
        const int ly = k / W, lx = k - ly * W;
        tile[ly][lx] = v[i];
      }
    }
  }
}

// Stage the (ROWS) x (TX+4) neighbourhood of a tile (ROWS = tile height + 4)
// in LDS; outside the grid the value is 0 (never read by a regular cell).
// Branch-free: an outside entry loads u[0] and discards it.
template <typename T, int ROWS = LH>
__device__ __forceinline__ void load_tile(T (*tile)[LW], const T* __restrict__ u, int nx, int ny, int bx, int by) {
  stage_tile<T, ROWS>(tile, [&](int ly, int lx) {
    const int gx = bx + lx - HALO, gy = by + ly - HALO;
    const bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    const T x = u[in ? (size_t)gy * nx + gx : 0];
    return in ? x : (T)0;
  });
}

// Workgroups of a launch are handed to the 8 XCDs round-robin (workgroup id
// mod 8) and every XCD has its own L2.  xcd_tile maps the 1-D workgroup id b
// of an nb-workgroup launch to a tile index so that XCD x processes one
// contiguous range of tiles, i.e. a band of tile rows: horizontally and
// vertically adjacent tiles, whose halos overlap, then share an L2.  The map
// is a bijection of [0, nb): XCD x owns ceil(nb/8) tiles if x < nb mod 8
// (or nb mod 8 == 0), one fewer otherwise.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int per = (nb + NXCD - 1) / NXCD, rem = nb % NXCD;
  const int x = b % NXCD, k = b / NXCD;
  int start = x * per;
  if (rem != 0 && x > rem) start -= x - rem;
  return start + k;
}

// Raw buffer views of one array (gfx9 buffer descriptor: base address, size
// in bytes, word 3 = 0x00020000, i.e. 32-bit data format, no swizzle).  The
// hardware checks every access against the size: a load at a byte offset
// outside [0, size) returns 0 and a store there is dropped.  Offsets are
// 32-bit; callers keep arrays below 2^31 bytes and give a cell outside the
// grid an offset of at least 2^31 (as unsigned), so it reads 0 and writes
// nothing without a select or a branch.
using bufrsrc = __amdgpu_buffer_rsrc_t;
constexpr int BUF_OUT = (int)0x80000000u;   // an offset no array reaches
__device__ __forceinline__ bufrsrc make_buf(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
typedef unsigned int bufu2 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ T buf_ld(bufrsrc r, int off);
template <>
__device__ __forceinline__ double buf_ld<double>(bufrsrc r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float buf_ld<float>(bufrsrc r, int off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ uint8_t buf_ld<uint8_t>(bufrsrc r, int off) {
  return __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
}
__device__ __forceinline__ void buf_st(bufrsrc r, int off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bufu2, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_st(bufrsrc r, int off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
}

// Stage the ROWS x (TX + 2 H) neighbourhood of a tile in LDS: rows
// by - H .. by - H + ROWS - 1, columns bx - H .. bx + TX + H - 1 of the
// nx x ny plane viewed by bu, 0 outside the grid (ROWS a multiple of 4).
// Thread (w, tx) loads tile column tx in rows w, w + 4, ... (32-bit
// offsets stepping by 4 rows; a column past nx reads from BUF_OUT), threads
// q < 2 H ROWS load the side columns; every load is issued before the
// first LDS write.
template <typename T, int ROWS, int H>
__device__ __forceinline__ void stage_cols(T (*tile)[TX + 2 * H], bufrsrc bu, int nx, int ny, int bx, int by) {
  static_assert(ROWS % 4 == 0, "rows in steps of 4");
  constexpr int SZ = (int)sizeof(T), M = ROWS / 4, NS = 2 * H * ROWS, NIS = (NS + BLOCK - 1) / BLOCK;
  const int tx = threadIdx.x & (TX - 1), w = threadIdx.x >> 6, q = threadIdx.x;
  const int gx = bx + tx;
  const int o0 = (unsigned)gx < (unsigned)nx ? ((by - H + w) * nx + gx) * SZ : BUF_OUT;
  T v[M], vs[NIS];
#pragma unroll
  for (int i = 0; i < M; ++i) v[i] = buf_ld<T>(bu, o0 + 4 * i * nx * SZ);
#pragma unroll
  for (int i = 0; i < NIS; ++i) {
    const int qq = q + i * BLOCK, cc = qq & (2 * H - 1), ly = qq / (2 * H);
    const int gxs = bx - H + (cc < H ? cc : TX + cc), gys = by - H + ly;
    const bool in = qq < NS && (unsigned)gxs < (unsigned)nx && (unsigned)gys < (unsigned)ny;
    vs[i] = buf_ld<T>(bu, in ? (gys * nx + gxs) * SZ : BUF_OUT);
  }
#pragma unroll
  for (int i = 0; i < M; ++i) tile[w + 4 * i][tx + H] = v[i];
#pragma unroll
  for (int i = 0; i < NIS; ++i) {
    const int qq = q + i * BLOCK, cc = qq & (2 * H - 1), ly = qq / (2 * H);
    if (qq < NS) tile[ly][cc < H ? cc : TX + cc] = vs[i];
  }
}

// x if keep, else +0.0, as a bit mask: a select between a loaded value and
// a constant can be compiled into a branch around the load that waits for
// it inside, which serializes the loads of a gather.
__device__ __forceinline__ double keep_or_zero(double x, bool keep) {
  return __longlong_as_double(__double_as_longlong(x) & (keep ? ~0LL : 0LL));
}

// Maximum that keeps a NaN (fmax drops it): a non-finite residual must
// survive the norm reductions so that the host sees it.
__device__ __forceinline__ double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

// Residual-norm accumulators of a thread, then of a workgroup: the maximum
// of |r| (NaN kept) and the sum of r^2.  Every norm-taking launch stores
// one pair per workgroup, (max, sum of squares), at 2 * (z * G + b); the
// host reduces the pairs of a plane in workgroup order.
struct NormAcc {
  double m = 0.0, s = 0.0;
  __device__ __forceinline__ void add(double r) {
    m = nanmax(m, fabs(r));
    s += r * r;
  }
};

// The workgroup's pair (valid in thread 0): shuffle reduction within each
// wavefront, then the wavefronts in order through red (2 * BLOCK / 64
// doubles of LDS).  Every thread must call it.
__device__ __forceinline__ NormAcc block_norm(NormAcc a, double* red) {
  for (int off = 32; off > 0; off >>= 1) {
    a.m = nanmax(a.m, __shfl_xor(a.m, off, 64));
    a.s += __shfl_xor(a.s, off, 64);
  }
  if ((threadIdx.x & 63) == 0) red[2 * (threadIdx.x >> 6)] = a.m, red[2 * (threadIdx.x >> 6) + 1] = a.s;
  __syncthreads();
  NormAcc o;
  o.m = red[0], o.s = red[1];
  for (int w = 1; w < BLOCK / 64; ++w) o.m = nanmax(o.m, red[2 * w]), o.s += red[2 * w + 1];
  return o;
}

// (L u) at a cell from a value accessor at(dy, dx) (neighbour offsets in
// -2..2), difference form.  The one arithmetic sequence shared by the LDS
// tile form and the register-window form below.
template <typename T, bool CROSS, typename At>
__device__ __forceinline__ T regular_row(const At& at, const CoefT<T>& c) {
  const T uc = at(0, 0);
  const T two = (T)2 * uc;
  T acc = c.ax1 * ((at(0, 1) + at(0, -1)) - two) + c.ax2 * ((at(0, 2) + at(0, -2)) - two) +
          c.cy1 * ((at(1, 0) + at(-1, 0)) - two) + c.cy2 * ((at(2, 0) + at(-2, 0)) - two);
  if (CROSS) {
    // sum_{m1,m2} g(m1) g(m2) u, g(+-1) = +-8, g(+-2) = -+1, as nested differences
    T d[5];
#pragma unroll
    for (int m = -2; m <= 2; ++m) {
      if (m == 0) continue;
      d[m + 2] = (T)8 * (at(1, m) - at(-1, m)) - (at(2, m) - at(-2, m));
    }
    acc += c.bxy * ((T)8 * (d[3] - d[1]) - (d[4] - d[0]));
  }
  return acc;
}

// The same row with the y-differences of the cross term given:
// dy(m) = 8 (u(1, m) - u(-1, m)) - (u(2, m) - u(-2, m)) for m = +-1, +-2,
// and the axis values uc = u(0, 0), xp1 = u(0, 1), xm1 = u(0, -1), ...,
// yp1 = u(1, 0), ... (same operations in the same order as regular_row).
template <typename T, typename Dy>
__device__ __forceinline__ T regular_row_dy(T uc, T xp1, T xm1, T xp2, T xm2, T yp1, T ym1, T yp2, T ym2,
                                            const Dy& dy, const CoefT<T>& c) {
  const T two = (T)2 * uc;
  T acc = c.ax1 * ((xp1 + xm1) - two) + c.ax2 * ((xp2 + xm2) - two) + c.cy1 * ((yp1 + ym1) - two) +
          c.cy2 * ((yp2 + ym2) - two);
  acc += c.bxy * ((T)8 * (dy(1) - dy(-1)) - (dy(2) - dy(-2)));
  return acc;
}

// (L u) at tile position (ly, lx) (already offset by HALO), difference form.
template <typename T, bool CROSS>
__device__ __forceinline__ T apply_regular(const T (*t)[LW], int ly, int lx, const CoefT<T>& c) {
  return regular_row<T, CROSS>([&](int dy, int dx) { return t[ly + dy][lx + dx]; }, c);
}

// y-differences of the cross term on the NR x (TX + 4) cells of a tile
// whose u neighbourhood (NR + 4 rows) is staged in t:
// dy[y][x] = 8 (t[y+3][x] - t[y+1][x]) - (t[y+4][x] - t[y][x]).
template <typename T, int NR>
__device__ __forceinline__ void fill_dy(T (*dy)[LW], const T (*t)[LW]) {
  for (int k = threadIdx.x; k < NR * LW; k += BLOCK) {
    const int y = k / LW, x = k - y * LW;
    dy[y][x] = (T)8 * (t[y + 3][x] - t[y + 1][x]) - (t[y + 4][x] - t[y][x]);
  }
}

// (L u) at tile position (ly, lx) (already offset by HALO) with the cross
// term's y-differences taken from dy (tile rows without the HALO offset).
template <typename T>
__device__ __forceinline__ T apply_regular_dy(const T (*t)[LW], const T (*dy)[LW], int ly, int lx,
                                              const CoefT<T>& c) {
  const T* row = t[ly] + lx;
  const T* dr = dy[ly - HALO] + lx;
  return regular_row_dy<T>(row[0], row[1], row[-1], row[2], row[-2], t[ly + 1][lx], t[ly - 1][lx], t[ly + 2][lx],
                           t[ly - 2][lx], [&](int dx) { return dr[dx]; }, c);
}

}  // namespace ccgk
