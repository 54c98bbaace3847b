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
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "ccgmg.h"
#include "kernels.hpp"
#include "diag_kernels.hpp"
#include "setup.hpp"
#include "vcycle_kernels.hpp"

using namespace ccgk;

// Device scratch of ccgmg_residual_norms_noalloc (partial maxima and sums of
// squares, then the per-plane totals), for callers that cannot allocate.  In
// host code `scratch` only names the symbol: its device address differs per
// GPU and is taken with hipGetSymbolAddress (scratch_on_current_device).
constexpr size_t SCRATCH_DOUBLES = (size_t)1 << 19;   // 4 MiB
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

// ===========================================================================
// Host side
// ===========================================================================
namespace {

thread_local std::string g_create_error;

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

#define HIP_OK(x)                                                                                          \
  do {                                                                                                     \
    hipError_t e_ = (x);                                                                                   \
    if (e_ != hipSuccess) throw ccg::Error(CCGMG_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Device address of the static scratch array on the current device, looked
// up once per device (with that device current) and kept.
double* scratch_on_current_device() {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) throw ccg::Error(CCGMG_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw ccg::Error(CCGMG_EDEVICE, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_ptr[dev] = p;
  }
  return (double*)g_scratch_ptr[dev];
}

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
  int32_t *ecell = nullptr, *ecols = nullptr;   // overlapped rows: cell; ELL columns [n_ext][ew]
  int ew = 0;                     // ELL width: longest overlapped row of this row set
  int32_t* ebt = nullptr;         // boundary-term index of each overlapped row (-1: none)
  int32_t* scell = nullptr;       // cell of every block row
  int32_t *epar = nullptr, *eqpar = nullptr;   // coarse parents (fused prolongation), -1: none
  int ns = 0;                     // block rows
  double* cbuf[2] = {nullptr, nullptr};   // compact copies of the block rows' values
  int cur = 0;                    // which copy is current while a cycle is recorded
  double *evals = nullptr, *ersum = nullptr;
  int64_t* inv_off = nullptr;
  float* inv = nullptr;           // dense block inverses (computed in FP64), stored in FP32 ...
  double* inv64 = nullptr;        // ... or in FP64 (options.inverse_fp32 = 0)
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
  int sweep2_ty[2] = {8, 8};      // the same for the two-sweep launch, tuned separately
  int npart_reg = 0, npart_irr = 0;
  // level 0: partials of a fused step that also takes the residual norm
  // (at most npart_fused per plane), and whether the SMO-1 cells and the
  // SMO-2 block rows together are exactly the non-empty cells (L, L^T)
  double* fpart = nullptr;
  int npart_fused = 0;
  bool norm_cover[2] = {false, false};
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
  float* minv = nullptr;            // inverse of the coarsest operator (computed in FP64), FP32 ...
  float* mtinv = nullptr;           // ... and of its transpose
  double *minv64 = nullptr, *mtinv64 = nullptr;   // the same in FP64 (options.inverse_fp32 = 0)
  double* mrg = nullptr;            // gathered coarsest right-hand sides [MAX_COARSE_UNKNOWNS][max_nrhs]
  struct Coarse {
    int nm;
    int32_t* cell;
    float *inv, *tinv;
    double *inv64, *tinv64;
  };
  std::map<int, Coarse> coarse_cache;   // per coarsest level index
  std::vector<double> tune_ms;          // autotune: solve time per depth (index = M)
  double* tune_rhs = nullptr;           // the tuner's seeded right-hand side (drawn once, device)
  int nfaces = 0;                   // level-0 boundary data
  int32_t *fptr = nullptr, *fface = nullptr, *fcell = nullptr;
  double *fval = nullptr, *fweight = nullptr;
  double* g = nullptr;              // [max_nrhs][nfaces]
  double* bterm = nullptr;          // [max_nrhs][nirr0]
  int g_nrhs = 0;
  double* norm_host = nullptr;      // pinned: partial maxima of the residual norm (level 0)
  double* norm_host2 = nullptr;     // a second one: cycles alternate between the two
  double* norm_host0 = nullptr;     // a third: the reference norm ||f - N g|| of the solve's start
  double setup_seconds = 0;
  double plg_max_cond = 0;
  std::string err;
  bool host_only = false;
  // solves run on a private stream (ordered after the caller's stream by
  // events) so that each V-cycle can be captured into a hipGraph
  hipStream_t ws = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipEvent_t ev_cyc[2] = {nullptr, nullptr};   // ends of the cycles in flight (alternating)
  hipEvent_t ev_pro = nullptr;      // end of a solve's prologue (reference norm read back)
  int device = 0;                   // the HIP device the context lives on
  double* scratch = nullptr;        // that device's static scratch array (no-alloc entry point)
  hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;   // device time of a solve (created once)
  struct GraphEntry {
    const void *u, *f, *bterm, *norm;
    int nrhs, precision, M;
    bool adjoint, pipe;
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
                size_t ncells, int bsize, int overlap, int threads, bool inv_fp32, Smo2Data& out,
                std::vector<void*>& owned) {
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
  // ELL layout (row e's entries at e * ew + k, padding: column 0, weight 0,
  // no parent), so a row's columns are addressed without its row pointer
  int ew = 1;
  for (size_t e = 0; e < eidx.size(); ++e) ew = std::max(ew, erp[e + 1] - erp[e]);
  std::vector<int32_t> lcols(eidx.size() * ew, 0), lpar(eidx.size() * ew, -1);
  std::vector<double> lvals(eidx.size() * ew, 0.0);
  for (size_t e = 0; e < eidx.size(); ++e)
    for (int t = erp[e]; t < erp[e + 1]; ++t) {
      const size_t d = e * ew + (t - erp[e]);
      lcols[d] = ecols[t];
      lpar[d] = epar[t];
      lvals[d] = evals[t];
    }
  out.ew = ew;
  out.ecols = upload(lcols, owned);
  out.epar = upload(lpar, owned);
  out.eqpar = upload(eqpar, owned);
  out.evals = upload(lvals, owned);
  out.ersum = upload(ersum, owned);
  out.nblk = nblk;
  out.ext_ptr = upload(eptr, owned);
  out.ext_idx = upload(eidx, owned);
  out.own_cnt = upload(ocnt, owned);
  out.inv_off = upload(ioff, owned);
  if (inv_fp32) {
    const std::vector<float> all32(all.begin(), all.end());
    out.inv = upload(all32, owned);
    out.inv_bytes = all32.size() * sizeof(float);
  } else {
    out.inv64 = upload(all, owned);
    out.inv_bytes = all.size() * sizeof(double);
  }
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
  build_smo2(S, bt, parent, ncells, opt.smo2_block, opt.smo2_overlap, opt.num_threads, opt.inverse_fp32 != 0, D.smo2,
             owned);
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

  // two consecutive plain SMO-1 sweeps in one launch
  template <typename T, bool CROSS, bool FIN>
  void sweep2_t(DevLevel& L, const T* u, const T* r, T* out, int ty) {
    CoefT<T> c(L.coef);
    const dim3 g = tiles1d(L.nx, L.ny, nrhs, ty);
    const int nbx = tiles_x(L.nx);
    const uint8_t rb = jacbit();
    switch (ty) {
      case 8: hipLaunchKernelGGL((k_sweep2<T, CROSS, FIN, 8>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, c, rb); break;
      case 32: hipLaunchKernelGGL((k_sweep2<T, CROSS, FIN, 32>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, c, rb); break;
      default: hipLaunchKernelGGL((k_sweep2<T, CROSS, FIN, 16>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, c, rb); break;
    }
  }

  // false (nothing launched) where it does not apply: the two-sweep kernel
  // addresses a plane through 32-bit buffer offsets, which needs planes
  // below 2^31 bytes; the caller then runs two sweeps
  template <typename T>
  static bool sweep2_fits(const DevLevel& L) {
    return (uint64_t)L.nx * (uint64_t)L.ny * sizeof(T) < (1ull << 31);
  }
  template <typename T>
  bool sweep2(DevLevel& L, const T* u, const T* r, T* out, int ty = 0) {
    if (!sweep2_fits<T>(L)) return false;
    if (ty == 0) ty = L.sweep2_ty[sizeof(T) == 8 ? 0 : 1];
    const bool fin = &L == &X->lv[0];
    if (L.cross) {
      if (fin) sweep2_t<T, true, true>(L, u, r, out, ty);
      else sweep2_t<T, true, false>(L, u, r, out, ty);
    } else {
      if (fin) sweep2_t<T, false, true>(L, u, r, out, ty);
      else sweep2_t<T, false, false>(L, u, r, out, ty);
    }
    return true;
  }

  // restriction into rc; also zeroes the coarse block rows' compact copy
  // (which becomes the current one) and sets the coarse iterate uc to zero,
  // or (first_sweep) to the result of one plain SMO-1 sweep from zero
  template <typename T>
  void restrict_(DevLevel& L, DevLevel& C, const T* u, const T* r, T* rc, T* uc, bool first_sweep = false) {
    CoefT<T> c(L.coef);
    const dim3 g = tiles1d(L.nx, L.ny, nrhs);
    const int nbx = tiles_x(L.nx);
    const bool fin = &L == &X->lv[0];
    const uint8_t rb = regbit(), jb = jacbit();
    Smo2Data& CS = rows(C).smo2;
    CS.cur = 0;
    double* cc = CS.cbuf[0];
    const int ncc = CS.ns;
    const uint8_t* ck = first_sweep ? C.kind : nullptr;
    const T cw = CoefT<T>(C.coef).omega_invD;
    if (L.cross) {
      if (fin) hipLaunchKernelGGL((k_restrict<T, T, true, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, rc, uc, cc, ncc, L.nx, L.ny, nbx, C.nx, C.ny, c, rb, ck, cw, jb);
      else hipLaunchKernelGGL((k_restrict<T, T, true, false>), g, dim3(BLOCK), 0, s, u, r, L.kind, rc, uc, cc, ncc, L.nx, L.ny, nbx, C.nx, C.ny, c, rb, ck, cw, jb);
    } else {
      if (fin) hipLaunchKernelGGL((k_restrict<T, T, false, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, rc, uc, cc, ncc, L.nx, L.ny, nbx, C.nx, C.ny, c, rb, ck, cw, jb);
      else hipLaunchKernelGGL((k_restrict<T, T, false, false>), g, dim3(BLOCK), 0, s, u, r, L.kind, rc, uc, cc, ncc, L.nx, L.ny, nbx, C.nx, C.ny, c, rb, ck, cw, jb);
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
    a.ecell = S.ecell, a.ecols = S.ecols, a.ew = S.ew;
    a.evals = S.evals, a.ersum = S.ersum;
    a.eidx = S.ext_idx, a.ebt = S.ebt, a.ext_ptr = S.ext_ptr, a.own_cnt = S.own_cnt;
    a.inv_off = S.inv_off, a.inv = S.inv, a.inv64 = S.inv64;
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

  // one fused smoothing step (SMO-1 and SMO-2 from the same iterate u);
  // part (finest level, FP64, no pending correction): also the residual
  // norm partials of u, fused_parts(L) per plane
  template <typename T, bool CROSS, bool FIN, bool PRO>
  void fused_t(DevLevel& L, const T* u, const T* r, T* out, const double* bterm, int ty, const T* e,
               const DevLevel* C, double* part = nullptr) {
    Smo2Data& S = rows(L).smo2;
    CoefT<T> c(L.coef);
    const int nbx = tiles_x(L.nx);
    const int ntiles = nbx * ((L.ny + ty - 1) / ty);
    const dim3 g(ntiles + S.nblk, 1, nrhs);
    const uint8_t rb = jacbit(), sb = adjoint ? F_S2_T : F_S2;
    const Smo2Args a = smo2_args(L, bterm);
    const int ncx = C ? C->nx : 0, ncy = C ? C->ny : 0;
    const uint8_t pb = regbit();
    if (part) {
      if constexpr (std::is_same<T, double>::value && FIN && !PRO) {
        switch (ty) {
          case 8: hipLaunchKernelGGL((k_smooth_fused<T, CROSS, FIN, 8, PRO, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, S.nblk, c, rb, sb, a, e, ncx, ncy, pb, part); break;
          case 32: hipLaunchKernelGGL((k_smooth_fused<T, CROSS, FIN, 32, PRO, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, S.nblk, c, rb, sb, a, e, ncx, ncy, pb, part); break;
          default: hipLaunchKernelGGL((k_smooth_fused<T, CROSS, FIN, 16, PRO, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, S.nblk, c, rb, sb, a, e, ncx, ncy, pb, part); break;
        }
        S.cur = 1 - S.cur;
        return;
      } else {
        throw ccg::Error(CCGMG_EINVAL, "residual partials only from the finest FP64 step");
      }
    }
    switch (ty) {
      case 8: hipLaunchKernelGGL((k_smooth_fused<T, CROSS, FIN, 8, PRO>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, S.nblk, c, rb, sb, a, e, ncx, ncy, pb, nullptr); break;
      case 32: hipLaunchKernelGGL((k_smooth_fused<T, CROSS, FIN, 32, PRO>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, S.nblk, c, rb, sb, a, e, ncx, ncy, pb, nullptr); break;
      default: hipLaunchKernelGGL((k_smooth_fused<T, CROSS, FIN, 16, PRO>), g, dim3(BLOCK), 0, s, u, r, L.kind, out, L.nx, L.ny, nbx, S.nblk, c, rb, sb, a, e, ncx, ncy, pb, nullptr); break;
    }
    S.cur = 1 - S.cur;
  }

  // partials per plane of a fused step of level L with norm partials
  int fused_parts(DevLevel& L) {
    const int ty = L.sweep_ty[0];
    return tiles_x(L.nx) * ((L.ny + ty - 1) / ty) + rows(L).smo2.nblk;
  }

  template <typename T, bool CROSS, bool FIN>
  void fused_p(DevLevel& L, const T* u, const T* r, T* out, const double* bterm, int ty, const T* e,
               const DevLevel* C, double* part) {
    if (e) fused_t<T, CROSS, FIN, true>(L, u, r, out, bterm, ty, e, C);
    else fused_t<T, CROSS, FIN, false>(L, u, r, out, bterm, ty, nullptr, nullptr, part);
  }

  // one fused step; with e, the pending coarse-grid correction P e (coarse
  // level C) is applied on the fly; with part (level 0, FP64, no e), the
  // residual norm partials of u are written there as well
  template <typename T>
  void fused_step(DevLevel& L, const T* u, const T* r, T* out, const double* bterm, const T* e = nullptr,
                  const DevLevel* C = nullptr, double* part = nullptr) {
    // the correction is read at the parent of every in-grid cell
    if (e && (!C || L.nx != 2 * C->nx || L.ny != 2 * C->ny))
      throw ccg::Error(CCGMG_EINVAL, "coarse level is not the fine level halved");
    const int ty = L.sweep_ty[sizeof(T) == 8 ? 0 : 1];
    const bool fin = &L == &X->lv[0];
    if (part && (!fin || e)) throw ccg::Error(CCGMG_EINVAL, "residual partials only from the finest FP64 step");
    if (L.cross) {
      if (fin) fused_p<T, true, true>(L, u, r, out, bterm, ty, e, C, part);
      else fused_p<T, true, false>(L, u, r, out, bterm, ty, e, C, part);
    } else {
      if (fin) fused_p<T, false, true>(L, u, r, out, bterm, ty, e, C, part);
      else fused_p<T, false, false>(L, u, r, out, bterm, ty, e, C, part);
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

  // a recorded cycle must leave the finest level's current copy where it
  // found it (its values carry over from one cycle to the next)
  void settle_rows(DevLevel& L) {
    Smo2Data& S = rows(L).smo2;
    if (S.cur != 0 && S.ns > 0) {
      HIP_OK(hipMemcpyAsync(S.cbuf[0], S.cbuf[1], sizeof(double) * S.ns * nrhs, hipMemcpyDeviceToDevice, s));
      S.cur = 0;
    }
  }

  bool fused(DevLevel& L) const { return X->opt.smoother_fused && rows(L).smo2.ns > 0; }

  // SMO-2 in step k of a phase of nsteps: every step (smo2_every_sweep =
  // 1), the last step of the phase only (0), or every s-th step counted
  // back from the last (s)
  bool with_smo2(int k, int nsteps) const {
    const int every = X->opt.smo2_every_sweep;
    return every >= 1 ? (nsteps - 1 - k) % every == 0 : k == nsteps - 1;
  }

  int pre_steps(int m) const { return (m > 0 && X->opt.nu1_coarse > 0) ? X->opt.nu1_coarse : X->opt.nu1; }

  // Whether the restriction onto level m (m > 0, starting from a zero
  // iterate) can also carry out that level's first pre-smoothing step:
  // true when the step's SMO-1 part is a plain sweep (it then maps the
  // zero iterate to omega D^-1 r on the SMO-1 cells and leaves the rest at
  // zero).  In fused mode that step must be one without SMO-2; unfused,
  // its SMO-2 pass still runs after it.
  bool fold_first_sweep(int m) {
    if (m >= X->M) return false;
    const int n1 = pre_steps(m);
    if (n1 < 1) return false;
    return !fused(X->lv[m]) || !with_smo2(0, n1);
  }

  // smooth nsteps times; returns pointer to the buffer holding the result.
  // Fused mode: e (if given) is the pending coarse-grid correction from
  // level C, applied by the first step.  first_done: the SMO-1 sweep of
  // step 0 has already been carried out (by the restriction; cur holds its
  // result).
  // Two steps k, k + 1 whose SMO-1 sweeps follow each other with no SMO-2
  // pass between them run as one two-sweep launch (sweep2) where the level
  // allows it.
  template <typename T>
  T* smooth(DevLevel& L, T* cur, T* other, const T* r, const double* bterm, int nsteps, const T* e = nullptr,
            const DevLevel* C = nullptr, bool first_done = false) {
    if (fused(L)) {
      for (int k = first_done ? 1 : 0; k < nsteps; ++k) {
        // the step that applies the coarse-grid correction is always fused;
        // in the other steps without SMO-2 the block rows keep their values
        if (with_smo2(k, nsteps) || (k == 0 && e))
          fused_step<T>(L, cur, r, other, bterm, k == 0 ? e : nullptr, C);
        else if (k + 1 < nsteps && !with_smo2(k + 1, nsteps) && sweep2<T>(L, cur, r, other))
          ++k;
        else
          sweep<T>(L, cur, r, other);
        std::swap(cur, other);
      }
      return cur;
    }
    for (int k = 0; k < nsteps; ++k) {
      if (!(k == 0 && first_done)) {
        if (!with_smo2(k, nsteps) && k + 1 < nsteps && sweep2<T>(L, cur, r, other))
          ++k;   // steps k and k + 1 swept; step k has no SMO-2 pass
        else
          sweep<T>(L, cur, r, other);
        std::swap(cur, other);
      }
      if (with_smo2(k, nsteps)) smo2<T>(L, cur, r, bterm);
    }
    return cur;
  }

  template <typename T>
  void fill(T* p, size_t n, T v) {
    hipLaunchKernelGGL((k_fill<T>), dim3(std::min<size_t>(4096, (n + 255) / 256)), dim3(256), 0, s, p, n, v);
  }

  template <typename T>
  void coarse(DevLevel& L, T* u, const T* r) {
    const float* inv = adjoint ? X->mtinv : X->minv;
    const double* inv64 = adjoint ? X->mtinv64 : X->minv64;
    const int nm = X->nm;
    if (nrhs == 1) {
      hipLaunchKernelGGL((k_coarse<T>), dim3((nm + COARSE_WAVES - 1) / COARSE_WAVES, 1), dim3(64 * COARSE_WAVES),
                         nm * sizeof(double), s, u, r, X->mcell, inv, inv64, nm, L.n);
      return;
    }
    // several right-hand sides: gather, then one product reading the inverse once
    hipLaunchKernelGGL((k_coarse_gather<T>), dim3((nm + 255) / 256, nrhs), dim3(256), 0, s, r, X->mcell, X->mrg,
                       nm, nrhs, L.n);
    hipLaunchKernelGGL((k_coarse_multi<T>), dim3((nm + CM_ROWS - 1) / CM_ROWS, (nrhs + CM_RHS - 1) / CM_RHS), dim3(64 * CMW), 0, s, u,
                       X->mrg, X->mcell, inv, inv64, nm, nrhs, L.n);
  }

  // Alg. 2 on level m with iterate in (u, spare v) and rhs r.  first_done:
  // the restriction onto this level has already carried out the SMO-1
  // sweep of its first pre-smoothing step (fold_first_sweep).
  template <typename T>
  T* vcycle(int m, T* u, T* v, const T* r, const double* bterm, bool first_done = false) {
    DevLevel& L = X->lv[m];
    if (m == X->M) {
      coarse<T>(L, u, r);
      return u;
    }
    // smoothing steps: nu1/nu2 on the finest level, nu1_coarse/nu2_coarse
    // (when positive) on the coarse levels
    const int n1 = pre_steps(m);
    const int n2 = (m > 0 && X->opt.nu2_coarse > 0) ? X->opt.nu2_coarse : X->opt.nu2;
    T* cur = smooth<T>(L, u, v, r, bterm, n1, nullptr, nullptr, first_done);
    T* oth = cur == u ? v : u;
    DevLevel& C = X->lv[m + 1];
    Buf<T> cb = bufs<T>(C);
    const bool fold = fold_first_sweep(m + 1);
    restrict_<T>(L, C, cur, r, cb.r, cb.u, fold);
    T* e = vcycle<T>(m + 1, cb.u, cb.v, cb.r, nullptr, fold);
    T* out;
    if (fused(L) && X->opt.prolongation == 0 && n2 > 0) {
      out = smooth<T>(L, cur, oth, r, bterm, n2, e, &C);   // correction applied by the first step
    } else {
      prolong<T>(L, C, cur, e);
      out = smooth<T>(L, cur, oth, r, bterm, n2);
    }
    // coarse levels need no settling: the restriction onto them rewrites
    // (zeroes) copy 0 and makes it current at the start of every visit
    if (m == 0) settle_rows(L);
    return out;
  }

  // One FMG cycle (Fig. 4) of level 0's problem A x = r with iterate u (the
  // boundary term bterm on level 0): the residual of u restricted to level
  // 1, then restricted level by level (zero iterates) to the coarsest
  // level, solved there; on the way up each level runs one V-cycle from the
  // prolonged solution of the level below (the descent left its iterate
  // and compact copy at zero), and level 0 runs one V-cycle from u + P e_1.
  // That equals u + FMG(r - bterm - A u), V-cycles being affine.  Returns
  // the buffer holding the new iterate (u or v).
  template <typename T>
  T* fmg(T* u, T* v, const T* r, const double* bterm) {
    const int M = X->M;
    if (M == 0) return vcycle<T>(0, u, v, r, bterm);
    {
      Buf<T> cb = bufs<T>(X->lv[1]);
      restrict_<T>(X->lv[0], X->lv[1], u, r, cb.r, cb.u);
    }
    for (int m = 1; m < M; ++m) {
      Buf<T> lb = bufs<T>(X->lv[m]), cb = bufs<T>(X->lv[m + 1]);
      restrict_<T>(X->lv[m], X->lv[m + 1], lb.u, lb.r, cb.r, cb.u);
    }
    Buf<T> mb = bufs<T>(X->lv[M]);
    coarse<T>(X->lv[M], mb.u, mb.r);
    T* e = mb.u;
    for (int m = M - 1; m >= 1; --m) {
      Buf<T> lb = bufs<T>(X->lv[m]);
      prolong<T>(X->lv[m], X->lv[m + 1], lb.u, e);
      e = vcycle<T>(m, lb.u, lb.v, lb.r, nullptr);
    }
    prolong<T>(X->lv[0], X->lv[1], u, e);
    return vcycle<T>(0, u, v, r, bterm);
  }

  // one cycle of the kind the options ask for
  template <typename T>
  T* cycle(T* u, T* v, const T* r, const double* bterm) {
    return X->opt.cycle == 1 ? fmg<T>(u, v, r, bterm) : vcycle<T>(0, u, v, r, bterm);
  }

  // partial maxima over non-empty cells of |r - bterm - A u| (zero_u: of
  // |r - bterm|), one launch, into L.part[z * norm_parts(L) + b]
  int norm_parts(DevLevel& L) {
    return tiles_x(L.nx) * ((L.ny + TY - 1) / TY) + (rows(L).n + BLOCK - 1) / BLOCK;
  }

  template <typename T>
  void resmax(DevLevel& L, const T* u, const T* r, const double* bterm, int zero_u, float* res_out,
              double* part = nullptr) {
    if (!part) part = L.part;
    const int nbx = tiles_x(L.nx);
    const int ntiles = nbx * ((L.ny + TY - 1) / TY);
    DevRows& R = rows(L);
    const int nrb = (R.n + BLOCK - 1) / BLOCK;
    const dim3 g(ntiles + nrb, 1, nrhs);
    CoefT<T> c(L.coef);
    const uint8_t rb = regbit();
    if (L.cross)
      hipLaunchKernelGGL((k_resnorm<T, true>), g, dim3(BLOCK), 0, s, u, r, L.kind, L.nx, L.ny, nbx, ntiles, c, zero_u,
                         rb, bterm, R.cell, R.rp, R.cols, R.vals, R.rowsum, R.n, res_out, part);
    else
      hipLaunchKernelGGL((k_resnorm<T, false>), g, dim3(BLOCK), 0, s, u, r, L.kind, L.nx, L.ny, nbx, ntiles, c,
                         zero_u, rb, bterm, R.cell, R.rp, R.cols, R.vals, R.rowsum, R.n, res_out, part);
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
  L.norm_cover[0] = L.norm_cover[1] = true;
  for (size_t k = 0; k < L.n; ++k) {
    const bool ne = kind[k] & F_NONEMPTY;
    const bool jf_ = kind[k] & F_JAC, sf_ = kind[k] & F_S2, jt_ = kind[k] & F_JAC_T, st_ = kind[k] & F_S2_T;
    if (ne ? jf_ == sf_ : (jf_ || sf_)) L.norm_cover[0] = false;
    if (ne ? jt_ == st_ : (jt_ || st_)) L.norm_cover[1] = false;
  }
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
  // norm partials: a (maximum, sum of squares) pair per workgroup
  L.part = dalloc<double>((size_t)2 * (L.npart_reg + L.npart_irr) * maxr, X->owned);
  if (m == 0) {
    L.npart_fused = ((L.nx + TX - 1) / TX) * ((L.ny + 7) / 8) + std::max(L.fwd.smo2.nblk, L.adj.smo2.nblk);
    L.fpart = dalloc<double>((size_t)2 * L.npart_fused * maxr, X->owned);
  }
}

void upload_coarsest(ccgmg_ctx* X) {
  auto hit = X->coarse_cache.find(X->M);
  if (hit != X->coarse_cache.end()) {
    X->nm = hit->second.nm, X->mcell = hit->second.cell, X->minv = hit->second.inv, X->mtinv = hit->second.tinv;
    X->minv64 = hit->second.inv64, X->mtinv64 = hit->second.tinv64;
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
  double amax = 0.0;
  for (double v : A) amax = std::max(amax, std::fabs(v));
  const double tiny = 1e-12 * amax;
  // inverse on the device: Gauss-Jordan with partial pivoting, 2 launches per
  // pivot on the private stream; the transpose's inverse is its transpose
  std::vector<void*> scratch;   // freed once the inverse is done
  double* dA = upload(A, scratch);
  double* colk = dalloc<double>(n, scratch);
  int* status = dalloc<int>(1, scratch);
  const bool fp32 = X->opt.inverse_fp32 != 0;
  double* dinv = dalloc<double>((size_t)n * n, fp32 ? scratch : X->owned);
  float *finv = nullptr, *ftinv = nullptr;
  double* dtinv = nullptr;
  if (fp32) {
    finv = dalloc<float>((size_t)n * n, X->owned);
    ftinv = dalloc<float>((size_t)n * n, X->owned);
  } else {
    dtinv = dalloc<double>((size_t)n * n, X->owned);
  }
  hipStream_t st = X->ws;
  HIP_OK(hipMemsetAsync(status, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_set_identity, dim3((unsigned)(((size_t)n * n + 255) / 256)), dim3(256), 0, st, dinv, n);
  const dim3 ge((2 * n + 1023) / 1024, n);
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, st, dA, dinv, n, k, colk, status, tiny);
    hipLaunchKernelGGL(k_gj_elim, ge, dim3(256), 0, st, dA, dinv, n, k, colk, status);
  }
  // stored in FP32 by default (applied in FP64): an inexact coarsest solve
  // (relative 1e-7) leaves the V-cycle's contraction unchanged and halves
  // the bytes
  if (fp32) {
    hipLaunchKernelGGL(k_transpose<float>, dim3((n + 31) / 32, (n + 31) / 32), dim3(32, 8), 0, st, dinv, ftinv, n);
    hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, st, (const double*)dinv, finv, (size_t)n * n);
  } else {
    hipLaunchKernelGGL(k_transpose<double>, dim3((n + 31) / 32, (n + 31) / 32), dim3(32, 8), 0, st, dinv, dtinv, n);
  }
  int singular = 0;
  HIP_OK(hipMemcpyAsync(&singular, status, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  for (void* q : scratch) (void)hipFree(q);
  if (singular) throw ccg::Error(CCGMG_ESINGULAR, "singular coarsest operator");
  X->nm = n;
  X->mcell = upload(cells, X->owned);
  X->minv = finv;
  X->mtinv = ftinv;
  X->minv64 = fp32 ? nullptr : dinv;
  X->mtinv64 = dtinv;
  X->coarse_cache[X->M] = {n, X->mcell, X->minv, X->mtinv, X->minv64, X->mtinv64};
}

// Tile-height autotuning of the SMO-1 sweep and of the two-sweep launch: on
// every level and in both precisions, time each admissible tile height (HIP
// events, private stream, work buffers of that level; best of two
// interleaved rounds) and keep the lowest one within 3% of the fastest:
// on small levels the candidates time alike within noise, and the lowest
// height gives the most workgroups.
void tune_tiles(ccgmg_ctx* X) {
  static const int cand[] = {8, 16, 32};
  Driver Dr{X, X->ws, 1, false};
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  const int reps = 20;   // per candidate and round; best of two interleaved rounds
  for (DevLevel& L : X->lv) {
    Dr.fill<double>(L.u, L.n, 1.0);
    Dr.fill<double>(L.r, L.n, 0.5);
    Dr.fill<float>(L.u32, L.n, 1.0f);
    Dr.fill<float>(L.r32, L.n, 0.5f);
    for (int kern = 0; kern < 2; ++kern)
    for (int prec = 0; prec < 2; ++prec) {
      if (kern == 1 && !(prec == 0 ? Dr.sweep2_fits<double>(L) : Dr.sweep2_fits<float>(L))) continue;
      float best[3] = {1e30f, 1e30f, 1e30f};
      int* pick = kern == 0 ? &L.sweep_ty[prec] : &L.sweep2_ty[prec];
      for (int round = 0; round < 2; ++round)
      for (int ci = 0; ci < 3; ++ci) {
        const int ty = cand[ci];
        auto launch = [&]() {
          if (kern == 0) {
            if (prec == 0) Dr.sweep<double>(L, L.u, L.r, L.v, ty);
            else Dr.sweep<float>(L, L.u32, L.r32, L.v32, ty);
          } else {
            if (prec == 0) Dr.sweep2<double>(L, L.u, L.r, L.v, ty);
            else Dr.sweep2<float>(L, L.u32, L.r32, L.v32, ty);
          }
        };
        launch();
        launch();
        HIP_OK(hipEventRecord(e0, X->ws));
        for (int k = 0; k < reps; ++k) launch();
        HIP_OK(hipEventRecord(e1, X->ws));
        HIP_OK(hipEventSynchronize(e1));
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, e0, e1));
        best[ci] = std::min(best[ci], ms);
      }
      const float fastest = std::min(best[0], std::min(best[1], best[2]));
      for (int ci = 2; ci >= 0; --ci)
        if (best[ci] <= 1.03f * fastest) *pick = cand[ci];
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

// One FP64 cycle (V-cycle or FMG) on level 0 (u = caller's iterate, v =
// spare buffer).
void fp64_cycle(Driver& Dr, double* u, const double* f, const double* bterm) {
  DevLevel& L0 = Dr.X->lv[0];
  double* res = Dr.cycle<double>(u, L0.v, f, bterm);
  if (res != u) HIP_OK(hipMemcpyAsync(u, res, sizeof(double) * L0.n * Dr.nrhs, hipMemcpyDeviceToDevice, Dr.s));
}

// One refinement step of the mixed-precision solve.  On entry L0.r32 holds
// the FP32 copy of the FP64 residual f - N g - A u (difference form), written
// by the residual check that ended the previous step (or by the prologue):
// one FP32 V-cycle (or FMG cycle) on A e = r32 from a zero guess (explicit rows and the
// coarsest solve in FP64 arithmetic), then u += e in FP64.
void mp_cycle(Driver& Dr, double* u) {
  ccgmg_ctx* X = Dr.X;
  DevLevel& L0 = X->lv[0];
  const int nr = Dr.nrhs;
  Dr.fill<float>(L0.u32, L0.n * nr, 0.0f);
  Dr.gather_rows<float>(L0, L0.u32);
  float* e = Dr.cycle<float>(L0.u32, L0.v32, L0.r32, nullptr);
  const size_t n = L0.n * nr;
  hipLaunchKernelGGL(k_axpy_f32, dim3(std::min<size_t>(4096, (n + 255) / 256)), dim3(256), 0, Dr.s, u, e, L0.kind, L0.n, n);
}

// Pieces of a solve shared by single and batched solves.  Residual norms are
// per-workgroup partial maxima of level 0, read back into the pinned buffer
// norm_host and reduced on the host.
double norm_of(ccgmg_ctx* X, int nparts, int z, const double* part = nullptr) {
  const double* p = part ? part : X->norm_host;
  double m = 0.0;
  for (int k = 0; k < nparts; ++k) {
    const double v = p[2 * ((size_t)z * nparts + k)];
    if (std::isnan(v)) return v;   // a NaN partial is the result
    m = std::max(m, v);
  }
  return m;
}

// The L2 norm from the same partials (their sums of squares, in workgroup
// order).
double l2_of(ccgmg_ctx* X, int nparts, int z, const double* part = nullptr) {
  const double* p = part ? part : X->norm_host;
  double s = 0.0;
  for (int k = 0; k < nparts; ++k) s += p[2 * ((size_t)z * nparts + k) + 1];
  return std::sqrt(s);
}

// Whether the solve takes each cycle's residual norm from the first
// smoothing step of the next cycle (norm_in_first_step): FP64 V-cycles
// whose first finest-level step is a fused one (SMO-1 and SMO-2 from the
// same iterate), on a level whose SMO-1 cells and SMO-2 block rows are
// exactly its non-empty cells.  That step computes the residual of the
// iterate it starts from on every non-empty cell anyway and writes its
// result to the spare buffer, so the checked iterate stays where it is.
bool norm_in_first_step(Driver& Dr) {
  ccgmg_ctx* X = Dr.X;
  DevLevel& L0 = X->lv[0];
  return X->opt.precision == 0 && X->opt.cycle == 0 && X->M > 0 && X->opt.nu1 >= 1 && Dr.fused(L0) &&
         Dr.with_smo2(0, X->opt.nu1) && L0.norm_cover[Dr.adjoint ? 1 : 0];
}

// The first smoothing step of a cycle with the residual norm partials of
// its starting iterate u: reads u, writes L0.v; the partials go to part,
// which may be the pinned host buffer the solve loop reads (the kernel
// writes it directly: the host reads it after the event that follows the
// launch, when the writes are visible), else to L0.fpart.
void first_step_norm(Driver& Dr, const double* u, const double* f, const double* bterm, double* part = nullptr) {
  DevLevel& L0 = Dr.X->lv[0];
  Dr.fused_step<double>(L0, u, f, L0.v, bterm, nullptr, nullptr, part ? part : L0.fpart);
}

// Start of a solve on stream Dr.s: boundary term, initial iterate, compact
// copies, and the norm of the initial residual read back (not waited for).
// pipe (norm_in_first_step): also the first step of the first cycle, whose
// partials give that norm from a zero start.  Returns the boundary term in
// use (or nullptr).
const double* solve_prologue(Driver& Dr, const double* f, double* u, bool pipe = false) {
  ccgmg_ctx* X = Dr.X;
  DevLevel& L0 = X->lv[0];
  const int nrhs = Dr.nrhs;
  const size_t n = L0.n * nrhs;
  const double* bterm = nullptr;
  if (!Dr.adjoint && X->nfaces > 0 && X->g_nrhs >= nrhs && L0.fwd.n > 0) {
    hipLaunchKernelGGL(k_bterm, dim3((L0.fwd.n + 255) / 256, nrhs), dim3(256), 0, Dr.s, X->g, X->fptr, X->fface,
                       X->fval, X->bterm, L0.fwd.n, X->nfaces);
    bterm = X->bterm;
  }
  if (!X->opt.use_initial_guess) Dr.fill<double>(u, n, 0.0);
  hipLaunchKernelGGL(k_mask_empty, dim3(std::min<size_t>(4096, (n + 255) / 256)), dim3(256), 0, Dr.s, u, L0.kind,
                     L0.n, n);
  const bool mp = X->opt.precision == 1;
  if (!mp) Dr.gather_rows<double>(L0, u);
  // reference norm ||f - N g||; for a zero start it is also the residual
  // the first mixed-precision step needs (stored as FP32)
  const bool zero_start = !X->opt.use_initial_guess;
  if (pipe) {
    // from a zero start the step's partials are those of |f - N g|,
    // written straight into the pinned buffer
    if (zero_start) {
      first_step_norm(Dr, u, f, bterm, X->norm_host0);
    } else {
      Dr.resmax<double>(L0, u, f, bterm, 1, nullptr, X->norm_host0);
      first_step_norm(Dr, u, f, bterm);
    }
    return bterm;
  }
  Dr.resmax<double>(L0, u, f, bterm, 1, (mp && zero_start) ? L0.r32 : nullptr, X->norm_host0);
  if (mp && !zero_start) Dr.resmax<double>(L0, u, f, bterm, 0, L0.r32);   // residual of the initial guess
  return bterm;
}

// One V-cycle (FP64, or FP32 inside one FP64 refinement step) and the FP64
// residual check, whose partial maxima the kernel writes straight into
// norm_dst (pinned; default norm_host), on stream Dr.s (recordable in a
// graph).
void solve_cycle(Driver& Dr, double* u, const double* f, const double* bterm, double* norm_dst = nullptr) {
  ccgmg_ctx* X = Dr.X;
  DevLevel& L0 = X->lv[0];
  const bool mp = X->opt.precision == 1;
  if (mp)
    mp_cycle(Dr, u);
  else
    fp64_cycle(Dr, u, f, bterm);
  // the residual check; in mixed precision it also leaves the FP32 residual
  // for the next refinement step
  Dr.resmax<double>(L0, u, f, bterm, 0, mp ? L0.r32 : nullptr, norm_dst ? norm_dst : X->norm_host);
}

// One FP64 V-cycle whose first step has already run (its result in L0.v,
// the compact copy advanced), then the first step of the next cycle, which
// writes the residual norm partials of this cycle's result u into the
// pinned buffer norm_dst (norm_in_first_step; recordable in a graph).
void solve_cycle_pipe(Driver& Dr, double* u, const double* f, const double* bterm, double* norm_dst) {
  ccgmg_ctx* X = Dr.X;
  DevLevel& L0 = X->lv[0];
  Dr.rows(L0).smo2.cur = 1;   // the state a first step leaves
  double* res = Dr.vcycle<double>(0, L0.v, u, f, bterm, true);
  if (res != u) HIP_OK(hipMemcpyAsync(u, res, sizeof(double) * L0.n * Dr.nrhs, hipMemcpyDeviceToDevice, Dr.s));
  first_step_norm(Dr, u, f, bterm, norm_dst);
}

// Convergence bookkeeping of one solve (host side, after each read-back).
struct Monitor {
  std::vector<double> rn, rn2;   // reference norms ||f - N g|| (L-infinity, L2)
  int nparts = 0, cycles = 0, hist = 0, slow = 0;
  double prev = 1e300, rel = 1.0, rel2 = 1.0;
  bool converged = false, stopped = false;
  bool guess = false;   // the solve starts from the caller's iterate
  // from the reference norms ||f - N g|| the prologue read back into
  // X->norm_host0; returns false if one of them is not finite (NaN or Inf
  // in f-hat or g-hat)
  bool start(ccgmg_ctx* X, int nrhs, int np, int np0 = -1) {
    if (np0 < 0) np0 = np;
    nparts = np;
    rn.assign(nrhs, 1.0);
    rn2.assign(nrhs, 1.0);
    rel = rel2 = 0.0;
    bool finite = true;
    for (int z = 0; z < nrhs; ++z) {
      const double m = norm_of(X, np0, z, X->norm_host0), m2 = l2_of(X, np0, z, X->norm_host0);
      finite = finite && std::isfinite(m);
      rn[z] = m > 0 ? m : 1.0;
      rn2[z] = m2 > 0 ? m2 : 1.0;
      if (m > 0) rel = rel2 = 1.0;
    }
    guess = X->opt.use_initial_guess != 0;
    return finite;
  }
  double fmin = 1.0;   // smallest contraction factor seen so far
  // after a cycle; returns true when this solve is finished
  bool step(ccgmg_ctx* X, ccgmg_report* rep, const double* part = nullptr) {
    converged = stopped = false;
    ++cycles;
    const double before = cycles > 1 ? prev : 1.0;
    rel = rel2 = 0;
    for (size_t z = 0; z < rn.size(); ++z) {
      rel = std::max(rel, norm_of(X, nparts, (int)z, part) / rn[z]);
      rel2 = std::max(rel2, l2_of(X, nparts, (int)z, part) / rn2[z]);
    }
    if (rep && hist < 64) rep->history[hist++] = rel;
    if (!std::isfinite(rel)) return stopped = true;
    if (rel <= X->opt.tol) return converged = stopped = true;
    if (before > 0.0) fmin = std::min(fmin, rel / before);
    if (rel > 0.95 * prev) {
      if (++slow >= 3) return stopped = true;
    } else {
      slow = 0;
    }
    prev = rel;
    if (cycles >= X->opt.max_cycles) return stopped = true;
    return false;
  }
  // true when the next cycle cannot end the solve, so the one after it may
  // be enqueued before its residual is read: it stays below max_cycles and
  // the stagnation count, and its residual cannot reach tol even if it
  // contracts 10x better than the best cycle so far (1e-3 before any cycle
  // is measured, and then only from a zero start with a non-zero residual:
  // the caller's iterate may already be close)
  bool next_not_final(ccgmg_ctx* X) const {
    if (stopped || cycles + 1 >= X->opt.max_cycles || slow + 1 >= 3) return false;
    if (cycles == 0 && guess) return false;
    const double f = cycles > 0 ? 0.1 * fmin : 1e-3;
    return std::isfinite(rel) && rel * f > X->opt.tol;
  }
};

// The captured graph of one cycle of this solve (cached per context, keyed
// by its arrays, norm read-back buffer, right-hand-side count, precision,
// depth and direction); recorded on stream Dr.s, launchable on any stream.
hipGraphExec_t cycle_graph(Driver& Dr, double* u, const double* f, const double* bterm,
                           double* norm_dst = nullptr, bool pipe = false) {
  ccgmg_ctx* X = Dr.X;
  if (!norm_dst) norm_dst = X->norm_host;
  for (auto& g : X->graphs)
    if (g.u == u && g.f == f && g.bterm == bterm && g.norm == norm_dst && g.nrhs == Dr.nrhs &&
        g.precision == X->opt.precision && g.M == X->M && g.adjoint == Dr.adjoint && g.pipe == pipe)
      return g.exec;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph;
  HIP_OK(hipStreamBeginCapture(Dr.s, hipStreamCaptureModeThreadLocal));
  if (pipe)
    solve_cycle_pipe(Dr, u, f, bterm, norm_dst);
  else
    solve_cycle(Dr, u, f, bterm, norm_dst);
  HIP_OK(hipStreamEndCapture(Dr.s, &graph));
  HIP_OK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  (void)hipGraphDestroy(graph);
  if (X->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(X->graphs.front().exec);
    X->graphs.erase(X->graphs.begin());
  }
  X->graphs.push_back({u, f, bterm, norm_dst, Dr.nrhs, X->opt.precision, X->M, Dr.adjoint, pipe, exec});
  return exec;
}

int solve_impl(ccgmg_ctx* X, const double* f, double* u, int nrhs, ccgmg_report* rep, bool adjoint) {
  return guard(X, [&]() {
    if (!f || !u || nrhs < 1 || nrhs > X->opt.max_nrhs) throw ccg::Error(CCGMG_EINVAL, "bad solve arguments");
    hipStream_t ws = X->ws;
    Driver Dr{X, ws, nrhs, adjoint};
    HIP_OK(hipEventRecord(X->ev_in, X->stream));
    HIP_OK(hipStreamWaitEvent(ws, X->ev_in, 0));
    HIP_OK(hipEventRecord(X->ev_t0, ws));
    // pipe: cycle k's residual norm comes from the first step of cycle k + 1
    // (each recorded cycle ends with the next cycle's first step); a solve
    // that ends after cycle k returns its result, which that step only read
    const bool pipe = norm_in_first_step(Dr);
    const double* bterm = solve_prologue(Dr, f, u, pipe);
    HIP_OK(hipEventRecord(X->ev_pro, ws));
    // cycle k reads its residual back into buffer k mod 2 and records event
    // k mod 2; while the host checks cycle k, cycle k + 1 may already run
    // (enqueued only when cycle k cannot end the solve), which hides the
    // host's round trip without running a cycle more than a synchronous
    // loop would.  The first cycle is queued before the reference norm is
    // read (it is needed only for the first check).
    double* nb[2] = {X->norm_host, X->norm_host2};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    if (X->opt.use_graph)
      for (int k = 0; k < 2; ++k) exec[k] = cycle_graph(Dr, u, f, bterm, nb[k], pipe);
    if (rep) std::memset(rep, 0, sizeof(*rep));
    int launched = 0, done = 0;
    auto launch = [&]() {
      const int k = launched++ & 1;
      if (exec[k])
        HIP_OK(hipGraphLaunch(exec[k], ws));
      else if (pipe)
        solve_cycle_pipe(Dr, u, f, bterm, nb[k]);
      else
        solve_cycle(Dr, u, f, bterm, nb[k]);
      HIP_OK(hipEventRecord(X->ev_cyc[k], ws));
    };
    launch();
    HIP_OK(hipEventSynchronize(X->ev_pro));
    Monitor mon;
    DevLevel& L0 = X->lv[0];
    const int np = pipe ? Dr.fused_parts(L0) : Dr.norm_parts(L0);
    const int np0 = (pipe && !X->opt.use_initial_guess) ? Dr.fused_parts(L0) : Dr.norm_parts(L0);
    if (!mon.start(X, nrhs, np, np0)) {
      HIP_OK(hipStreamSynchronize(ws));
      HIP_OK(hipEventRecord(X->ev_out, ws));
      HIP_OK(hipStreamWaitEvent(X->stream, X->ev_out, 0));
      throw ccg::Error(CCGMG_EINVAL, "non-finite right-hand side or boundary data");
    }
    for (;;) {
      if (launched == done + 1 && mon.next_not_final(X)) launch();
      HIP_OK(hipEventSynchronize(X->ev_cyc[done & 1]));
      const bool fin = mon.step(X, rep, nb[done & 1]);
      ++done;
      if (launched > done) continue;   // a later cycle already ran: its check decides
      if (fin) break;
      launch();
    }
    HIP_OK(hipEventRecord(X->ev_t1, ws));
    HIP_OK(hipEventRecord(X->ev_out, ws));
    HIP_OK(hipStreamWaitEvent(X->stream, X->ev_out, 0));
    HIP_OK(hipEventSynchronize(X->ev_t1));
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, X->ev_t0, X->ev_t1));
    if (rep) {
      rep->cycles = mon.cycles;
      rep->outer_iters = X->opt.precision == 1 ? mon.cycles : 0;
      rep->rel_res_inf = mon.rel;
      rep->rel_res_2 = mon.rel2;
      rep->seconds = ms * 1e-3;
    }
    if (!mon.converged) throw ccg::Error(CCGMG_ENOCONV, "tolerance not reached");
  });
}

// A solve from zero with the current schedule and depth, timed as the
// solves run (graph replay; a first call captures the graph).  f: the
// right-hand side (device, one plane), or nullptr for a seeded N(0,1)
// right-hand side on the non-empty cells without boundary term.  Returns
// the geometric-mean contraction per cycle (1e300 if tol > 0 is not
// reached); *seconds: device time; *score: time per cycle x cycles per
// 1e10 at the asymptotic rate (the cycles after the first two).
double timed_solve(ccgmg_ctx* X, const double* f, double tol, int max_cycles, double* seconds,
                   bool keep_graphs = false, double* score = nullptr) {
  DevLevel& L0 = X->lv[0];
  double* ud = L0.u;   // level-0 scratch buffers (level 0 of a solve uses the caller's arrays)
  const double* rd = f;
  int g_saved = X->g_nrhs;
  if (!f) {
    // drawn once per context (the draw takes longer than the solves)
    if (!X->tune_rhs) {
      std::vector<double> r(L0.n, 0.0);
      std::mt19937_64 gen(12345);
      std::normal_distribution<double> nd(0.0, 1.0);
      const ccg::Discretization& D = X->H.disc[0];
      for (size_t k = 0; k < L0.n; ++k) r[k] = D.nonempty[k] ? nd(gen) : 0.0;
      X->tune_rhs = upload(r, X->owned);
    }
    rd = X->tune_rhs;
    X->g_nrhs = 0;
  }
  ccgmg_options saved = X->opt;
  X->opt.max_cycles = max_cycles;
  X->opt.tol = tol;
  X->opt.use_initial_guess = 0;
  X->opt.precision = 0;
  X->opt.use_graph = 1;   // timed as the solves will run: graph replays
  ccgmg_report rep;
  solve_impl(X, rd, ud, 1, &rep, false);
  X->opt = saved;
  X->g_nrhs = g_saved;
  if (!keep_graphs) X->clear_graphs();
  if (seconds) *seconds = rep.seconds;
  double last = rep.cycles > 0 ? rep.history[std::min(rep.cycles, 64) - 1] : 1.0;
  if (score) {
    const int nc = std::min(rep.cycles, 64);
    double tail = 1.0;
    if (nc >= 4) tail = std::pow(rep.history[nc - 1] / rep.history[1], 1.0 / (nc - 2));
    *score = (tail > 0.0 && tail < 1.0) ? rep.seconds / rep.cycles * std::log(1e-10) / std::log(tail) : 1e300;
  }
  if (tol > 0.0 && !(rep.rel_res_inf <= tol)) return 1e300;
  return (std::isfinite(last) && rep.cycles > 0) ? std::pow(last, 1.0 / rep.cycles) : 1e300;
}

// The SMO-1 weight omega of every level (omega / D of the regular rows; the
// graphs captured with the former value are dropped).
void set_omega(ccgmg_ctx* X, double omega) {
  X->opt.omega = omega;
  for (DevLevel& L : X->lv) {
    if (L.n == 0) continue;
    const double h2 = L.h * L.h;
    L.coef.omega_invD = omega / (-30.0 * (X->a + X->c) / (12.0 * h2));
  }
  X->clear_graphs();
}

// Measured choice of smoothing schedule and depth: every candidate schedule
// (with tune_schedule) at every admissible coarsest level (<= the dense
// inverse limit), solved three times (capture, then two timed replays, the
// faster counting), then the SMO-1 weight (see below).  With f == 0
// (set-up) the seeded random right-hand side is used and candidates are
// ranked by the asymptotic-rate estimate; with the caller's f they are
// ranked by the measured time of the solve itself.
void tune_schedule_depth(ccgmg_ctx* X, const double* f) {
  struct Sched {
    int fused, nu1, nu2, c1, c2;   // c1, c2: coarse-level steps (0: as nu1, nu2)
    int every;                     // SMO-2 in every step (1) or every s-th step from the last (s)
  };
  std::vector<Sched> cands;
  if (X->opt.tune_schedule)
    cands = {{0, 3, 3, 0, 0, 1}, {1, 3, 3, 0, 0, 1}, {1, 4, 4, 0, 0, 1}, {1, 5, 5, 0, 0, 1},
             {1, 4, 4, 2, 2, 1}, {1, 5, 5, 2, 2, 1}, {1, 5, 5, 3, 3, 1}, {1, 6, 6, 3, 3, 1},
             {1, 4, 4, 3, 4, 1}, {1, 4, 4, 2, 5, 1},   // fewer pre- than post-steps on the coarse levels
             // SMO-2 blocks in every second or third step only (the others are
             // plain SMO-1 sweeps at the sweep's cost)
             {1, 5, 5, 2, 5, 2}, {1, 4, 4, 2, 5, 3}, {1, 6, 6, 3, 4, 3}, {1, 5, 5, 3, 3, 2},
             // lighter schedules (with a tuned SMO-1 weight fewer steps may do)
             {1, 3, 3, 2, 3, 1}, {1, 3, 3, 2, 4, 3}, {1, 4, 4, 2, 4, 3}, {1, 3, 3, 2, 2, 1},
             {1, 2, 3, 2, 3, 1}, {1, 3, 3, 1, 3, 1}};
  else
    cands = {{X->opt.smoother_fused, X->opt.nu1, X->opt.nu2, X->opt.nu1_coarse, X->opt.nu2_coarse,
              X->opt.smo2_every_sweep}};
  const int Mmax = (int)X->H.disc.size() - 1;
  X->tune_ms.assign(Mmax + 1, -1.0);
  double best = 1e300;
  int bestM = X->M;
  Sched bestS = {X->opt.smoother_fused, X->opt.nu1, X->opt.nu2, X->opt.nu1_coarse, X->opt.nu2_coarse,
                 X->opt.smo2_every_sweep};
  // the current schedule at depth Mc: captured, then replayed twice, the
  // faster replay counting (the timing noise of one replay, a few per cent,
  // is as large as the differences between the best candidates); false if
  // it does not converge fast enough
  auto measure = [&](int Mc, double& cost) {
    X->M = Mc;
    upload_coarsest(X);
    double sec = 0, score = 0, sec2 = 0, score2 = 0;
    timed_solve(X, f, 1e-10, 60, &sec, true);   // captures the graph
    const double rate = timed_solve(X, f, 1e-10, 60, &sec, true, &score);
    timed_solve(X, f, 1e-10, 60, &sec2, false, &score2);
    cost = f ? std::min(sec, sec2) : std::min(score, score2);
    return rate <= X->opt.depth_max_rate;
  };
  auto search = [&]() {
    for (const Sched& sc : cands) {
      X->opt.smoother_fused = sc.fused, X->opt.nu1 = sc.nu1, X->opt.nu2 = sc.nu2;
      X->opt.nu1_coarse = sc.c1, X->opt.nu2_coarse = sc.c2, X->opt.smo2_every_sweep = sc.every;
      for (int Mc = Mmax; Mc >= 1; --Mc) {
        long nu = 0;
        for (uint8_t v : X->H.disc[Mc].nonempty) nu += v;
        if (nu > MAX_COARSE_UNKNOWNS) break;
        double cost = 0;
        const bool ok = measure(Mc, cost);
        if (ok && (X->tune_ms[Mc] < 0 || 1e3 * cost < X->tune_ms[Mc])) X->tune_ms[Mc] = 1e3 * cost;
        if (ok && cost < best) best = cost, bestM = Mc, bestS = sc;
      }
    }
    X->opt.smoother_fused = bestS.fused, X->opt.nu1 = bestS.nu1, X->opt.nu2 = bestS.nu2;
    X->opt.nu1_coarse = bestS.c1, X->opt.nu2_coarse = bestS.c2, X->opt.smo2_every_sweep = bestS.every;
  };
  search();
  if (X->opt.tune_schedule) {
    // the SMO-1 weight at the chosen schedule and depth (the paper's
    // experiments use 0.5; for the fourth-order stencil with b = 0 a Fourier
    // analysis of weighted Jacobi puts the best high-frequency damping near
    // 0.77, and above 2/2.13 = 0.94 the highest frequency grows, so such a
    // weight fails the rate check there), then the schedules again at the
    // chosen weight
    const double om0 = X->opt.omega;
    double bestOm = om0;
    for (double om : {0.5, 0.6, 0.7, 0.77, 0.85, 0.92, 1.0}) {
      if (om == om0) continue;
      set_omega(X, om);
      double cost = 0;
      if (measure(bestM, cost) && cost < best) best = cost, bestOm = om;
    }
    set_omega(X, bestOm);
    if (bestOm != om0) search();
  }
  X->M = bestM;
  upload_coarsest(X);
  X->clear_graphs();
}

// Many geometries in one captured launch: the V-cycles of all contexts of a
// batch are recorded into one hipGraph whose branches (forked streams) run
// concurrently; geometries are placed largest first onto the least-loaded
// branch.  Every
// replay advances every geometry by one cycle and reads back all residual
// norms; a geometry that has converged keeps cycling (its residual only
// shrinks) until all have finished.
struct BatchGraph {
  std::vector<const void*> key;   // f and u pointers and nrhs of every geometry
  hipGraphExec_t exec = nullptr;
};

}  // namespace

struct ccgmg_batch {
  std::vector<ccgmg_ctx*> ctx;
  // lockstep mode (nbranches == 0 at creation): one launch per V-cycle step
  // for all geometries
  bool lockstep = false;
  int nu = 4;
  int every = 1;                    // SMO-2 in every every-th step counted back from the last
  bool pair = false;                // consecutive plain steps as one two-sweep launch
  int* active_d = nullptr;          // per geometry: 1 while it still cycles
  int* active_h = nullptr;          // pinned copy
  double* part_d = nullptr;         // residual-norm partials of all geometries
  double* part_h = nullptr;         // pinned copy
  size_t part_cap = 0;
  std::vector<size_t> part_off;     // per geometry
  std::vector<void*> desc_bufs;     // descriptor tables of captured cycles
  hipStream_t caller = nullptr, main = nullptr;
  std::vector<hipStream_t> br;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;   // device time of a batch solve (created once)
  std::vector<hipEvent_t> ev_fork;   // [0]: fork, [1 + b]: join of branch b
  std::vector<BatchGraph> graphs;
  std::string err;
  void clear_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
    for (void* q : desc_bufs) (void)hipFree(q);
    desc_bufs.clear();
  }
};

namespace {

// ---------------------------------------------------------------------------
// Lockstep batch planner: walks one V-cycle of every geometry level by level
// (down: nu fused steps, restriction, coarsest solves of the geometries whose
// hierarchy ends there; up: nu fused steps, the first applying the coarse
// correction) and emits one batched launch per step with a descriptor per
// geometry taking part.
// ---------------------------------------------------------------------------
struct LRec {
  int kind;                       // 0 fused, 1 restrict, 2 coarse, 3 coarse (many RHS), 4 norm, 5 aux,
                                  // 6 two plain sweeps
  bool pro = false;
  int mode = 0;                   // aux mode
  BStarts st{};
  size_t off = 0, bytes = 0;      // descriptor table in the blob
  size_t smem = 0;
  int total = 0;                  // workgroups
  // many-RHS coarsest solve of one geometry
  ccgmg_ctx* X = nullptr;
  void* u = nullptr;
  const void* r = nullptr;
  int nr = 0;
};

struct Planner {
  std::vector<LRec> recs;
  std::vector<char> blob;
  template <typename D>
  void add(LRec rec, const std::vector<D>& ds, const std::vector<int>& wg) {
    if (ds.empty()) return;
    if ((int)ds.size() > BMAX) throw ccg::Error(CCGMG_EINVAL, "too many geometries in one batch");
    rec.st.n = (int)ds.size();
    rec.st.start[0] = 0;
    for (size_t k = 0; k < ds.size(); ++k) rec.st.start[k + 1] = rec.st.start[k] + wg[k];
    rec.total = rec.st.start[ds.size()];
    if (rec.total == 0) return;
    while (blob.size() % 64) blob.push_back(0);
    rec.off = blob.size();
    rec.bytes = sizeof(D) * ds.size();
    blob.resize(blob.size() + rec.bytes);
    std::memcpy(blob.data() + rec.off, ds.data(), rec.bytes);
    recs.push_back(rec);
  }
};

template <typename T>
T* lvbuf(DevLevel& L, int which) {   // 0 u, 1 v, 2 r in the precision T
  if constexpr (sizeof(T) == 8)
    return which == 0 ? (T*)L.u : which == 1 ? (T*)L.v : (T*)L.r;
  else
    return which == 0 ? (T*)L.u32 : which == 1 ? (T*)L.v32 : (T*)L.r32;
}

Smo2Args lock_smo2_args(DevLevel& L, int cur, const double* bterm) {
  Smo2Data& S = L.fwd.smo2;
  Smo2Args a;
  a.bterm = bterm;
  a.ecell = S.ecell, a.ecols = S.ecols, a.ew = S.ew;
  a.evals = S.evals, a.ersum = S.ersum;
  a.eidx = S.ext_idx, a.ebt = S.ebt, a.ext_ptr = S.ext_ptr, a.own_cnt = S.own_cnt;
  a.inv_off = S.inv_off, a.inv = S.inv, a.inv64 = S.inv64;
  a.c_in = S.cbuf[cur], a.c_out = S.cbuf[1 - cur];
  a.ns = S.ns, a.nbt = L.fwd.n;
  a.epar = S.epar, a.eqpar = S.eqpar;
  return a;
}

constexpr int LOCK_TY = 16;   // SMO-1 tile height of batched fused steps

// Whether step k (of nu, in a phase) of a lockstep batch has its SMO-2 part
// (the same rule as a single solve's with_smo2).
bool lock_smo2_step(const ccgmg_batch* B, int k) {
  return B->every >= 1 ? (B->nu - 1 - k) % B->every == 0 : k == B->nu - 1;
}

// One V-cycle in precision T on level-0 arrays (u0, v0, r0, bterm0) of every
// geometry; the result ends in u0 (an even number of steps per level).
template <typename T>
void plan_vcycle(ccgmg_batch* B, Planner& P, const std::vector<void*>& u0, const std::vector<void*>& v0,
                 const std::vector<const void*>& r0, const std::vector<const double*>& bterm0,
                 const std::vector<int>& planes) {
  const int G = (int)B->ctx.size();
  int Mmax = 0;
  for (auto* X : B->ctx) Mmax = std::max(Mmax, X->M);
  std::vector<std::vector<void*>> cur(G), oth(G);
  std::vector<std::vector<const void*>> rr(G);
  std::vector<std::vector<int>> cc(G);
  for (int g = 0; g < G; ++g) {
    ccgmg_ctx* X = B->ctx[g];
    cur[g].resize(X->M + 1), oth[g].resize(X->M + 1), rr[g].resize(X->M + 1), cc[g].assign(X->M + 1, 0);
    for (int m = 0; m <= X->M; ++m) {
      cur[g][m] = m == 0 ? u0[g] : (void*)lvbuf<T>(X->lv[m], 0);
      oth[g][m] = m == 0 ? v0[g] : (void*)lvbuf<T>(X->lv[m], 1);
      rr[g][m] = m == 0 ? r0[g] : (const void*)lvbuf<T>(X->lv[m], 2);
    }
  }
  // one step (blocks: with its SMO-2 part; a step without it writes the
  // block rows unchanged, s2bit = 0) or, sweeps2, two plain steps in one
  // two-sweep launch
  auto fused = [&](int m, bool pro, bool blocks, bool sweeps2) {
    std::vector<BFused> ds;
    std::vector<int> wg;
    for (int g = 0; g < G; ++g) {
      ccgmg_ctx* X = B->ctx[g];
      if (m >= X->M) continue;
      DevLevel& L = X->lv[m];
      BFused d{};
      d.u = cur[g][m], d.r = rr[g][m], d.out = oth[g][m], d.kind = L.kind, d.c = L.coef;
      d.plane = L.n;
      d.nx = L.nx, d.ny = L.ny, d.nbx = tiles_x(L.nx), d.ntiles = d.nbx * ((L.ny + LOCK_TY - 1) / LOCK_TY);
      d.nblk = blocks ? L.fwd.smo2.nblk : 0;
      d.regbit = F_JAC, d.s2bit = blocks ? F_S2 : 0, d.probit = F_REG;
      d.geo = g;
      d.a = lock_smo2_args(L, cc[g][m], m == 0 ? bterm0[g] : nullptr);
      if (pro) {
        DevLevel& C = X->lv[m + 1];
        d.e = cur[g][m + 1], d.ncx = C.nx, d.ncy = C.ny, d.cplane = C.n;
      }
      ds.push_back(d);
      wg.push_back((d.nblk + d.ntiles) * planes[g]);
      std::swap(cur[g][m], oth[g][m]);
      if (blocks && L.fwd.smo2.ns > 0) cc[g][m] ^= 1;
    }
    LRec rec{};
    rec.kind = sweeps2 ? 6 : 0, rec.pro = pro;
    P.add(rec, ds, wg);
  };
  // the nu steps of one phase on level m (up: the first applies the
  // coarse-grid correction and always has its SMO-2 part)
  auto phase = [&](int m, bool up) {
    for (int k = 0; k < B->nu; ++k) {
      const bool pro = up && k == 0;
      const bool blk = pro || lock_smo2_step(B, k);
      if (!blk && B->pair && k + 1 < B->nu && !lock_smo2_step(B, k + 1)) {
        fused(m, false, false, true);
        ++k;
      } else {
        fused(m, pro, blk, false);
      }
    }
  };
  for (int m = 0; m <= Mmax; ++m) {
    phase(m, false);
    std::vector<BRestrict> rs;
    std::vector<int> rw;
    std::vector<BCoarse> cs;
    std::vector<int> cw;
    for (int g = 0; g < G; ++g) {
      ccgmg_ctx* X = B->ctx[g];
      if (m < X->M) {
        DevLevel& L = X->lv[m];
        DevLevel& C = X->lv[m + 1];
        BRestrict d{};
        d.u = cur[g][m], d.r = rr[g][m], d.kind = L.kind;
        d.rc = lvbuf<T>(C, 2), d.uc = lvbuf<T>(C, 0), d.cc = C.fwd.smo2.cbuf[0];
        d.c = L.coef, d.plane = L.n, d.cplane = C.n;
        d.ncc = C.fwd.smo2.ns, d.nx = L.nx, d.ny = L.ny, d.nbx = tiles_x(L.nx), d.ncx = C.nx, d.ncy = C.ny;
        d.ntiles = d.nbx * ((L.ny + TY - 1) / TY);
        d.regbit = F_REG, d.geo = g;
        rs.push_back(d);
        rw.push_back(d.ntiles * planes[g]);
        cc[g][m + 1] = 0;
      } else if (m == X->M) {
        if (planes[g] > 4) {
          LRec rec{};
          rec.kind = 3, rec.X = X, rec.u = cur[g][m], rec.r = rr[g][m], rec.nr = planes[g];
          rec.total = 1;
          P.recs.push_back(rec);
        } else {
          BCoarse d{};
          d.u = cur[g][m], d.r = rr[g][m], d.cell = X->mcell, d.inv = X->minv, d.inv64 = X->minv64;
          d.plane = X->lv[m].n;
          d.nm = X->nm, d.nwg = (X->nm + 3) / 4, d.geo = g;
          cs.push_back(d);
          cw.push_back(d.nwg * planes[g]);
        }
      }
    }
    LRec r1{};
    r1.kind = 1;
    P.add(r1, rs, rw);
    LRec r2{};
    r2.kind = 2;
    for (auto& d : cs) r2.smem = std::max(r2.smem, sizeof(double) * (size_t)d.nm);
    P.add(r2, cs, cw);
  }
  for (int m = Mmax - 1; m >= 0; --m) phase(m, true);
}

template <typename T, bool CROSS>
void launch_recs(ccgmg_batch* B, const std::vector<LRec>& recs, const char* dblob, hipStream_t s) {
  for (const LRec& r : recs) {
    const void* d = dblob + r.off;
    const dim3 g(r.total), b(BLOCK);
    switch (r.kind) {
      case 0:
        if (r.pro)
          hipLaunchKernelGGL((k_fused_batched<T, CROSS, true, LOCK_TY>), g, b, 0, s, (const BFused*)d, r.st,
                             B->active_d);
        else
          hipLaunchKernelGGL((k_fused_batched<T, CROSS, false, LOCK_TY>), g, b, 0, s, (const BFused*)d, r.st,
                             B->active_d);
        break;
      case 1:
        hipLaunchKernelGGL((k_restrict_batched<T, CROSS>), g, b, 0, s, (const BRestrict*)d, r.st, B->active_d);
        break;
      case 6:
        hipLaunchKernelGGL((k_sweep2_batched<T, CROSS, LOCK_TY>), g, b, 0, s, (const BFused*)d, r.st, B->active_d);
        break;
      case 2:
        hipLaunchKernelGGL((k_coarse_batched<T>), g, b, r.smem, s, (const BCoarse*)d, r.st, B->active_d);
        break;
      case 3: {
        ccgmg_ctx* X = r.X;
        const int nm = X->nm;
        hipLaunchKernelGGL((k_coarse_gather<T>), dim3((nm + 255) / 256, r.nr), dim3(256), 0, s, (const T*)r.r,
                           X->mcell, X->mrg, nm, r.nr, X->lv[X->M].n);
        hipLaunchKernelGGL((k_coarse_multi<T>), dim3((nm + CM_ROWS - 1) / CM_ROWS, (r.nr + CM_RHS - 1) / CM_RHS), dim3(64 * CMW), 0, s, (T*)r.u,
                           X->mrg, X->mcell, X->minv, X->minv64, nm, r.nr, X->lv[X->M].n);
        break;
      }
      case 4:
        hipLaunchKernelGGL((k_resnorm_batched<CROSS>), g, b, 0, s, (const BNorm*)d, r.st, B->active_d);
        break;
      default:
        hipLaunchKernelGGL(k_aux_batched, g, b, 0, s, (const BAux*)d, r.st, B->active_d, r.mode);
        break;
    }
  }
}

int batch_guard(ccgmg_batch* B, const std::function<void()>& body) {
  if (!B) return CCGMG_EINVAL;
  try {
    body();
  } catch (const ccg::Error& e) {
    B->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    B->err = e.what();
    return CCGMG_EINVAL;
  }
  return CCGMG_OK;
}

// Residual-norm partials of one geometry's plane in a lockstep batch.
// Appends the SMO-1 weight of a context and, with schedule, its smoothing
// schedule to a graph-cache key (batch graphs capture both; ccgmg_tune may
// change them).
void push_tuning_key(std::vector<const void*>& key, const ccgmg_ctx* X, bool schedule) {
  uint64_t w;
  std::memcpy(&w, &X->opt.omega, sizeof(w));
  key.push_back((const void*)(uintptr_t)w);
  if (!schedule) return;
  const ccgmg_options& o = X->opt;
  for (int v : {o.smoother_fused, o.nu1, o.nu2, o.nu1_coarse, o.nu2_coarse, o.smo2_every_sweep})
    key.push_back((const void*)(intptr_t)v);
}

int lockstep_parts(ccgmg_ctx* X) {
  DevLevel& L0 = X->lv[0];
  return (L0.fwd.n + BLOCK - 1) / BLOCK + tiles_x(L0.nx) * ((L0.ny + TY - 1) / TY);
}

// Lockstep batch solve (see ccgmg_batch_create with nbranches == 0).
void lockstep_solve(ccgmg_batch* B, const double* const* f, double* const* u, const int* nrhs,
                    ccgmg_report* reps) {
  const int n = (int)B->ctx.size();
  const bool mp = B->ctx[0]->opt.precision == 1;
  bool cross = false;
  for (auto* X : B->ctx) cross = cross || X->b != 0.0;
  HIP_OK(hipEventRecord(B->ev_in, B->caller));
  HIP_OK(hipStreamWaitEvent(B->main, B->ev_in, 0));
  HIP_OK(hipEventRecord(B->ev_t0, B->main));
  std::vector<const double*> bterm(n);
  for (int g = 0; g < n; ++g) {
    Driver Dr{B->ctx[g], B->main, nrhs[g], false};
    bterm[g] = solve_prologue(Dr, f[g], u[g]);
  }
  // residual-norm partials of all geometries in one buffer (laid out for
  // max_nrhs planes each at batch creation)
  std::vector<int> nparts(n);
  for (int g = 0; g < n; ++g) nparts[g] = lockstep_parts(B->ctx[g]);
  const size_t total = B->part_cap;
  HIP_OK(hipStreamSynchronize(B->main));
  std::vector<Monitor> mon(n);
  for (int g = 0; g < n; ++g)
    if (!mon[g].start(B->ctx[g], nrhs[g], nparts[g]))
      throw ccg::Error(CCGMG_EINVAL, "non-finite right-hand side or boundary data for geometry " + std::to_string(g));
  // the captured cycle fixes the arrays, the right-hand-side counts,
  // whether each geometry has a boundary term, and each geometry's depth and
  // SMO-1 weight (ccgmg_tune may change both after a first batch solve)
  std::vector<const void*> key;
  for (int g = 0; g < n; ++g) {
    key.push_back(f[g]);
    key.push_back(u[g]);
    key.push_back((const void*)(intptr_t)nrhs[g]);
    key.push_back(bterm[g]);
    key.push_back((const void*)(intptr_t)B->ctx[g]->M);
    push_tuning_key(key, B->ctx[g], false);
  }
  hipGraphExec_t exec = nullptr;
  for (auto& gr : B->graphs)
    if (gr.key == key) exec = gr.exec;
  if (!exec) {
    Planner P;
    std::vector<int> planes(nrhs, nrhs + n);
    if (mp) {
      std::vector<BAux> zs;
      std::vector<int> zw;
      for (int g = 0; g < n; ++g) {
        DevLevel& L0 = B->ctx[g]->lv[0];
        BAux a{};
        a.u32 = L0.u32, a.cc = L0.fwd.smo2.cbuf[0], a.n = L0.n * nrhs[g], a.ncc = (size_t)L0.fwd.smo2.ns * nrhs[g];
        a.plane = L0.n, a.geo = g;
        zs.push_back(a);
        zw.push_back(BAUX_WG);
      }
      LRec r0{};
      r0.kind = 5, r0.mode = 0;
      P.add(r0, zs, zw);
      std::vector<void*> u0(n), v0(n);
      std::vector<const void*> rr(n);
      std::vector<const double*> bt(n, nullptr);
      for (int g = 0; g < n; ++g) {
        DevLevel& L0 = B->ctx[g]->lv[0];
        u0[g] = L0.u32, v0[g] = L0.v32, rr[g] = L0.r32;
      }
      plan_vcycle<float>(B, P, u0, v0, rr, bt, planes);
      std::vector<BAux> as;
      for (int g = 0; g < n; ++g) {
        BAux a = zs[g];
        a.u = u[g], a.kind = B->ctx[g]->lv[0].kind;
        as.push_back(a);
      }
      LRec r1{};
      r1.kind = 5, r1.mode = 1;
      P.add(r1, as, zw);
    } else {
      std::vector<void*> u0(n), v0(n);
      std::vector<const void*> rr(n);
      for (int g = 0; g < n; ++g) u0[g] = u[g], v0[g] = B->ctx[g]->lv[0].v, rr[g] = f[g];
      plan_vcycle<double>(B, P, u0, v0, rr, bterm, planes);
    }
    std::vector<BNorm> ns;
    std::vector<int> nw;
    for (int g = 0; g < n; ++g) {
      DevLevel& L0 = B->ctx[g]->lv[0];
      BNorm d{};
      d.u = u[g], d.r = f[g], d.kind = L0.kind, d.c = L0.coef, d.plane = L0.n;
      d.nx = L0.nx, d.ny = L0.ny, d.nbx = tiles_x(L0.nx), d.ntiles = d.nbx * ((L0.ny + TY - 1) / TY);
      d.nrb = (L0.fwd.n + BLOCK - 1) / BLOCK;
      d.bterm = bterm[g];
      d.cell = L0.fwd.cell, d.rp = L0.fwd.rp, d.cols = L0.fwd.cols, d.vals = L0.fwd.vals, d.rowsum = L0.fwd.rowsum;
      d.nrows = L0.fwd.n, d.res_out = mp ? L0.r32 : nullptr, d.partial = B->part_d + B->part_off[g];
      d.regbit = F_REG, d.geo = g;
      ns.push_back(d);
      nw.push_back(nparts[g] * nrhs[g]);
    }
    LRec rn{};
    rn.kind = 4;
    P.add(rn, ns, nw);
    void* dblob = nullptr;
    HIP_OK(hipMalloc(&dblob, std::max<size_t>(P.blob.size(), 64)));
    B->desc_bufs.push_back(dblob);
    HIP_OK(hipMemcpy(dblob, P.blob.data(), P.blob.size(), hipMemcpyHostToDevice));
    hipGraph_t graph;
    HIP_OK(hipStreamBeginCapture(B->main, hipStreamCaptureModeThreadLocal));
    if (mp) {
      if (cross)
        launch_recs<float, true>(B, P.recs, (const char*)dblob, B->main);
      else
        launch_recs<float, false>(B, P.recs, (const char*)dblob, B->main);
    } else {
      if (cross)
        launch_recs<double, true>(B, P.recs, (const char*)dblob, B->main);
      else
        launch_recs<double, false>(B, P.recs, (const char*)dblob, B->main);
    }
    HIP_OK(hipMemcpyAsync(B->part_h, B->part_d, sizeof(double) * total, hipMemcpyDeviceToHost, B->main));
    HIP_OK(hipStreamEndCapture(B->main, &graph));
    HIP_OK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    B->graphs.push_back({key, exec});
  }
  for (int g = 0; g < n; ++g) B->active_h[g] = 1;
  HIP_OK(hipMemcpyAsync(B->active_d, B->active_h, sizeof(int) * n, hipMemcpyHostToDevice, B->main));
  if (reps) std::memset(reps, 0, sizeof(ccgmg_report) * n);
  for (;;) {
    HIP_OK(hipGraphLaunch(exec, B->main));
    HIP_OK(hipStreamSynchronize(B->main));
    bool all = true, changed = false;
    for (int g = 0; g < n; ++g) {
      if (!mon[g].stopped && mon[g].step(B->ctx[g], reps ? &reps[g] : nullptr, B->part_h + B->part_off[g])) {
        B->active_h[g] = 0;
        changed = true;
      }
      all = all && mon[g].stopped;
    }
    if (all) break;
    if (changed) HIP_OK(hipMemcpyAsync(B->active_d, B->active_h, sizeof(int) * n, hipMemcpyHostToDevice, B->main));
  }
  HIP_OK(hipEventRecord(B->ev_t1, B->main));
  HIP_OK(hipEventRecord(B->ev_out, B->main));
  HIP_OK(hipStreamWaitEvent(B->caller, B->ev_out, 0));
  HIP_OK(hipEventSynchronize(B->ev_t1));
  float ms = 0;
  HIP_OK(hipEventElapsedTime(&ms, B->ev_t0, B->ev_t1));
  bool ok = true;
  for (int g = 0; g < n; ++g) {
    if (reps) {
      reps[g].cycles = mon[g].cycles;
      reps[g].outer_iters = mp ? mon[g].cycles : 0;
      reps[g].rel_res_inf = mon[g].rel;
      reps[g].rel_res_2 = mon[g].rel2;
      reps[g].seconds = ms * 1e-3;
    }
    ok = ok && mon[g].converged;
  }
  if (!ok) throw ccg::Error(CCGMG_ENOCONV, "tolerance not reached for every geometry");
}

// ---------------------------------------------------------------------------
// Tuning cache (options.tune_cache): the measured tile heights, schedule and
// depth of a context, kept per (GPU architecture, level sizes, precision,
// b != 0 and the options the measurement depends on) for the rest of the
// process and, when the environment variable CCGMG_TUNE_CACHE names a file,
// in that file (one "key<TAB>values" line per entry, read once, appended).
// ---------------------------------------------------------------------------
struct TuneEntry {
  std::vector<int> ty64, ty32, ty2_64, ty2_32;   // SMO-1 and two-sweep tile heights per level
  int fused = 0, nu1 = 0, nu2 = 0, c1 = 0, c2 = 0, M = 0, every = 1;
  int omega_milli = 500;                         // SMO-1 weight x 1000
};
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;
bool g_tune_loaded = false;

std::string tune_key(ccgmg_ctx* X) {
  hipDeviceProp_t p;
  HIP_OK(hipGetDeviceProperties(&p, X->device));
  const ccgmg_options& o = X->opt;
  std::string k = std::string(p.gcnArchName) + "|";
  for (const auto& D : X->H.disc) k += std::to_string(D.nx) + "x" + std::to_string(D.ny) + ",";
  char buf[256];
  std::snprintf(buf, sizeof(buf), "|prec%d|cross%d|nrhs%d|cycle%d|depth%d/%g|sched%d:%d,%d,%d,%d,%d|w%g|s2%d,%d,%d,%d,%d,%d|pro%d|inv%d",
                o.precision, X->b != 0.0 ? 1 : 0, o.max_nrhs, o.cycle, o.auto_depth, o.depth_max_rate,
                o.tune_schedule, o.smoother_fused, o.nu1, o.nu2, o.nu1_coarse, o.nu2_coarse, o.omega,
                o.smo2_every_sweep, o.smo2_iters, o.smo2_block, o.smo2_overlap, o.smo2_widen, o.tune_tiles,
                o.prolongation, o.inverse_fp32);
  return k + buf;
}

void tune_cache_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("CCGMG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return;
  char line[4096];
  while (std::fgets(line, sizeof(line), fp)) {
    char* tab = std::strchr(line, '\t');
    if (!tab) continue;
    *tab = 0;
    std::vector<int> v;
    for (char* q = tab + 1; *q;) {
      char* end = nullptr;
      const long x = std::strtol(q, &end, 10);
      if (end == q) break;
      v.push_back((int)x);
      q = end;
    }
    // values: nlev, ty64[nlev], ty32[nlev], fused, nu1, nu2, c1, c2, M, every,
    // ty2_64[nlev], ty2_32[nlev], omega x 1000 (lines of another layout are
    // skipped)
    if (v.empty() || v[0] < 1 || (int)v.size() != 1 + 4 * v[0] + 8) continue;
    TuneEntry e;
    const int nl = v[0];
    e.ty64.assign(v.begin() + 1, v.begin() + 1 + nl);
    e.ty32.assign(v.begin() + 1 + nl, v.begin() + 1 + 2 * nl);
    const int* t = v.data() + 1 + 2 * nl;
    e.fused = t[0], e.nu1 = t[1], e.nu2 = t[2], e.c1 = t[3], e.c2 = t[4], e.M = t[5], e.every = t[6];
    e.ty2_64.assign(v.begin() + 8 + 2 * nl, v.begin() + 8 + 3 * nl);
    e.ty2_32.assign(v.begin() + 8 + 3 * nl, v.begin() + 8 + 4 * nl);
    e.omega_milli = v[8 + 4 * nl];
    // a line whose values the launches could not take (a tile height the
    // kernels are not built for, a weight outside (0, 2), negative step
    // counts) is skipped like one of another layout: set-up then tunes anew
    auto tile_ok = [](const std::vector<int>& t) {
      for (int x : t)
        if (x != 8 && x != 16 && x != 32) return false;
      return true;
    };
    if (!tile_ok(e.ty64) || !tile_ok(e.ty32) || !tile_ok(e.ty2_64) || !tile_ok(e.ty2_32) || e.fused < 0 ||
        e.fused > 1 || e.nu1 < 0 || e.nu2 < 0 || e.c1 < 0 || e.c2 < 0 || e.every < 0 ||
        e.M < 0 || e.omega_milli <= 0 || e.omega_milli >= 2000)
      continue;
    g_tune[line] = e;
  }
  std::fclose(fp);
}

bool tune_cache_get(const std::string& key, TuneEntry& e) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_cache_load_locked();
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  e = it->second;
  return true;
}

void tune_cache_put(const std::string& key, const TuneEntry& e) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_cache_load_locked();
  g_tune[key] = e;
  const char* path = std::getenv("CCGMG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* fp = std::fopen(path, "a");
  if (!fp) return;
  std::string v = std::to_string(e.ty64.size());
  for (int t : e.ty64) v += " " + std::to_string(t);
  for (int t : e.ty32) v += " " + std::to_string(t);
  for (int t : {e.fused, e.nu1, e.nu2, e.c1, e.c2, e.M, e.every}) v += " " + std::to_string(t);
  for (int t : e.ty2_64) v += " " + std::to_string(t);
  for (int t : e.ty2_32) v += " " + std::to_string(t);
  v += " " + std::to_string(e.omega_milli);
  std::fprintf(fp, "%s\t%s\n", key.c_str(), v.c_str());
  std::fclose(fp);
}

// Host part of context creation: arguments checked, options taken, the
// hierarchy built on the host (threads: set-up threads, -1 = as the
// options say).
void create_host(ccgmg_ctx* X, const ccgmg_grid* grid, const ccgmg_curve* curves, int ncurves, double a, double b,
               double c, const ccgmg_options* opts, int threads) {
  if (!grid || !curves || ncurves <= 0 || grid->nx <= 0 || grid->ny <= 0 || !(grid->h > 0))
    throw ccg::Error(CCGMG_EINVAL, "invalid grid or curves");
  // the kernels address one plane of a level with signed 32-bit byte
  // offsets, including rows up to 40 beyond the grid (tile halos): keep
  // (ny + 64) * nx FP64 values below 2^31 bytes
  if ((uint64_t)grid->nx * ((uint64_t)grid->ny + 64) * sizeof(double) >= (1ull << 31))
    throw ccg::Error(CCGMG_EINVAL, "grid too large: (ny + 64) * nx FP64 cell values must stay below 2^31 bytes");
  if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(c))
    throw ccg::Error(CCGMG_EINVAL, "non-finite coefficient");
  if (b * b - 4.0 * a * c >= 0.0) throw ccg::Error(CCGMG_ENOTELLIPTIC, "b^2 - 4ac >= 0");
  if (opts)
    X->opt = *opts;
  else
    ccgmg_default_options(&X->opt);
  if (X->opt.max_nrhs < 1) X->opt.max_nrhs = 1;
  if (X->opt.smo2_block < 1 || X->opt.smo2_block > 64) throw ccg::Error(CCGMG_EINVAL, "smo2_block must be in 1..64");
  // weighted Jacobi reduces no error at omega <= 0, and from omega = 2 on
  // |1 - omega lambda/D| exceeds 1 at every mode with lambda/D > 1 (the
  // highest frequencies of the stencil)
  if (!(X->opt.omega > 0.0 && X->opt.omega < 2.0)) throw ccg::Error(CCGMG_EINVAL, "omega must be in (0, 2)");
  if (X->opt.nu1 < 0 || X->opt.nu2 < 0 || X->opt.smo2_iters < 1 || X->opt.smo2_overlap < 0 ||
      X->opt.smo2_widen < 0 || X->opt.smo2_widen > 4 || X->opt.inverse_fp32 < 0 || X->opt.inverse_fp32 > 1 ||
      X->opt.cycle < 0 || X->opt.cycle > 1)
    throw ccg::Error(CCGMG_EINVAL, "bad smoothing parameters");
  // Alg. 1 merges interface cells of volume <= theta h^2, a fraction of a
  // full cell; the weights of eq. weightDef are at least w_min, so the
  // centre row of a least-squares problem keeps a positive weight
  if (!(X->opt.theta >= 0.0 && X->opt.theta < 1.0)) throw ccg::Error(CCGMG_EINVAL, "theta must be in [0, 1)");
  if (!(X->opt.w_min > 0.0 && std::isfinite(X->opt.w_min))) throw ccg::Error(CCGMG_EINVAL, "w_min must be positive");
  if (X->opt.max_cycles < 1 || !(X->opt.tol >= 0.0)) throw ccg::Error(CCGMG_EINVAL, "max_cycles must be >= 1 and tol >= 0");
  if (X->opt.precision < 0 || X->opt.precision > 1 || X->opt.prolongation < 0 || X->opt.prolongation > 1 ||
      X->opt.smoother_fused < 0 || X->opt.smoother_fused > 1 || X->opt.auto_depth < 0 || X->opt.auto_depth > 2 ||
      X->opt.smo2_every_sweep < 0)
    throw ccg::Error(CCGMG_EINVAL, "precision, prolongation, smoother_fused, auto_depth or smo2_every_sweep out of range");
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
    if (cs[k].bc < 0 || cs[k].bc > 2) throw ccg::Error(CCGMG_EINVAL, "unknown boundary condition");
    if (cs[k].bc == 2) {
      cs[k].robin[0] = curves[k].robin[0], cs[k].robin[1] = curves[k].robin[1];
      if (!std::isfinite(cs[k].robin[0]) || !std::isfinite(cs[k].robin[1]) ||
          (cs[k].robin[0] == 0.0 && cs[k].robin[1] == 0.0))
        throw ccg::Error(CCGMG_EINVAL, "Robin coefficients must be finite and not both zero");
    }
    cs[k].index = k;
  }
  ccg::Options so;
  so.theta = X->opt.theta;
  so.w_min = X->opt.w_min;
  so.coarsest_min_n = std::max(2, X->opt.coarsest_min_n);
  so.max_levels = std::max(1, X->opt.max_levels);
  so.threads = threads >= 0 ? threads : X->opt.num_threads;
  X->H.build(cs, grid->nx, grid->ny, grid->x0, grid->y0, grid->h, a, b, c, so);
  for (double v : X->H.disc[0].cond) X->plg_max_cond = std::max(X->plg_max_cond, v);
  X->M = (int)X->H.disc.size() - 1;
}

// Device part of context creation on the current device: streams and
// events, the level data, boundary-data buffers, the coarsest inverse, and
// the measured choices of tile heights, schedule and depth.
void create_device(ccgmg_ctx* X) {
  X->stream = (hipStream_t)X->opt.hip_stream;
  HIP_OK(hipGetDevice(&X->device));
  X->scratch = scratch_on_current_device();
  HIP_OK(hipStreamCreateWithFlags(&X->ws, hipStreamNonBlocking));
  HIP_OK(hipEventCreateWithFlags(&X->ev_in, hipEventDisableTiming));
  HIP_OK(hipEventCreateWithFlags(&X->ev_out, hipEventDisableTiming));
  for (hipEvent_t& e : X->ev_cyc) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIP_OK(hipEventCreateWithFlags(&X->ev_pro, hipEventDisableTiming));
  HIP_OK(hipEventCreate(&X->ev_t0));
  HIP_OK(hipEventCreate(&X->ev_t1));
  const int maxr = X->opt.max_nrhs;
  X->lv.resize(X->H.disc.size());
  for (size_t m = 0; m < X->H.disc.size(); ++m) upload_level(X, (int)m, maxr);
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
  if (maxr > 1) X->mrg = dalloc<double>((size_t)MAX_COARSE_UNKNOWNS * maxr, X->owned);
  for (double** p : {&X->norm_host, &X->norm_host2, &X->norm_host0})
    HIP_OK(hipHostMalloc((void**)p,
                         2 * sizeof(double) *
                             std::max(X->lv[0].npart_reg + X->lv[0].npart_irr, X->lv[0].npart_fused) * maxr,
                         hipHostMallocDefault));
  // the coarsest level must be small enough for the dense inverse
  while (X->M > 0) {
    long nu = 0;
    for (uint8_t v : X->H.disc[X->M].nonempty) nu += v;
    if (nu <= MAX_COARSE_UNKNOWNS) break;
    throw ccg::Error(CCGMG_EINVAL, "coarsest level has too many unknowns; allow more levels");
  }
  if (X->opt.sweep_tile_rows) {
    const int ty = X->opt.sweep_tile_rows;
    if (ty != 8 && ty != 16 && ty != 32) throw ccg::Error(CCGMG_EINVAL, "sweep_tile_rows must be 0, 8, 16 or 32");
    for (DevLevel& L : X->lv) L.sweep_ty[0] = L.sweep_ty[1] = L.sweep2_ty[0] = L.sweep2_ty[1] = ty;
  }
  std::string key;
  TuneEntry cached;
  if (X->opt.tune_cache) {
    key = tune_key(X);
    auto fits = [&](int M) {   // the cached depth's coarsest level must suit the dense inverse here too
      if (M < 0 || M >= (int)X->lv.size()) return false;
      long nu = 0;
      for (uint8_t v : X->H.disc[M].nonempty) nu += v;
      return nu <= MAX_COARSE_UNKNOWNS;
    };
    if (tune_cache_get(key, cached) && cached.ty64.size() == X->lv.size() && cached.ty32.size() == X->lv.size() &&
        cached.ty2_64.size() == X->lv.size() && cached.ty2_32.size() == X->lv.size() && fits(cached.M)) {
      for (size_t m = 0; m < X->lv.size(); ++m) {
        X->lv[m].sweep_ty[0] = cached.ty64[m], X->lv[m].sweep_ty[1] = cached.ty32[m];
        X->lv[m].sweep2_ty[0] = cached.ty2_64[m], X->lv[m].sweep2_ty[1] = cached.ty2_32[m];
      }
      X->opt.smoother_fused = cached.fused, X->opt.nu1 = cached.nu1, X->opt.nu2 = cached.nu2;
      X->opt.nu1_coarse = cached.c1, X->opt.nu2_coarse = cached.c2, X->opt.smo2_every_sweep = cached.every;
      set_omega(X, cached.omega_milli / 1000.0);
      X->M = cached.M;
      upload_coarsest(X);
      return;
    }
  }
  upload_coarsest(X);
  if (!X->opt.sweep_tile_rows && X->opt.tune_tiles) tune_tiles(X);
  if (X->opt.auto_depth == 2 && X->M > 1) {
    tune_schedule_depth(X, nullptr);
  } else if (X->opt.auto_depth == 1 && X->M > 1) {
    for (;;) {
      const double rate = timed_solve(X, nullptr, 0.0, 6, nullptr);
      if (rate <= X->opt.depth_max_rate || X->M <= 1) break;
      long next = 0;
      for (uint8_t v : X->H.disc[X->M - 1].nonempty) next += v;
      if (next > MAX_COARSE_UNKNOWNS) break;
      X->M -= 1;
      upload_coarsest(X);
    }
    X->clear_graphs();
  }
  if (X->opt.tune_cache) {
    TuneEntry e;
    for (const DevLevel& L : X->lv) {
      e.ty64.push_back(L.sweep_ty[0]), e.ty32.push_back(L.sweep_ty[1]);
      e.ty2_64.push_back(L.sweep2_ty[0]), e.ty2_32.push_back(L.sweep2_ty[1]);
    }
    e.fused = X->opt.smoother_fused, e.nu1 = X->opt.nu1, e.nu2 = X->opt.nu2;
    e.c1 = X->opt.nu1_coarse, e.c2 = X->opt.nu2_coarse, e.M = X->M, e.every = X->opt.smo2_every_sweep;
    e.omega_milli = (int)std::lround(1000.0 * X->opt.omega);
    tune_cache_put(key, e);
  }
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
  o->inverse_fp32 = 1;
  o->host_only = 0;
  o->cycle = 0;
  o->tune_cache = 0;
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
    const double t0 = now();
    create_host(X.get(), grid, curves, ncurves, a, b, c, opts, -1);
    if (!X->host_only) create_device(X.get());
    X->setup_seconds = now() - t0;
  } catch (const ccg::Error& e) {
    g_create_error = e.what();
    ccgmg_destroy(X.release());
    return e.code;
  } catch (const std::bad_alloc&) {
    g_create_error = "out of host memory";
    ccgmg_destroy(X.release());
    return CCGMG_ENOMEM;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    ccgmg_destroy(X.release());
    return CCGMG_EINVAL;
  }
  *out = X.release();
  return CCGMG_OK;
}

int ccgmg_create_many(const ccgmg_problem* probs, int n, const ccgmg_options* opts, int host_threads,
                      ccgmg_ctx** out) {
  if (!out || !probs || n < 1) return CCGMG_EINVAL;
  g_create_error.clear();
  for (int k = 0; k < n; ++k) out[k] = nullptr;
  std::vector<std::unique_ptr<ccgmg_ctx>> X(n);
  for (auto& x : X) x.reset(new ccgmg_ctx());
  // host phase: geometries largest first (cells) onto a pool of workers,
  // each building with an equal share of the host threads; the calling
  // thread takes each finished geometry's device phase in that order
  int T = host_threads > 0 ? host_threads : (int)std::max(1u, std::thread::hardware_concurrency());
  const int W = std::max(1, std::min(n, std::max(1, T / 2)));
  const int per = std::max(1, T / W);
  std::vector<int> order(n);
  for (int k = 0; k < n; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int p, int q) {
    return (long)probs[p].grid.nx * probs[p].grid.ny > (long)probs[q].grid.nx * probs[q].grid.ny;
  });
  std::vector<int> status(n, 1);                // 1 pending, 0 built, < 0 failed
  std::vector<std::string> msg(n);
  std::vector<double> host_s(n, 0.0);
  std::mutex mu;
  std::condition_variable cv;
  std::atomic<int> next{0};
  std::atomic<bool> abort{false};
  auto worker = [&]() {
    for (;;) {
      const int slot = next.fetch_add(1);
      if (slot >= n) return;
      const int k = order[slot];
      int st = CCGMG_OK;
      std::string m;
      const double t0 = now();
      if (!abort.load()) {
        try {
          const ccgmg_problem& P = probs[k];
          create_host(X[k].get(), &P.grid, P.curves, P.ncurves, P.a, P.b, P.c, opts ? &opts[k] : nullptr, per);
        } catch (const ccg::Error& e) {
          st = e.code, m = e.what();
        } catch (const std::bad_alloc&) {
          st = CCGMG_ENOMEM, m = "out of host memory";
        } catch (const std::exception& e) {
          st = CCGMG_EINVAL, m = e.what();
        }
      } else {
        st = CCGMG_EINVAL, m = "not built: an earlier geometry failed";
      }
      {
        std::lock_guard<std::mutex> lock(mu);
        status[k] = st == CCGMG_OK ? 0 : st;
        msg[k] = m;
        host_s[k] = now() - t0;
      }
      cv.notify_all();
    }
  };
  std::vector<std::thread> pool;
  for (int w = 0; w < W; ++w) pool.emplace_back(worker);
  int code = CCGMG_OK;
  std::string err;
  for (int slot = 0; slot < n; ++slot) {
    const int k = order[slot];
    {
      std::unique_lock<std::mutex> lock(mu);
      cv.wait(lock, [&]() { return status[k] != 1; });
    }
    if (code != CCGMG_OK) continue;
    if (status[k] != 0) {
      code = status[k];
      err = "geometry " + std::to_string(k) + ": " + msg[k];
      abort.store(true);
      continue;
    }
    try {
      const double t0 = now();
      if (!X[k]->host_only) create_device(X[k].get());
      X[k]->setup_seconds = host_s[k] + (now() - t0);
    } catch (const ccg::Error& e) {
      code = e.code, err = "geometry " + std::to_string(k) + ": " + e.what();
    } catch (const std::exception& e) {
      code = CCGMG_EINVAL, err = "geometry " + std::to_string(k) + ": " + e.what();
    }
    if (code != CCGMG_OK) abort.store(true);
  }
  for (auto& t : pool) t.join();
  if (code != CCGMG_OK) {
    for (auto& x : X) ccgmg_destroy(x.release());
    g_create_error = err;
    return code;
  }
  for (int k = 0; k < n; ++k) out[k] = X[k].release();
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
  info->nu1_coarse = X->opt.nu1_coarse > 0 ? X->opt.nu1_coarse : X->opt.nu1;
  info->nu2_coarse = X->opt.nu2_coarse > 0 ? X->opt.nu2_coarse : X->opt.nu2;
  info->smo2_every_sweep = X->opt.smo2_every_sweep;
  info->omega = X->opt.omega;
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

int ccgmg_get_stencils(const ccgmg_ctx* X, int level, int32_t* rows, int32_t* cols, double* vals) {
  return ccgmg_get_irregular(X, level, rows, cols, vals, nullptr);
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

int ccgmg_residual_norms(ccgmg_ctx* X, const double* f, const double* u, int nrhs, double* rel_inf, double* rel_l2) {
  return guard(X, [&]() {
    if (!f || !u || nrhs < 1 || nrhs > X->opt.max_nrhs || (!rel_inf && !rel_l2))
      throw ccg::Error(CCGMG_EINVAL, "bad residual-norm arguments");
    DevLevel& L0 = X->lv[0];
    const DevRows& R = L0.fwd;
    hipStream_t ws = X->ws;
    HIP_OK(hipEventRecord(X->ev_in, X->stream));
    HIP_OK(hipStreamWaitEvent(ws, X->ev_in, 0));
    const double* bterm = nullptr;
    if (X->nfaces > 0 && X->g_nrhs >= nrhs && R.n > 0) {
      hipLaunchKernelGGL(k_bterm, dim3((R.n + 255) / 256, nrhs), dim3(256), 0, ws, X->g, X->fptr, X->fface, X->fval,
                         X->bterm, R.n, X->nfaces);
      bterm = X->bterm;
    }
    const int nbx = tiles_x(L0.nx);
    const int ntiles = nbx * ((L0.ny + TY - 1) / TY);
    const int nrb = (R.n + BLOCK - 1) / BLOCK;
    const int np = ntiles + nrb;
    const dim3 g(np, 1, nrhs);
    const size_t per = (size_t)2 * np * nrhs;   // (max, sum of squares) per workgroup and plane
    double* part = nullptr;
    HIP_OK(hipMalloc((void**)&part, sizeof(double) * 2 * per));
    std::unique_ptr<double, void (*)(double*)> hold(part, [](double* p) { (void)hipFree(p); });
    CoefT<double> c(L0.coef);
    for (int zero_u = 1; zero_u >= 0; --zero_u) {
      double* out = part + (zero_u ? 0 : per);
      if (L0.cross)
        hipLaunchKernelGGL((k_res_norms<true>), g, dim3(BLOCK), 0, ws, u, f, L0.kind, L0.nx, L0.ny, nbx, ntiles, c,
                           zero_u, bterm, R.cell, R.rp, R.cols, R.vals, R.rowsum, R.n, out);
      else
        hipLaunchKernelGGL((k_res_norms<false>), g, dim3(BLOCK), 0, ws, u, f, L0.kind, L0.nx, L0.ny, nbx, ntiles, c,
                           zero_u, bterm, R.cell, R.rp, R.cols, R.vals, R.rowsum, R.n, out);
    }
    HIP_OK(hipGetLastError());
    std::vector<double> h(2 * per);
    HIP_OK(hipMemcpyAsync(h.data(), part, sizeof(double) * 2 * per, hipMemcpyDeviceToHost, ws));
    HIP_OK(hipStreamSynchronize(ws));
    for (int z = 0; z < nrhs; ++z) {
      double m[2] = {0.0, 0.0}, q[2] = {0.0, 0.0};   // [reference, residual]
      for (int k = 0; k < 2; ++k)
        for (int b = 0; b < np; ++b) {
          const double* e = h.data() + k * per + 2 * ((size_t)z * np + b);
          m[k] = std::isnan(m[k]) ? m[k] : (std::isnan(e[0]) ? e[0] : std::max(m[k], e[0]));
          q[k] += e[1];
        }
      if (rel_inf) rel_inf[z] = m[1] / (m[0] > 0 ? m[0] : 1.0);
      if (rel_l2) rel_l2[z] = std::sqrt(q[1]) / (q[0] > 0 ? std::sqrt(q[0]) : 1.0);
    }
  });
}

// As ccgmg_residual_norms, with every intermediate in the device's static
// scratch array (X->scratch, found at set-up) and the totals reduced on the
// device: no device or host allocation on the way to a result.  Calls that
// overlap on one device share the array and race.
int ccgmg_residual_norms_noalloc(ccgmg_ctx* X, const double* f, const double* u, int nrhs, double* rel_inf,
                                 double* rel_l2) {
  if (!X) return CCGMG_EINVAL;
  try {
    if (X->host_only) throw ccg::Error(CCGMG_EINVAL, "context was created with host_only");
    if (!f || !u || nrhs < 1 || nrhs > X->opt.max_nrhs || (!rel_inf && !rel_l2))
      throw ccg::Error(CCGMG_EINVAL, "bad residual-norm arguments");
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev != X->device) throw ccg::Error(CCGMG_EINVAL, "the current device is not the context's device");
    DevLevel& L0 = X->lv[0];
    const DevRows& R = L0.fwd;
    const int nbx = tiles_x(L0.nx);
    const int ntiles = nbx * ((L0.ny + TY - 1) / TY);
    const int nrb = (R.n + BLOCK - 1) / BLOCK;
    const int np = ntiles + nrb;
    const size_t per = (size_t)2 * np * nrhs;   // (max, sum of squares) per workgroup and plane
    const size_t need = 2 * per + 4 * (size_t)nrhs;
    if (need > SCRATCH_DOUBLES)
      throw ccg::Error(CCGMG_EINVAL, "needs " + std::to_string(need * sizeof(double)) +
                                         " bytes of scratch; the static scratch holds " +
                                         std::to_string(SCRATCH_DOUBLES * sizeof(double)) + " (fewer planes fit)");
    double* part = X->scratch;
    double* tot = part + 2 * per;
    hipStream_t ws = X->ws;
    HIP_OK(hipEventRecord(X->ev_in, X->stream));
    HIP_OK(hipStreamWaitEvent(ws, X->ev_in, 0));
    const double* bterm = nullptr;
    if (X->nfaces > 0 && X->g_nrhs >= nrhs && R.n > 0) {
      hipLaunchKernelGGL(k_bterm, dim3((R.n + 255) / 256, nrhs), dim3(256), 0, ws, X->g, X->fptr, X->fface, X->fval,
                         X->bterm, R.n, X->nfaces);
      bterm = X->bterm;
    }
    const dim3 g(np, 1, nrhs);
    CoefT<double> c(L0.coef);
    for (int zero_u = 1; zero_u >= 0; --zero_u) {
      double* out = part + (zero_u ? 0 : per);
      if (L0.cross)
        hipLaunchKernelGGL((k_res_norms<true>), g, dim3(BLOCK), 0, ws, u, f, L0.kind, L0.nx, L0.ny, nbx, ntiles, c,
                           zero_u, bterm, R.cell, R.rp, R.cols, R.vals, R.rowsum, R.n, out);
      else
        hipLaunchKernelGGL((k_res_norms<false>), g, dim3(BLOCK), 0, ws, u, f, L0.kind, L0.nx, L0.ny, nbx, ntiles, c,
                           zero_u, bterm, R.cell, R.rp, R.cols, R.vals, R.rowsum, R.n, out);
    }
    hipLaunchKernelGGL(k_norm_finish, dim3(2, nrhs), dim3(BLOCK), 0, ws, part, per, np, tot);
    HIP_OK(hipGetLastError());
    // totals back in chunks of 64 planes through a stack buffer
    double hb[4 * 64];
    for (int z0 = 0; z0 < nrhs; z0 += 64) {
      const int cnt = std::min(64, nrhs - z0);
      HIP_OK(hipMemcpyAsync(hb, tot + 4 * (size_t)z0, sizeof(double) * 4 * cnt, hipMemcpyDeviceToHost, ws));
      HIP_OK(hipStreamSynchronize(ws));
      for (int k = 0; k < cnt; ++k) {
        const double* e = hb + 4 * k;   // reference max, sum; residual max, sum
        if (rel_inf) rel_inf[z0 + k] = e[2] / (e[0] > 0 ? e[0] : 1.0);
        if (rel_l2) rel_l2[z0 + k] = std::sqrt(e[3]) / (e[1] > 0 ? std::sqrt(e[1]) : 1.0);
      }
    }
  } catch (const ccg::Error& e) {
    X->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    X->err = e.what();
    return CCGMG_EINVAL;
  }
  return CCGMG_OK;
}

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

int ccgmg_tune(ccgmg_ctx* X, const double* f) {
  return guard(X, [&]() {
    if (!f) throw ccg::Error(CCGMG_EINVAL, "bad tune arguments");
    if (X->H.disc.size() < 2) return;
    tune_schedule_depth(X, f);
  });
}

int ccgmg_solve(ccgmg_ctx* X, const double* f, double* u, int nrhs, ccgmg_report* rep) {
  return solve_impl(X, f, u, nrhs, rep, false);
}

int ccgmg_batch_create(ccgmg_ctx* const* ctxs, int n, int nbranches, ccgmg_batch** out) {
  if (!out) return CCGMG_EINVAL;
  *out = nullptr;
  g_create_error.clear();
  std::unique_ptr<ccgmg_batch> B(new ccgmg_batch());
  try {
    if (!ctxs || n < 1 || nbranches < 0) throw ccg::Error(CCGMG_EINVAL, "invalid batch arguments");
    if (nbranches == 0 && n > BMAX) throw ccg::Error(CCGMG_EINVAL, "too many geometries for a lockstep batch");
    for (int g = 0; g < n; ++g) {
      if (!ctxs[g] || ctxs[g]->host_only) throw ccg::Error(CCGMG_EINVAL, "batch needs device contexts");
      for (int k = 0; k < g; ++k)
        if (ctxs[k] == ctxs[g]) throw ccg::Error(CCGMG_EINVAL, "a context appears twice in the batch");
    }
    B->ctx.assign(ctxs, ctxs + n);
    B->caller = ctxs[0]->stream;
    HIP_OK(hipStreamCreateWithFlags(&B->main, hipStreamNonBlocking));
    if (nbranches == 0) {
      // lockstep: one schedule for all (fused smoothing, nu steps before and
      // after on every level, piecewise-constant correction) and one precision
      B->lockstep = true;
      const ccgmg_options& o0 = ctxs[0]->opt;
      B->nu = (o0.smoother_fused && o0.nu1 == o0.nu2 && o0.nu1 > 0) ? o0.nu1 : 4;
      // the first context's SMO-2 schedule, where it keeps the cycle's
      // bookkeeping simple: an even number of SMO-2 passes per level (the
      // finest level's compact copy returns to where it started) and, for
      // two-sweep launches, as many of them going down as coming up (the
      // result returns to the first buffer); else SMO-2 in every step
      B->every = o0.smo2_every_sweep;
      int blk = 0, pd = 0, pu = 0;
      for (int up = 0; up < 2; ++up)
        for (int k = 0; k < B->nu; ++k) {
          const bool b1 = (up && k == 0) || lock_smo2_step(B.get(), k);
          blk += b1;
          if (!b1 && k + 1 < B->nu && !lock_smo2_step(B.get(), k + 1)) ++(up ? pu : pd), ++k;
        }
      if (blk % 2) B->every = 1;
      B->pair = B->every != 1 && pd == pu;
      for (int g = 0; g < n; ++g) {
        ccgmg_ctx* X = ctxs[g];
        if (X->opt.precision != o0.precision) throw ccg::Error(CCGMG_EINVAL, "lockstep batch needs one precision");
        X->opt.smoother_fused = 1, X->opt.nu1 = X->opt.nu2 = B->nu;
        X->opt.nu1_coarse = X->opt.nu2_coarse = 0, X->opt.prolongation = 0, X->opt.cycle = 0;
        X->clear_graphs();
      }
      HIP_OK(hipMalloc((void**)&B->active_d, sizeof(int) * n));
      // the partials of every geometry's residual checks, max_nrhs planes
      // each, so that a solve allocates nothing
      B->part_off.assign(n, 0);
      size_t total = 0;
      for (int g = 0; g < n; ++g) {
        B->part_off[g] = total;
        total += (size_t)2 * lockstep_parts(ctxs[g]) * ctxs[g]->opt.max_nrhs;
      }
      HIP_OK(hipMalloc((void**)&B->part_d, sizeof(double) * total));
      HIP_OK(hipHostMalloc((void**)&B->part_h, sizeof(double) * total, hipHostMallocDefault));
      B->part_cap = total;
      HIP_OK(hipHostMalloc((void**)&B->active_h, sizeof(int) * n, hipHostMallocDefault));
    }
    const int nb = std::min(n, std::max(1, nbranches));
    B->br.resize(nb);
    for (auto& st : B->br) HIP_OK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
    HIP_OK(hipEventCreate(&B->ev_t0));
    HIP_OK(hipEventCreate(&B->ev_t1));
    B->ev_fork.resize(1 + nb);
    for (auto& e : B->ev_fork) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  } catch (const ccg::Error& e) {
    g_create_error = e.what();
    ccgmg_batch_destroy(B.release());
    return e.code;
  }
  *out = B.release();
  return CCGMG_OK;
}

int ccgmg_batch_solve(ccgmg_batch* B, const double* const* f, double* const* u, const int* nrhs,
                      ccgmg_report* reps) {
  return batch_guard(B, [&]() {
    const int n = (int)B->ctx.size();
    if (!f || !u || !nrhs) throw ccg::Error(CCGMG_EINVAL, "bad batch solve arguments");
    for (int g = 0; g < n; ++g)
      if (!f[g] || !u[g] || nrhs[g] < 1 || nrhs[g] > B->ctx[g]->opt.max_nrhs)
        throw ccg::Error(CCGMG_EINVAL, "bad solve arguments for geometry " + std::to_string(g));
    if (B->lockstep) {
      lockstep_solve(B, f, u, nrhs, reps);
      return;
    }
    HIP_OK(hipEventRecord(B->ev_in, B->caller));
    HIP_OK(hipStreamWaitEvent(B->main, B->ev_in, 0));
    HIP_OK(hipEventRecord(B->ev_t0, B->main));
    std::vector<const double*> bterm(n);
    for (int g = 0; g < n; ++g) {
      Driver Dr{B->ctx[g], B->main, nrhs[g], false};
      bterm[g] = solve_prologue(Dr, f[g], u[g]);
    }
    HIP_OK(hipStreamSynchronize(B->main));
    std::vector<Monitor> mon(n);
    for (int g = 0; g < n; ++g) {
      Driver Dr{B->ctx[g], B->main, nrhs[g], false};
      if (!mon[g].start(B->ctx[g], nrhs[g], Dr.norm_parts(B->ctx[g]->lv[0])))
        throw ccg::Error(CCGMG_EINVAL, "non-finite right-hand side or boundary data for geometry " + std::to_string(g));
    }
    // longest-processing-time-first: geometries by decreasing work (cells x
    // right-hand sides), each onto the least-loaded branch
    const int nb = (int)B->br.size();
    std::vector<int> plan_order(n), plan_branch(n);
    {
      for (int g = 0; g < n; ++g) plan_order[g] = g;
      auto work = [&](int g) { return (double)B->ctx[g]->lv[0].n * nrhs[g]; };
      std::stable_sort(plan_order.begin(), plan_order.end(), [&](int x, int y) { return work(x) > work(y); });
      std::vector<double> load(nb, 0.0);
      for (int g : plan_order) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[b] += work(g);
        plan_branch[g] = b;
      }
    }
    std::vector<const void*> key;
    for (int g = 0; g < n; ++g) {
      key.push_back(f[g]);
      key.push_back(u[g]);
      key.push_back((const void*)(intptr_t)nrhs[g]);
      key.push_back((const void*)(intptr_t)(B->ctx[g]->opt.precision * 64 + B->ctx[g]->M));
      key.push_back(bterm[g]);
      push_tuning_key(key, B->ctx[g], true);
    }
    hipGraphExec_t exec = nullptr;
    for (auto& gr : B->graphs)
      if (gr.key == key) exec = gr.exec;
    if (!exec) {
      hipGraph_t graph;
      HIP_OK(hipStreamBeginCapture(B->main, hipStreamCaptureModeThreadLocal));
      HIP_OK(hipEventRecord(B->ev_fork[0], B->main));
      for (int b = 0; b < nb; ++b) HIP_OK(hipStreamWaitEvent(B->br[b], B->ev_fork[0], 0));
      for (int g : plan_order)
        if (true) {
          Driver Dr{B->ctx[g], B->br[plan_branch[g]], nrhs[g], false};
          solve_cycle(Dr, u[g], f[g], bterm[g]);
        }
      for (int b = 0; b < nb; ++b) {
        HIP_OK(hipEventRecord(B->ev_fork[1 + b], B->br[b]));
        HIP_OK(hipStreamWaitEvent(B->main, B->ev_fork[1 + b], 0));
      }
      HIP_OK(hipStreamEndCapture(B->main, &graph));
      HIP_OK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      (void)hipGraphDestroy(graph);
      if (B->graphs.size() >= 4) {
        (void)hipGraphExecDestroy(B->graphs.front().exec);
        B->graphs.erase(B->graphs.begin());
      }
      B->graphs.push_back({key, exec});
    }
    if (reps) std::memset(reps, 0, sizeof(ccgmg_report) * n);
    // while every geometry is active the whole batch cycle is one graph
    // launch; once some have finished, only the active geometries' own cycle
    // graphs are launched, on their branches
    std::vector<hipGraphExec_t> own(n, nullptr);
    bool all_active = true;
    for (;;) {
      if (all_active) {
        HIP_OK(hipGraphLaunch(exec, B->main));
      } else {
        HIP_OK(hipEventRecord(B->ev_fork[0], B->main));
        for (int b = 0; b < nb; ++b) HIP_OK(hipStreamWaitEvent(B->br[b], B->ev_fork[0], 0));
        for (int g : plan_order) {
          if (mon[g].stopped) continue;
          hipStream_t sb = B->br[plan_branch[g]];
          if (!own[g]) {
            Driver Dr{B->ctx[g], sb, nrhs[g], false};
            own[g] = cycle_graph(Dr, u[g], f[g], bterm[g]);
          }
          HIP_OK(hipGraphLaunch(own[g], sb));
        }
        for (int b = 0; b < nb; ++b) {
          HIP_OK(hipEventRecord(B->ev_fork[1 + b], B->br[b]));
          HIP_OK(hipStreamWaitEvent(B->main, B->ev_fork[1 + b], 0));
        }
      }
      HIP_OK(hipStreamSynchronize(B->main));
      bool all = true;
      for (int g = 0; g < n; ++g) {
        if (!mon[g].stopped && mon[g].step(B->ctx[g], reps ? &reps[g] : nullptr)) all_active = false;
        all = all && mon[g].stopped;
      }
      if (all) break;
    }
    HIP_OK(hipEventRecord(B->ev_t1, B->main));
    HIP_OK(hipEventRecord(B->ev_out, B->main));
    HIP_OK(hipStreamWaitEvent(B->caller, B->ev_out, 0));
    HIP_OK(hipEventSynchronize(B->ev_t1));
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, B->ev_t0, B->ev_t1));
    bool ok = true;
    for (int g = 0; g < n; ++g) {
      if (reps) {
        reps[g].cycles = mon[g].cycles;
        reps[g].outer_iters = B->ctx[g]->opt.precision == 1 ? mon[g].cycles : 0;
        reps[g].rel_res_inf = mon[g].rel;
        reps[g].rel_res_2 = mon[g].rel2;
        reps[g].seconds = ms * 1e-3;
      }
      ok = ok && mon[g].converged;
    }
    if (!ok) throw ccg::Error(CCGMG_ENOCONV, "tolerance not reached for every geometry");
  });
}

const char* ccgmg_batch_last_error(const ccgmg_batch* B) { return B ? B->err.c_str() : g_create_error.c_str(); }

void ccgmg_batch_destroy(ccgmg_batch* B) {
  if (!B) return;
  if (B->main) (void)hipStreamSynchronize(B->main);
  B->clear_graphs();
  if (B->active_d) (void)hipFree(B->active_d);
  if (B->active_h) (void)hipHostFree(B->active_h);
  if (B->part_d) (void)hipFree(B->part_d);
  if (B->part_h) (void)hipHostFree(B->part_h);
  for (auto st : B->br)
    if (st) (void)hipStreamDestroy(st);
  if (B->main) (void)hipStreamDestroy(B->main);
  for (auto e : B->ev_fork)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : {B->ev_in, B->ev_out, B->ev_t0, B->ev_t1})
    if (e) (void)hipEventDestroy(e);
  delete B;
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
    if (!avg_us || reps < 1 || level < 0 || level > X->M || kernel < 0 || kernel > 11)
      throw ccg::Error(CCGMG_EINVAL, "bad profile arguments");
    Driver Dr{X, X->stream, 1, false};
    DevLevel& L = X->lv[level];
    Dr.fill<double>(L.u, L.n, 1.0);
    Dr.fill<double>(L.r, L.n, 0.5);
    Dr.fill<double>(L.v, L.n, 0.0);
    Dr.fill<float>(L.u32, L.n, 1.0f);
    Dr.fill<float>(L.r32, L.n, 0.5f);
    DevLevel* C = level < X->M ? &X->lv[level + 1] : nullptr;
    if ((kernel == 1 || kernel == 2 || kernel == 9) && !C) throw ccg::Error(CCGMG_EINVAL, "no coarser level");
    if (kernel == 9) Dr.fill<double>(C->u, C->n, 0.25);
    if ((kernel == 10 || kernel == 11) && level != 0)
      throw ccg::Error(CCGMG_EINVAL, "the norm-taking step is a fused step of level 0");
    if (kernel == 4 && level != X->M) throw ccg::Error(CCGMG_EINVAL, "coarsest solve only on the coarsest level");
    auto launch = [&]() {
      switch (kernel) {
        case 0: Dr.sweep<double>(L, L.u, L.r, L.v); break;
        case 1: Dr.restrict_<double>(L, *C, L.u, L.r, C->r, C->u); break;
        case 2: Dr.prolong<double>(L, *C, L.u, C->u); break;
        case 3:   // the compact copies alternate between launches; settled after the loop
          if (L.fwd.smo2.ns > 0) Dr.smo2_pass<double>(L, L.u, L.r, nullptr);
          break;
        case 4: Dr.coarse<double>(L, L.u, L.r); break;
        case 7:
          Dr.fused_step<double>(L, L.u, L.r, L.v, nullptr);
          break;
        case 8: Dr.sweep2<double>(L, L.u, L.r, L.v); break;
        case 9:
          Dr.fused_step<double>(L, L.u, L.r, L.v, nullptr, C->u, C);
          break;
        case 10:
          Dr.fused_step<double>(L, L.u, L.r, L.v, nullptr, nullptr, nullptr, X->norm_host);
          break;
        case 11:
          Dr.fused_step<double>(L, L.u, L.r, L.v, nullptr, nullptr, nullptr, L.fpart);
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
    if (kernel == 3 || kernel == 7) Dr.settle_rows(L);
    HIP_OK(hipEventSynchronize(e1));
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_OK(hipStreamSynchronize(X->stream));
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
    for (hipEvent_t e : X->ev_cyc)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : {X->ev_pro, X->ev_t0, X->ev_t1})
      if (e) (void)hipEventDestroy(e);
    for (double* p : {X->norm_host, X->norm_host2, X->norm_host0})
      if (p) (void)hipHostFree(p);
  }
  delete X;
}

}  // extern "C"
