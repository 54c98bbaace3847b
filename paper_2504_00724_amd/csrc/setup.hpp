// Host-side construction of the cut-cell grid hierarchy: geometry and
// merging (Section 3.1, Alg. 1), classification (Section 3.2), poised
// lattices and least-squares weights (Sections 2.2-2.3, 3.3), Alg. 3
// ordering (Section 4.2) and the SMO-2 block data (Section 4.1).
#pragma once

#include <cmath>
#include <array>
#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

namespace ccg {

constexpr int DEG = 4;                    // moments / basis up to total degree 4
constexpr int NB = 15;                    // dim Pi_4 in 2-D
using Mom = std::array<double, 25>;       // m[a * 5 + b] = int X^a Y^b (scaled)

enum CurveKind { K_BOX = 0, K_CIRCLE = 1, K_ELLIPSE = 2, K_POLAR_SIN = 3, K_POLAR_COS = 4, K_POLYGON = 5 };
enum CellState : int8_t { S_EMPTY = 0, S_MERGED = 1, S_PURE = 2, S_CUT = 3 };
enum CellKind : int8_t { C_EMPTY = 0, C_MERGED = 1, C_REGULAR = 2, C_IRR_PURE = 3, C_IRR_CUT = 4 };

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

struct Curve {
  int kind = 0, inside = 0, bc = 0, index = 0;   // bc: 0 Dirichlet, 1 Neumann, 2 Robin
  double p[8] = {0};
  double robin[2] = {0, 0};                      // Robin: robin[0] u + robin[1] du/dn
  void point(double t, double& x, double& y) const;
  void deriv(double t, double& dx, double& dy) const;
  bool contains(double x, double y) const;
  std::vector<double> breakpoints() const;
};

// Robin rows: the least-squares column is N phi / s, s = |gamma1| + |gamma2| / h.
inline double robin_scale(const Curve& c, double h) { return std::fabs(c.robin[0]) + std::fabs(c.robin[1]) / h; }

struct Face {                 // one boundary curve's piece of a cell
  int curve = -1;
  double len = 0.0;
  Mom m{}, mx{}, my{};        // int X^aY^b ds, int X^aY^b n_x ds, int X^aY^b n_y ds
};

struct CellArc {              // a run of one curve inside one cell, domain on its left
  int curve = 0, sigma = 1;
  std::vector<std::pair<double, double>> pieces;  // parameter intervals (curve direction)
  double pin[2], pout[2];
  double s_in = 0, s_out = 0;
};

struct LoopItem {             // arc (index into the cell's arc list) or perimeter walk
  bool is_arc;
  int arc;
  double sa, sb;
};

struct Comp {                 // a connected component of a cut cell
  int own = -1;               // grid cell it was traced in
  Mom mom{};                  // area moments about the own cell centre
  double edge_len[4] = {0, 0, 0, 0};  // inside length per edge: bottom, right, top, left
  std::vector<Face> faces;    // sorted by curve
  std::vector<LoopItem> loop; // empty for a full square
  double volume() const { return mom[0]; }
};

struct ControlVolume {        // non-empty cell after merging (not a plain pure cell)
  std::vector<int> members;   // indices into Geometry::comps
  Mom mom{};                  // about the host cell centre
  std::vector<Face> faces;    // sorted by curve, moments about the host centre
};

struct Geometry {
  int nx = 0, ny = 0;
  double x0 = 0, y0 = 0, h = 0, theta = 0.3;
  int threads = 0;                  // host threads for the cut-cell pass (0: all)
  int q = 16;                 // Gauss-Legendre nodes per arc piece
  std::vector<Curve> curves;
  int box = -1;               // index of the box curve or -1
  std::unordered_map<int, std::vector<CellArc>> arcs;
  std::vector<Comp> comps;
  std::unordered_map<int, std::vector<int>> native_comps;
  std::vector<int8_t> native;   // 0 empty, 1 pure, 2 cut
  std::vector<int8_t> state;    // CellState
  std::vector<int32_t> host;
  std::vector<double> vol;      // units of h^2
  std::unordered_map<int, ControlVolume> cv;
  std::unordered_map<int, std::vector<Face>> pure_faces;

  void build(const std::vector<Curve>& cs, int nx_, int ny_, double x0_, double y0_, double h_,
             double theta_, int threads_ = 0);
  const Mom& moments(int idx) const;
  const std::vector<Face>& faces(int idx) const;
  bool on_border(int i, int j, int edge) const;
  Comp trace(int idx, const std::vector<LoopItem>& loop) const;
  bool in_domain(double x, double y) const;

 private:
  void validate();
  void intersect();
  void classify_native();
  void merge();
  std::vector<std::vector<LoopItem>> loops(int idx) const;
};

Mom square_moments();
Mom shift(const Mom& m, double d, double e);
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

struct Discretization {
  int nx = 0, ny = 0;
  double h = 0, a = 1, b = 0, c = 1, w_min = 0.5;
  const Geometry* g = nullptr;
  std::vector<int8_t> kind;     // CellKind
  std::vector<uint8_t> nonempty, regular;
  std::vector<int32_t> irr;     // increasing linear index
  std::vector<int32_t> irr_pos; // cell -> position in irr or -1
  std::vector<std::pair<int, int>> faces;  // (cell, curve)
  std::vector<int32_t> sten;    // irr.size() * 15
  std::vector<double> wts;      // irr.size() * 15, units 1/h^2
  std::vector<double> cond;
  std::vector<int32_t> fw_ptr;  // CSR over irregular rows into (fw_face, fw_val)
  std::vector<int32_t> fw_face;
  std::vector<double> fw_val;   // physical units
  std::vector<int32_t> order;   // Alg. 3: position -> irregular cell index (linear)
  std::vector<int32_t> block;   // Alg. 3: curve block of each position (-1 leftovers)
  double coef[5][5];            // regular stencil, coef[dy+2][dx+2], units 1/h^2
  double diag = 0;

  void build(const Geometry& geo, double a_, double b_, double c_, double w_min_, int threads);
  void alg3();
};

struct Options {
  double theta = 0.3, w_min = 0.5;
  int coarsest_min_n = 16, max_levels = 16, threads = 0;
};

struct Hierarchy {
  std::vector<Geometry> geo;
  std::vector<Discretization> disc;
  void build(const std::vector<Curve>& curves, int nx, int ny, double x0, double y0, double h,
             double a, double b, double c, const Options& opt);
};

// Rows of an operator that the V-cycle treats explicitly (everything but the
// constant-stencil rows): cell of each row, CSR columns/values, and the
// numbering used to cut the SMO-2 blocks (positions into `cell`).
struct RowSet {
  std::vector<int32_t> cell, rp, cols;
  std::vector<double> vals;
  std::vector<int32_t> order;
};

// Irregular rows of L in increasing cell index, numbered by Alg. 3.
void forward_rows(const Discretization& D, RowSet& out);

// Rows of L^T.  A cell keeps the regular (symmetric) stencil in L^T when its
// whole 5x5 box is regular and no irregular row references it; those cells
// are flagged in `adj_regular`.  Every other non-empty cell gets an explicit
// row: stencil coefficients of its regular neighbours' rows plus the
// weights of the irregular rows that reference it.  Rows are numbered by
// visiting the Alg. 3 order of the irregular cells and taking the still
// unnumbered rows within infinity-distance 4 (the lattice reach).
void transposed_rows(const Discretization& D, RowSet& out, std::vector<uint8_t>& adj_regular);

// Rows of the SMO-2 block solve: `base` plus the (regular-stencil) rows of
// every cell flagged in `stencil_mask` within infinity-distance `widen` of a
// base row.  `jacobi_mask` receives the stencil cells left to SMO-1.  The
// numbering visits the base rows in their order and takes the still
// unnumbered rows within distance max(widen, 1) of each.
void smoother_rows(const Discretization& D, const RowSet& base, const std::vector<uint8_t>& stencil_mask,
                   int widen, RowSet& out, std::vector<int32_t>& base_index, std::vector<uint8_t>& jacobi_mask);

int cell_quadrature(const Geometry& G, long* count, int32_t* cell_of, double* x, double* y, double* w);
int face_quadrature(const Geometry& G, const Discretization& D, long* count, int32_t* face_of, double* x, double* y,
                    double* w, double* nxo, double* nyo);

// Dense inverse (Gauss-Jordan with partial pivoting), row-major n x n, threads.
bool dense_inverse(std::vector<double>& A, int n, int threads);

void parallel_for(int n, int threads, const std::function<void(int, int)>& body);

}  // namespace ccg
