// Host set-up of the cut-cell hierarchy.  See setup.hpp.
//
// Geometry (Section 3.1): every analytic curve is cut at the parameters
// where x'(t) or y'(t) vanishes, so that each piece is monotone in both
// coordinates; grid-line crossings inside a piece are found by bisection.
// The resulting sub-arcs lie in single cells.  A cut cell's boundary is
// traced as loops (arc, then counter-clockwise along the cell perimeter to
// the next arc), each loop bounding one connected component.  Area and
// boundary moments come from Green's formula with the x-primitive (eq.
// volumeIntegral, eq. iteratedIntegral): vertical cell edges are integrated
// in closed form, arcs by Gauss-Legendre in the curve parameter.
//
// Merging (Alg. 1): extra components of a cell move to the edge neighbour
// sharing the longest edge stretch; then, in increasing linear index with
// live volumes, interface cells of volume <= theta h^2 merge into the
// non-empty edge neighbour with the longest common cut face (ties -x, +x,
// -y, +y; lengths within MERGE_TIE of each other tie, so that faces equal
// in exact arithmetic are not told apart by rounding).
//
// Lattices (R-PLG; the paper cites its PLG algorithm without stating it):
// principal-lattice images q + g(T0 - t) and line lattices (5 rows or
// columns holding 5, 4, 3, 2, 1 feasible cells picked nearest-first to q)
// inside the infinity-ball of radius 4, ranked by compactness; the 16 most
// compact are fitted; a fit is acceptable if its cell sample matrix has
// condition <= 1e8 and q's own weight is <= -(a+c)/2 (1/h^2 units); the
// acceptable fit of least W^{-1}-norm (the norm eq. derivedCoefAgain
// minimises) is taken.
#include "setup.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <numeric>
#include <set>
#include <thread>
#include <tuple>

namespace ccg {

static const double TWO_PI = 2.0 * M_PI;
static const int POLAR_SAMPLES = 8192;
static const double DEGENERATE_CHORD = 1e-10;
static const double PERIM_SNAP = 1e-9;
static const double EXTREMUM_REL = 1e-8;   // |x'| (|y'|) <= this * |c'|: x (y) is extremal there
static const double MERGE_TIE = 1e-12;     // cut-face lengths (units of h) this close tie in Alg. 1
static const int PLG_RADIUS = 4;
static const double COND_MAX = 1e8;
static const int PLG_POOL = 16;
static const double OWN_WEIGHT_MAX = -0.5;
static const double NORM_TIE = 1e-9;

static inline double pymod(double a, double b) {
  double r = std::fmod(a, b);
  if (r < 0) r += b;
  return r;
}

void parallel_for(int n, int threads, const std::function<void(int, int)>& body) {
  if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
  threads = std::min(threads, std::max(1, n));
  if (threads <= 1) {
    body(0, n);
    return;
  }
  std::vector<std::thread> pool;
  std::atomic<int> next(0);
  const int chunk = std::max(1, n / (threads * 8));
  std::vector<std::exception_ptr> errs(threads);
  for (int t = 0; t < threads; ++t) {
    pool.emplace_back([&, t]() {
      try {
        for (;;) {
          int s = next.fetch_add(chunk);
          if (s >= n) break;
          body(s, std::min(n, s + chunk));
        }
      } catch (...) {
        errs[t] = std::current_exception();
      }
    });
  }
  for (auto& th : pool) th.join();
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
}

// ---------------------------------------------------------------------------
// Gauss-Legendre nodes by Newton's method on P_n
// ---------------------------------------------------------------------------
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = pk;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[n - 1 - i] = z;           // ascending order
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// ---------------------------------------------------------------------------
// Curves
// ---------------------------------------------------------------------------
// Polygon (a convex quadrilateral, vertices counter-clockwise in p): edge k
// is traversed for t in [k pi/2, (k+1) pi/2), linearly.
static void polygon_edge(const double* p, double t, double& ax, double& ay, double& bx, double& by, double& s) {
  const double q = 0.5 * M_PI;
  const double tt = pymod(t, TWO_PI);
  const int k = std::min(3, std::max(0, (int)std::floor(tt / q)));
  s = tt / q - k;
  ax = p[2 * k], ay = p[2 * k + 1];
  bx = p[(2 * k + 2) % 8], by = p[(2 * k + 3) % 8];
}

void Curve::point(double t, double& x, double& y) const {
  switch (kind) {
    case K_POLYGON: {
      double ax, ay, bx, by, s;
      polygon_edge(p, t, ax, ay, bx, by, s);
      x = ax + s * (bx - ax);
      y = ay + s * (by - ay);
      return;
    }
    case K_CIRCLE:
      x = p[0] + p[2] * std::cos(t);
      y = p[1] + p[2] * std::sin(t);
      return;
    case K_ELLIPSE: {
      double u = p[2] * std::cos(t), v = p[3] * std::sin(t);
      double cr = std::cos(p[4]), sr = std::sin(p[4]);
      x = p[0] + cr * u - sr * v;
      y = p[1] + sr * u + cr * v;
      return;
    }
    default: {
      double r = p[2] + p[3] * (kind == K_POLAR_SIN ? std::sin(p[4] * t + p[5]) : std::cos(p[4] * t + p[5]));
      x = p[0] + r * std::cos(t);
      y = p[1] + r * std::sin(t);
    }
  }
}

void Curve::deriv(double t, double& dx, double& dy) const {
  switch (kind) {
    case K_POLYGON: {
      double ax, ay, bx, by, s;
      polygon_edge(p, t, ax, ay, bx, by, s);
      dx = (bx - ax) / (0.5 * M_PI);
      dy = (by - ay) / (0.5 * M_PI);
      return;
    }
    case K_CIRCLE:
      dx = -p[2] * std::sin(t);
      dy = p[2] * std::cos(t);
      return;
    case K_ELLIPSE: {
      double du = -p[2] * std::sin(t), dv = p[3] * std::cos(t);
      double cr = std::cos(p[4]), sr = std::sin(p[4]);
      dx = cr * du - sr * dv;
      dy = sr * du + cr * dv;
      return;
    }
    default: {
      double r, dr;
      if (kind == K_POLAR_SIN) {
        r = p[2] + p[3] * std::sin(p[4] * t + p[5]);
        dr = p[3] * p[4] * std::cos(p[4] * t + p[5]);
      } else {
        r = p[2] + p[3] * std::cos(p[4] * t + p[5]);
        dr = -p[3] * p[4] * std::sin(p[4] * t + p[5]);
      }
      double c = std::cos(t), s = std::sin(t);
      dx = dr * c - r * s;
      dy = dr * s + r * c;
    }
  }
}

bool Curve::contains(double x, double y) const {
  switch (kind) {
    case K_POLYGON: {
      for (int k = 0; k < 4; ++k) {
        const double ax = p[2 * k], ay = p[2 * k + 1], bx = p[(2 * k + 2) % 8], by = p[(2 * k + 3) % 8];
        if ((bx - ax) * (y - ay) - (by - ay) * (x - ax) <= 0.0) return false;
      }
      return true;
    }
    case K_CIRCLE: {
      double dx = x - p[0], dy = y - p[1];
      return dx * dx + dy * dy < p[2] * p[2];
    }
    case K_ELLIPSE: {
      double cr = std::cos(p[4]), sr = std::sin(p[4]);
      double dx = x - p[0], dy = y - p[1];
      double u = cr * dx + sr * dy, v = -sr * dx + cr * dy;
      double uu = u / p[2], vv = v / p[3];
      return uu * uu + vv * vv < 1.0;
    }
    default: {
      double dx = x - p[0], dy = y - p[1];
      double rho = std::hypot(dx, dy);
      double th = std::atan2(dy, dx);
      double r = p[2] + p[3] * (kind == K_POLAR_SIN ? std::sin(p[4] * th + p[5]) : std::cos(p[4] * th + p[5]));
      return rho < r;
    }
  }
}

static std::vector<double> dedupe_params(std::vector<double> ts) {
  std::sort(ts.begin(), ts.end());
  std::vector<double> out;
  for (double t : ts)
    if (out.empty() || t - out.back() > 1e-14) out.push_back(t);
  if (out.size() > 1 && out.front() + TWO_PI - out.back() <= 1e-14) out.pop_back();
  return out;
}

template <class F>
static double bisect_sign(F g, double lo, double hi) {
  double glo = g(lo);
  for (int it = 0; it < 100; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double gm = g(mid);
    if (gm == 0.0) return mid;
    if ((gm < 0.0) == (glo < 0.0)) {
      lo = mid;
      glo = gm;
    } else {
      hi = mid;
    }
  }
  return 0.5 * (lo + hi);
}

std::vector<double> Curve::breakpoints() const {
  if (kind == K_CIRCLE || kind == K_POLYGON) return {0.0, 0.5 * M_PI, M_PI, 1.5 * M_PI};   // polygon: its vertices
  std::vector<double> ts;
  if (kind == K_ELLIPSE) {
    double cr = std::cos(p[4]), sr = std::sin(p[4]);
    double tx = std::atan2(-p[3] * sr, p[2] * cr);
    double ty = std::atan2(p[3] * cr, p[2] * sr);
    for (double t : {tx, tx + M_PI, ty, ty + M_PI}) ts.push_back(pymod(t, TWO_PI));
    return dedupe_params(ts);
  }
  for (int comp = 0; comp < 2; ++comp) {
    auto g = [&](double t) {
      double dx, dy;
      deriv(t, dx, dy);
      return comp == 0 ? dx : dy;
    };
    double pt = 0.0, pv = g(0.0);
    for (int s = 1; s <= POLAR_SAMPLES; ++s) {
      double t = TWO_PI * s / POLAR_SAMPLES;
      double v = g(t);
      if (pv == 0.0)
        ts.push_back(pt);
      else if (pv * v < 0.0)
        ts.push_back(bisect_sign(g, pt, t));
      pt = t;
      pv = v;
    }
  }
  for (double& t : ts) t = pymod(t, TWO_PI);
  return dedupe_params(ts);
}

// ---------------------------------------------------------------------------
// Moments
// ---------------------------------------------------------------------------
Mom square_moments() {
  Mom m{};
  auto I = [](int a) { return (std::pow(0.5, a + 1) - std::pow(-0.5, a + 1)) / (a + 1); };
  for (int a = 0; a <= DEG; ++a)
    for (int b = 0; a + b <= DEG; ++b) m[a * 5 + b] = I(a) * I(b);
  return m;
}

static void shift_matrix(double d, double S[5][5]) {
  static const double C[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0}, {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};
  double pw[5] = {1, d, d * d, d * d * d, d * d * d * d};
  for (int a = 0; a < 5; ++a)
    for (int p = 0; p < 5; ++p) S[a][p] = p <= a ? C[a][p] * pw[a - p] : 0.0;
}

Mom shift(const Mom& m, double d, double e) {
  double Sx[5][5], Sy[5][5], T[5][5];
  shift_matrix(d, Sx);
  shift_matrix(e, Sy);
  for (int a = 0; a < 5; ++a)
    for (int q = 0; q < 5; ++q) {
      double s = 0;
      for (int p = 0; p <= a; ++p) s += Sx[a][p] * m[p * 5 + q];
      T[a][q] = s;
    }
  Mom out{};
  for (int a = 0; a < 5; ++a)
    for (int b = 0; a + b <= DEG; ++b) {
      double s = 0;
      for (int q = 0; q <= b; ++q) s += T[a][q] * Sy[b][q];
      out[a * 5 + b] = s;
    }
  return out;
}

static void add_shifted(Mom& acc, const Mom& m, double d, double e) {
  Mom s = shift(m, d, e);
  for (int k = 0; k < 25; ++k) acc[k] += s[k];
}

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
static double perimeter_coord(double X, double Y) {
  double d[4] = {std::fabs(Y), std::fabs(1.0 - X), std::fabs(1.0 - Y), std::fabs(X)};
  int e = 0;
  for (int k = 1; k < 4; ++k)
    if (d[k] < d[e]) e = k;
  auto cl = [](double v) { return std::min(1.0, std::max(0.0, v)); };
  double s;
  if (e == 0)
    s = cl(X);
  else if (e == 1)
    s = 1.0 + cl(Y);
  else if (e == 2)
    s = 2.0 + (1.0 - cl(X));
  else
    s = 3.0 + (1.0 - cl(Y));
  return pymod(s, 4.0);
}

bool Geometry::on_border(int i, int j, int edge) const {
  return (edge == 0 && j == 0) || (edge == 1 && i == nx - 1) || (edge == 2 && j == ny - 1) ||
         (edge == 3 && i == 0);
}

bool Geometry::in_domain(double x, double y) const {
  for (const Curve& c : curves) {
    if (c.kind == K_BOX) continue;
    bool ins = c.contains(x, y);
    if (c.inside && !ins) return false;
    if (!c.inside && ins) return false;
  }
  return true;
}

void Geometry::validate() {
  double xl = x0, yl = y0, xr = x0 + nx * h, yr = y0 + ny * h;
  int outer = 0;
  box = -1;
  for (const Curve& c : curves) {
    if (c.inside) ++outer;
    if (c.kind == K_BOX) {
      if (!c.inside) throw Error(-3, "a box must be the outer boundary");
      if (!(std::fabs(c.p[0] - xl) <= 1e-12 && std::fabs(c.p[1] - yl) <= 1e-12 &&
            std::fabs(c.p[2] - xr) <= 1e-12 && std::fabs(c.p[3] - yr) <= 1e-12))
        throw Error(-3, "the box must coincide with the grid extent");
      box = c.index;
    } else {
      if (c.kind < 0 || c.kind > 5) throw Error(-1, "unknown curve kind");
      if (c.kind == K_POLYGON) {
        // convex, counter-clockwise, no edge along a grid direction
        for (int k = 0; k < 4; ++k) {
          const double ax = c.p[2 * k], ay = c.p[2 * k + 1], bx = c.p[(2 * k + 2) % 8], by = c.p[(2 * k + 3) % 8];
          const double cx = c.p[(2 * k + 4) % 8], cy = c.p[(2 * k + 5) % 8];
          if ((bx - ax) * (cy - by) - (by - ay) * (cx - bx) <= 0.0)
            throw Error(-3, "a polygon must be a convex quadrilateral with counter-clockwise vertices");
          if (bx == ax || by == ay) throw Error(-3, "polygon edges must not be parallel to the grid lines");
        }
      }
      auto bp = c.breakpoints();
      double mnx = 1e300, mxx = -1e300, mny = 1e300, mxy = -1e300;
      for (double t : bp) {
        double x, y;
        c.point(t, x, y);
        mnx = std::min(mnx, x);
        mxx = std::max(mxx, x);
        mny = std::min(mny, y);
        mxy = std::max(mxy, y);
      }
      if (!(mnx > xl && mxx < xr && mny > yl && mxy < yr))
        throw Error(-3, "curve " + std::to_string(c.index) + " leaves the grid");
    }
  }
  if (outer > 1) throw Error(-3, "more than one outer boundary");
  if (outer == 0) throw Error(-3, "no outer boundary");
}

namespace {
struct Event {
  double t;
  double x, y;
};
struct Sub {
  int i, j;
  double ta, tb;
  double pa[2], pb[2];
};
}  // namespace

void Geometry::intersect() {
  arcs.clear();
  for (const Curve& c : curves) {
    if (c.kind == K_BOX) continue;
    std::vector<double> bps = c.breakpoints();
    std::vector<Event> ev;
    for (double tb : bps) {
      Event e;
      e.t = tb;
      c.point(tb, e.x, e.y);
      ev.push_back(e);
    }
    const int nb = (int)bps.size();
    for (int b = 0; b < nb; ++b) {
      double ta = bps[b], tb = b + 1 < nb ? bps[b + 1] : bps[0] + TWO_PI;
      double pa[2], pb[2], da[2], db[2];
      c.point(ta, pa[0], pa[1]);
      c.point(tb, pb[0], pb[1]);
      c.deriv(ta, da[0], da[1]);
      c.deriv(tb, db[0], db[1]);
      for (int comp = 0; comp < 2; ++comp) {
        double org = comp == 0 ? x0 : y0;
        double lo = std::min(pa[comp], pb[comp]), hi = std::max(pa[comp], pb[comp]);
        // ends where this coordinate is extremal: a grid line that close to
        // such an end is touched (tangency), not crossed
        const bool ext_a = std::fabs(da[comp]) <= EXTREMUM_REL * std::hypot(da[0], da[1]);
        const bool ext_b = std::fabs(db[comp]) <= EXTREMUM_REL * std::hypot(db[0], db[1]);
        long k0 = (long)std::floor((lo - org) / h), k1 = (long)std::ceil((hi - org) / h);
        for (long k = k0; k <= k1; ++k) {
          double xk = org + k * h;
          if (!(lo < xk && xk < hi)) continue;
          if ((ext_a && std::fabs(xk - pa[comp]) <= DEGENERATE_CHORD * h) ||
              (ext_b && std::fabs(xk - pb[comp]) <= DEGENERATE_CHORD * h))
            continue;
          auto fn = [&](double t) {
            double x, y;
            c.point(t, x, y);
            return (comp == 0 ? x : y) - xk;
          };
          double t = bisect_sign(fn, ta, tb);
          Event e;
          e.t = t;
          c.point(t, e.x, e.y);
          if (comp == 0)
            e.x = xk;
          else
            e.y = xk;
          ev.push_back(e);
        }
      }
    }
    std::stable_sort(ev.begin(), ev.end(), [](const Event& a, const Event& b) { return a.t < b.t; });
    Event first = ev[0];
    first.t += TWO_PI;
    ev.push_back(first);
    std::vector<Sub> subs;
    for (size_t e = 0; e + 1 < ev.size(); ++e) {
      const Event &A = ev[e], &B = ev[e + 1];
      if (std::hypot(B.x - A.x, B.y - A.y) <= DEGENERATE_CHORD * h) continue;
      double xm, ym;
      c.point(0.5 * (A.t + B.t), xm, ym);
      Sub s;
      s.i = (int)std::floor((xm - x0) / h);
      s.j = (int)std::floor((ym - y0) / h);
      s.ta = A.t;
      s.tb = B.t;
      s.pa[0] = A.x;
      s.pa[1] = A.y;
      s.pb[0] = B.x;
      s.pb[1] = B.y;
      subs.push_back(s);
    }
    if (subs.empty()) throw Error(-3, "degenerate curve");
    bool single = true;
    for (auto& s : subs)
      if (s.i != subs[0].i || s.j != subs[0].j) single = false;
    if (single) throw Error(-3, "curve " + std::to_string(c.index) + " lies inside a single cell");
    size_t start = 0;
    auto same = [](const Sub& a, const Sub& b) { return a.i == b.i && a.j == b.j; };
    while (same(subs[start], subs[(start + subs.size() - 1) % subs.size()])) ++start;
    std::rotate(subs.begin(), subs.begin() + start, subs.end());
    size_t r = 0;
    while (r < subs.size()) {
      size_t e = r;
      while (e + 1 < subs.size() && same(subs[e + 1], subs[r])) ++e;
      int i = subs[r].i, j = subs[r].j;
      if (i < 0 || i >= nx || j < 0 || j >= ny) throw Error(-3, "curve leaves the grid");
      CellArc arc;
      arc.curve = c.index;
      for (size_t k = r; k <= e; ++k) arc.pieces.push_back({subs[k].ta, subs[k].tb});
      const double* pf = subs[r].pa;
      const double* pl = subs[e].pb;
      if (c.inside) {
        arc.sigma = 1;
        arc.pin[0] = pf[0], arc.pin[1] = pf[1], arc.pout[0] = pl[0], arc.pout[1] = pl[1];
      } else {
        arc.sigma = -1;
        arc.pin[0] = pl[0], arc.pin[1] = pl[1], arc.pout[0] = pf[0], arc.pout[1] = pf[1];
      }
      double xi = x0 + i * h, yj = y0 + j * h;
      arc.s_in = perimeter_coord((arc.pin[0] - xi) / h, (arc.pin[1] - yj) / h);
      arc.s_out = perimeter_coord((arc.pout[0] - xi) / h, (arc.pout[1] - yj) / h);
      arcs[j * nx + i].push_back(arc);
      r = e + 1;
    }
  }
}

std::vector<std::vector<LoopItem>> Geometry::loops(int idx) const {
  const std::vector<CellArc>& A = arcs.at(idx);
  std::vector<int> ord(A.size());
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int x, int y) {
    return std::make_tuple(A[x].s_in, A[x].curve, A[x].pieces[0].first) <
           std::make_tuple(A[y].s_in, A[y].curve, A[y].pieces[0].first);
  });
  std::vector<char> used(A.size(), 0);
  std::vector<std::vector<LoopItem>> out;
  for (size_t st = 0; st < ord.size(); ++st) {
    if (used[st]) continue;
    std::vector<LoopItem> loop;
    size_t a = st;
    for (;;) {
      used[a] = 1;
      double so = A[ord[a]].s_out;
      size_t best = 0;
      double bd = -1;
      for (size_t b = 0; b < ord.size(); ++b) {
        double d = A[ord[b]].s_in - so;
        if (d < 0.0) d += 4.0;
        if (d > 4.0 - PERIM_SNAP) d = 0.0;
        if (bd < 0 || d < bd) {
          best = b;
          bd = d;
        }
      }
      loop.push_back({true, ord[a], 0, 0});
      loop.push_back({false, -1, so, so + bd});
      if (best == st) break;
      if (used[best]) throw Error(-3, "inconsistent boundary in cell " + std::to_string(idx));
      a = best;
    }
    out.push_back(loop);
  }
  return out;
}

static Face& face_of(std::vector<Face>& fs, int curve) {
  for (Face& f : fs)
    if (f.curve == curve) return f;
  fs.push_back(Face());
  fs.back().curve = curve;
  return fs.back();
}

static void segment_moments(Face& f, double P0x, double P0y, double P1x, double P1y, double nx_, double ny_) {
  double L = std::hypot(P1x - P0x, P1y - P0y);
  if (L <= 0.0) return;
  f.len += L;
  bool horizontal = P0y == P1y;
  for (int a = 0; a <= DEG; ++a)
    for (int b = 0; a + b <= DEG; ++b) {
      double v;
      if (horizontal) {
        double lo = std::min(P0x, P1x), hi = std::max(P0x, P1x);
        v = (std::pow(hi, a + 1) - std::pow(lo, a + 1)) / (a + 1) * std::pow(P0y, b);
      } else {
        double lo = std::min(P0y, P1y), hi = std::max(P0y, P1y);
        v = std::pow(P0x, a) * (std::pow(hi, b + 1) - std::pow(lo, b + 1)) / (b + 1);
      }
      f.m[a * 5 + b] += v;
      f.mx[a * 5 + b] += v * nx_;
      f.my[a * 5 + b] += v * ny_;
    }
}

// Perimeter path [sa, sb] split per edge: (e0, e1, edge) with edge-local coordinates.
static void split_perimeter(double sa, double sb, std::vector<std::tuple<double, double, int>>& out) {
  out.clear();
  double s = sa;
  while (s < sb) {
    double es = std::floor(s);
    double nxt = std::min(sb, es + 1.0);
    double e0 = s - es, e1 = nxt - es;
    if (e1 > e0) out.emplace_back(std::max(0.0, e0), std::min(1.0, e1), ((int)es % 4 + 4) % 4);
    s = nxt;
  }
}

Comp Geometry::trace(int idx, const std::vector<LoopItem>& loop) const {
  Comp comp;
  comp.own = idx;
  comp.loop = loop;
  const int i = idx % nx, j = idx / nx;
  const double cx = x0 + (i + 0.5) * h, cy = y0 + (j + 0.5) * h;
  std::vector<double> tq, wq;
  gauss_legendre(q, tq, wq);
  std::vector<std::tuple<double, double, int>> pieces;
  for (const LoopItem& it : loop) {
    if (it.is_arc) {
      const CellArc& arc = arcs.at(idx)[it.arc];
      const Curve& c = curves[arc.curve];
      Face& f = face_of(comp.faces, arc.curve);
      for (auto& pc : arc.pieces) {
        double half = 0.5 * (pc.second - pc.first), mid = 0.5 * (pc.first + pc.second);
        for (int qn = 0; qn < q; ++qn) {
          double t = mid + half * tq[qn], w = wq[qn] * half;
          double px, py, dx, dy;
          c.point(t, px, py);
          c.deriv(t, dx, dy);
          double X = (px - cx) / h, Y = (py - cy) / h;
          double dY = arc.sigma * dy / h;
          double speed = std::hypot(dx, dy) / h;
          double nxds = arc.sigma * dy / h, nyds = -arc.sigma * dx / h;
          f.len += w * speed;
          double Xp[6] = {1, X, X * X, X * X * X, X * X * X * X, X * X * X * X * X};
          double Yp[5] = {1, Y, Y * Y, Y * Y * Y, Y * Y * Y * Y};
          for (int a = 0; a <= DEG; ++a)
            for (int b = 0; a + b <= DEG; ++b) {
              comp.mom[a * 5 + b] += w * Xp[a + 1] / (a + 1) * Yp[b] * dY;
              f.m[a * 5 + b] += w * Xp[a] * Yp[b] * speed;
              f.mx[a * 5 + b] += w * Xp[a] * Yp[b] * nxds;
              f.my[a * 5 + b] += w * Xp[a] * Yp[b] * nyds;
            }
        }
      }
    } else {
      split_perimeter(it.sa, it.sb, pieces);
      for (auto& pc : pieces) {
        double e0 = std::get<0>(pc), e1 = std::get<1>(pc);
        int edge = std::get<2>(pc);
        comp.edge_len[edge] += e1 - e0;
        double P0x, P0y, P1x, P1y;
        if (edge == 0) {
          P0x = e0 - 0.5, P0y = -0.5, P1x = e1 - 0.5, P1y = -0.5;
        } else if (edge == 1) {
          P0x = 0.5, P0y = e0 - 0.5, P1x = 0.5, P1y = e1 - 0.5;
        } else if (edge == 2) {
          P0x = 0.5 - e0, P0y = 0.5, P1x = 0.5 - e1, P1y = 0.5;
        } else {
          P0x = -0.5, P0y = 0.5 - e0, P1x = -0.5, P1y = 0.5 - e1;
        }
        if (edge == 1 || edge == 3) {
          for (int a = 0; a <= DEG; ++a)
            for (int b = 0; a + b <= DEG; ++b)
              comp.mom[a * 5 + b] += std::pow(P0x, a + 1) / (a + 1) * (std::pow(P1y, b + 1) - std::pow(P0y, b + 1)) / (b + 1);
        }
        if (box >= 0 && on_border(i, j, edge)) {
          static const double NRM[4][2] = {{0, -1}, {1, 0}, {0, 1}, {-1, 0}};
          segment_moments(face_of(comp.faces, box), P0x, P0y, P1x, P1y, NRM[edge][0], NRM[edge][1]);
        }
      }
    }
  }
  std::sort(comp.faces.begin(), comp.faces.end(), [](const Face& x, const Face& y) { return x.curve < y.curve; });
  return comp;
}

void Geometry::classify_native() {
  native.assign((size_t)nx * ny, 0);
  std::vector<int> cut;
  for (auto& kv : arcs) cut.push_back(kv.first);
  std::sort(cut.begin(), cut.end());
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double x = x0 + (i + 0.5) * h, y = y0 + (j + 0.5) * h;
      native[(size_t)j * nx + i] = in_domain(x, y) ? 1 : 0;
    }
  comps.clear();
  native_comps.clear();
  std::vector<std::vector<Comp>> traced(cut.size());
  parallel_for((int)cut.size(), threads, [&](int s, int e) {
    for (int k = s; k < e; ++k) {
      for (auto& lp : loops(cut[k])) traced[k].push_back(trace(cut[k], lp));
    }
  });
  for (size_t k = 0; k < cut.size(); ++k) {
    int idx = cut[k];
    native[idx] = 2;
    for (Comp& cp : traced[k]) {
      if (cp.volume() <= 0.0) throw Error(-3, "non-positive component volume in cell " + std::to_string(idx));
      native_comps[idx].push_back((int)comps.size());
      comps.push_back(std::move(cp));
    }
  }
}

void Geometry::merge() {
  const size_t n = (size_t)nx * ny;
  vol.assign(n, 0.0);
  for (size_t k = 0; k < n; ++k) vol[k] = native[k] == 1 ? 1.0 : 0.0;
  std::map<int, std::vector<int>> members;
  auto neighbours = [&](int idx, int out[4][2]) {
    int i = idx % nx, j = idx / nx, m = 0;
    if (i > 0) out[m][0] = idx - 1, out[m][1] = 3, ++m;
    if (i < nx - 1) out[m][0] = idx + 1, out[m][1] = 1, ++m;
    if (j > 0) out[m][0] = idx - nx, out[m][1] = 0, ++m;
    if (j < ny - 1) out[m][0] = idx + nx, out[m][1] = 2, ++m;
    return m;
  };
  std::vector<int> cut;
  for (auto& kv : native_comps) cut.push_back(kv.first);
  std::sort(cut.begin(), cut.end());
  for (int idx : cut) {
    const std::vector<int>& cs = native_comps[idx];
    int keep = 0;
    for (size_t k = 1; k < cs.size(); ++k)
      if (comps[cs[k]].volume() > comps[cs[keep]].volume()) keep = (int)k;
    members[idx].push_back(cs[keep]);
    for (size_t k = 0; k < cs.size(); ++k) {
      if ((int)k == keep) continue;
      int nb[4][2];
      int m = neighbours(idx, nb);
      int best = -1;
      double bl = -1.0;
      for (int t = 0; t < m; ++t)
        if (comps[cs[k]].edge_len[nb[t][1]] > bl + MERGE_TIE) best = nb[t][0], bl = comps[cs[k]].edge_len[nb[t][1]];
      if (best < 0 || bl <= 0.0) throw Error(-3, "isolated component in cell " + std::to_string(idx));
      members[best].push_back(cs[k]);
    }
  }
  // pure cells that received components: their square goes first
  std::map<int, int> square_comp;
  auto square_of = [&](int idx) {
    auto it = square_comp.find(idx);
    if (it != square_comp.end()) return it->second;
    std::vector<LoopItem> lp{{false, -1, 0.0, 4.0}};
    comps.push_back(trace(idx, lp));
    comps.back().loop.clear();
    square_comp[idx] = (int)comps.size() - 1;
    return (int)comps.size() - 1;
  };
  for (auto& kv : members)
    if (native[kv.first] == 1) kv.second.insert(kv.second.begin(), square_of(kv.first));
  for (auto& kv : members) {
    double v = 0;
    for (int c : kv.second) v += comps[c].volume();
    vol[kv.first] = v;
  }
  host.assign(n, -1);
  // cells whose host is a given cell, so that re-pointing them when that
  // cell merges in turn touches only them
  std::unordered_map<int, std::vector<int>> hosted;
  auto aperture = [&](int idx, int edge) {
    if (native[idx] == 0) return 0.0;
    if (native[idx] == 1) return 1.0;
    double s = 0;
    for (int c : native_comps.at(idx)) s += comps[c].edge_len[edge];
    return s;
  };
  for (size_t idx = 0; idx < n; ++idx) {
    if (vol[idx] <= 0.0 || vol[idx] > theta) continue;
    if (native[idx] == 1 && !members.count((int)idx)) continue;
    int nb[4][2];
    int m = neighbours((int)idx, nb);
    int best = -1;
    double bl = 0.0;
    for (int t = 0; t < m; ++t) {
      if (vol[nb[t][0]] <= 0.0) continue;
      double ap = aperture((int)idx, nb[t][1]);
      if (ap > bl + MERGE_TIE) best = nb[t][0], bl = ap;   // a tie keeps the earlier of -x, +x, -y, +y
    }
    if (best < 0) throw Error(-3, "small cell " + std::to_string(idx) + " has no neighbour to merge into");
    if (!members.count(best)) members[best].push_back(square_of(best));
    auto it = members.find((int)idx);
    if (it != members.end()) {
      members[best].insert(members[best].end(), it->second.begin(), it->second.end());
      members.erase(it);
    }
    vol[best] += vol[idx];
    vol[idx] = 0.0;
    host[idx] = best;
    std::vector<int>& into = hosted[best];
    into.push_back((int)idx);
    auto hs = hosted.find((int)idx);
    if (hs != hosted.end()) {
      for (int k : hs->second) host[k] = best;
      into.insert(into.end(), hs->second.begin(), hs->second.end());
      hosted.erase(hs);
    }
  }
  state.assign(n, S_EMPTY);
  for (size_t k = 0; k < n; ++k) {
    if (vol[k] > 0.0)
      state[k] = (native[k] == 1 && !members.count((int)k)) ? S_PURE : S_CUT;
    else if (native[k] != 0)
      state[k] = S_MERGED;
  }
  cv.clear();
  for (auto& kv : members) {
    int idx = kv.first;
    if (vol[idx] <= 0.0) continue;
    ControlVolume c;
    c.members = kv.second;
    int i = idx % nx, j = idx / nx;
    for (int ci : kv.second) {
      const Comp& cp = comps[ci];
      double d = cp.own % nx - i, e = cp.own / nx - j;
      add_shifted(c.mom, cp.mom, d, e);
      for (const Face& f : cp.faces) {
        Face& g = face_of(c.faces, f.curve);
        g.len += f.len;
        add_shifted(g.m, f.m, d, e);
        add_shifted(g.mx, f.mx, d, e);
        add_shifted(g.my, f.my, d, e);
      }
    }
    std::sort(c.faces.begin(), c.faces.end(), [](const Face& x, const Face& y) { return x.curve < y.curve; });
    cv[idx] = std::move(c);
  }
  // pure border cells own their box edges
  pure_faces.clear();
  if (box >= 0) {
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        if (!(i == 0 || j == 0 || i == nx - 1 || j == ny - 1)) continue;
        int idx = j * nx + i;
        if (state[idx] != S_PURE) continue;
        std::vector<LoopItem> lp{{false, -1, 0.0, 4.0}};
        pure_faces[idx] = trace(idx, lp).faces;
      }
  }
}

void Geometry::build(const std::vector<Curve>& cs, int nx_, int ny_, double x0_, double y0_, double h_,
                     double theta_, int threads_) {
  curves = cs;
  for (size_t k = 0; k < curves.size(); ++k) curves[k].index = (int)k;
  nx = nx_, ny = ny_, x0 = x0_, y0 = y0_, h = h_, theta = theta_, threads = threads_;
  validate();
  intersect();
  classify_native();
  merge();
}

static const Mom SQUARE = square_moments();
static const std::vector<Face> NO_FACES;

const Mom& Geometry::moments(int idx) const {
  if (state[idx] == S_PURE) return SQUARE;
  return cv.at(idx).mom;
}

const std::vector<Face>& Geometry::faces(int idx) const {
  if (state[idx] == S_PURE) {
    auto it = pure_faces.find(idx);
    return it == pure_faces.end() ? NO_FACES : it->second;
  }
  return cv.at(idx).faces;
}

// ---------------------------------------------------------------------------
// Small dense linear algebra for the least-squares rows
// ---------------------------------------------------------------------------
// 2-norm condition number of an n x n matrix (column-major a[col*n+row]) by
// one-sided Jacobi rotations.
static double cond2(std::vector<double> a, int n) {
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double al = 0, be = 0, ga = 0;
        double* cp = &a[p * n];
        double* cq = &a[q * n];
        for (int i = 0; i < n; ++i) al += cp[i] * cp[i], be += cq[i] * cq[i], ga += cp[i] * cq[i];
        if (std::fabs(ga) <= 1e-15 * std::sqrt(al * be)) continue;
        rotated = true;
        double zeta = (be - al) / (2.0 * ga);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (int i = 0; i < n; ++i) {
          double x = cp[i], y = cq[i];
          cp[i] = cs * x - sn * y;
          cq[i] = sn * x + cs * y;
        }
      }
    if (!rotated) break;
  }
  double smax = 0, smin = 1e300;
  for (int p = 0; p < n; ++p) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += a[p * n + i] * a[p * n + i];
    s = std::sqrt(s);
    smax = std::max(smax, s);
    smin = std::min(smin, s);
  }
  return smin > 0 ? smax / smin : 1e300;
}

// beta = W M^T (M W M^T)^{-1} L with W^{-1} = diag(w): M is N x m (row-major
// M[j*m+k], N = 15 basis functions, m = 15 + faces).  Householder QR of
// A = W^{1/2} M^T (m x N), then beta = W^{1/2} Q R^{-T} L.
static void weighted_min_norm(const std::vector<double>& M, int m, const std::vector<double>& w,
                              const double* L, std::vector<double>& beta) {
  const int N = NB;
  std::vector<double> A((size_t)m * N);  // column-major A[col*m + row]
  std::vector<double> s(m);
  for (int k = 0; k < m; ++k) s[k] = 1.0 / std::sqrt(w[k]);
  for (int j = 0; j < N; ++j)
    for (int k = 0; k < m; ++k) A[(size_t)j * m + k] = s[k] * M[(size_t)j * m + k];
  std::vector<double> V((size_t)m * N, 0.0), tau(N, 0.0);
  for (int j = 0; j < N; ++j) {
    double* col = &A[(size_t)j * m];
    double nrm = 0;
    for (int i = j; i < m; ++i) nrm += col[i] * col[i];
    nrm = std::sqrt(nrm);
    double alpha = col[j] >= 0 ? -nrm : nrm;
    double* v = &V[(size_t)j * m];
    for (int i = 0; i < m; ++i) v[i] = 0;
    v[j] = col[j] - alpha;
    for (int i = j + 1; i < m; ++i) v[i] = col[i];
    double vn = 0;
    for (int i = j; i < m; ++i) vn += v[i] * v[i];
    tau[j] = vn > 0 ? 2.0 / vn : 0.0;
    for (int c2 = j; c2 < N; ++c2) {
      double* cc = &A[(size_t)c2 * m];
      double d = 0;
      for (int i = j; i < m; ++i) d += v[i] * cc[i];
      d *= tau[j];
      for (int i = j; i < m; ++i) cc[i] -= d * v[i];
    }
  }
  // R is the upper triangle of A (N x N); solve R^T y = L (forward substitution)
  std::vector<double> y(m, 0.0);
  for (int i = 0; i < N; ++i) {
    double t = L[i];
    for (int k = 0; k < i; ++k) t -= A[(size_t)i * m + k] * y[k];
    y[i] = t / A[(size_t)i * m + i];
  }
  // z = Q [y; 0] = H_0 H_1 ... H_{N-1} [y; 0]
  for (int j = N - 1; j >= 0; --j) {
    const double* v = &V[(size_t)j * m];
    double d = 0;
    for (int i = j; i < m; ++i) d += v[i] * y[i];
    d *= tau[j];
    for (int i = j; i < m; ++i) y[i] -= d * v[i];
  }
  beta.assign(m, 0.0);
  for (int k = 0; k < m; ++k) beta[k] = s[k] * y[k];
}

// ---------------------------------------------------------------------------
// Candidate lattices
// ---------------------------------------------------------------------------
namespace {
struct Offs {
  std::array<std::pair<int, int>, NB> o;
  int sumsq, maxinf;
};
struct LineAssign {
  int lines[5];
  int counts[5];
};
std::vector<Offs> principal_images() {
  std::vector<std::pair<int, int>> T0;
  for (int p1 = 0; p1 < 5; ++p1)
    for (int p2 = 0; p1 + p2 < 5; ++p2) T0.push_back({p1, p2});
  auto g = [](int gi, int x, int y) -> std::pair<int, int> {
    switch (gi) {
      case 0: return {x, y};
      case 1: return {-y, x};
      case 2: return {-x, -y};
      case 3: return {y, -x};
      case 4: return {-x, y};
      case 5: return {x, -y};
      case 6: return {y, x};
      default: return {-y, -x};
    }
  };
  std::vector<Offs> out;
  std::set<std::array<std::pair<int, int>, NB>> seen;
  for (int gi = 0; gi < 8; ++gi)
    for (auto& t : T0) {
      Offs o;
      for (int k = 0; k < NB; ++k) o.o[k] = g(gi, T0[k].first - t.first, T0[k].second - t.second);
      std::sort(o.o.begin(), o.o.end());
      if (!seen.insert(o.o).second) continue;
      o.sumsq = 0;
      o.maxinf = 0;
      for (auto& d : o.o) {
        o.sumsq += d.first * d.first + d.second * d.second;
        o.maxinf = std::max(o.maxinf, std::max(std::abs(d.first), std::abs(d.second)));
      }
      out.push_back(o);
    }
  return out;
}
std::vector<LineAssign> line_assignments() {
  std::vector<int> others;
  for (int d = -PLG_RADIUS; d <= PLG_RADIUS; ++d)
    if (d != 0) others.push_back(d);
  std::vector<LineAssign> out;
  const int no = (int)others.size();
  for (int a = 0; a < no; ++a)
    for (int b = a + 1; b < no; ++b)
      for (int c = b + 1; c < no; ++c)
        for (int d = c + 1; d < no; ++d) {
          int ls[5] = {0, others[a], others[b], others[c], others[d]};
          std::sort(ls, ls + 5);
          int perm[5] = {0, 1, 2, 3, 4};
          static const int VALS[5] = {5, 4, 3, 2, 1};
          do {
            LineAssign la;
            for (int k = 0; k < 5; ++k) la.lines[k] = ls[k], la.counts[k] = VALS[perm[k]];
            out.push_back(la);
          } while (std::next_permutation(perm, perm + 5));
        }
  return out;
}
const std::vector<Offs>& PRINCIPAL() {
  static const std::vector<Offs> v = principal_images();
  return v;
}
const std::vector<LineAssign>& LINES() {
  static const std::vector<LineAssign> v = line_assignments();
  return v;
}
}  // namespace

// ---------------------------------------------------------------------------
// Discretization of one level
// ---------------------------------------------------------------------------
namespace {
struct RowResult {
  std::vector<int32_t> cells;
  std::vector<double> beta;  // scaled: cells then faces
  double cond = 0;
  bool ok = false;
};

struct Fitter {
  const Geometry& g;
  const Discretization& D;
  std::map<std::pair<int, int>, std::array<double, NB>> pure_cache;  // key: 2*offsets

  Fitter(const Geometry& g_, const Discretization& D_) : g(g_), D(D_) {}

  static void basis_from(const Mom& m, double* out) {
    double vol = m[0];
    int k = 0;
    for (int d = 0; d <= DEG; ++d)
      for (int a = d; a >= 0; --a) out[k++] = m[a * 5 + (d - a)] / vol;
  }
  void basis_averages(int cell, double px, double py, double* out) {
    double d = cell % D.nx + 0.5 - px, e = cell / D.nx + 0.5 - py;
    if (g.state[cell] == S_PURE) {
      auto key = std::make_pair((int)std::lround(2 * d), (int)std::lround(2 * e));
      auto it = pure_cache.find(key);
      if (it == pure_cache.end()) {
        std::array<double, NB> v;
        basis_from(shift(SQUARE, d, e), v.data());
        it = pure_cache.emplace(key, v).first;
      }
      std::copy(it->second.begin(), it->second.end(), out);
      return;
    }
    basis_from(shift(g.moments(cell), d, e), out);
  }
  void operator_averages(int cell, double px, double py, double* out) {
    double d = cell % D.nx + 0.5 - px, e = cell / D.nx + 0.5 - py;
    Mom m = shift(g.moments(cell), d, e);
    double vol = m[0];
    int k = 0;
    for (int dg = 0; dg <= DEG; ++dg)
      for (int a1 = dg; a1 >= 0; --a1) {
        int a2 = dg - a1;
        double v = 0;
        if (a1 >= 2) v += D.a * a1 * (a1 - 1) * m[(a1 - 2) * 5 + a2];
        if (a1 >= 1 && a2 >= 1) v += D.b * a1 * a2 * m[(a1 - 1) * 5 + (a2 - 1)];
        if (a2 >= 2) v += D.c * a2 * (a2 - 1) * m[a1 * 5 + (a2 - 2)];
        out[k++] = v / vol;
      }
  }
  // Face average of N phi over a boundary face (the last column of the
  // least-squares system): phi itself (Dirichlet), its xi-gradient along the
  // outward normal (Neumann, h times du/dn), or (gamma1 phi + gamma2 dphi/dn)
  // / s with s = |gamma1| + |gamma2| / h (Robin: O(1), and the Dirichlet or
  // Neumann column when one coefficient is 0).
  void face_column(int cell, const Face& f, double px, double py, double* out) {
    double d = cell % D.nx + 0.5 - px, e = cell / D.nx + 0.5 - py;
    const Curve& cv = g.curves[f.curve];
    const double s = cv.bc == 2 ? robin_scale(cv, D.h) : 1.0;
    const double wd = cv.bc == 0 ? 1.0 : cv.bc == 2 ? cv.robin[0] / s : 0.0;          // weight of the value part
    const double wn = cv.bc == 1 ? 1.0 : cv.bc == 2 ? cv.robin[1] / D.h / s : 0.0;   // of the gradient part
    Mom m = shift(f.m, d, e), mx = shift(f.mx, d, e), my = shift(f.my, d, e);
    int k = 0;
    for (int dg = 0; dg <= DEG; ++dg)
      for (int a1 = dg; a1 >= 0; --a1) {
        int a2 = dg - a1;
        double v = 0;
        if (a1 >= 1) v += a1 * mx[(a1 - 1) * 5 + a2];
        if (a2 >= 1) v += a2 * my[a1 * 5 + (a2 - 1)];
        double val = 0.0;
        if (wd != 0.0) val += wd * (m[a1 * 5 + a2] / f.len);
        if (wn != 0.0) val += wn * (v / f.len);
        out[k++] = val;
      }
  }

  bool feasible(int i, int j) const {
    return i >= 0 && i < D.nx && j >= 0 && j < D.ny && D.nonempty[(size_t)j * D.nx + i];
  }

  std::vector<std::vector<int32_t>> pool(int q) {
    const int nx = D.nx, qi = q % nx, qj = q / nx, R = PLG_RADIUS;
    bool win[9][9];
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) win[dy + R][dx + R] = feasible(qi + dx, qj + dy);
    typedef std::tuple<int, int, int, int> Key;
    std::vector<std::pair<Key, std::vector<int32_t>>> ranked;
    const auto& P = PRINCIPAL();
    for (size_t e = 0; e < P.size(); ++e) {
      bool ok = true;
      for (auto& d : P[e].o)
        if (!win[d.second + R][d.first + R]) {
          ok = false;
          break;
        }
      if (!ok) continue;
      std::vector<int32_t> cells;
      for (auto& d : P[e].o) cells.push_back((qj + d.second) * nx + qi + d.first);
      std::sort(cells.begin(), cells.end());
      ranked.push_back({Key(P[e].sumsq, P[e].maxinf, 0, (int)e), cells});
    }
    // offsets along a line, nearest first (ties: negative side first);
    // initialised once, thread-safely, by the first row to get here
    static const std::array<int, 9> ALONG = []() {
      std::vector<int> al;
      for (int v = -PLG_RADIUS; v <= PLG_RADIUS; ++v) al.push_back(v);
      std::stable_sort(al.begin(), al.end(), [](int x, int y) {
        return std::make_pair(std::abs(x), x) < std::make_pair(std::abs(y), y);
      });
      std::array<int, 9> a{};
      for (int k = 0; k < 9; ++k) a[k] = al[k];
      return a;
    }();
    const auto& LA = LINES();
    for (int axis = 0; axis < 2; ++axis) {
      std::vector<std::pair<int, int32_t>> lines[9];  // (along, cell)
      int cost[9][6], reach[9][6], avail[9];
      for (int d = -R; d <= R; ++d) {
        auto& cl = lines[d + R];
        for (int k = 0; k < 9; ++k) {
          int t = ALONG[k];
          int dx = axis == 0 ? t : d, dy = axis == 0 ? d : t;
          if (win[dy + R][dx + R]) cl.push_back({t, (qj + dy) * nx + qi + dx});
        }
        avail[d + R] = (int)cl.size();
        cost[d + R][0] = 0;
        reach[d + R][0] = 0;
        for (int k = 1; k <= 5; ++k) {
          if (k <= (int)cl.size()) {
            int t = cl[k - 1].first;
            cost[d + R][k] = cost[d + R][k - 1] + t * t + d * d;
            reach[d + R][k] = std::max(reach[d + R][k - 1], std::max(std::abs(t), std::abs(d)));
          } else {
            cost[d + R][k] = 0;
            reach[d + R][k] = 0;
          }
        }
      }
      std::vector<std::tuple<int, int, int>> feas;  // (cost, max, e)
      feas.reserve(LA.size());
      for (size_t e = 0; e < LA.size(); ++e) {
        bool ok = true;
        int tot = 0, mx = 0;
        for (int k = 0; k < 5; ++k) {
          int li = LA[e].lines[k] + R, cn = LA[e].counts[k];
          if (avail[li] < cn) {
            ok = false;
            break;
          }
          tot += cost[li][cn];
          mx = std::max(mx, reach[li][cn]);
        }
        if (ok) feas.emplace_back(tot, mx, (int)e);
      }
      // only the best 3 * PLG_POOL in (cost, max, e) order are used: a
      // partial sort gives them in the same order as a full sort (the keys
      // are distinct through e)
      const size_t keep = std::min(feas.size(), (size_t)(3 * PLG_POOL));
      std::partial_sort(feas.begin(), feas.begin() + keep, feas.end());
      for (size_t f = 0; f < keep; ++f) {
        int e = std::get<2>(feas[f]);
        std::vector<int32_t> cells;
        for (int k = 0; k < 5; ++k) {
          auto& cl = lines[LA[e].lines[k] + R];
          for (int c = 0; c < LA[e].counts[k]; ++c) cells.push_back(cl[c].second);
        }
        std::sort(cells.begin(), cells.end());
        ranked.push_back({Key(std::get<0>(feas[f]), std::get<1>(feas[f]), 1 + axis, e), cells});
      }
    }
    std::stable_sort(ranked.begin(), ranked.end(),
                     [](const std::pair<Key, std::vector<int32_t>>& x, const std::pair<Key, std::vector<int32_t>>& y) {
                       return x.first < y.first;
                     });
    std::vector<std::vector<int32_t>> out;
    std::set<std::vector<int32_t>> seen;
    for (auto& r : ranked) {
      if (!seen.insert(r.second).second) continue;
      out.push_back(r.second);
      if ((int)out.size() == PLG_POOL) break;
    }
    return out;
  }

  // fit lattice `cells` for row q: scaled weights (cells then faces) and the
  // cell sample matrix (column-major, for its condition number)
  void fit(int q, const std::vector<int32_t>& cells, std::vector<double>& beta, std::vector<double>& w,
           std::vector<double>& colmaj) {
    const std::vector<Face>& fs = g.faces(q);
    const int nf = (int)fs.size(), m = NB + nf;
    int imin = 1 << 30, imax = -1, jmin = 1 << 30, jmax = -1;
    for (int c : cells) {
      imin = std::min(imin, c % D.nx), imax = std::max(imax, c % D.nx);
      jmin = std::min(jmin, c / D.nx), jmax = std::max(jmax, c / D.nx);
    }
    const double px = 0.5 * (imin + imax + 1), py = 0.5 * (jmin + jmax + 1);
    std::vector<double> M((size_t)NB * m);          // row-major M[j*m + k]
    colmaj.assign((size_t)NB * NB, 0.0);            // cell block, column-major
    double col[NB];
    for (int k = 0; k < NB; ++k) {
      basis_averages(cells[k], px, py, col);
      for (int j = 0; j < NB; ++j) M[(size_t)j * m + k] = col[j], colmaj[(size_t)k * NB + j] = col[j];
    }
    for (int f = 0; f < nf; ++f) {
      face_column(q, fs[f], px, py, col);
      for (int j = 0; j < NB; ++j) M[(size_t)j * m + NB + f] = col[j];
    }
    double L[NB];
    operator_averages(q, px, py, L);
    const int qi = q % D.nx, qj = q / D.nx;
    w.assign(m, D.w_min);
    for (int k = 0; k < NB; ++k)
      w[k] = std::max(std::hypot((double)(cells[k] % D.nx - qi), (double)(cells[k] / D.nx - qj)), D.w_min);
    weighted_min_norm(M, m, w, L, beta);
  }

  // The candidates in pool order; one replaces the current choice when it is
  // acceptable and its norm beats the choice's by the tie margin.  The
  // condition number (the costly part of acceptability) is computed only for
  // candidates that pass the other tests, so the choice is the same as with
  // every condition number computed.
  RowResult row(int q) {
    RowResult best;
    double best_norm = 0;
    const double bound = OWN_WEIGHT_MAX * (D.a + D.c);
    std::vector<double> beta, w, colmaj;
    for (auto& cells : pool(q)) {
      fit(q, cells, beta, w, colmaj);
      int qpos = (int)(std::find(cells.begin(), cells.end(), q) - cells.begin());
      if (beta[qpos] > bound) continue;
      double nrm = 0;
      for (size_t k = 0; k < beta.size(); ++k) nrm += w[k] * beta[k] * beta[k];
      if (best.ok && !(nrm < best_norm * (1.0 - NORM_TIE))) continue;
      const double cond = cond2(colmaj, NB);
      if (cond > COND_MAX) continue;
      best.ok = true;
      best_norm = nrm;
      best.cells = cells;
      best.beta = beta;
      best.cond = cond;
    }
    return best;
  }
};
}  // namespace

void Discretization::build(const Geometry& geo, double a_, double b_, double c_, double w_min_, int threads) {
  g = &geo;
  nx = geo.nx, ny = geo.ny, h = geo.h, a = a_, b = b_, c = c_, w_min = w_min_;
  const size_t n = (size_t)nx * ny;
  nonempty.assign(n, 0);
  regular.assign(n, 0);
  kind.assign(n, C_EMPTY);
  for (size_t k = 0; k < n; ++k) nonempty[k] = geo.state[k] == S_PURE || geo.state[k] == S_CUT;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t k = (size_t)j * nx + i;
      if (!nonempty[k]) {
        kind[k] = geo.state[k] == S_MERGED ? C_MERGED : C_EMPTY;
        continue;
      }
      bool reg = true;
      for (int dy = -2; dy <= 2 && reg; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
          int ii = i + dx, jj = j + dy;
          if (ii < 0 || jj < 0 || ii >= nx || jj >= ny || geo.state[(size_t)jj * nx + ii] != S_PURE) {
            reg = false;
            break;
          }
        }
      regular[k] = reg;
      kind[k] = reg ? C_REGULAR : (geo.state[k] == S_PURE ? C_IRR_PURE : C_IRR_CUT);
    }
  irr.clear();
  irr_pos.assign(n, -1);
  for (size_t k = 0; k < n; ++k)
    if (nonempty[k] && !regular[k]) {
      irr_pos[k] = (int32_t)irr.size();
      irr.push_back((int32_t)k);
    }
  faces.clear();
  std::map<std::pair<int, int>, int> face_index;
  for (int q : irr)
    for (const Face& f : geo.faces(q)) {
      face_index[{q, f.curve}] = (int)faces.size();
      faces.push_back({q, f.curve});
    }
  // regular stencil (eq. stdLap; cross term from eq. stdGrad applied twice)
  for (auto& r : coef)
    for (double& v : r) v = 0;
  const double s = 1.0 / (12.0 * h * h);
  coef[2][2] = -30.0 * (a + c) * s;
  coef[2][3] = coef[2][1] = 16.0 * a * s;
  coef[2][4] = coef[2][0] = -1.0 * a * s;
  coef[3][2] = coef[1][2] = 16.0 * c * s;
  coef[4][2] = coef[0][2] = -1.0 * c * s;
  if (b != 0.0) {
    const double gg[5] = {1.0, -8.0, 0.0, 8.0, -1.0};  // g(m) for m = -2..2
    for (int m2 = -2; m2 <= 2; ++m2)
      for (int m1 = -2; m1 <= 2; ++m1)
        if (m1 != 0 && m2 != 0) coef[m2 + 2][m1 + 2] = b * gg[m1 + 2] * gg[m2 + 2] / (144.0 * h * h);
  }
  diag = coef[2][2];
  // irregular rows
  const size_t ni = irr.size();
  std::vector<RowResult> rows(ni);
  std::atomic<int> failed(-1);
  parallel_for((int)ni, threads, [&](int s0, int s1) {
    Fitter F(geo, *this);
    for (int k = s0; k < s1; ++k) {
      rows[k] = F.row(irr[k]);
      if (!rows[k].ok) failed = irr[k];
    }
  });
  if (failed >= 0) throw Error(-4, "no acceptable lattice for cell " + std::to_string((int)failed));
  sten.assign(ni * NB, 0);
  wts.assign(ni * NB, 0.0);
  cond.assign(ni, 0.0);
  fw_ptr.assign(ni + 1, 0);
  fw_face.clear();
  fw_val.clear();
  for (size_t k = 0; k < ni; ++k) {
    const int q = irr[k];
    for (int t = 0; t < NB; ++t) {
      sten[k * NB + t] = rows[k].cells[t];
      wts[k * NB + t] = rows[k].beta[t] / (h * h);
    }
    cond[k] = rows[k].cond;
    const std::vector<Face>& fs = geo.faces(q);
    for (size_t f = 0; f < fs.size(); ++f) {
      double bf = rows[k].beta[NB + f];
      fw_face.push_back(face_index[{q, fs[f].curve}]);
      // Neumann columns are in xi-gradient units (h du/dn), Dirichlet
      // columns in the datum's units, Robin columns the datum over s
      const Curve& cv = geo.curves[fs[f].curve];
      fw_val.push_back(cv.bc == 1 ? bf / h : cv.bc == 2 ? bf / (robin_scale(cv, h) * h * h) : bf / (h * h));
    }
    fw_ptr[k + 1] = (int32_t)fw_face.size();
  }
  alg3();
}

// Alg. 3 with the boundary parameter of each boundary cell (see the oracle's
// documentation of the same rule): box cells by the counter-clockwise
// perimeter position of the cell centre's projection, curve cells by the
// midpoint parameter of their own arc.
void Discretization::alg3() {
  const Geometry& geo = *g;
  std::vector<std::tuple<int, double, int>> keys;  // (curve, param, cell)
  for (int q : irr) {
    const std::vector<Face>& fs = geo.faces(q);
    if (fs.empty()) continue;
    int cv_ = fs[0].curve;
    double par = 0;
    if (cv_ == geo.box) {
      int i = q % nx, j = q / nx;
      std::vector<std::pair<int, double>> cand;
      auto add_for = [&](int ii, int jj) {
        double X = (ii + 0.5) / nx, Y = (jj + 0.5) / ny;
        if (jj == 0) cand.push_back({0, X});
        if (ii == nx - 1) cand.push_back({1, 1.0 + Y});
        if (jj == ny - 1) cand.push_back({2, 2.0 + (1.0 - X)});
        if (ii == 0) cand.push_back({3, 3.0 + (1.0 - Y)});
      };
      add_for(i, j);
      if (cand.empty()) {
        for (int ci : geo.cv.at(q).members) {
          int own = geo.comps[ci].own, oi = own % nx, oj = own / nx;
          double s0[4] = {(oi + 0.5) / nx, 1.0 + (oj + 0.5) / ny, 2.0 + 1.0 - (oi + 0.5) / nx, 3.0 + 1.0 - (oj + 0.5) / ny};
          for (int e = 0; e < 4; ++e)
            if (geo.on_border(oi, oj, e)) cand.push_back({e, s0[e]});
        }
      }
      par = std::min_element(cand.begin(), cand.end())->second;
    } else {
      bool have = false;
      for (int ci : geo.cv.at(q).members) {
        const Comp& cp = geo.comps[ci];
        for (const LoopItem& it : cp.loop) {
          if (!it.is_arc) continue;
          const CellArc& arc = geo.arcs.at(cp.own)[it.arc];
          if (arc.curve != cv_) continue;
          double t = pymod(0.5 * (arc.pieces.front().first + arc.pieces.back().second), TWO_PI);
          par = have ? std::min(par, t) : t;
          have = true;
        }
      }
    }
    keys.emplace_back(cv_, par, q);
  }
  std::sort(keys.begin(), keys.end());
  std::vector<int32_t> num(irr.size(), -1), blk(irr.size(), -1);
  int k = 0;
  for (auto& key : keys) {
    int q = std::get<2>(key), i = q % nx, j = q / nx;
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        int ii = i + dx, jj = j + dy;
        if (ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
        int p = irr_pos[(size_t)jj * nx + ii];
        if (p >= 0 && num[p] < 0) num[p] = k++, blk[p] = std::get<0>(key);
      }
  }
  for (size_t p = 0; p < irr.size(); ++p)
    if (num[p] < 0) num[p] = k++;
  order.assign(irr.size(), 0);
  block.assign(irr.size(), -1);
  for (size_t p = 0; p < irr.size(); ++p) order[num[p]] = irr[p], block[num[p]] = blk[p];
}

void Hierarchy::build(const std::vector<Curve>& curves, int nx, int ny, double x0, double y0, double h,
                      double a, double b, double c, const Options& opt) {
  geo.clear();
  disc.clear();
  geo.emplace_back();
  geo.back().build(curves, nx, ny, x0, y0, h, opt.theta, opt.threads);
  disc.emplace_back();
  disc.back().build(geo.back(), a, b, c, opt.w_min, opt.threads);
  int cx = nx, cy = ny;
  double ch = h;
  while ((int)geo.size() < opt.max_levels) {
    if (cx % 2 || cy % 2 || cx / 2 < opt.coarsest_min_n || cy / 2 < opt.coarsest_min_n) break;
    cx /= 2, cy /= 2, ch *= 2;
    Geometry G;
    Discretization D;
    try {
      G.build(curves, cx, cy, x0, y0, ch, opt.theta, opt.threads);
      D.build(G, a, b, c, opt.w_min, opt.threads);
    } catch (const Error&) {
      break;
    }
    geo.push_back(std::move(G));
    disc.push_back(std::move(D));
    disc.back().g = &geo.back();
  }
  for (size_t k = 0; k < geo.size(); ++k) disc[k].g = &geo[k];
}

void forward_rows(const Discretization& D, RowSet& out) {
  const int ni = (int)D.irr.size();
  out.cell = D.irr;
  out.rp.resize(ni + 1);
  for (int k = 0; k <= ni; ++k) out.rp[k] = NB * k;
  out.cols = D.sten;
  out.vals = D.wts;
  out.order.resize(ni);
  for (int p = 0; p < ni; ++p) out.order[p] = D.irr_pos[D.order[p]];
}

void transposed_rows(const Discretization& D, RowSet& out, std::vector<uint8_t>& adj_regular) {
  const int nx = D.nx, ny = D.ny;
  const size_t n = (size_t)nx * ny;
  const int ni = (int)D.irr.size();
  // irregular-row entries grouped by column
  std::vector<std::vector<std::pair<int32_t, double>>> by_col(n);
  std::vector<uint8_t> ref(n, 0);
  for (int k = 0; k < ni; ++k)
    for (int t = 0; t < NB; ++t) {
      const int c = D.sten[NB * k + t];
      by_col[c].push_back({D.irr[k], D.wts[NB * k + t]});
      ref[c] = 1;
    }
  adj_regular.assign(n, 0);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t g = (size_t)j * nx + i;
      if (!D.regular[g] || ref[g]) continue;
      bool all = true;
      for (int dy = -2; dy <= 2 && all; ++dy)
        for (int dx = -2; dx <= 2; ++dx)
          if (!D.regular[(size_t)(j + dy) * nx + (i + dx)]) {
            all = false;
            break;
          }
      adj_regular[g] = all;
    }
  out.cell.clear();
  out.rp.assign(1, 0);
  out.cols.clear();
  out.vals.clear();
  std::vector<int32_t> pos(n, -1);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const size_t g = (size_t)j * nx + i;
      if (!D.nonempty[g] || adj_regular[g]) continue;
      std::map<int32_t, double> e;
      for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
          const int ii = i + dx, jj = j + dy;
          if (ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
          const size_t r = (size_t)jj * nx + ii;
          // L(r, g) for a regular row r: coefficient at offset g - r
          const double w = D.coef[2 - dy][2 - dx];
          if (D.regular[r] && w != 0.0) e[(int32_t)r] += w;
        }
      for (auto& pr : by_col[g]) e[pr.first] += pr.second;
      pos[g] = (int32_t)out.cell.size();
      out.cell.push_back((int32_t)g);
      for (auto& kv : e) {
        out.cols.push_back(kv.first);
        out.vals.push_back(kv.second);
      }
      out.rp.push_back((int32_t)out.cols.size());
    }
  const int nt = (int)out.cell.size();
  std::vector<int32_t> num(nt, -1);
  int k = 0;
  for (int p = 0; p < ni; ++p) {
    const int q = D.order[p], i = q % nx, j = q / nx;
    for (int dy = -4; dy <= 4; ++dy)
      for (int dx = -4; dx <= 4; ++dx) {
        const int ii = i + dx, jj = j + dy;
        if (ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
        const int t = pos[(size_t)jj * nx + ii];
        if (t >= 0 && num[t] < 0) num[t] = k++;
      }
  }
  for (int t = 0; t < nt; ++t)
    if (num[t] < 0) num[t] = k++;
  out.order.assign(nt, 0);
  for (int t = 0; t < nt; ++t) out.order[num[t]] = t;
}

void smoother_rows(const Discretization& D, const RowSet& base, const std::vector<uint8_t>& stencil_mask,
                   int widen, RowSet& out, std::vector<int32_t>& base_index, std::vector<uint8_t>& jacobi_mask) {
  const int nx = D.nx, ny = D.ny;
  const size_t n = (size_t)nx * ny;
  const int nb = (int)base.cell.size();
  std::vector<int32_t> bpos(n, -1);
  for (int k = 0; k < nb; ++k) bpos[base.cell[k]] = k;
  std::vector<uint8_t> in(n, 0);
  for (int k = 0; k < nb; ++k) in[base.cell[k]] = 1;
  if (widen > 0)
    for (int k = 0; k < nb; ++k) {
      const int q = base.cell[k], i = q % nx, j = q / nx;
      for (int dy = -widen; dy <= widen; ++dy)
        for (int dx = -widen; dx <= widen; ++dx) {
          const int ii = i + dx, jj = j + dy;
          if (ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
          const size_t c = (size_t)jj * nx + ii;
          if (stencil_mask[c]) in[c] = 1;
        }
    }
  jacobi_mask.assign(n, 0);
  for (size_t c = 0; c < n; ++c) jacobi_mask[c] = stencil_mask[c] && !in[c];
  out.cell.clear();
  out.rp.assign(1, 0);
  out.cols.clear();
  out.vals.clear();
  base_index.clear();
  std::vector<int32_t> pos(n, -1);
  for (size_t c = 0; c < n; ++c) {
    if (!in[c]) continue;
    pos[c] = (int32_t)out.cell.size();
    out.cell.push_back((int32_t)c);
    const int b = bpos[c];
    base_index.push_back(b);
    if (b >= 0) {
      for (int t = base.rp[b]; t < base.rp[b + 1]; ++t) {
        out.cols.push_back(base.cols[t]);
        out.vals.push_back(base.vals[t]);
      }
    } else {
      const int i = (int)(c % nx), j = (int)(c / nx);
      for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
          const double w = D.coef[dy + 2][dx + 2];
          if (w == 0.0) continue;
          out.cols.push_back((j + dy) * nx + i + dx);
          out.vals.push_back(w);
        }
    }
    out.rp.push_back((int32_t)out.cols.size());
  }
  const int ns = (int)out.cell.size();
  const int rad = std::max(widen, 1);
  std::vector<int32_t> num(ns, -1);
  int k = 0;
  for (int p = 0; p < nb; ++p) {
    const int q = base.cell[base.order[p]], i = q % nx, j = q / nx;
    for (int dy = -rad; dy <= rad; ++dy)
      for (int dx = -rad; dx <= rad; ++dx) {
        const int ii = i + dx, jj = j + dy;
        if (ii < 0 || jj < 0 || ii >= nx || jj >= ny) continue;
        const int t = pos[(size_t)jj * nx + ii];
        if (t >= 0 && num[t] < 0) num[t] = k++;
      }
  }
  for (int t = 0; t < ns; ++t)
    if (num[t] < 0) num[t] = k++;
  out.order.assign(ns, 0);
  for (int t = 0; t < ns; ++t) out.order[num[t]] = t;
}

bool dense_inverse(std::vector<double>& A, int n, int threads) {
  // Gauss-Jordan with partial pivoting on [A | I], row-major.
  std::vector<double> B((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) B[(size_t)i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    double best = std::fabs(A[(size_t)k * n + k]);
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + k]) > best) best = std::fabs(A[(size_t)r * n + k]), piv = r;
    if (best == 0.0 || !std::isfinite(best)) return false;
    if (piv != k)
      for (int cc = 0; cc < n; ++cc) {
        std::swap(A[(size_t)k * n + cc], A[(size_t)piv * n + cc]);
        std::swap(B[(size_t)k * n + cc], B[(size_t)piv * n + cc]);
      }
    const double inv = 1.0 / A[(size_t)k * n + k];
    for (int cc = 0; cc < n; ++cc) A[(size_t)k * n + cc] *= inv, B[(size_t)k * n + cc] *= inv;
    const double* Ak = &A[(size_t)k * n];
    const double* Bk = &B[(size_t)k * n];
    parallel_for(n, n > 256 ? threads : 1, [&](int r0, int r1) {
      for (int r = r0; r < r1; ++r) {
        if (r == k) continue;
        double f = A[(size_t)r * n + k];
        if (f == 0.0) continue;
        double* Ar = &A[(size_t)r * n];
        double* Br = &B[(size_t)r * n];
        for (int cc = 0; cc < n; ++cc) Ar[cc] -= f * Ak[cc], Br[cc] -= f * Bk[cc];
      }
    });
  }
  A.swap(B);
  return true;
}

}  // namespace ccg
