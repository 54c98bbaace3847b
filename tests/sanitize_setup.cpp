// Host set-up under AddressSanitizer and UndefinedBehaviorSanitizer: the
// library's hierarchy construction (cut cells and Alg. 1, classification,
// lattices and least-squares rows on every level), the explicit row sets
// of L and L^T and of the SMO-2 blocks, and both quadrature exports, on a
// set of geometries covering every curve kind and boundary condition.
// Built and run by tests/test_host_sanitizers.py with g++ (no GPU code).
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "setup.hpp"

using ccg::Curve;

static Curve curve(int kind, std::vector<double> p, int inside, int bc, double g1 = 0, double g2 = 0) {
  Curve c;
  c.kind = kind, c.inside = inside, c.bc = bc;
  for (size_t k = 0; k < p.size() && k < 8; ++k) c.p[k] = p[k];
  c.robin[0] = g1, c.robin[1] = g2;
  return c;
}

struct Case {
  const char* name;
  int n;
  double x0, h, a, b, c;
  std::vector<Curve> curves;
};

int main(int argc, char** argv) {
  // "small": the first cases on half the grid, 4 set-up threads (for the
  // slower thread-sanitizer build)
  const bool small = argc > 1 && std::string(argv[1]) == "small";
  const double pi = std::acos(-1.0);
  std::vector<Case> cases;
  cases.push_back({"disk inside the square", 64, 0.0, 1.0 / 64, 1, 0, 1,
                   {curve(ccg::K_CIRCLE, {0.5, 0.5, 0.3}, 1, 0)}});
  cases.push_back({"flower hole, Neumann, b != 0", 64, 0.0, 1.0 / 64, 1, 0.5, 1,
                   {curve(ccg::K_BOX, {0, 0, 1, 1}, 1, 0), curve(ccg::K_POLAR_SIN, {0.5, 0.5, 0.25, 0.05, 5, 0}, 0, 1)}});
  cases.push_back({"three circles", 128, 0.0, 1.0 / 128, 1, 0, 1,
                   {curve(ccg::K_BOX, {0, 0, 1, 1}, 1, 0), curve(ccg::K_CIRCLE, {0.3, 0.3, 0.12}, 0, 0),
                    curve(ccg::K_CIRCLE, {0.7, 0.35, 0.1}, 0, 0), curve(ccg::K_CIRCLE, {0.5, 0.72, 0.14}, 0, 0)}});
  cases.push_back({"rotated ellipses, b = 1.2", 64, 0.0, 1.0 / 64, 1, 1.2, 1,
                   {curve(ccg::K_BOX, {0, 0, 1, 1}, 1, 0), curve(ccg::K_ELLIPSE, {0.35, 0.4, 0.12, 0.06, 0.7}, 0, 0),
                    curve(ccg::K_ELLIPSE, {0.7, 0.65, 0.08, 0.11, 2.1}, 0, 0)}});
  cases.push_back({"flower box (Problem 1 shape), Neumann", 40, -0.5, 1.0 / 40, 1, 0, 1,
                   {curve(ccg::K_BOX, {-0.5, -0.5, 0.5, 0.5}, 1, 0),
                    curve(ccg::K_POLAR_COS, {0.0, 0.0, 0.25, 0.05, 6, 0}, 0, 1)}});
  cases.push_back({"Robin ellipse", 64, 0.0, 1.0 / 64, 1, 0, 1,
                   {curve(ccg::K_BOX, {0, 0, 1, 1}, 1, 0), curve(ccg::K_ELLIPSE, {0.5, 0.5, 0.125, 0.25, 0}, 0, 2, 1.0, 0.5)}});
  {
    const double c = std::cos(pi / 6), s = std::sin(pi / 6);
    std::vector<double> p;
    for (auto v : {std::pair<double, double>{-0.5, -0.5}, {0.5, -0.5}, {0.5, 0.5}, {-0.5, 0.5}}) {
      p.push_back(0.5 + c * v.first - s * v.second);
      p.push_back(0.5 + s * v.first + c * v.second);
    }
    cases.push_back({"rotated box (polygon)", 96, -0.25, 1.5 / 96, 1, 0, 2, {curve(ccg::K_POLYGON, p, 1, 0)}});
  }
  if (small) {
    cases.resize(3);
    for (Case& cs : cases) cs.n /= 2, cs.h *= 2;
  }
  int checked = 0;
  for (const Case& cs : cases) {
    ccg::Options opt;
    opt.threads = small ? 4 : 2;
    ccg::Hierarchy H;
    try {
      H.build(cs.curves, cs.n, cs.n, cs.x0, cs.x0, cs.h, cs.a, cs.b, cs.c, opt);
    } catch (const ccg::Error& e) {
      std::printf("%s: set-up error %d: %s\n", cs.name, e.code, e.what());
      return 2;
    }
    long rows = 0;
    for (const ccg::Discretization& D : H.disc) {
      ccg::RowSet fwd, adj, sm;
      std::vector<uint8_t> adj_regular, jac;
      std::vector<int32_t> base;
      ccg::forward_rows(D, fwd);
      ccg::transposed_rows(D, adj, adj_regular);
      std::vector<uint8_t> mask(D.nonempty.size(), 0);
      for (size_t k = 0; k < mask.size(); ++k) mask[k] = D.regular[k];
      ccg::smoother_rows(D, fwd, mask, 1, sm, base, jac);
      rows += (long)fwd.cell.size() + (long)adj.cell.size() + (long)sm.cell.size();
    }
    long nc = 0, nf = 0;
    ccg::cell_quadrature(H.geo[0], &nc, nullptr, nullptr, nullptr, nullptr);
    std::vector<int32_t> ci(nc), fi;
    std::vector<double> x(nc), y(nc), w(nc);
    ccg::cell_quadrature(H.geo[0], &nc, ci.data(), x.data(), y.data(), w.data());
    ccg::face_quadrature(H.geo[0], H.disc[0], &nf, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    fi.resize(nf);
    std::vector<double> fx(nf), fy(nf), fw(nf), fnx(nf), fny(nf);
    ccg::face_quadrature(H.geo[0], H.disc[0], &nf, fi.data(), fx.data(), fy.data(), fw.data(), fnx.data(), fny.data());
    std::printf("%s: %zu levels, %ld explicit rows, %ld cell and %ld face nodes\n", cs.name, H.disc.size(), rows, nc, nf);
    ++checked;
  }
  std::printf("checked %d geometries\n", checked);
  return 0;
}
