// Quadrature nodes for callers that average their own data over cut cells
// and boundary faces (Green's formula with the x-primitive, eq.
// iteratedIntegral): for an outer node t_q on a boundary piece the inner
// integral from the member cell's centre xi0 to x(t_q) is a second
// Gauss-Legendre rule, giving 2-D nodes with weights w_q y'(t_q) (x - xi0)/2 w_r.
#include <algorithm>
#include <cmath>
#include <vector>

#include "setup.hpp"

namespace ccg {
namespace {
struct QuadSink {
  std::vector<int32_t> owner;
  std::vector<double> x, y, w, nx, ny;
};

void cell_nodes(const Geometry& G, int idx, QuadSink& S, int q) {
  std::vector<double> tq, wq;
  gauss_legendre(q, tq, wq);
  const double h = G.h;
  auto emit_loop = [&](const Comp& cp) {
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
    for (const LoopItem& it : cp.loop) {
      if (it.is_arc) {
        const CellArc& arc = G.arcs.at(own)[it.arc];
        const Curve& c = G.curves[arc.curve];
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

int cell_quadrature(const Geometry& G, long* count, int32_t* cell_of, double* x, double* y, double* w) {
  if (!count) return -1;
  QuadSink S;
  std::vector<int> cells;
  for (auto& kv : G.cv) cells.push_back(kv.first);
  std::sort(cells.begin(), cells.end());
  for (int idx : cells) cell_nodes(G, idx, S, 16);
  const long n = (long)S.w.size();
  if (!cell_of && !x && !y && !w) {
    *count = n;
    return 0;
  }
  if (*count < n) return -1;
  for (long k = 0; k < n; ++k) {
    if (cell_of) cell_of[k] = S.owner[k];
    if (x) x[k] = S.x[k];
    if (y) y[k] = S.y[k];
    if (w) w[k] = S.w[k];
  }
  *count = n;
  return 0;
}

int face_quadrature(const Geometry& G, const Discretization& D, long* count, int32_t* face_of, double* x, double* y,
                    double* w, double* nxo, double* nyo) {
  if (!count) return -1;
  const int q = 16;
  std::vector<double> tq, wq;
  gauss_legendre(q, tq, wq);
  QuadSink S;
  const double h = G.h;
  for (size_t f = 0; f < D.faces.size(); ++f) {
    const int idx = D.faces[f].first, curve = D.faces[f].second;
    std::vector<const Comp*> members;
    std::vector<Comp> tmp;
    if (G.state[idx] == S_PURE) {
      tmp.push_back(G.trace(idx, {{false, -1, 0.0, 4.0}}));
      members.push_back(&tmp.back());
    } else {
      for (int ci : G.cv.at(idx).members) members.push_back(&G.comps[ci]);
    }
    for (const Comp* cp : members) {
      const int own = cp->own, i = own % G.nx, j = own / G.nx;
      const double cx = G.x0 + (i + 0.5) * h, cy = G.y0 + (j + 0.5) * h;
      std::vector<LoopItem> loop = cp->loop;
      if (loop.empty()) loop.push_back({false, -1, 0.0, 4.0});
      for (const LoopItem& it : loop) {
        if (it.is_arc) {
          const CellArc& arc = G.arcs.at(own)[it.arc];
          if (arc.curve != curve) continue;
          const Curve& c = G.curves[arc.curve];
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
    return 0;
  }
  if (*count < n) return -1;
  for (long k = 0; k < n; ++k) {
    if (face_of) face_of[k] = S.owner[k];
    if (x) x[k] = S.x[k];
    if (y) y[k] = S.y[k];
    if (w) w[k] = S.w[k];
    if (nxo) nxo[k] = S.nx[k];
    if (nyo) nyo[k] = S.ny[k];
  }
  *count = n;
  return 0;
}


}  // namespace ccg
