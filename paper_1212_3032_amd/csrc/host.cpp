// Host-side geometry, quadrature nodes, cluster tree and block partition.
#include "host.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>
#include <stdexcept>

namespace ewbem {

void radon7(double bary[7][3], double w[7]) {
  // Radon's rule: the centroid and two orbits (a, a, 1-2a) with
  // a = (6 -+ sqrt 15)/21; weights 9/40 and (155 -+ sqrt 15)/1200.
  const double r15 = std::sqrt(15.0);
  const double a = (6.0 - r15) / 21.0, b = (6.0 + r15) / 21.0;
  const double wa = (155.0 - r15) / 1200.0, wb = (155.0 + r15) / 1200.0;
  const double third = 1.0 / 3.0;
  double pts[7][3] = {{third, third, third},
                      {a, a, 1 - 2 * a}, {a, 1 - 2 * a, a}, {1 - 2 * a, a, a},
                      {b, b, 1 - 2 * b}, {b, 1 - 2 * b, b}, {1 - 2 * b, b, b}};
  double ww[7] = {9.0 / 40.0, wa, wa, wa, wb, wb, wb};
  for (int i = 0; i < 7; ++i) {
    for (int k = 0; k < 3; ++k) bary[i][k] = pts[i][k];
    w[i] = ww[i];
  }
}

void gauss_legendre01(int n, double* x, double* w) {
  // Newton iteration on P_n from the Chebyshev-like initial guesses.
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? t : p1;
      double pm = (n == 1) ? 1.0 : p0;
      dp = n * (t * pn - pm) / (t * t - 1.0);
      double dt = pn / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double pn = (n == 1) ? t : p1, pm = (n == 1) ? 1.0 : p0;
    dp = n * (t * pn - pm) / (t * t - 1.0);
    x[i] = 0.5 * (1.0 - t);
    w[i] = 1.0 / ((1.0 - t * t) * dp * dp);   // (2/((1-t^2)P'^2)) / 2
  }
}

void build_geometry(int nv, const double* xyz, int nt, const int32_t* tri, bool exterior,
                    const std::vector<int>& perm, HostGeom& g) {
  g.ne = nt;
  g.perm = perm;
  g.iperm.assign(nt, 0);
  for (int t = 0; t < nt; ++t) g.iperm[perm[t]] = t;
  g.cen.assign(3 * nt, 0);
  g.nrm.assign(3 * nt, 0);
  g.area.assign(nt, 0);
  g.qp.assign(21 * nt, 0);
  g.qw.assign(7 * nt, 0);
  g.vtx.assign(9 * nt, 0);
  double bary[7][3], w[7];
  radon7(bary, w);
  for (int t = 0; t < nt; ++t) {
    const int e = perm[t];
    const double* p[3];
    for (int k = 0; k < 3; ++k) {
      int vi = tri[3 * e + k];
      if (vi < 0 || vi >= nv) throw std::invalid_argument("triangle vertex index out of range");
      p[k] = xyz + 3 * vi;
    }
    double e1[3], e2[3], c[3];
    for (int k = 0; k < 3; ++k) {
      e1[k] = p[1][k] - p[0][k];
      e2[k] = p[2][k] - p[0][k];
    }
    c[0] = e1[1] * e2[2] - e1[2] * e2[1];
    c[1] = e1[2] * e2[0] - e1[0] * e2[2];
    c[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double len = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    if (!(len > 0)) throw std::invalid_argument("degenerate triangle");
    double sgn = exterior ? -1.0 : 1.0;
    g.area[t] = 0.5 * len;
    for (int k = 0; k < 3; ++k) {
      g.nrm[3 * t + k] = sgn * c[k] / len;
      g.cen[3 * t + k] = (p[0][k] + p[1][k] + p[2][k]) / 3.0;
      for (int v = 0; v < 3; ++v) g.vtx[9 * t + 3 * v + k] = p[v][k];
    }
    for (int q = 0; q < 7; ++q) {
      for (int k = 0; k < 3; ++k)
        g.qp[21 * t + 3 * q + k] = bary[q][0] * p[0][k] + bary[q][1] * p[1][k] + bary[q][2] * p[2][k];
      g.qw[7 * t + q] = w[q] * g.area[t];
    }
  }
}

std::vector<int> build_tree(int nv, const double* xyz, int nt, const int32_t* tri, int leaf_size,
                            std::vector<Cluster>& clusters) {
  if (leaf_size < 1) throw std::invalid_argument("leaf_size must be positive");
  std::vector<int> order(nt);
  std::iota(order.begin(), order.end(), 0);
  std::vector<double> cen(3 * nt), lo(3 * nt), hi(3 * nt);
  for (int e = 0; e < nt; ++e) {
    for (int k = 0; k < 3; ++k) {
      double a = xyz[3 * tri[3 * e] + k], b = xyz[3 * tri[3 * e + 1] + k], c = xyz[3 * tri[3 * e + 2] + k];
      cen[3 * e + k] = (a + b + c) / 3.0;
      lo[3 * e + k] = std::min(a, std::min(b, c));
      hi[3 * e + k] = std::max(a, std::max(b, c));
    }
  }
  clusters.clear();
  std::function<int(int, int, int)> rec = [&](int b, int e, int level) -> int {
    Cluster c;
    c.begin = b;
    c.end = e;
    c.level = level;
    double clo[3] = {1e300, 1e300, 1e300}, chi[3] = {-1e300, -1e300, -1e300};
    double mlo[3] = {1e300, 1e300, 1e300}, mhi[3] = {-1e300, -1e300, -1e300};
    for (int i = b; i < e; ++i) {
      int el = order[i];
      for (int k = 0; k < 3; ++k) {
        c.lo[k] = 0;
        clo[k] = std::min(clo[k], lo[3 * el + k]);
        chi[k] = std::max(chi[k], hi[3 * el + k]);
        mlo[k] = std::min(mlo[k], cen[3 * el + k]);
        mhi[k] = std::max(mhi[k], cen[3 * el + k]);
      }
    }
    for (int k = 0; k < 3; ++k) {
      c.lo[k] = clo[k];
      c.hi[k] = chi[k];
    }
    int id = (int)clusters.size();
    clusters.push_back(c);
    if (e - b > leaf_size) {
      int axis = 0;
      double ext = -1;
      for (int k = 0; k < 3; ++k)
        if (mhi[k] - mlo[k] > ext) {
          ext = mhi[k] - mlo[k];
          axis = k;
        }
      int mid = b + (e - b) / 2;
      std::nth_element(order.begin() + b, order.begin() + mid, order.begin() + e,
                       [&](int u, int v) {
                         double cu = cen[3 * u + axis], cv = cen[3 * v + axis];
                         return cu < cv || (cu == cv && u < v);
                       });
      int c0 = rec(b, mid, level + 1);
      int c1 = rec(mid, e, level + 1);
      clusters[id].child[0] = c0;
      clusters[id].child[1] = c1;
    }
    return id;
  };
  rec(0, nt, 0);
  return order;
}

static double bbox_diam(const Cluster& c) {
  double s = 0;
  for (int k = 0; k < 3; ++k) s += (c.hi[k] - c.lo[k]) * (c.hi[k] - c.lo[k]);
  return std::sqrt(s);
}

static double bbox_dist(const Cluster& a, const Cluster& b) {
  double s = 0;
  for (int k = 0; k < 3; ++k) {
    double d = std::max(0.0, std::max(a.lo[k] - b.hi[k], b.lo[k] - a.hi[k]));
    s += d * d;
  }
  return std::sqrt(s);
}

void build_partition(double eta, Partition& p, int max_far) {
  p.near.clear();
  p.far.clear();
  p.leaves.clear();
  for (int i = 0; i < (int)p.clusters.size(); ++i)
    if (p.clusters[i].leaf()) p.leaves.push_back(i);
  std::sort(p.leaves.begin(), p.leaves.end(),
            [&](int a, int b) { return p.clusters[a].begin < p.clusters[b].begin; });
  std::function<void(int, int)> rec = [&](int t, int s) {
    const Cluster& ct = p.clusters[t];
    const Cluster& cs = p.clusters[s];
    if (eta > 0) {
      double d = bbox_dist(ct, cs);
      // an admissible pair larger than max_far elements on a side is split
      // further: its child pairs are admissible too (their boxes are no
      // larger and no closer)
      if (std::min(bbox_diam(ct), bbox_diam(cs)) <= eta * d &&
          ((ct.size() <= max_far && cs.size() <= max_far) || (ct.leaf() && cs.leaf()))) {
        p.far.push_back({t, s});
        return;
      }
    }
    if (ct.leaf() && cs.leaf()) {
      p.near.push_back({t, s});
      return;
    }
    if (ct.leaf()) {
      rec(t, cs.child[0]);
      rec(t, cs.child[1]);
    } else if (cs.leaf()) {
      rec(ct.child[0], s);
      rec(ct.child[1], s);
    } else {
      rec(ct.child[0], cs.child[0]);
      rec(ct.child[0], cs.child[1]);
      rec(ct.child[1], cs.child[0]);
      rec(ct.child[1], cs.child[1]);
    }
  };
  rec(0, 0);
}

}  // namespace ewbem
