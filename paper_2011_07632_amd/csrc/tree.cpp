// Partition tree and admissibility lists (host).
//
// A perfect binary tree (Section 2 assumes a perfect tree) in heap order, of
// one of two kinds:
// * kd: depth D is the smallest integer with N <= leaf * 2^D; a node is split
//   on the axis of its largest bounding-box extent (lowest axis on ties), its
//   points ordered by (coordinate, original index), the left child taking
//   floor(n/2) of them;
// * box: the 2^d-ary box-bisection tree of Section 6 for d = 3, as three
//   binary levels per 2^d-ary level: a node at depth t is bisected along axis
//   t mod 3 at the midpoint of its points' extent on that axis (points below
//   it go left, in the same order as above), and D is the smallest multiple of
//   3 at which no node holds more than leaf points.  The box of a node is the
//   tight box of its points, so no child is empty and the tree stays perfect.
// Far-field sets (Section 5.1) use the admissibility rule
// r_i + r_j <= eta * |c_i - c_j| on bounding-box centres c and half-diagonals
// r; near (Type-1) and coupling (Type-3) lists are built top-down from the
// children of the parent's near list (Section 5.2.2).
//
// Floating-point contraction is disabled here so that every comparison that
// decides the tree or a list is evaluated in plain IEEE double arithmetic.
#pragma clang fp contract(off)

#include "model.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace spd {

static int depth_for(int64_t n, int leaf) {
  int d = 0;
  while (n > (int64_t)leaf * ((int64_t)1 << d)) ++d;
  return d;
}

// Split node v into 2v+1 and 2v+2 (appended to start/end); axis < 0 takes the
// axis of largest extent (kd), otherwise the node is bisected along axis (box).
void TreeHost::split(const double* pts, int v, int axis) {
  const int64_t s = start[v], e = end[v];
  double lo3[3] = {INFINITY, INFINITY, INFINITY}, hi3[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = s; i < e; ++i)
    for (int a = 0; a < 3; ++a) {
      const double x = pts[3 * perm[i] + a];
      lo3[a] = std::min(lo3[a], x);
      hi3[a] = std::max(hi3[a], x);
    }
  const bool box = axis >= 0;
  if (!box) {
    axis = 0;
    if (e > s) {
      double best = hi3[0] - lo3[0];
      for (int a = 1; a < 3; ++a)
        if (hi3[a] - lo3[a] > best) { best = hi3[a] - lo3[a]; axis = a; }
    }
  }
  std::sort(perm.begin() + s, perm.begin() + e, [&](int64_t a, int64_t b) {
    const double xa = pts[3 * a + axis], xb = pts[3 * b + axis];
    return xa < xb || (xa == xb && a < b);
  });
  int64_t m = (e - s) / 2;
  if (box) {
    const double mid = 0.5 * (lo3[axis] + hi3[axis]);
    m = std::partition_point(perm.begin() + s, perm.begin() + e,
                             [&](int64_t a) { return pts[3 * a + axis] < mid; }) -
        (perm.begin() + s);
    SPD_REQUIRE(m > 0 && m < e - s, SPD_E_INVALID,
                "box bisection: node " + std::to_string(v) + " (" + std::to_string(e - s) +
                    " points) has no extent along axis " + std::to_string(axis));
  }
  start.push_back(s);
  end.push_back(s + m);
  start.push_back(s + m);
  end.push_back(e);
}

void TreeHost::build(const double* pts, int64_t n, int leaf_size, double eta_, int kind_) {
  SPD_REQUIRE(n >= 1, SPD_E_INVALID, "empty point set");
  SPD_REQUIRE(leaf_size >= 1, SPD_E_INVALID, "leaf size must be positive");
  N = n;
  leaf = leaf_size;
  eta = eta_;
  kind = kind_;
  perm.resize(n);
  std::iota(perm.begin(), perm.end(), (int64_t)0);
  start.assign(1, 0);
  end.assign(1, n);
  if (kind == SPD_TREE_KD) {
    D = depth_for(n, leaf);
    SPD_REQUIRE(D <= 24, SPD_E_INVALID, "tree too deep");
    for (int v = 0; v < (1 << D) - 1; ++v) split(pts, v, -1);
  } else {
    SPD_REQUIRE(kind == SPD_TREE_BOX, SPD_E_INVALID, "unknown tree kind");
    D = 0;
    auto largest = [&]() {
      int64_t m = 0;
      for (int v = (1 << D) - 1; v < (1 << (D + 1)) - 1; ++v) m = std::max(m, end[v] - start[v]);
      return m;
    };
    while (largest() > leaf) {
      SPD_REQUIRE(D + 3 <= 24, SPD_E_INVALID, "tree too deep");
      for (int t = D; t < D + 3; ++t)
        for (int v = (1 << t) - 1; v < (1 << (t + 1)) - 1; ++v) split(pts, v, t % 3);
      D += 3;
    }
  }
  L = D + 1;
  nnodes = (1 << (D + 1)) - 1;
  lo.assign(3 * nnodes, 0.0);
  hi.assign(3 * nnodes, 0.0);
  for (int v = nnodes - 1; v >= 0; --v) {
    if (is_leaf(v)) {
      if (end[v] > start[v]) {
        for (int a = 0; a < 3; ++a) { lo[3 * v + a] = INFINITY; hi[3 * v + a] = -INFINITY; }
        for (int64_t i = start[v]; i < end[v]; ++i)
          for (int a = 0; a < 3; ++a) {
            const double x = pts[3 * perm[i] + a];
            lo[3 * v + a] = std::min(lo[3 * v + a], x);
            hi[3 * v + a] = std::max(hi[3 * v + a], x);
          }
      }
    } else {
      const int c1 = 2 * v + 1, c2 = 2 * v + 2;
      const bool e1 = end[c1] > start[c1], e2 = end[c2] > start[c2];
      for (int a = 0; a < 3; ++a) {
        if (e1 && e2) {
          lo[3 * v + a] = std::min(lo[3 * c1 + a], lo[3 * c2 + a]);
          hi[3 * v + a] = std::max(hi[3 * c1 + a], hi[3 * c2 + a]);
        } else if (e1 || e2) {
          const int c = e1 ? c1 : c2;
          lo[3 * v + a] = lo[3 * c + a];
          hi[3 * v + a] = hi[3 * c + a];
        }
      }
    }
  }
  center.assign(3 * nnodes, 0.0);
  radius.assign(nnodes, 0.0);
  for (int v = 0; v < nnodes; ++v) {
    double d[3];
    for (int a = 0; a < 3; ++a) {
      center[3 * v + a] = 0.5 * (lo[3 * v + a] + hi[3 * v + a]);
      d[a] = hi[3 * v + a] - lo[3 * v + a];
    }
    radius[v] = 0.5 * std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  }
  build_lists();
}

bool TreeHost::admissible(int i, int j) const {
  if (i == j) return false;
  const double dx = center[3 * i] - center[3 * j];
  const double dy = center[3 * i + 1] - center[3 * j + 1];
  const double dz = center[3 * i + 2] - center[3 * j + 2];
  const double dist = std::sqrt(dx * dx + dy * dy + dz * dz);
  return radius[i] + radius[j] <= eta * dist;
}

void TreeHost::build_lists() {
  std::vector<std::vector<int>> nearl(nnodes), coupl(nnodes);
  nearl[0] = {0};
  for (int d = 1; d <= D; ++d) {
    for (int v = (1 << d) - 1; v < (1 << (d + 1)) - 1; ++v) {
      const int p = (v - 1) / 2;
      for (int q : nearl[p])
        for (int j = 2 * q + 1; j <= 2 * q + 2; ++j)
          (admissible(v, j) ? coupl[v] : nearl[v]).push_back(j);
      std::sort(nearl[v].begin(), nearl[v].end());
      std::sort(coupl[v].begin(), coupl[v].end());
    }
  }
  near_ptr.assign(nnodes + 1, 0);
  coup_ptr.assign(nnodes + 1, 0);
  near_idx.clear();
  coup_idx.clear();
  for (int v = 0; v < nnodes; ++v) {
    near_ptr[v] = (int64_t)near_idx.size();
    coup_ptr[v] = (int64_t)coup_idx.size();
    near_idx.insert(near_idx.end(), nearl[v].begin(), nearl[v].end());
    coup_idx.insert(coup_idx.end(), coupl[v].begin(), coupl[v].end());
  }
  near_ptr[nnodes] = (int64_t)near_idx.size();
  coup_ptr[nnodes] = (int64_t)coup_idx.size();
}

int TreeHost::lca_level(int i, int j) const {
  int k = level(i);
  while (i != j) {
    i = (i - 1) / 2;
    j = (j - 1) / 2;
    ++k;
  }
  return k;
}

int64_t TreeHost::near_pos(int i, int j) const {
  const int* b = near_idx.data() + near_ptr[i];
  const int* e = near_idx.data() + near_ptr[i + 1];
  const int* it = std::lower_bound(b, e, j);
  return (it != e && *it == j) ? near_ptr[i] + (it - b) : -1;
}

int64_t TreeHost::coup_pos(int i, int j) const {
  const int* b = coup_idx.data() + coup_ptr[i];
  const int* e = coup_idx.data() + coup_ptr[i + 1];
  const int* it = std::lower_bound(b, e, j);
  return (it != e && *it == j) ? coup_ptr[i] + (it - b) : -1;
}

// Proxy radii of a node: from the nearest box of its far field (couplings of
// the node and all ancestors) to the farthest corner of the root box.
bool TreeHost::proxy_radii(int v, double& rin, double& rout) const {
  rin = INFINITY;
  bool any = false;
  const double* c = &center[3 * v];
  int a = v;
  while (true) {
    for (int64_t e = coup_ptr[a]; e < coup_ptr[a + 1]; ++e) {
      const int j = coup_idx[e];
      double d[3];
      for (int q = 0; q < 3; ++q)
        d[q] = std::max(std::max(lo[3 * j + q] - c[q], 0.0), c[q] - hi[3 * j + q]);
      rin = std::min(rin, std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]));
      any = true;
    }
    if (a == 0) break;
    a = (a - 1) / 2;
  }
  if (!any) return false;
  rout = 0.0;
  for (int ix = 0; ix < 2; ++ix)
    for (int iy = 0; iy < 2; ++iy)
      for (int iz = 0; iz < 2; ++iz) {
        const double dx = (ix ? hi[0] : lo[0]) - c[0];
        const double dy = (iy ? hi[1] : lo[1]) - c[1];
        const double dz = (iz ? hi[2] : lo[2]) - c[2];
        rout = std::max(rout, std::sqrt(dx * dx + dy * dy + dz * dz));
      }
  rout = std::max(rout, rin);
  return true;
}

// Points per proxy sphere of a node whose innermost sphere has radius rin:
// density * (rin / ell)^2 rounded up to a multiple of 64, clamped to [lo, hi]
// (density 0 keeps lo).  Evaluated without contraction, as the oracle does.
int proxy_count(double rin, double ell, int lo, int hi, double density) {
  if (!(density > 0.0)) return lo;
  const double t = rin / ell;
  const double x = density * (t * t) / 64.0;
  const double n = 64.0 * std::ceil(x);
  if (!(n < (double)hi)) return hi;
  return std::max((int)n, lo);
}

}  // namespace spd
