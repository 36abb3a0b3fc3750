// Host-only check of the partition tree and admissibility lists (TreeHost),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py.  For seeded random point sets of several
// sizes and leaf sizes it builds the tree (kd and box bisection) and lists and
// checks, exiting non-zero on the first violation:
//   - perm is a permutation and node ranges nest (children split the parent);
//   - every leaf holds at most leaf_size points and the tree is perfect;
//   - near and coupling lists are symmetric, sorted, and disjoint;
//   - every pair of leaves is covered exactly once by a near pair of leaves or
//     a coupling pair of some ancestors (the lists tile the matrix);
//   - near_pos / coup_pos / lca_level agree with the lists.
#include "model.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

using spd::TreeHost;

static int fail(const char* what, int n, int leaf) {
  std::fprintf(stderr, "FAIL %s (n=%d leaf=%d)\n", what, n, leaf);
  return 1;
}

static int check(int n, int leaf, unsigned seed, int kind) {
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  std::vector<double> pts((size_t)3 * n);
  for (double& x : pts) x = U(rng);
  TreeHost T;
  try {
    T.build(pts.data(), n, leaf, 1.0, kind);
  } catch (const spd::Error&) {
    return fail("build failed", n, leaf);
  }
  if (kind == SPD_TREE_BOX && T.D % 3 != 0) return fail("box tree depth not a multiple of 3", n, leaf);
  std::vector<int64_t> p(T.perm.begin(), T.perm.end());
  std::sort(p.begin(), p.end());
  for (int i = 0; i < n; ++i)
    if (p[i] != i) return fail("perm is not a permutation", n, leaf);
  if (T.nnodes != (1 << (T.L)) - 1) return fail("tree is not perfect", n, leaf);
  for (int v = 0; v < T.nnodes; ++v) {
    if (T.is_leaf(v)) {
      if (T.size(v) > leaf) return fail("leaf too large", n, leaf);
      continue;
    }
    const int c1 = 2 * v + 1, c2 = 2 * v + 2;
    if (T.start[c1] != T.start[v] || T.end[c1] != T.start[c2] || T.end[c2] != T.end[v])
      return fail("children do not split the parent", n, leaf);
  }
  auto in = [](const std::vector<int>& idx, int64_t a, int64_t b, int x) {
    return std::binary_search(idx.begin() + a, idx.begin() + b, x);
  };
  for (int v = 0; v < T.nnodes; ++v) {
    for (int64_t e = T.near_ptr[v]; e < T.near_ptr[v + 1]; ++e) {
      const int j = T.near_idx[e];
      if (e > T.near_ptr[v] && T.near_idx[e - 1] >= j) return fail("near list not sorted", n, leaf);
      if (!in(T.near_idx, T.near_ptr[j], T.near_ptr[j + 1], v)) return fail("near not symmetric", n, leaf);
      if (T.near_pos(v, j) != e) return fail("near_pos", n, leaf);
      if (in(T.coup_idx, T.coup_ptr[v], T.coup_ptr[v + 1], j)) return fail("near and coupling overlap", n, leaf);
    }
    for (int64_t e = T.coup_ptr[v]; e < T.coup_ptr[v + 1]; ++e) {
      const int j = T.coup_idx[e];
      if (e > T.coup_ptr[v] && T.coup_idx[e - 1] >= j) return fail("coupling list not sorted", n, leaf);
      if (!in(T.coup_idx, T.coup_ptr[j], T.coup_ptr[j + 1], v)) return fail("coupling not symmetric", n, leaf);
      if (T.coup_pos(v, j) != e) return fail("coup_pos", n, leaf);
      if (!T.admissible(v, j)) return fail("coupling pair not admissible", n, leaf);
    }
  }
  // every leaf pair covered exactly once
  const int lf = T.first_at(1), lc = T.count_at(1);
  std::vector<int> cover((size_t)lc * lc, 0);
  auto leaves_under = [&](int v, std::vector<int>& out) {
    std::vector<int> st{v};
    while (!st.empty()) {
      const int u = st.back();
      st.pop_back();
      if (T.is_leaf(u)) out.push_back(u - lf);
      else { st.push_back(2 * u + 1); st.push_back(2 * u + 2); }
    }
  };
  for (int v = 0; v < T.nnodes; ++v) {
    if (T.is_leaf(v))
      for (int64_t e = T.near_ptr[v]; e < T.near_ptr[v + 1]; ++e) {
        const int j = T.near_idx[e];
        if (!T.is_leaf(j)) return fail("near partner of a leaf is not a leaf", n, leaf);
        cover[(size_t)(v - lf) * lc + (j - lf)] += 1;
      }
    for (int64_t e = T.coup_ptr[v]; e < T.coup_ptr[v + 1]; ++e) {
      std::vector<int> a, b;
      leaves_under(v, a);
      leaves_under(T.coup_idx[e], b);
      for (int x : a)
        for (int y : b) cover[(size_t)x * lc + y] += 1;
      if (T.lca_level(v, T.coup_idx[e]) <= T.level(v)) return fail("lca below the pair", n, leaf);
    }
  }
  for (int c : cover)
    if (c != 1) return fail("leaf pairs not tiled exactly once", n, leaf);
  return 0;
}

int main() {
  const int sizes[][2] = {{1, 4}, {5, 8}, {17, 4}, {600, 32}, {1000, 7}, {3001, 50}, {4096, 64}};
  unsigned seed = 1;
  for (const auto& s : sizes)
    if (check(s[0], s[1], seed++, SPD_TREE_KD)) return 1;
  const int box[][2] = {{1, 4}, {5, 8}, {600, 64}, {3001, 128}, {4096, 100}};
  for (const auto& s : box)
    if (check(s[0], s[1], seed++, SPD_TREE_BOX)) return 1;
  std::printf("tree_check ok\n");
  return 0;
}
