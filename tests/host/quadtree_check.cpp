// Checks of the adaptive quadtree and its FMM interaction lists (quadtree.h),
// built with the host compiler under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// For every ordered pair of leaves (T, S) it checks against a brute-force
// reading of the definitions that the pair is served exactly once: either S is
// in T's direct (U) list, or exactly one level holds an M2L term from S's
// ancestor to T's ancestor, and that the U list is exactly the set of leaves
// whose ancestors at the coarser of the two levels are adjacent.  It also checks
// the leaf sizes, that the leaves partition the nodes, and the parent / child /
// range consistency of every box.  Exit status 0 when every check passes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <set>
#include <vector>

#include "quadtree.h"

using namespace yq::qt;

static int failures = 0;
#define CHECK(c, ...)                          \
  do {                                         \
    if (!(c)) {                                \
      if (failures < 20) {                     \
        std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
        std::printf(__VA_ARGS__);              \
        std::printf("\n");                     \
      }                                        \
      ++failures;                              \
    }                                          \
  } while (0)

// Morton keys of points on the 2^dmax grid of their bounding square, sorted.
static std::vector<uint32_t> keys_of(const std::vector<double>& x, const std::vector<double>& y,
                                     int dmax) {
  const size_t n = x.size();
  double x0 = x[0], x1 = x[0], y0 = y[0], y1 = y[0];
  for (size_t i = 0; i < n; ++i) {
    x0 = std::min(x0, x[i]);
    x1 = std::max(x1, x[i]);
    y0 = std::min(y0, y[i]);
    y1 = std::max(y1, y[i]);
  }
  const double W = std::max(x1 - x0, y1 - y0) * (1.0 + 1e-9) + 1e-12;
  const double cx = 0.5 * (x0 + x1) - 0.5 * W, cy = 0.5 * (y0 + y1) - 0.5 * W;
  const int64_t m = 1LL << dmax;
  std::vector<uint32_t> k(n);
  for (size_t i = 0; i < n; ++i) {
    int64_t ix = (int64_t)((x[i] - cx) / W * m), iy = (int64_t)((y[i] - cy) / W * m);
    ix = std::min(std::max(ix, (int64_t)0), m - 1);
    iy = std::min(std::max(iy, (int64_t)0), m - 1);
    k[i] = (uint32_t)morton(ix, iy);
  }
  std::sort(k.begin(), k.end());
  return k;
}

static int ancestor(const Tree& t, int level, int box, int m) {
  for (int l = level; l > m; --l) box = t.lv[l].parent[box];
  return box;
}

static void check_tree(const char* name, const std::vector<uint32_t>& k, int dmax, int leaf_max,
                       int min_level) {
  const int64_t n = (int64_t)k.size();
  Tree t = build(k.data(), n, dmax, leaf_max, min_level);
  const int nl = (int)t.leaf_level.size();
  // boxes: ranges, parents, children
  for (int l = 0; l <= t.depth; ++l) {
    const Level& L = t.lv[l];
    CHECK((int)L.start.size() == L.nbox() && (int)L.child.size() == 4 * L.nbox(), "%s sizes", name);
    for (int b = 0; b < L.nbox(); ++b) {
      CHECK(L.count[b] > 0 || n == 0, "%s empty box", name);
      for (int j = L.start[b]; j < L.start[b] + L.count[b]; ++j)
        CHECK((int64_t)(k[j] >> (2 * (dmax - l))) == L.key[b], "%s node outside its box", name);
      if (b > 0) CHECK(L.key[b] > L.key[b - 1] && L.start[b] >= L.start[b - 1] + L.count[b - 1],
                       "%s level order", name);
      if (l > 0) {
        const Level& P = t.lv[l - 1];
        CHECK(P.child[4 * (size_t)L.parent[b] + L.cpos[b]] == b, "%s parent/child", name);
        CHECK(L.key[b] >> 2 == P.key[L.parent[b]], "%s parent key", name);
      }
      int sum = 0, nch = 0;
      for (int q = 0; q < 4; ++q) {
        const int c = L.child[4 * (size_t)b + q];
        if (c >= 0) {
          sum += t.lv[l + 1].count[c];
          ++nch;
        }
      }
      if (nch) CHECK(sum == L.count[b], "%s children do not cover the parent", name);
      CHECK((nch == 0) == (L.leaf[b] >= 0), "%s leaf flag", name);
      if (nch) CHECK(L.count[b] > leaf_max || l < min_level, "%s split below leaf_max", name);
      if (!nch) CHECK(L.count[b] <= leaf_max || l == dmax, "%s leaf over leaf_max", name);
      if (!nch && n > 0) CHECK(l >= min_level || l == dmax, "%s leaf above min_level", name);
    }
  }
  // leaves partition the sorted nodes in order
  int64_t pos = 0;
  for (int s = 0; s < nl; ++s) {
    CHECK(t.leaf_start[s] == pos, "%s leaves do not partition the nodes", name);
    pos += t.leaf_cnt[s];
  }
  CHECK(pos == n, "%s leaves miss nodes", name);
  // every ordered pair of leaves: U membership and M2L coverage
  std::vector<std::set<int>> V(t.depth + 1);
  std::vector<std::vector<std::set<int>>> Vset(t.depth + 1);
  for (int l = 2; l <= t.depth; ++l) {
    const Level& L = t.lv[l];
    Vset[l].resize(L.nbox());
    for (int b = 0; b < L.nbox(); ++b) {
      for (int e = L.ilp[b]; e < L.ilp[b + 1]; ++e) {
        const int sb = L.ils[e];
        const int ox = L.ix[sb] - L.ix[b], oy = L.iy[sb] - L.iy[b];
        CHECK(std::max(std::abs(ox), std::abs(oy)) >= 2 && std::max(std::abs(ox), std::abs(oy)) <= 3,
              "%s V entry not well separated", name);
        CHECK(L.ilo[e] == (ox + 3) * 7 + (oy + 3), "%s V offset", name);
        const int pb = L.parent[b], ps = L.parent[sb];
        const Level& P = t.lv[l - 1];
        CHECK(std::abs(P.ix[pb] - P.ix[ps]) <= 1 && std::abs(P.iy[pb] - P.iy[ps]) <= 1,
              "%s V entry's parents not adjacent", name);
        Vset[l][b].insert(sb);
      }
    }
  }
  int64_t upairs = 0;
  for (int T = 0; T < nl; ++T) {
    std::set<int> U(t.nbi.begin() + t.nbp[T], t.nbi.begin() + t.nbp[T + 1]);
    CHECK((int)U.size() == t.nbp[T + 1] - t.nbp[T], "%s duplicate U entry", name);
    for (int S = 0; S < nl; ++S) {
      const int dT = t.leaf_level[T], dS = t.leaf_level[S];
      const int m = std::min(dT, dS);
      const int aT = ancestor(t, dT, t.leaf_box[T], m), aS = ancestor(t, dS, t.leaf_box[S], m);
      const Level& L = t.lv[m];
      const bool adj = std::abs(L.ix[aT] - L.ix[aS]) <= 1 && std::abs(L.iy[aT] - L.iy[aS]) <= 1;
      CHECK(adj == (U.count(S) > 0), "%s U list of leaf %d vs %d (adjacent %d)", name, T, S, adj);
      int m2l = 0;
      for (int l = 2; l <= m; ++l) {
        const int bT = ancestor(t, dT, t.leaf_box[T], l), bS = ancestor(t, dS, t.leaf_box[S], l);
        m2l += (int)Vset[l][bT].count(bS);
      }
      CHECK(m2l == (adj ? 0 : 1), "%s pair (%d, %d) served by %d M2L terms (adjacent %d)", name, T,
            S, m2l, adj);
      upairs += adj ? (int64_t)t.leaf_cnt[T] * t.leaf_cnt[S] : 0;
    }
  }
  CHECK(upairs == t.p2p_pairs, "%s P2P pair count", name);
  std::printf("%-28s n=%-7lld depth=%-2d leaves=%-5d max_leaf=%-4d p2p_pairs=%lld\n", name,
              (long long)n, t.depth, nl, t.max_leaf, (long long)t.p2p_pairs);
}

int main() {
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U01(0.0, 1.0);
  const double pi = 3.14159265358979323846;
  // ellipse boundaries (nodes clustered on curves, as in the solver)
  {
    std::vector<double> x, y;
    for (int e = 0; e < 24; ++e) {
      const double cx = 30 * U01(rng), cy = 30 * U01(rng), th = 2 * pi * U01(rng);
      const double A = 0.8 + 0.4 * U01(rng), B = 0.4 + 0.2 * U01(rng);
      for (int j = 0; j < 512; ++j) {
        const double t = 2 * pi * (j + 0.5) / 512;
        const double u = A * std::cos(t), v = B * std::sin(t);
        x.push_back(cx + std::cos(th) * u - std::sin(th) * v);
        y.push_back(cy + std::sin(th) * u + std::cos(th) * v);
      }
    }
    check_tree("24 ellipses, leaf 64", keys_of(x, y, 14), 14, 64, 2);
    check_tree("24 ellipses, leaf 16", keys_of(x, y, 14), 14, 16, 2);
    check_tree("24 ellipses, dmax 6", keys_of(x, y, 6), 6, 16, 2);
  }
  // uniform points
  {
    std::vector<double> x(6000), y(6000);
    for (size_t i = 0; i < x.size(); ++i) {
      x[i] = U01(rng);
      y[i] = U01(rng);
    }
    check_tree("uniform, leaf 32", keys_of(x, y, 14), 14, 32, 2);
  }
  // one dense cluster in a wide box: deep, strongly non-uniform
  {
    std::vector<double> x, y;
    for (int i = 0; i < 3000; ++i) {
      x.push_back(0.5 + 1e-3 * U01(rng));
      y.push_back(0.5 + 1e-3 * U01(rng));
    }
    for (int i = 0; i < 400; ++i) {
      x.push_back(U01(rng));
      y.push_back(U01(rng));
    }
    check_tree("cluster + background", keys_of(x, y, 14), 14, 24, 2);
  }
  // coincident points (cannot be split below leaf_max: leaves at dmax)
  {
    std::vector<double> x(200, 0.25), y(200, 0.75);
    x.push_back(0.0);
    y.push_back(0.0);
    x.push_back(1.0);
    y.push_back(1.0);
    check_tree("coincident points", keys_of(x, y, 10), 10, 8, 2);
  }
  // small inputs
  {
    std::vector<double> x{0.3}, y{0.6};
    check_tree("one node", keys_of(x, y, 14), 14, 64, 2);
    std::vector<double> x2(64), y2(64);
    for (int i = 0; i < 64; ++i) {
      x2[i] = U01(rng);
      y2[i] = U01(rng);
    }
    check_tree("leaf_max nodes", keys_of(x2, y2, 14), 14, 64, 2);
    check_tree("no forced levels", keys_of(x2, y2, 14), 14, 8, 0);
  }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
