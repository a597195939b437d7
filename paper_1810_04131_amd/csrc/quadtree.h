// Adaptive quadtree of Morton-sorted nodes and the interaction lists of the
// FMM (host code only: no HIP types, so it also builds with a plain C++ compiler).
//
// Boxes: the root is the bounding square; a box is split into its (non-empty)
// quadrants while it holds more than leaf_max nodes, and always on levels below
// min_level, down to level dmax.  The nodes are sorted by their Morton keys on
// the 2^dmax x 2^dmax grid of the root, so every box holds a contiguous range of
// the sorted nodes and the boxes of a level are sorted by key.
//
// Lists (levels need not be equal between interacting leaves):
//   V (M2L, per box at levels >= 2): children of the parent's colleagues (the
//     adjacent boxes of the same level, the parent included) that are not
//     adjacent to the box.  Only boxes that exist appear, so a colleague that is a
//     leaf contributes nothing.
//   U (P2P, per leaf T): every leaf S whose ancestor at level min(level T, level
//     S) is adjacent to (or equal to) T's ancestor at that level.
// Every ordered pair of leaves (T, S) is then served exactly once: by U(T), or
// by the M2L at the first level where their ancestors are not adjacent (the
// parents there are adjacent, so the source ancestor is in the target
// ancestor's V list; the multipole reaches it by M2M and the local expansion
// reaches T by L2L).  A leaf coarser than a neighbour's subtree interacts with
// that whole subtree directly, which replaces the W and X lists of the classical
// adaptive FMM by direct sums.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <unordered_map>
#include <vector>

namespace yq {
namespace qt {

// Bit interleaving for Morton keys (x in the even bits), grid coordinates < 2^31.
inline uint64_t spread_bits(uint64_t v) {
  v &= 0x7fffffffULL;
  v = (v | (v << 16)) & 0x0000ffff0000ffffULL;
  v = (v | (v << 8)) & 0x00ff00ff00ff00ffULL;
  v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0fULL;
  v = (v | (v << 2)) & 0x3333333333333333ULL;
  v = (v | (v << 1)) & 0x5555555555555555ULL;
  return v;
}
inline uint64_t gather_bits(uint64_t v) {
  v &= 0x5555555555555555ULL;
  v = (v | (v >> 1)) & 0x3333333333333333ULL;
  v = (v | (v >> 2)) & 0x0f0f0f0f0f0f0f0fULL;
  v = (v | (v >> 4)) & 0x00ff00ff00ff00ffULL;
  v = (v | (v >> 8)) & 0x0000ffff0000ffffULL;
  v = (v | (v >> 16)) & 0x00000000ffffffffULL;
  return v;
}
inline int64_t morton(int64_t ix, int64_t iy) {
  return (int64_t)(spread_bits((uint64_t)ix) | (spread_bits((uint64_t)iy) << 1));
}
inline void unmorton(int64_t k, int64_t& ix, int64_t& iy) {
  ix = (int64_t)gather_bits((uint64_t)k);
  iy = (int64_t)gather_bits((uint64_t)k >> 1);
}

// Lookup of the boxes of one level by grid position: a dense table while the
// level's grid is small, a hash map above that.
struct BoxIndex {
  std::vector<int> dense;
  std::unordered_map<int64_t, int> sparse;
  void init(int level, const std::vector<int64_t>& keys) {
    const int64_t cells = 1LL << (2 * level);
    dense.clear();
    sparse.clear();
    if (cells <= (1LL << 24)) {
      dense.assign((size_t)cells, -1);
      for (size_t b = 0; b < keys.size(); ++b) dense[(size_t)keys[b]] = (int)b;
    } else {
      sparse.reserve(keys.size() * 2);
      for (size_t b = 0; b < keys.size(); ++b) sparse[keys[b]] = (int)b;
    }
  }
  int find(int64_t key) const {
    if (!dense.empty()) return key >= 0 && key < (int64_t)dense.size() ? dense[(size_t)key] : -1;
    auto it = sparse.find(key);
    return it == sparse.end() ? -1 : it->second;
  }
};

struct Level {
  std::vector<int64_t> key;     // Morton keys at this level, ascending
  std::vector<int> start, count;  // sorted-node range of each box
  std::vector<int> parent, cpos;  // box at the level above, position 0..3 in it (-1, 0 at the root)
  std::vector<int> child;       // [4 * nbox]: boxes at the level below, -1 where none
  std::vector<int> leaf;        // leaf index of a leaf box, -1 for split boxes
  std::vector<int> ix, iy;      // grid coordinates
  std::vector<int> col;         // [9 * nbox]: colleagues in (dx, dy) order, -1 where none
  std::vector<int> ilp, ils, ilo;  // V lists: CSR over boxes, source box, offset (ox+3)*7+(oy+3)
  int nbox() const { return (int)key.size(); }
};

struct Tree {
  int depth = 0;                 // deepest level holding a box
  std::vector<Level> lv;         // 0..depth
  // leaves in node order
  std::vector<int> leaf_level, leaf_box, leaf_start, leaf_cnt;
  std::vector<int> nbp, nbi;     // U lists over leaves (CSR; the leaf itself included)
  int max_leaf = 0;              // largest leaf (nodes)
  int64_t p2p_pairs = 0;         // sum over leaves of targets x U-list sources
};

// Builds the tree of n nodes whose Morton keys (on the 2^dmax grid) are skey,
// sorted ascending.  1 <= dmax <= 15, leaf_max >= 1, 0 <= min_level <= dmax.
inline Tree build(const uint32_t* skey, int64_t n, int dmax, int leaf_max, int min_level) {
  Tree t;
  t.lv.emplace_back();
  {
    Level& r = t.lv[0];
    r.key.push_back(0);
    r.start.push_back(0);
    r.count.push_back((int)n);
    r.parent.push_back(-1);
    r.cpos.push_back(0);
  }
  // top-down: split while over leaf_max (or above min_level)
  for (int l = 0;; ++l) {
    Level& L = t.lv[l];
    const int nb = L.nbox();
    L.child.assign(4 * (size_t)nb, -1);
    L.leaf.assign(nb, -1);
    std::vector<int> split(nb, 0);
    bool any = false;
    for (int b = 0; b < nb; ++b) {
      split[b] = l < dmax && (L.count[b] > leaf_max || l < min_level) && L.count[b] > 0;
      any = any || split[b];
    }
    if (!any) break;
    t.lv.emplace_back();
    Level& C = t.lv[l + 1];
    Level& P = t.lv[l];   // (the emplace may have moved the level)
    const int shift = 2 * (dmax - l - 1);
    for (int b = 0; b < nb; ++b) {
      if (!split[b]) continue;
      const uint32_t* lo = skey + P.start[b];
      const uint32_t* hi = lo + P.count[b];
      for (int q = 0; q < 4; ++q) {
        const int64_t ck = 4 * P.key[b] + q;
        const uint32_t* e = std::partition_point(lo, hi, [&](uint32_t k) {
          return (int64_t)(k >> shift) <= ck;
        });
        if (e > lo) {
          P.child[4 * (size_t)b + q] = C.nbox();
          C.key.push_back(ck);
          C.start.push_back((int)(lo - skey));
          C.count.push_back((int)(e - lo));
          C.parent.push_back(b);
          C.cpos.push_back(q);
        }
        lo = e;
      }
    }
  }
  t.depth = (int)t.lv.size() - 1;
  // leaves, in node order (boxes of one level are in node order; merge by start)
  {
    std::vector<std::pair<int, std::pair<int, int>>> lf;   // (start, (level, box))
    for (int l = 0; l <= t.depth; ++l) {
      Level& L = t.lv[l];
      if (L.child.empty()) L.child.assign(4 * (size_t)L.nbox(), -1);
      if (L.leaf.empty()) L.leaf.assign(L.nbox(), -1);
      for (int b = 0; b < L.nbox(); ++b) {
        bool has = false;
        for (int q = 0; q < 4; ++q) has = has || L.child[4 * (size_t)b + q] >= 0;
        if (!has && L.count[b] > 0) lf.push_back({L.start[b], {l, b}});
      }
    }
    std::sort(lf.begin(), lf.end());
    for (size_t k = 0; k < lf.size(); ++k) {
      const int l = lf[k].second.first, b = lf[k].second.second;
      t.lv[l].leaf[b] = (int)k;
      t.leaf_level.push_back(l);
      t.leaf_box.push_back(b);
      t.leaf_start.push_back(t.lv[l].start[b]);
      t.leaf_cnt.push_back(t.lv[l].count[b]);
      t.max_leaf = std::max(t.max_leaf, t.lv[l].count[b]);
    }
  }
  // grid coordinates and colleagues
  for (int l = 0; l <= t.depth; ++l) {
    Level& L = t.lv[l];
    const int nb = L.nbox();
    L.ix.resize(nb);
    L.iy.resize(nb);
    for (int b = 0; b < nb; ++b) {
      int64_t x, y;
      unmorton(L.key[b], x, y);
      L.ix[b] = (int)x;
      L.iy[b] = (int)y;
    }
    BoxIndex idx;
    idx.init(l, L.key);
    const int64_t lim = 1LL << l;
    L.col.assign(9 * (size_t)nb, -1);
    for (int b = 0; b < nb; ++b)
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy) {
          const int64_t qx = L.ix[b] + dx, qy = L.iy[b] + dy;
          if (qx < 0 || qy < 0 || qx >= lim || qy >= lim) continue;
          L.col[9 * (size_t)b + (dx + 1) * 3 + (dy + 1)] = idx.find(morton(qx, qy));
        }
  }
  // V lists
  for (int l = 0; l <= t.depth; ++l) {
    Level& L = t.lv[l];
    L.ilp.assign(1, 0);
    L.ils.clear();
    L.ilo.clear();
    if (l < 2) continue;
    const Level& Pl = t.lv[l - 1];
    for (int b = 0; b < L.nbox(); ++b) {
      const int* pc = &Pl.col[9 * (size_t)L.parent[b]];
      for (int e = 0; e < 9; ++e) {
        if (pc[e] < 0) continue;
        for (int q = 0; q < 4; ++q) {
          const int sb = Pl.child[4 * (size_t)pc[e] + q];
          if (sb < 0) continue;
          const int ox = L.ix[sb] - L.ix[b], oy = L.iy[sb] - L.iy[b];
          if (std::abs(ox) <= 1 && std::abs(oy) <= 1) continue;
          L.ils.push_back(sb);
          L.ilo.push_back((ox + 3) * 7 + (oy + 3));
        }
      }
      L.ilp.push_back((int)L.ils.size());
    }
  }
  // U lists
  const int nleaf = (int)t.leaf_level.size();
  t.nbp.assign(1, 0);
  std::vector<int> lst;
  for (int k = 0; k < nleaf; ++k) {
    const int dT = t.leaf_level[k], bT = t.leaf_box[k];
    lst.clear();
    // (i) leaves at the levels of T's ancestors (T included) adjacent to the ancestor
    int a = bT;
    for (int m = dT; m >= 0; --m) {
      const Level& L = t.lv[m];
      for (int e = 0; e < 9; ++e) {
        const int c = L.col[9 * (size_t)a + e];
        if (c >= 0 && L.leaf[c] >= 0) lst.push_back(L.leaf[c]);
      }
      if (m > 0) a = L.parent[a];
    }
    // (ii) every leaf below a split colleague of T
    const Level& LT = t.lv[dT];
    for (int e = 0; e < 9; ++e) {
      const int c = LT.col[9 * (size_t)bT + e];
      if (c < 0 || LT.leaf[c] >= 0) continue;
      const int s0 = LT.start[c], s1 = s0 + LT.count[c];
      auto it = std::lower_bound(t.leaf_start.begin(), t.leaf_start.end(), s0);
      for (; it != t.leaf_start.end() && *it < s1; ++it) lst.push_back((int)(it - t.leaf_start.begin()));
    }
    std::sort(lst.begin(), lst.end());
    lst.erase(std::unique(lst.begin(), lst.end()), lst.end());
    for (int s : lst) {
      t.nbi.push_back(s);
      t.p2p_pairs += (int64_t)t.leaf_cnt[k] * t.leaf_cnt[s];
    }
    t.nbp.push_back((int)t.nbi.size());
  }
  return t;
}

}  // namespace qt
}  // namespace yq
