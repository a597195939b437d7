// Quadtree Yukawa FMM for the double-layer far field (fmm.hip).
#pragma once

#include <vector>

#include "common.h"

namespace yq {

struct FmmLevel {
  int nbox = 0;
  double w = 0.0;                 // box width
  int64_t off = 0;                // first box of the level in the expansion arrays
  DevBuf<double> cx, cy;          // centres
  DevBuf<int> parent;             // index at level - 1
  DevBuf<int> cpos;               // position (0..3) in the parent
  DevBuf<int> ch;                 // children indices at level + 1 [4 * nbox], -1 if empty
  DevBuf<int> tord;               // M2M / L2L order: boxes sorted by which children they have
  DevBuf<int> ilp, ils, ilo;      // interaction list: CSR over targets, source box, offset id
  DevBuf<int> ild;                // the same as a dense table [nbox * 49] (-1: none), its rows
                                  // in the M2L order below
  DevBuf<int> ord;                // M2L order: boxes grouped by the sets of offsets holding a source
  std::vector<uint64_t> occ;      // host: each box's set of far offsets holding a source (bit
                                  // i: the i-th far offset), in the M2L order
  double2* M = nullptr;           // expansions [nbox * (p + 1)], views into Fmm::Mall / Lall
  double2* L = nullptr;
};

constexpr int DMAX = 14;   // deepest quadtree level

// Per-level views of one tree for the M2L kernels.
struct M2LLevels {
  const int* ild[DMAX + 1];
  const int* ord[DMAX + 1];
  const double2* M[DMAX + 1];
  double2* L[DMAX + 1];
  int nbox[DMAX + 1];
  int64_t off[DMAX + 2];     // first box of each level in the packed multipoles (off[depth + 1] = total)
};

struct Fmm {
  int p = 20;
  int depth = 0;
  int leaf_max = 64;
  double x0 = 0.0, y0 = 0.0, W = 1.0, kappa = 1.0;
  int64_t N = 0;
  std::vector<FmmLevel> lv;       // 0..depth
  int64_t nbox_total = 0;         // boxes of every level
  DevBuf<double2> Mall, Lall;     // multipole and local expansions of every box, level by level
  DevBuf<int> perm;               // sorted position -> node index
  DevBuf<double> xs, ys, wnxs, wnys, qx, qy, outs;
  // leaves (boxes of any level that are not split), in node order
  int nleaf = 0;
  DevBuf<int> leaf_start, leaf_cnt;   // sorted-node range
  DevBuf<int> leaf_gid;               // box index in Mall / Lall
  DevBuf<double> leaf_cx, leaf_cy;    // box centre
  DevBuf<double> leaf_r;              // largest distance of a leaf node from the box centre
  DevBuf<int> leaf_of;                // sorted node -> its leaf
  DevBuf<int> nbp, nbi;               // P2P leaves (CSR, self included): every leaf whose
                                      // ancestor at the coarser of the two levels is adjacent
  int64_t p2p_pairs = 0;              // source-target pairs of one P2P pass
  int64_t p2p_srcs = 0;               // sum over the P2P entries of their source counts
  int64_t m2l_pairs = 0;              // box pairs of one M2L pass
  // Near-field cache: the leaf pass's pair coefficients K1(z)/z ((x - y) . w nu) for
  // this geometry, so that the pass reads them instead of evaluating them.  Entry e
  // of the P2P lists (target leaf b, source leaf nbi[e]) owns the block of
  // cnt(b) x cnt(nbi[e]) coefficients at blk_off[e], target-fastest.
  DevBuf<int64_t> blk_off;
  DevBuf<int2> ent;                   // entry e's source range: (first sorted node, count)
  DevBuf<float> nc32;                 // FP32 coefficients (the inner operator's leaf pass)
  DevBuf<double> nc64;                // FP64 coefficients (the FP64 leaf pass)
  int nc_kind = 0;                    // 0 none, 1 FP32, 2 FP64
  // the cache also holds the QBX corrections of these weights (set by whoever folds
  // them in; cleared with the cache)
  const void* nc_folded = nullptr;
  DevBuf<double> ss;                  // the density in sorted node order (cached passes)
  // P2M coefficients (with the FP32 cache): M_n of a leaf = sum over its sorted nodes
  // k of sigma_k pc32[k 2 (p + 1) + 2 n + (0: re, 1: im)]
  DevBuf<float> pc32;
  DevBuf<double2> tg;  // M2M / L2L tables: [level][cpos 0..3][k + 2p], k in -2p..2p
  DevBuf<double2> ts;  // M2L tables: [level][offset 0..48][k + 2p]
  int max_leaf = 0;
  bool built = false;
  bool use_mfma = true;   // M2M, M2L, L2L on the matrix cores (FP64 MFMA)
  int R16 = 0;            // 2 (p + 1) rounded up to a multiple of 16
  DevBuf<double> amat;    // M2L matrices [level][offset][R16 * R16] in MFMA operand order
  DevBuf<double> gmat;    // M2M / L2L matrices [level][child position][R16 * R16], same order
  DevBuf<int4> m2l_tiles; // every 16-box M2L tile: (level, first position in the level's M2L
                          // order, the union of its boxes' offset sets as two 32-bit halves)
  int n_m2l_tiles = 0;
  // FP32 M2L for the inner (FP32-class) applies: with s_n = n! (2 / (kappa w))^n per
  // level, the products run on M_n s_n and A_mn / (s_m s_n) in FP32 and give L_m / s_m
  bool want_m2l32 = false;
  DevBuf<float> amat32;   // scaled M2L matrices, the operand order of amat
  DevBuf<double> msc;     // s_n per level [level][n]
  DevBuf<double> mpk64;   // multipoles packed as M2L operands, FP64 [box][R16]
  DevBuf<float> mpk32;    // the same scaled by s_n, FP32
  PinnedBuf stage_up, stage_dn;   // set-up transfers (grow-only, reused by every build)
  DevBuf<char> stage_dev;         // device side of the batched uploads and copies
  DevBuf<double> bbox;            // node bounding box (xmin, xmax, ymin, ymax)
  DevBuf<uint32_t> keys, skeys;   // finest-level Morton keys, unsorted / sorted
  DevBuf<int> iota;               // 0..N-1 (sort payload)
  DevBuf<char> sort_tmp;          // radix-sort scratch

  hipEvent_t dn_done = nullptr;   // recorded after download()

  Fmm() = default;
  Fmm(const Fmm&) = delete;
  Fmm& operator=(const Fmm&) = delete;
  ~Fmm();
  // Queues the device part of the tree build (bounding box, Morton keys, their
  // stable sort, the sorted copies of positions and w nu) and the copy of the
  // sorted keys to the host; build() waits for that copy, so kernels queued in
  // between run while the host builds the levels and lists.
  void download(const double* dx, const double* dy, const double* dwnx, const double* dwny,
                int64_t n, hipStream_t s);
  void build(int64_t n, double kappa, int order, int leaf_max, const double* tab, hipStream_t s);
  void set_order(int q, const double* tab, hipStream_t s);
  void copy_tree(const Fmm& o, int q, const double* tab, hipStream_t s);
  // partial[i] = (2 pi / kappa^2) * far field at node i (the far-field kernels' scaling)
  // stop (optional device flag): the heavy kernels do nothing once it is set
  M2LLevels m2l_levels() const;
  template <typename T>
  void m2l_run(hipStream_t s, const int* stop, DevBuf<T>& mp, const T* A);
  void m2l_mfma(hipStream_t s, const int* stop = nullptr);
  void m2l_mfma32(hipStream_t s, const int* stop = nullptr);
  void tree_mfma(bool gather, int l, hipStream_t s);
  void expansions(const double* sigma, hipStream_t s, bool m2l32 = false,
                  const int* stop = nullptr);
  // gpart[i], gpart[N + i] = (2 pi / kappa^2) * gradient of the far field at node i (FP64)
  void apply_grad(const double* sigma, double* gpart, const double* tab, hipStream_t s);
  void apply(const double* sigma, double* partial, bool p2p_fp32, const double* tab,
             hipStream_t s, const int* stop = nullptr);
  // computes the near-field cache (FP64 coefficients, else FP32) for the current
  // geometry; p2p_pairs x 8 (or 4) bytes.  drop_near_cache frees it.
  void build_near_cache(bool f64, const double* tab, hipStream_t s);
  void drop_near_cache();
  // device bytes build_near_cache(f64) takes
  // The cached leaf pass hands a source leaf's densities to the lanes through one
  // wavefront exchange, so it needs leaves of at most 64 nodes (a tree built with a
  // larger leaf_max, or one whose depth limit left a bigger leaf, stays uncached).
  bool near_cacheable() const { return built && max_leaf <= 64; }
  int64_t near_cache_bytes(bool f64) const {
    return p2p_pairs * (f64 ? 8 : 4) + N * 8 + (f64 ? 0 : N * 2 * (p + 1) * 4);
  }
};

// One tree of an FMM forest as the forest kernels see it (device copy): the
// member's own sorted nodes, leaves, lists, expansions and tables, the batch
// configuration it belongs to (mask, Krylov column) and where its density and its
// far field live.
struct FmmDev {
  int cfg;                 // configuration index in the batch engine
  int depth, nleaf;
  int64_t N, off;          // nodes; offset of the configuration in the batch vectors
  int64_t p2p_pairs;       // source-target pairs of one leaf pass
  int64_t p2p_srcs;        // sum over its P2P entries of their source counts
  const int64_t* blk_off;  // near-field cache (nc_kind 1: float, 2: double; 0: none)
  const int2* ent;
  const void* nc;
  int nc_kind;
  double* ss;
  const float* pc32;       // P2M coefficients (FP32 cache), or null
  double kappa;
  const int* perm;
  const double *xs, *ys, *wnxs, *wnys;
  double *qx, *qy;
  const int *leaf_start, *leaf_cnt, *leaf_gid, *nbp, *nbi;
  const double *leaf_cx, *leaf_cy, *leaf_r;
  const int* leaf_of;
  double2 *Mall, *Lall;
  M2LLevels lv;
  const int* ch[DMAX + 1];
  const int* tord[DMAX + 1];
  const double* gmat;      // M2M / L2L matrices
  const void* amat;        // M2L matrices (FP64, or the scaled FP32 copy)
  void* mpk;               // packed multipoles (FP64 or FP32)
  const double* msc;
  const int4* m2l_tiles;
  const double* tab;
  double* out;             // far field of the member's nodes, node order (2 pi / kappa^2 scaling)
  double* gout;            // its gradient [2 N] (x, then y), the gradient kernels' scaling
};

// Many quadtrees (one per batch configuration, all of one expansion order) whose
// FMM passes run as one launch per pass over every tree: gather, P2M, M2M per
// level, multipole packing, M2L (all levels), L2L per level, L2P + P2P.  Each
// tree's arithmetic is that of Fmm::apply on it alone; a block whose
// configuration's mask entry is 0 does nothing, so the launch sequence is fixed
// and can be captured in a graph.
struct FmmForest {
  int p = 0, R16 = 0, depth = 0;
  bool f32 = false;              // FP32 leaf pairs (the inner operator)
  int nmem = 0;
  DevBuf<FmmDev> dev;
  // work items (member, index within the member's launch of that pass)
  DevBuf<int2> it_gather, it_p2m, it_pack, it_m2l, it_leaf2, it_leaf4, it_leaves;
  DevBuf<int2> it_cleaf;         // leaves of the trees whose near-field cache the pass reads
  DevBuf<int2> it_cp2m;          // leaves of the trees holding P2M coefficients
  int n_cp2m = 0;
  int n_cleaf = 0, n_leaves = 0; // n_leaves: every leaf (it_leaves)
  std::vector<DevBuf<int2>> it_tree;   // per parent level l: M2M into / L2L out of level l
  int n_gather = 0, n_p2m = 0, n_pack = 0, n_m2l = 0, n_leaf2 = 0, n_leaf4 = 0;
  std::vector<int> n_tree;
  bool m2l32 = false;            // FP32 M2L (the trees' want_m2l32, inner operator only)
  // A member: its built FMM, its batch configuration, the offset of that
  // configuration in the batch vectors, the far-field output (FP64, node order,
  // the far-field kernels' 2 pi / kappa^2 scaling) and its FP64 Bessel table.
  struct Tree {
    Fmm* fmm;
    int cfg;
    int64_t off;
    double* out;
    double* gout;   // gradient output [2 N] (FP64 forests; may be null otherwise)
    const double* tab;
  };
  // p2p32: FP32 leaf pairs (and FP32 M2L where the trees were set up for it), as
  // the inner operator's Fmm::apply; else FP64 throughout.  All trees must share
  // one order and use the MFMA translations.  Synchronises s.
  void build(const std::vector<Tree>& trees, bool p2p32, hipStream_t s);
  // far field of every masked member for the density V + col[cfg] * T + off
  void apply(const int* mask, const double* V, const int* col, int64_t T, hipStream_t s) const;
  // its gradient (FP64 forests), as Fmm::apply_grad of each tree
  void apply_grad(const int* mask, const double* V, const int* col, int64_t T,
                  hipStream_t s) const;
  // the passes up to the local expansions (gather, P2M, M2M, M2L, L2L), and the leaf
  // passes after them: far field (leaves) or its gradient (leaves_grad, FP64 forests)
  void expansions(const int* mask, const double* V, const int* col, int64_t T,
                  hipStream_t s) const;
  // the local expansions' values at the nodes (out = L2P), then the leaf pass adds the
  // direct interactions.  pairs (may be null): adds the source-target pairs the leaf
  // pass evaluates and, into pairs[1], the algorithmic bytes of its cached trees
  // (coefficients once, each target's output read and written, each entry's source
  // densities once)
  void l2p(const int* mask, hipStream_t s) const;
  void leaves(const int* mask, hipStream_t s, unsigned long long* pairs = nullptr) const;
  void leaves_grad(const int* mask, hipStream_t s) const;
};

}  // namespace yq
