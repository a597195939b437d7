// Internal batch engine (batch.hip): fused kernels over many configurations.
#pragma once

#include <vector>

#include "common.h"
#include "problem.h"

namespace yq {

constexpr int SC = 1024;   // nodes per chunk of the symmetric FP32 far field (bsym32)

// matvec parts: the FMM members' expansions (and the FP32 source records), the
// forest's leaf pass, the direct members' fused far field, the finish; the timers
// bracket the two middle ones
constexpr int NPART = 4;
constexpr int PART_LEAF = 1, PART_DIRECT = 2;
constexpr int PK_DIRECT = 0, PK_LEAF = 1;

// What the fused kernels need of one configuration (device copy, one per config).
struct ConfDev {
  const double* x;
  const double* y;
  const double* wnx;
  const double* wny;
  Far32View f32;          // FP32 far-field view (its src is the configuration's own records)
  const float2* rel;      // scaled relative positions (pack input)
  const double* W;
  const float* W32;       // W in FP32 for the inner operator (null: W)
  const int* xrow;
  const int* xpan;
  const double* xvals;
  int qfold32, qfold64;   // the QBX correction is in the tree's FP32 / FP64 near-field cache
  const uint32_t* qumask; // then: the panels left out of the fold (qf_umask, qf_xmask)
  const uint8_t* qxmask;
  const double* tab;
  double* part64;
  float* part32;
  int64_t N;      // nodes
  int64_t off;    // offset of its nodes in the arena vectors
  double kappa;
  double kap2;
  int P, win;
  int tblocks, chunks, chunk;
  int chunks32;   // FP32 partial slots: chunks (bfar32) or ceil(N / SC) (bsym32)
  int kb;         // Krylov reduction blocks
  int64_t kpoff;  // offset of its multi-dot partials
  int fmm;        // far field from the FMM forest (part64, one chunk), not the fused sums
  // forces: node normals and weights, the particle table, the gradient rows of the
  // window correction and of the extra near panels, the gradient far-field partials
  const double* nx;
  const double* ny;
  const double* w;
  const double* pc;
  const double* WGx;
  const double* WGy;
  const double* xgvals;
  double* gpart;
  int n;          // particles
  int64_t poff;   // first particle in the batch's particle order
};

struct Member {
  yq_problem* pb = nullptr;  // not owned
  int64_t off = 0;
  int64_t poff = 0;          // first particle in the batch's particle order (forces)
};

struct Engine {
  yq_params prm{};
  int m = 100;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool use_graphs = true;
  int persist_blocks = 0;   // 0: default (2048)
  int64_t T = 0;            // arena capacity (nodes)
  std::vector<Member> members;

  DevBuf<double> tab64;       // FP64 Bessel coefficients (shared by all configurations)
  DevBuf<ConfDev> conf;
  DevBuf<int4> items;
  // symmetric FP32 far field: (configuration, chunk p, chunk q >= p) items
  bool sym32 = true;
  DevBuf<int4> sitems;
  int nsitems = 0;
  DevBuf<int2> kblk;
  DevBuf<int> node_conf;
  int nitems = 0, nkblk = 0;
  DevBuf<double> kpart;
  DevBuf<int> active, inc, jc, kc, conv, pmask, fmask;
  DevBuf<double> hb, H, cs, sn, gv, yv, scale, bnorm, rtol, res, nrm;
  DevBuf<double> V, w, r, tmp, delta, f;
  DevBuf<float> V32;             // the basis in FP32 (mixed solves' orthogonalisation)
  DevBuf<double> gx, gy, pen;   // forces: surface gradient [T], per-particle energies
  DevBuf<int2> fitems;          // forces: (configuration, particle) blocks
  int nfitems = 0;
  DevBuf<int2> litems;          // (configuration, node) of the QBX corrections left out of folds
  int nlitems = 0;
  // members with an FMM far field, as one forest per operator: the inner (FP32
  // leaf pairs and M2L) and the FP64 residual operator (the members' order-40 FMMs)
  FmmForest forest_in, forest_hi;
  // near-field caches of the forest trees (FP32 coefficients for the inner operator
  // first, then FP64 for the residual operator): at most this many bytes; -1: the
  // device memory free at the rebuild (with the caches already held) less a reserve of
  // a tenth of the device memory (at least 8 GiB)
  int64_t near_budget = -1;
  int64_t near_bytes = 0;      // bytes the caches hold
  int near_trees32 = 0, near_trees64 = 0;
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};   // FP64, mixed iteration
  hipGraphExec_t graph_part[2 * NPART] = {};            // the same in parts (timers on)
  // timers: events around every launch of the direct members' fused far field (kind
  // PK_DIRECT) and of the forest's leaf pass (PK_LEAF), and the number of
  // source-target pairs the launches evaluated, per precision and kind
  bool prof_on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[2][2];
  std::vector<hipEvent_t> ev_pool;
  DevBuf<unsigned long long> prof_pairs;   // [(precision * 2 + kind) * 2 + (pairs, bytes)]
  unsigned long long* prof_counter(int prec, int kind) const;
  void prof_record(int prec, int kind, hipEvent_t a, hipEvent_t b);

  ~Engine();
  void init(const yq_params& p);
  void rebuild();
  int grid_blocks(int n) const;   // persistent blocks for n work items
  void matvec(int prec, const int* mask, const double* Vin, const int* col, double* out);
  void matvec_part(int part, int prec, const int* mask, const double* Vin, const int* col,
                   double* out);
  void iteration_part(int prec, int part);
  void drop_graphs();
  hipEvent_t prof_event();
  void set_profiling(bool on);
  void read_profile(int prec, int kind, int64_t& launches, double& ms, double& pairs,
                    double& bytes, bool reset);
  void dots(const int* mask, const double* x, const double* y);
  void axpby(const int* mask, double a, const double* x, double b, const double* y, double* out);
  void iteration(int prec);
  void run_iteration(int prec);
  // captures the iteration graphs of both precisions now (when graphs are on)
  void ensure_graphs();
  int count_active(std::vector<int>& h);
  void solve_cycle(const int* mask, double* x);
  void clear_active(const int* mask);
  std::vector<double> read_nrm();
  void upload_mask(DevBuf<int>& d, const std::vector<int>& h);
  void gmres(int prec, const double* b, double* x, const std::vector<int>& incl,
             const std::vector<double>& tolv, std::vector<int>& iters, std::vector<int>& budget,
             std::vector<int>& converged, int& matvecs);
  // fuse (mixed precision): the FP64 residual expected to be the last one also
  // computes the gradient far field for the forces (grad_ok[c] when it holds that of
  // the returned solution)
  void solve(std::vector<yq_solve_info>& info, double* x_out, bool fuse = false);
  std::vector<char> grad_ok;
  // FP64 operator for plain and fused configurations (fused: with the gradient far field)
  void resid(const std::vector<int>& plain, const std::vector<int>& fused, const double* x,
             double* out);
  // forces, torques and energy of every member's particles for the density sigma
  // (arena layout): force [2 P], torque [P] at each member's particle offset;
  // energy[c] per member (eqs. stress, force_torque, scalar-torque, main)
  void forces(const double* sigma, double gamma, double* force, double* torque,
              std::vector<double>& energy, const std::vector<char>* grad_done = nullptr);
};

}  // namespace yq
