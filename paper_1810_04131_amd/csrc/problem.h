// Internal definition of the problem handle (shared by api.hip and batch.hip).
#pragma once

#include <utility>
#include <vector>

#include "common.h"
#include "fmm.h"
#include <memory>

using namespace yq;

struct yq_problem {
  yq_params prm{};
  hipStream_t stream = nullptr;
  std::string err;

  int n = 0;
  int64_t N = 0;
  int64_t npan = 0;   // panels (n * P unless refined)
  bool refined = false;   // pan / poff describe the panels (adaptive refinement)
  double kappa = 0.0;
  bool ready = false;
  bool have_f = false;
  bool batch_member = false;  // workspace for GMRES/forces comes from the batch
  std::unique_ptr<Fmm> fmm;     // far-field FMM (inner operator) when enabled
  std::unique_ptr<Fmm> fmm_hi;  // higher-order FP64 FMM for residuals (fmm_resid_order > 0)
  int far_want = 16384;       // far-field plan parameter (far_plan)
  // cutoff far field: kappa x gap beyond which tile pairs are skipped, for the FP64
  // value sums, the FP64 gradient sums and the FP32 sums (HUGE_VAL: exact sums)
  double zcut64 = HUGE_VAL, zcut64g = HUGE_VAL, zcut32 = HUGE_VAL;

  std::vector<double> h_pc;  // [n*5]
  DevBuf<double> pc, x, y, nx, ny, w, wnx, wny, panel_h, pcx, pcy, pr;
  // FP32 far field: tile / group bounding circles, scaled relative positions,
  // per-matvec packed sources
  DevBuf<double4> ftile, fgrp, fpan;
  DevBuf<float2> frel;
  DevBuf<float4> fsrc;
  DevBuf<double> pot_partial;
  DevBuf<double> pfx, pfy, pfwx, pfwy, pfs;   // oversampled potential rule (PotFine)
  DevBuf<double> qfx, qfy, qfwx, qfwy;         // oversampled points of the QBX build
  bool pot_fine_ready = false;                // pf* hold this geometry's points
  DevBuf<int> nb_ptr, nb_idx, bad, ncnt;
  DevBuf<int4> pan;   // refined panels: (particle, base panel, level, index)
  DevBuf<int> poff;   // refined panels: first panel of every particle [n + 1]
  DevBuf<int> xrow, xpan;
  int64_t x_total = 0;
  DevBuf<double> xvals, xgvals;
  DevBuf<double> W, WGx, WGy;
  DevBuf<float> W32;   // W rounded to FP32 (the batch engine's inner operator)
  // QBX corrections folded into a near-field cache of this geometry: per node, bit sl
  // set where window panel sl was left out of the fold (some node outside the leaf's
  // P2P list), bit 31 where some extra panel was; per extra-panel entry, 1 where left out
  DevBuf<uint32_t> qf_umask;
  DevBuf<uint8_t> qf_xmask;
  DevBuf<int> qf_left;            // the nodes with a panel left out (qf_nleft of them)
  DevBuf<int> qf_cnt;
  int64_t qf_nleft = 0;
  const double* W32_src = nullptr;   // the W it was rounded from
  DevBuf<double> Lqbx, Lnear, Lpot, tab;
  Consts consts{};
  FarPlan fp{};
  DevBuf<double> partial, gpartial;
  DevBuf<float> partial32;
  DevBuf<double> f;
  // Krylov workspace
  DevBuf<double> V, kw, kr, kd, kpart, kred;
  PinnedBuf hpart;   // host copy of Krylov partial dot products
  PinnedBuf stage;   // set-up: staged host inputs
  PinnedBuf hflags;  // set-up: geometry check flag and near-panel total
  DevBuf<char> scan_tmp;
  bool interp_ready = false;   // Lqbx, Lnear, Lpot uploaded
  bool qbx_valid = false;      // W, WGx, WGy hold the current set-up's window correction
  DevBuf<double> wrot;         // per particle (cos, sin) of a rigid turn (time stepping)
  PinnedBuf rstage;
  // device-side Arnoldi bookkeeping (H, rotations, g, 1 / h_{j+1,j}, step status)
  DevBuf<double> gm;
  DevBuf<int> gstop;            // set when the GMRES cycle has stopped
  PinnedBuf hstat;              // host copy of the step status
  hipEvent_t step_ev[2] = {nullptr, nullptr};
  const int* stop_dev = nullptr;   // passed to the far-field launches while set
  const double* src_for = nullptr; // fsrc already holds the FP32 records of this vector
  DevBuf<double> gx, gy, en;
  DevBuf<double> delta;   // refinement correction
  // time stepping: circles of the repulsion model, per-particle potential, new
  // configuration, hydrophobic force and torque of the step, overlap flag
  DevBuf<double4> dcc;
  DevBuf<double> drad, dphi, dpnew, dfh, dth;
  DevBuf<int> dbad;
  PinnedBuf dstage;
  bool grad_ready = false;  // gpartial holds the direct gradient far field of the solve's sigma

  // per-phase timers
  static constexpr int NPHASE = 8;
  uint32_t prof_mask = 0;   // bit p: time the launches of phase p
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[NPHASE];
  std::vector<hipEvent_t> pool;

  hipEvent_t event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    YQ_HIP(hipEventCreate(&e));
    return e;
  }
  ~yq_problem() {
    for (auto& v : ev)
      for (auto& p : v) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
      }
    for (auto e : pool) (void)hipEventDestroy(e);
    for (auto e : step_ev)
      if (e) (void)hipEventDestroy(e);
  }

  Far32View far32() const {
    Far32View v;
    v.x = x.p;
    v.y = y.p;
    v.tile = ftile.p;
    v.grp = fgrp.p;
    v.pan = fpan.p;
    v.src = fsrc.p;
    v.N = N;
    v.s = kappa * LOG2E;
    v.kappa = kappa;
    v.qc = SQRT_LOG2E / kappa;   // the same expression as in pack32
    v.kap2 = (float)(kappa * kappa);
    v.nscale = (float)(kappa / SQRT_LOG2E);
    v.zcut = zcut32;
    return v;
  }

  // packs sigma into the FP32 source records (before every FP32 far field)
  void pack32(const double* sigma) {
    launch_pack32(frel.p, wnx.p, wny.p, sigma, N, SQRT_LOG2E / kappa, fsrc.p, stream);
  }

  GeomView view() const {
    GeomView g;
    g.n = n;
    g.P = prm.panels_per_particle;
    g.N = N;
    g.kappa = kappa;
    g.pc = pc.p;
    g.x = x.p;
    g.y = y.p;
    g.nx = nx.p;
    g.ny = ny.p;
    g.w = w.p;
    g.wnx = wnx.p;
    g.wny = wny.p;
    g.panel_h = panel_h.p;
    g.tab = tab.p;
    g.ftile = ftile.p;
    g.fgrp = fgrp.p;
    g.fpan = fpan.p;
    g.zcut = zcut64;
    g.zcut_g = zcut64g;
    g.eta = prm.sl_coupling;
    g.npan = npan;
    if (refined) {
      g.pan = pan.p;
      g.poff = poff.p;
    }
    return g;
  }
};

