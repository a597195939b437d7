// C ABI of the batch engine (include/yqbx.h, "Batched solves").
//
// Configurations below the FMM threshold are members of the fused engine (one
// persistent far-field launch per GMRES iteration for all of them); those at or
// above it get their own problem with the FMM far field and are solved by
// worker threads, largest first, each on its own stream, while the engine runs.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <limits>
#include <memory>
#include <numeric>
#include <string>

#include "batch.h"
#include "common.h"
#include "problem.h"

using namespace yq;

struct yq_batch {
  yq_params prm{};
  Engine eng;
  std::vector<std::unique_ptr<yq_problem, void (*)(yq_problem*)>> probs;
  std::vector<int64_t> offsets;       // [nconf + 1]
  std::vector<int64_t> poffsets;      // particle offsets [nconf + 1]
  int far_want = 4096;
  std::string err;
  bool ready = false;
  bool have_f = false;
  // configurations from fmm_min_nodes on take the FMM: as trees of the engine's
  // forest (fmm_in_engine), or as standalone problems solved by worker threads
  int64_t fmm_min_nodes = std::numeric_limits<int64_t>::max();
  int fmm_workers = 6;
  bool fmm_in_engine = true;
  std::vector<int> direct_idx;            // engine members (fused sums or forest trees)
  std::vector<int> fmm_idx;               // worker-thread (lane) configurations
  std::vector<hipStream_t> streams;       // one per worker (default priority)
  int device = 0;
  ~yq_batch() {
    for (hipStream_t s : streams) (void)hipStreamDestroy(s);
  }
};

namespace {

thread_local std::string g_batch_err;

template <class F>
int bguard(yq_batch* b, F&& fn) {
  try {
    fn();
    return YQ_OK;
  } catch (const Error& e) {
    if (b) b->err = e.msg;
    g_batch_err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    if (b) b->err = e.what();
    g_batch_err = e.what();
    return YQ_EDEVICE;
  } catch (...) {
    if (b) b->err = "unknown error";
    return YQ_EDEVICE;
  }
}

void require(const yq_batch* b) {
  YQ_REQUIRE(b != nullptr, YQ_EINVAL, "null batch");
  YQ_REQUIRE(b->ready, YQ_ESTATE, "yq_batch_set_configs has not been called");
}

// Waits for the work queued on every FMM-lane problem's stream (every batch call
// returns with its work done, so a later solve on a worker stream sees it).
void sync_lane(yq_batch* b) {
  for (int c : b->fmm_idx) YQ_HIP(hipStreamSynchronize(b->probs[c]->stream));
}

// Runs job(c, pb) for every configuration c of idx (the FMM lane's problems) on
// the worker threads (in order, from a shared queue), each problem on its worker's
// stream, while local() runs on this thread; then waits for the workers and raises
// the first failure (codes other than YQ_OK and YQ_ENOCONV).
template <class Job, class Local>
void run_workers(yq_batch* b, const std::vector<int>& idx, Job&& job, Local&& local) {
  const int nf = (int)idx.size();
  std::vector<int> codes(nf, YQ_OK);
  std::vector<std::string> errs(nf);
  std::atomic<int> next{0};
  {
    std::vector<std::unique_ptr<HostThread>> workers;   // joined on every exit path
    for (size_t w = 0; w < b->streams.size() && nf > 0; ++w) {
      workers.push_back(std::make_unique<HostThread>([&, w] {
        (void)hipSetDevice(b->device);
        for (int k = next++; k < nf; k = next++) {
          const int c = idx[k];
          yq_problem* pb = b->probs[c].get();
          pb->stream = b->streams[w];   // earlier work on its stream is done (sync_lane)
          const int st = job(c, pb);
          codes[k] = st;
          if (st != YQ_OK && st != YQ_ENOCONV) errs[k] = yq_last_error(pb);
        }
      }));
    }
    local();
  }
  for (int k = 0; k < nf; ++k)
    YQ_REQUIRE(codes[k] == YQ_OK || codes[k] == YQ_ENOCONV, codes[k],
               "configuration " + std::to_string(idx[k]) + ": " + errs[k]);
}

void rebuild_plans(yq_batch* b) {
  for (int c : b->direct_idx) {
    yq_problem* pb = b->probs[c].get();
    if (pb->fmm) continue;   // a forest tree: no fused far-field plan
    pb->far_want = b->far_want;
    pb->fp = far_plan(pb->N, pb->N, 256, b->far_want);
    pb->partial.alloc((size_t)pb->fp.chunks * pb->N);
    pb->partial32.alloc((size_t)pb->fp.chunks * pb->N);
  }
  b->eng.rebuild();
}

}  // namespace

extern "C" {

int yq_batch_create(const yq_params* params, yq_batch** out) {
  return bguard(nullptr, [&] {
    YQ_REQUIRE(params && out, YQ_EINVAL, "null argument");
    yq_problem* probe = nullptr;
    int st = yq_create(params, &probe);  // validates the parameters
    YQ_REQUIRE(st == YQ_OK, st, std::string("bad parameters: ") + yq_last_error(nullptr));
    yq_destroy(probe);
    YQ_REQUIRE(params->far_mode != YQ_FAR_CUTOFF, YQ_EINVAL,
               "the cutoff far field is available to single problems only");
    YQ_REQUIRE(params->sl_coupling == 0.0, YQ_EINVAL,
               "the combined representation (sl_coupling > 0) is available to single problems only");
    YQ_REQUIRE(params->refine_levels == 0, YQ_EINVAL,
               "adaptive panel refinement is available to single problems only");
    auto b = std::make_unique<yq_batch>();
    b->prm = *params;
    b->eng.init(*params);
    YQ_HIP(hipGetDevice(&b->device));
    if (params->far_mode == YQ_FAR_FMM)
      b->fmm_min_nodes = 0;
    else if (params->far_mode == YQ_FAR_AUTO)
      b->fmm_min_nodes = kFmmAutoNodes;
    *out = b.release();
  });
}

void yq_batch_destroy(yq_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->eng.stream);
  b->probs.clear();
  delete b;
}

const char* yq_batch_last_error(const yq_batch* b) { return b ? b->err.c_str() : g_batch_err.c_str(); }

int yq_batch_set_configs(yq_batch* b, int32_t nconf, const int32_t* np, const double* center_xy,
                         const double* angle, const double* semi_axes, const double* kappa) {
  return bguard(b, [&] {
    YQ_REQUIRE(b && np && center_xy && angle && semi_axes && kappa, YQ_EINVAL, "null argument");
    YQ_REQUIRE(nconf >= 1, YQ_EINVAL, "need at least one configuration");
    b->ready = false;
    b->have_f = false;
    b->probs.clear();
    b->eng.members.clear();
    b->direct_idx.clear();
    b->fmm_idx.clear();
    b->offsets.assign(nconf + 1, 0);
    b->poffsets.assign(nconf + 1, 0);
    int64_t pofs = 0;
    for (int c = 0; c < nconf; ++c) {
      YQ_REQUIRE(np[c] >= 1, YQ_EINVAL, "configuration " + std::to_string(c) + " has no particles");
      const int64_t Nc = (int64_t)np[c] * b->prm.panels_per_particle * Q;
      const bool big = Nc >= b->fmm_min_nodes;
      // a forest tree needs the MFMA translations and the FP64 residual FMM
      const bool tree = big && b->fmm_in_engine && b->prm.fmm_resid_order > 0 &&
                        b->prm.fmm_m2l != YQ_M2L_VALU;
      const bool lane = big && !tree;
      yq_params p = b->prm;
      if (big) p.far_mode = YQ_FAR_FMM;
      yq_problem* pb = nullptr;
      int st = yq_create(&p, &pb);
      YQ_REQUIRE(st == YQ_OK, st, "yq_create failed");
      b->probs.emplace_back(pb, yq_destroy);
      pb->far_want = b->far_want;
      if (lane) {
        b->fmm_idx.push_back(c);
      } else {
        pb->batch_member = true;
        pb->stream = b->eng.stream;
        b->direct_idx.push_back(c);
      }
      st = yq_set_particles(pb, np[c], center_xy + 2 * pofs, angle + pofs, semi_axes + 2 * pofs,
                            kappa[c]);
      YQ_REQUIRE(st == YQ_OK, st,
                 "configuration " + std::to_string(c) + ": " + yq_last_error(pb));
      // a lane problem's set-up is queued on its own stream; it is solved later on a
      // worker's stream, which does not order itself after that one
      if (lane) YQ_HIP(hipStreamSynchronize(pb->stream));
      b->offsets[c + 1] = b->offsets[c] + pb->N;
      pofs += np[c];
      b->poffsets[c + 1] = pofs;
    }
    b->eng.T = b->offsets[nconf];
    for (int c : b->direct_idx)
      b->eng.members.push_back(Member{b->probs[c].get(), b->offsets[c], b->poffsets[c]});
    if (!b->direct_idx.empty()) b->eng.rebuild();
    // worker threads take the largest configurations first; one stream per worker
    auto largest_first = [&](int x, int y) {
      const int64_t nx = b->offsets[x + 1] - b->offsets[x], ny = b->offsets[y + 1] - b->offsets[y];
      return nx != ny ? nx > ny : x < y;
    };
    std::sort(b->fmm_idx.begin(), b->fmm_idx.end(), largest_first);
    const int nw = std::min<int>(b->fmm_workers, (int)b->fmm_idx.size());
    while ((int)b->streams.size() < nw) {
      hipStream_t s = nullptr;
      YQ_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      b->streams.push_back(s);
    }
    b->ready = true;
  });
}

int yq_batch_num_nodes(const yq_batch* b, int64_t* total, int64_t* offsets) {
  if (!b || !total) return YQ_EINVAL;
  if (!b->ready) return YQ_ESTATE;
  *total = b->eng.T;
  if (offsets)
    for (size_t c = 0; c < b->offsets.size(); ++c) offsets[c] = b->offsets[c];
  return YQ_OK;
}

int yq_batch_boundary_label(yq_batch* b, int32_t kind, double a, double bb, double* f) {
  return bguard(b, [&] {
    require(b);
    YQ_REQUIRE(f, YQ_EINVAL, "null f");
    for (size_t c = 0; c < b->probs.size(); ++c) {
      int st = yq_boundary_label(b->probs[c].get(), kind, a, bb, f + b->offsets[c]);
      YQ_REQUIRE(st == YQ_OK, st, yq_last_error(b->probs[c].get()));
    }
    sync_lane(b);
  });
}

int yq_batch_set_boundary_data(yq_batch* b, const double* f) {
  return bguard(b, [&] {
    require(b);
    YQ_REQUIRE(f, YQ_EINVAL, "null f");
    if (!b->direct_idx.empty())     // the engine holds f only when it has members
      YQ_HIP(hipMemcpyAsync(b->eng.f.p, f, b->eng.T * sizeof(double), hipMemcpyDeviceToDevice,
                            b->eng.stream));
    for (size_t c = 0; c < b->probs.size(); ++c) {
      int st = yq_set_boundary_data(b->probs[c].get(), f + b->offsets[c]);
      YQ_REQUIRE(st == YQ_OK, st, yq_last_error(b->probs[c].get()));
    }
    YQ_HIP(hipStreamSynchronize(b->eng.stream));
    sync_lane(b);   // the lane problems' copies of f are queued on their own streams
    b->have_f = true;
  });
}

int yq_batch_apply_operator(yq_batch* b, const double* sigma, double* out, int32_t precision) {
  return bguard(b, [&] {
    require(b);
    YQ_REQUIRE(sigma && out && sigma != out, YQ_EINVAL, "null or aliased argument");
    YQ_REQUIRE(precision == YQ_FP64 || precision == YQ_MIXED, YQ_EINVAL, "bad precision");
    Engine& e = b->eng;
    if (!b->direct_idx.empty()) {
      std::vector<int> all(e.members.size(), 1);
      e.upload_mask(e.inc, all);
      e.matvec(precision, e.inc.p, sigma, nullptr, out);
    }
    for (int c : b->fmm_idx) {
      yq_problem* pb = b->probs[c].get();
      const int st = yq_apply_operator(pb, sigma + b->offsets[c], out + b->offsets[c], precision);
      YQ_REQUIRE(st == YQ_OK, st, yq_last_error(pb));
      YQ_HIP(hipStreamSynchronize(pb->stream));
    }
    YQ_HIP(hipStreamSynchronize(e.stream));
  });
}

}  // extern "C"

namespace {

struct ForcesOut {
  double gamma;
  double* force;
  double* torque;
  double* energy;
};

// yq_batch_solve, and with fo its forces: the lane problems through
// yq_solve_forces, the engine's members with the FP64 residual expected to be the
// last one also giving the gradient far field (no separate gradient pass for them).
int batch_solve(yq_batch* b, double* sigma, yq_solve_info* info, const ForcesOut* fo) {
  int status = YQ_OK;
  int rc = bguard(b, [&] {
    require(b);
    YQ_REQUIRE(sigma, YQ_EINVAL, "null sigma");
    YQ_REQUIRE(b->have_f, YQ_ESTATE, "boundary data not set");
    YQ_REQUIRE(!fo || (fo->force && fo->torque), YQ_EINVAL, "null argument");
    const int nconf = (int)b->probs.size();
    std::vector<yq_solve_info> all(nconf);
    std::vector<double> en(nconf, 0.0);
    // the fused iteration's graphs are captured before any worker starts, so no
    // capture overlaps the workers' allocations
    if (!b->direct_idx.empty()) b->eng.ensure_graphs();
    run_workers(
        b, b->fmm_idx,
        [&](int c, yq_problem* pb) {
          if (!fo) return yq_solve(pb, nullptr, sigma + b->offsets[c], &all[c]);
          return yq_solve_forces(pb, nullptr, sigma + b->offsets[c], &all[c], fo->gamma,
                                 fo->force + 2 * b->poffsets[c], fo->torque + b->poffsets[c],
                                 &en[c]);
        },
        [&] {   // the engine on this thread
          if (b->direct_idx.empty()) return;
          std::vector<yq_solve_info> inf;
          b->eng.solve(inf, sigma, fo != nullptr);
          for (size_t k = 0; k < inf.size(); ++k) all[b->direct_idx[k]] = inf[k];
          if (fo) {
            std::vector<double> ee;
            b->eng.forces(sigma, fo->gamma, fo->force, fo->torque, ee, &b->eng.grad_ok);
            for (size_t k = 0; k < ee.size(); ++k) en[b->direct_idx[k]] = ee[k];
          }
          YQ_HIP(hipStreamSynchronize(b->eng.stream));
        });
    for (int c = 0; c < nconf; ++c) {
      if (info) info[c] = all[c];
      if (!(all[c].residual <= b->prm.tol)) status = YQ_ENOCONV;
    }
    if (fo && fo->energy)
      for (int c = 0; c < nconf; ++c) fo->energy[c] = en[c];
  });
  if (rc != YQ_OK) return rc;
  if (status != YQ_OK) b->err = "at least one configuration did not reach the tolerance";
  return status;
}

}  // namespace

extern "C" {

int yq_batch_solve(yq_batch* b, double* sigma, yq_solve_info* info) {
  return batch_solve(b, sigma, info, nullptr);
}

int yq_batch_solve_forces(yq_batch* b, double* sigma, yq_solve_info* info, double gamma,
                          double* force, double* torque, double* energy) {
  const ForcesOut fo{gamma, force, torque, energy};
  return batch_solve(b, sigma, info, &fo);
}

int yq_batch_forces(yq_batch* b, const double* sigma, double gamma, double* force, double* torque,
                    double* energy) {
  return bguard(b, [&] {
    require(b);
    YQ_REQUIRE(b->have_f, YQ_ESTATE, "boundary data not set");
    YQ_REQUIRE(sigma && force && torque, YQ_EINVAL, "null argument");
    std::vector<double> en(b->probs.size(), 0.0);
    // the lane problems' forces on the worker threads; the engine members' (fused
    // sums and forest trees) as one batched pass here
    run_workers(
        b, b->fmm_idx,
        [&](int c, yq_problem* pb) {
          return yq_forces(pb, sigma + b->offsets[c], gamma, force + 2 * b->poffsets[c],
                           torque + b->poffsets[c], &en[c]);
        },
        [&] {
          if (b->direct_idx.empty()) return;
          std::vector<double> ee;
          b->eng.forces(sigma, gamma, force, torque, ee);
          for (size_t k = 0; k < ee.size(); ++k) en[b->direct_idx[k]] = ee[k];
        });

    if (energy)
      for (size_t c = 0; c < en.size(); ++c) energy[c] = en[c];
  });
}

int yq_batch_set_fmm(yq_batch* b, int64_t min_nodes, int32_t workers) {
  return bguard(b, [&] {
    YQ_REQUIRE(b, YQ_EINVAL, "null batch");
    YQ_REQUIRE(min_nodes >= 0 && workers >= 1 && workers <= 8, YQ_EINVAL,
               "min_nodes >= 0 and 1 <= workers <= 8");
    YQ_REQUIRE(!b->ready, YQ_ESTATE, "the FMM lane is set before yq_batch_set_configs");
    b->fmm_min_nodes = min_nodes;
    b->fmm_workers = workers;
  });
}

int yq_batch_set_fmm_engine(yq_batch* b, int32_t enable) {
  return bguard(b, [&] {
    YQ_REQUIRE(b, YQ_EINVAL, "null batch");
    YQ_REQUIRE(!b->ready, YQ_ESTATE, "the FMM mode is set before yq_batch_set_configs");
    b->fmm_in_engine = enable != 0;
  });
}

int yq_batch_set_near_cache(yq_batch* b, int64_t max_bytes) {
  return bguard(b, [&] {
    YQ_REQUIRE(b, YQ_EINVAL, "null batch");
    YQ_REQUIRE(max_bytes >= -1, YQ_EINVAL, "max_bytes must be >= -1");
    YQ_REQUIRE(!b->ready, YQ_ESTATE, "the near-field cache budget is set before yq_batch_set_configs");
    b->eng.near_budget = max_bytes;
  });
}

int yq_batch_near_cache_info(const yq_batch* b, int64_t* bytes, int32_t* trees32,
                             int32_t* trees64) {
  return bguard(const_cast<yq_batch*>(b), [&] {
    YQ_REQUIRE(b, YQ_EINVAL, "null batch");
    if (bytes) *bytes = b->eng.near_bytes;
    if (trees32) *trees32 = b->eng.near_trees32;
    if (trees64) *trees64 = b->eng.near_trees64;
  });
}

int yq_batch_set_symmetric_far(yq_batch* b, int32_t enable) {
  return bguard(b, [&] {
    YQ_REQUIRE(b, YQ_EINVAL, "null batch");
    YQ_REQUIRE(!b->ready, YQ_ESTATE, "the far-field kernel is set before yq_batch_set_configs");
    b->eng.sym32 = enable != 0;
  });
}

int yq_batch_profile_enable(yq_batch* b, int32_t enable) {
  return bguard(b, [&] {
    YQ_REQUIRE(b, YQ_EINVAL, "null batch");
    b->eng.set_profiling(enable != 0);
  });
}

namespace {
int profile_read(yq_batch* b, int kind, int32_t precision, int64_t* launches, double* total_ms,
                 double* pairs, double* bytes, int32_t reset) {
  return bguard(b, [&] {
    YQ_REQUIRE(b && launches && total_ms && pairs, YQ_EINVAL, "null argument");
    YQ_REQUIRE(precision == YQ_FP64 || precision == YQ_MIXED, YQ_EINVAL, "bad precision");
    int64_t n = 0;
    double ms = 0.0, pc = 0.0, by = 0.0;
    if (b->eng.prof_on || !b->eng.prof_ev[precision == YQ_MIXED ? 1 : 0][kind].empty())
      b->eng.read_profile(precision, kind, n, ms, pc, by, reset != 0);
    *launches = n;
    *total_ms = ms;
    *pairs = pc;
    if (bytes) *bytes = by;
  });
}
}  // namespace

int yq_batch_profile_read(yq_batch* b, int32_t precision, int64_t* launches, double* total_ms,
                          double* pairs, int32_t reset) {
  return profile_read(b, PK_DIRECT, precision, launches, total_ms, pairs, nullptr, reset);
}

int yq_batch_profile_read_leaf(yq_batch* b, int32_t precision, int64_t* launches,
                               double* total_ms, double* pairs, double* bytes, int32_t reset) {
  return profile_read(b, PK_LEAF, precision, launches, total_ms, pairs, bytes, reset);
}

int yq_batch_use_graphs(yq_batch* b, int32_t enable) {
  if (!b) return YQ_EINVAL;
  b->eng.use_graphs = enable != 0;
  return YQ_OK;
}

int yq_batch_autotune(yq_batch* b, int32_t* persist_out, int32_t* want_out) {
  return bguard(b, [&] {
    require(b);
    Engine& e = b->eng;
    if (b->direct_idx.empty()) {   // nothing runs through the fused engine
      if (persist_out) *persist_out = e.persist_blocks;
      if (want_out) *want_out = b->far_want;
      return;
    }
    const int persist_c[] = {1024, 2048, 4096, 8192};
    const int want_c[] = {2048, 4096, 8192};
    std::vector<int> all(e.members.size(), 1);
    e.upload_mask(e.inc, all);
    DevBuf<double> s, o;
    s.alloc(e.T);
    o.alloc(e.T);
    YQ_HIP(hipMemsetAsync(s.p, 0, e.T * sizeof(double), e.stream));
    hipEvent_t a, z;
    YQ_HIP(hipEventCreate(&a));
    YQ_HIP(hipEventCreate(&z));
    float best = 1e30f;
    int bp = 2048, bw = b->far_want;
    for (int wv : want_c) {
      b->far_want = wv;
      rebuild_plans(b);
      e.upload_mask(e.inc, all);
      for (int pv : persist_c) {
        e.persist_blocks = pv;
        e.matvec(YQ_MIXED, e.inc.p, s.p, nullptr, o.p);  // warm
        YQ_HIP(hipEventRecord(a, e.stream));
        for (int rep = 0; rep < 2; ++rep) e.matvec(YQ_MIXED, e.inc.p, s.p, nullptr, o.p);
        YQ_HIP(hipEventRecord(z, e.stream));
        YQ_HIP(hipEventSynchronize(z));
        float ms = 0.0f;
        YQ_HIP(hipEventElapsedTime(&ms, a, z));
        if (ms < best) {
          best = ms;
          bp = pv;
          bw = wv;
        }
      }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(z);
    b->far_want = bw;
    rebuild_plans(b);
    e.persist_blocks = bp;
    if (persist_out) *persist_out = bp;
    if (want_out) *want_out = bw;
  });
}

}  // extern "C"
