// A continuous-batching solve server.
//
// Requests (particle configurations of any size) are queued on submit.  Each
// call to step() is one scheduling tick:
//   1. admission: queued requests, in arrival order, are admitted while a free
//      node range of the arena (first fit) and device-memory budget allow;
//      admission builds the request's geometry, near lists and QBX correction
//      and its boundary label;
//   2. residual: requests between refinement steps get r = f - A sigma with
//      the FP64 operator (one fused launch for all of them), and either finish
//      or start a GMRES cycle on r (per-request inner tolerance);
//   3. iteration: one Arnoldi step for every request inside a cycle (the
//      captured batch iteration graph: fused far field, correction, CGS2,
//      device-side Givens);
//   4. cycle end: requests whose cycle converged or filled the Krylov space
//      update sigma += V y and return to step 2;
//   5. finish: forces, torques and energy; the request's results are copied
//      to the host and its arena range, slot and memory are released.
// Requests therefore join and leave the running set between iterations, their
// work shares every fused launch, and each request's arithmetic is the same as
// when it runs alone (its plans depend only on its own size).
//
// Requests of at least fmm_min_nodes nodes take the FMM lane instead: admitted
// by the memory budget alone, each is solved as a standalone problem with the
// FMM far field (mixed precision, FP64 FMM residuals and forces) by one of a
// few worker threads, each on its own stream, so that their kernels overlap on
// the device with the fused iterations of the small requests.  A request's
// result depends only on the request.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>

#include "arena.h"
#include "batch.h"
#include "common.h"
#include "problem.h"

using namespace yq;

namespace yq {

// Starts a GMRES cycle for the listed slots: V0 = r / beta, fresh Hessenberg state.
__global__ void sstart_kernel(int ns, const int* __restrict__ slots, const double* __restrict__ beta,
                              const double* __restrict__ bn, const double* __restrict__ rt, int m,
                              int* __restrict__ active, int* __restrict__ jc, int* __restrict__ kc,
                              int* __restrict__ conv, double* __restrict__ scale,
                              double* __restrict__ gv, double* __restrict__ bnorm,
                              double* __restrict__ rtol) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  const int c = slots[t];
  active[c] = 1;
  jc[c] = 0;
  kc[c] = 0;
  conv[c] = 0;
  scale[c] = 1.0 / beta[t];
  double* g = gv + (int64_t)c * (m + 1);
  g[0] = beta[t];
  for (int k = 1; k <= m; ++k) g[k] = 0.0;
  bnorm[c] = bn[t];
  rtol[c] = rt[t];
}

// V0 = r scale (and its FP32 copy in V32 when given, for the mixed solves'
// Gram-Schmidt passes).
__global__ void sscale_kernel(const int* __restrict__ node_conf, int64_t T,
                              const int* __restrict__ mask, const double* __restrict__ scale,
                              const double* __restrict__ r, double* __restrict__ V,
                              float* __restrict__ V32) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= T) return;
  const int c = node_conf[g];
  if (c < 0 || !mask[c]) return;
  const double v = r[g] * scale[c];
  V[g] = v;
  if (V32) V32[g] = (float)v;
}

}  // namespace yq

namespace {

enum Phase { QUEUED = 0, RUNNING = 1, DONE = 2, FAILED = 3 };
enum Step { RESID = 0, ITER = 1, FINISH = 2 };

double now_s() {
  static const auto t0 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Request {
  int64_t id = 0;
  int phase = QUEUED;
  int step = RESID;
  int n = 0;
  std::vector<double> center, angle, axes;
  double kappa = 1.0;
  int label_kind = YQ_LABEL_ARC;
  double p0 = 0.0, p1 = 0.0;
  int64_t N = 0;
  double est_bytes = 0.0;
  double t_submit = 0.0, t_done = 0.0;
  bool fmm_lane = false;
  std::atomic<bool> cancel{false};
  // running state
  int slot = -1;
  int64_t off = 0;
  std::unique_ptr<yq_problem, void (*)(yq_problem*)> pb{nullptr, yq_destroy};
  bool x_zero = true;
  int budget = 0;
  double fnorm = 0.0, rel = 1.0;
  yq_solve_info info{};
  // results
  std::vector<double> sigma, force, torque;
  double energy = 0.0;
  int status = YQ_OK;
  std::string err;
};

}  // namespace

struct yq_server {
  yq_params prm{};
  Engine eng;
  int64_t capacity = 0;
  int max_slots = 0;
  MemBudget budget;     // device bytes of admitted requests (estimates)
  NodeArena arena;      // node ranges of the fused lane's requests
  std::vector<Request*> slots;
  std::deque<Request*> queue;
  std::map<int64_t, std::unique_ptr<Request>> reqs;
  int64_t next_id = 1;
  std::string err;
  DevBuf<int> d_slots;
  DevBuf<double> d_vals;
  int64_t completed_total = 0;
  // FMM lane
  int device = 0;
  int64_t fmm_min_nodes = std::numeric_limits<int64_t>::max();
  int fmm_workers = 2;
  int fmm_inflight = 0;                 // admitted to the lane and not yet collected
  std::mutex mu;
  std::condition_variable cv;           // work for the workers
  std::condition_variable cv_done;      // a worker finished a request
  std::deque<Request*> fmm_queue;       // waiting for a worker (guarded by mu)
  std::vector<Request*> fmm_done;       // finished by a worker (guarded by mu)
  bool stop = false;                    // guarded by mu
  std::vector<std::unique_ptr<HostThread>> workers;
};

namespace {

thread_local std::string g_srv_err;

template <class F>
int sguard(yq_server* s, F&& fn) {
  try {
    fn();
    return YQ_OK;
  } catch (const Error& e) {
    if (s) s->err = e.msg;
    g_srv_err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    if (s) s->err = e.what();
    g_srv_err = e.what();
    return YQ_EDEVICE;
  } catch (...) {
    if (s) s->err = "unknown error";
    return YQ_EDEVICE;
  }
}

// Device bytes a request of N nodes will hold (geometry, QBX correction and its
// gradient twins, partial sums), an upper estimate used for admission.
double estimate_bytes(const yq_params& p, int64_t N) {
  const double per_node = 7 * 8 + 2 * 4 + 3.0 * (2 * p.qbx_window + 1) * Q * 8 + 8 * 6 + 4 * 2;
  const FarPlan fp = far_plan(N, N, 256, 4096);
  return N * per_node + (double)fp.chunks * N * 12 + (double)fp.chunks * 2 * N * 8 + (1 << 20);
}

// The same for an FMM-lane request: geometry and QBX correction, the Krylov
// basis and work vectors, the two FMM instances.
double estimate_fmm_bytes(const yq_params& p, int64_t N) {
  const double per_node = 7 * 8 + 2 * 4 + 3.0 * (2 * p.qbx_window + 1) * Q * 8 + 8 * 6 + 4 * 2;
  return N * (per_node + 8.0 * (p.restart + 8) + 160.0) + (128 << 20);
}

// Solves one FMM-lane request on the calling worker's stream; fills its results.
void run_fmm_request(const yq_params& prm, Request* r, hipStream_t st) {
  yq_params p = prm;
  p.far_mode = YQ_FAR_FMM;
  yq_problem* raw = nullptr;
  int status = yq_create(&p, &raw);
  std::unique_ptr<yq_problem, void (*)(yq_problem*)> pb(raw, yq_destroy);
  std::string err = status == YQ_OK ? "" : yq_last_error(nullptr);
  try {
    if (status == YQ_OK) status = yq_set_stream(pb.get(), st);
    if (status == YQ_OK)
      status = yq_set_particles(pb.get(), r->n, r->center.data(), r->angle.data(), r->axes.data(),
                                r->kappa);
    DevBuf<double> f, sg, F, Tq;
    if (status == YQ_OK) {
      f.alloc(r->N);
      sg.alloc(r->N);
      F.alloc(2 * r->n);
      Tq.alloc(r->n);
      status = yq_boundary_label(pb.get(), r->label_kind, r->p0, r->p1, f.p);
    }
    if (status == YQ_OK) status = yq_set_boundary_data(pb.get(), f.p);
    int solved = YQ_EDEVICE;
    if (status == YQ_OK) {
      solved = yq_solve(pb.get(), nullptr, sg.p, &r->info);
      status = (solved == YQ_OK || solved == YQ_ENOCONV) ? YQ_OK : solved;
    }
    if (status == YQ_OK) status = yq_forces(pb.get(), sg.p, 1.0, F.p, Tq.p, &r->energy);
    if (status == YQ_OK) {
      r->sigma.assign(r->N, 0.0);
      r->force.assign(2 * r->n, 0.0);
      r->torque.assign(r->n, 0.0);
      YQ_HIP(hipMemcpyAsync(r->sigma.data(), sg.p, r->N * sizeof(double), hipMemcpyDeviceToHost, st));
      YQ_HIP(hipMemcpyAsync(r->force.data(), F.p, 2 * r->n * sizeof(double), hipMemcpyDeviceToHost,
                            st));
      YQ_HIP(hipMemcpyAsync(r->torque.data(), Tq.p, r->n * sizeof(double), hipMemcpyDeviceToHost,
                            st));
      YQ_HIP(hipStreamSynchronize(st));
      status = solved;      // YQ_OK or YQ_ENOCONV
    } else if (pb) {
      err = yq_last_error(pb.get());
    }
  } catch (const Error& e) {
    status = e.code;
    err = e.msg;
  } catch (const std::exception& e) {
    status = YQ_EDEVICE;
    err = e.what();
  }
  r->status = status;
  r->err = err;
  r->rel = r->info.residual;
}

void fmm_worker(yq_server* s) {
  (void)hipSetDevice(s->device);
  hipStream_t st = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] { return s->stop || !s->fmm_queue.empty(); });
      if (s->stop) break;
      r = s->fmm_queue.front();
      s->fmm_queue.pop_front();
    }
    if (r->cancel.load()) {
      r->status = YQ_ESTATE;
      r->err = "cancelled";
    } else if (!have_stream) {
      r->status = YQ_EDEVICE;
      r->err = "worker stream creation failed";
    } else {
      run_fmm_request(s->prm, r, st);
    }
    r->t_done = now_s();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->fmm_done.push_back(r);
    }
    s->cv_done.notify_all();
  }
  if (have_stream) (void)hipStreamDestroy(st);
}

void stop_workers(yq_server* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto& t : s->workers) t->join();
  s->workers.clear();
}

void sync_members(yq_server* s) {
  Engine& e = s->eng;
  for (int c = 0; c < s->max_slots; ++c) {
    Request* r = s->slots[c];
    e.members[c] = Member{r ? r->pb.get() : nullptr, r ? r->off : 0};
  }
  e.rebuild();
}

std::vector<double> masked_norms(yq_server* s, const std::vector<int>& mask, const double* x) {
  Engine& e = s->eng;
  e.upload_mask(e.inc, mask);
  e.dots(e.inc.p, x, x);
  std::vector<double> v = e.read_nrm();
  for (double& q : v) q = std::sqrt(std::max(q, 0.0));
  return v;
}

void fail_request(yq_server* s, Request* r, int code, const std::string& msg) {
  r->phase = FAILED;
  r->status = code;
  r->err = msg;
  r->t_done = now_s();
  (void)s;
}

}  // namespace

extern "C" {

int yq_server_create(const yq_params* params, int64_t node_capacity, int32_t max_slots,
                     double mem_budget_bytes, yq_server** out) {
  return sguard(nullptr, [&] {
    YQ_REQUIRE(params && out, YQ_EINVAL, "null argument");
    YQ_REQUIRE(node_capacity > 0 && max_slots >= 1 && mem_budget_bytes > 0, YQ_EINVAL,
               "capacity, slots and budget must be positive");
    yq_problem* probe = nullptr;
    int st = yq_create(params, &probe);
    YQ_REQUIRE(st == YQ_OK, st, std::string("bad parameters: ") + yq_last_error(nullptr));
    yq_destroy(probe);
    YQ_REQUIRE(params->far_mode != YQ_FAR_CUTOFF, YQ_EINVAL,
               "the cutoff far field is available to single problems only");
    YQ_REQUIRE(params->sl_coupling == 0.0, YQ_EINVAL,
               "the combined representation (sl_coupling > 0) is available to single problems only");
    YQ_REQUIRE(params->refine_levels == 0, YQ_EINVAL,
               "adaptive panel refinement is available to single problems only");
    auto s = std::make_unique<yq_server>();
    s->prm = *params;
    s->capacity = node_capacity;
    s->max_slots = max_slots;
    s->budget.limit = mem_budget_bytes;
    s->arena.reset(node_capacity);
    s->slots.assign(max_slots, nullptr);
    s->eng.init(*params);
    s->eng.T = node_capacity;
    s->eng.members.assign(max_slots, Member{});
    s->eng.rebuild();
    // arena vectors start at zero
    s->eng.upload_mask(s->eng.inc, std::vector<int>(max_slots, 0));
    s->d_slots.alloc(max_slots);
    s->d_vals.alloc(3 * (size_t)max_slots);
    YQ_HIP(hipGetDevice(&s->device));
    if (params->far_mode == YQ_FAR_FMM)
      s->fmm_min_nodes = 0;
    else if (params->far_mode == YQ_FAR_AUTO)
      s->fmm_min_nodes = kFmmAutoNodes;
    *out = s.release();
  });
}

void yq_server_destroy(yq_server* s) {
  if (!s) return;
  stop_workers(s);
  (void)hipStreamSynchronize(s->eng.stream);
  for (auto& kv : s->reqs) kv.second->pb.reset();
  delete s;
}

const char* yq_server_last_error(const yq_server* s) { return s ? s->err.c_str() : g_srv_err.c_str(); }

int yq_server_set_fmm(yq_server* s, int64_t min_nodes, int32_t workers) {
  return sguard(s, [&] {
    YQ_REQUIRE(s, YQ_EINVAL, "null server");
    YQ_REQUIRE(min_nodes >= 0 && workers >= 1 && workers <= 8, YQ_EINVAL,
               "min_nodes >= 0 and 1 <= workers <= 8");
    YQ_REQUIRE(s->next_id == 1, YQ_ESTATE, "the FMM lane is set before the first submit");
    s->fmm_min_nodes = min_nodes;
    s->fmm_workers = workers;
  });
}

int yq_server_submit(yq_server* s, int32_t n, const double* center_xy, const double* angle,
                     const double* semi_axes, double kappa, int32_t label_kind, double p0,
                     double p1, int64_t* ticket) {
  return sguard(s, [&] {
    YQ_REQUIRE(s && center_xy && angle && semi_axes && ticket, YQ_EINVAL, "null argument");
    YQ_REQUIRE(n >= 1, YQ_EINVAL, "request without particles");
    YQ_REQUIRE(label_kind == YQ_LABEL_ARC || label_kind == YQ_LABEL_JANUS, YQ_EINVAL,
               "unknown label kind");
    auto r = std::make_unique<Request>();
    r->id = s->next_id++;
    r->n = n;
    r->center.assign(center_xy, center_xy + 2 * n);
    r->angle.assign(angle, angle + n);
    r->axes.assign(semi_axes, semi_axes + 2 * n);
    r->kappa = kappa;
    r->label_kind = label_kind;
    r->p0 = p0;
    r->p1 = p1;
    r->N = (int64_t)n * s->prm.panels_per_particle * Q;
    r->fmm_lane = r->N >= s->fmm_min_nodes;
    r->est_bytes = r->fmm_lane ? estimate_fmm_bytes(s->prm, r->N) : estimate_bytes(s->prm, r->N);
    r->t_submit = now_s();
    r->budget = s->prm.maxiter;
    *ticket = r->id;
    Request* rp = r.get();
    s->reqs[r->id] = std::move(r);
    if ((!rp->fmm_lane && rp->N > s->capacity) || rp->est_bytes > s->budget.limit) {
      fail_request(s, rp, YQ_EADMIT, "request exceeds the node capacity or the memory budget");
      throw Error{YQ_EADMIT, "request " + std::to_string(rp->id) +
                                 " exceeds the node capacity or the memory budget"};
    }
    s->queue.push_back(rp);
  });
}

int yq_server_step(yq_server* s, int32_t* completed, int32_t* running, int32_t* queued) {
  return sguard(s, [&] {
    YQ_REQUIRE(s, YQ_EINVAL, "null server");
    Engine& e = s->eng;
    const int m = e.m;
    const int S = s->max_slots;
    int done_now = 0;
    bool changed = false;
    // ---- 1. admission (arrival order, first fit) ----
    for (auto it = s->queue.begin(); it != s->queue.end();) {
      Request* r = *it;
      if (r->fmm_lane) {
        if (s->fmm_inflight >= s->fmm_workers || !s->budget.fits(r->est_bytes)) {
          ++it;
          continue;
        }
        if (s->workers.empty()) {
          // Lane solves allocate and free device memory from other threads; a
          // graph capture on the engine's stream must not overlap such calls,
          // so from here on the fused iteration is launched eagerly.
          s->eng.use_graphs = false;
          while ((int)s->workers.size() < s->fmm_workers)
            s->workers.push_back(std::make_unique<HostThread>([s] { fmm_worker(s); }));
        }
        r->phase = RUNNING;
        s->budget.take(r->est_bytes);
        ++s->fmm_inflight;
        {
          std::lock_guard<std::mutex> lk(s->mu);
          s->fmm_queue.push_back(r);
        }
        s->cv.notify_one();
        it = s->queue.erase(it);
        continue;
      }
      int slot = -1;
      for (int c = 0; c < S; ++c)
        if (!s->slots[c]) {
          slot = c;
          break;
        }
      int64_t off = 0;
      if (slot < 0) {
        ++it;
        continue;
      }
      if (!s->budget.fits(r->est_bytes) || !s->arena.take(r->N, off)) {
        ++it;
        continue;
      }
      yq_problem* pb = nullptr;
      int st = yq_create(&s->prm, &pb);
      r->pb.reset(pb);
      if (st == YQ_OK) {
        pb->batch_member = true;
        pb->stream = e.stream;
        st = yq_set_particles(pb, r->n, r->center.data(), r->angle.data(), r->axes.data(), r->kappa);
      }
      if (st == YQ_OK) st = yq_boundary_label(pb, r->label_kind, r->p0, r->p1, e.f.p + off);
      if (st == YQ_OK) st = yq_set_boundary_data(pb, e.f.p + off);
      if (st != YQ_OK) {
        fail_request(s, r, st, pb ? yq_last_error(pb) : "create failed");
        r->pb.reset();
        s->arena.give(off, r->N);
        it = s->queue.erase(it);
        continue;
      }
      r->slot = slot;
      r->off = off;
      r->phase = RUNNING;
      r->step = RESID;
      r->x_zero = true;
      s->slots[slot] = r;
      s->budget.take(r->est_bytes);
      it = s->queue.erase(it);
      changed = true;
    }
    if (changed) sync_members(s);
    // ---- 2. residuals ----
    std::vector<int> need(S, 0), fresh(S, 0), mv(S, 0);
    int nneed = 0;
    for (int c = 0; c < S; ++c) {
      Request* r = s->slots[c];
      if (r && r->step == RESID) {
        need[c] = 1;
        ++nneed;
        if (r->x_zero) fresh[c] = 1;
        else mv[c] = 1;
      }
    }
    if (nneed) {
      // sigma = 0 for fresh requests; r = f - A sigma otherwise.  The arena vector
      // `delta` holds every running request's sigma.
      e.upload_mask(e.inc, fresh);
      e.axpby(e.inc.p, 0.0, e.f.p, 0.0, nullptr, e.delta.p);  // sigma lives in delta
      e.axpby(e.inc.p, 1.0, e.f.p, 0.0, nullptr, e.r.p);
      bool anymv = std::any_of(mv.begin(), mv.end(), [](int v) { return v; });
      if (anymv) {
        e.upload_mask(e.inc, mv);
        e.matvec(YQ_FP64, e.inc.p, e.delta.p, nullptr, e.tmp.p);
        e.axpby(e.inc.p, 1.0, e.f.p, -1.0, e.tmp.p, e.r.p);
      }
      std::vector<double> rn = masked_norms(s, need, e.r.p);
      std::vector<double> fnv;
      bool anyfresh = std::any_of(fresh.begin(), fresh.end(), [](int v) { return v; });
      if (anyfresh) fnv = masked_norms(s, fresh, e.f.p);
      std::vector<int> start_slots;
      std::vector<double> vals;  // beta, bnorm, rtol per started slot
      for (int c = 0; c < S; ++c) {
        if (!need[c]) continue;
        Request* r = s->slots[c];
        if (fresh[c]) r->fnorm = fnv[c];
        else ++r->info.matvecs_fp64;
        r->rel = r->fnorm > 0.0 ? rn[c] / r->fnorm : 0.0;
        if (r->rel <= s->prm.tol || r->budget <= 0 || r->info.outer_steps >= s->prm.max_refine) {
          r->step = FINISH;
          continue;
        }
        double itol = s->prm.tol;
        if (s->prm.precision == YQ_MIXED)
          itol = std::min(0.5, std::max(s->prm.inner_tol, 0.5 * s->prm.tol / r->rel));
        else
          itol = s->prm.tol * r->fnorm / std::max(rn[c], 1e-300);
        r->step = ITER;
        r->x_zero = false;
        ++r->info.outer_steps;
        start_slots.push_back(c);
        vals.push_back(rn[c]);
        vals.push_back(rn[c]);
        vals.push_back(std::min(itol, 0.5));
      }
      if (!start_slots.empty()) {
        const int ns = (int)start_slots.size();
        std::vector<double> beta(ns), bn(ns), rt(ns);
        for (int k = 0; k < ns; ++k) {
          beta[k] = vals[3 * k];
          bn[k] = vals[3 * k + 1];
          rt[k] = vals[3 * k + 2];
        }
        YQ_HIP(hipMemcpyAsync(s->d_slots.p, start_slots.data(), ns * sizeof(int),
                              hipMemcpyHostToDevice, e.stream));
        YQ_HIP(hipMemcpyAsync(s->d_vals.p, beta.data(), ns * sizeof(double), hipMemcpyHostToDevice,
                              e.stream));
        YQ_HIP(hipMemcpyAsync(s->d_vals.p + S, bn.data(), ns * sizeof(double), hipMemcpyHostToDevice,
                              e.stream));
        YQ_HIP(hipMemcpyAsync(s->d_vals.p + 2 * S, rt.data(), ns * sizeof(double),
                              hipMemcpyHostToDevice, e.stream));
        sstart_kernel<<<(ns + 63) / 64, 64, 0, e.stream>>>(
            ns, s->d_slots.p, s->d_vals.p, s->d_vals.p + S, s->d_vals.p + 2 * S, m, e.active.p,
            e.jc.p, e.kc.p, e.conv.p, e.scale.p, e.gv.p, e.bnorm.p, e.rtol.p);
        std::vector<int> st(S, 0);
        for (int c : start_slots) st[c] = 1;
        e.upload_mask(e.inc, st);
        sscale_kernel<<<(unsigned)((e.T + 255) / 256), 256, 0, e.stream>>>(
            e.node_conf.p, e.T, e.inc.p, e.scale.p, e.r.p, e.V.p,
            s->prm.precision == YQ_MIXED ? e.V32.p : nullptr);
        YQ_HIP(hipGetLastError());
      }
    }
    // ---- 3. one Arnoldi step for every request inside a cycle ----
    std::vector<int> initer(S, 0);
    int niter = 0;
    for (int c = 0; c < S; ++c)
      if (s->slots[c] && s->slots[c]->step == ITER) {
        initer[c] = 1;
        ++niter;
      }
    if (niter) {
      e.run_iteration(s->prm.precision == YQ_MIXED ? YQ_MIXED : YQ_FP64);
      std::vector<int> act;
      e.count_active(act);
      std::vector<int> ended(S, 0);
      int nend = 0;
      for (int c = 0; c < S; ++c)
        if (initer[c] && !act[c]) {
          ended[c] = 1;
          ++nend;
        }
      if (nend) {
        e.upload_mask(e.inc, ended);
        std::vector<int> hk(S);
        YQ_HIP(hipMemcpyAsync(hk.data(), e.kc.p, S * sizeof(int), hipMemcpyDeviceToHost, e.stream));
        // y = H^-1 g, sigma += V y
        e.solve_cycle(e.inc.p, e.delta.p);
        YQ_HIP(hipStreamSynchronize(e.stream));
        for (int c = 0; c < S; ++c)
          if (ended[c]) {
            Request* r = s->slots[c];
            r->info.iterations += hk[c];
            if (s->prm.precision == YQ_MIXED) r->info.matvecs_fp32 += hk[c];
            else r->info.matvecs_fp64 += hk[c];
            r->budget -= hk[c];
            r->step = RESID;
          }
      }
    }
    // ---- 5. finish ----
    bool released = false;
    for (int c = 0; c < S; ++c) {
      Request* r = s->slots[c];
      if (!r || r->step != FINISH) continue;
      const double* sg = e.delta.p + r->off;
      r->force.assign(2 * r->n, 0.0);
      r->torque.assign(r->n, 0.0);
      r->sigma.assign(r->N, 0.0);
      DevBuf<double> F, Tq;
      F.alloc(2 * r->n);
      Tq.alloc(r->n);
      int st = yq_forces(r->pb.get(), sg, 1.0, F.p, Tq.p, &r->energy);
      if (st == YQ_OK) {
        YQ_HIP(hipMemcpyAsync(r->force.data(), F.p, 2 * r->n * sizeof(double), hipMemcpyDeviceToHost,
                              e.stream));
        YQ_HIP(hipMemcpyAsync(r->torque.data(), Tq.p, r->n * sizeof(double), hipMemcpyDeviceToHost,
                              e.stream));
        YQ_HIP(hipMemcpyAsync(r->sigma.data(), sg, r->N * sizeof(double), hipMemcpyDeviceToHost,
                              e.stream));
        YQ_HIP(hipStreamSynchronize(e.stream));
      }
      r->info.residual = r->rel;
      r->t_done = now_s();
      r->info.seconds = r->t_done - r->t_submit;
      r->phase = st == YQ_OK ? DONE : FAILED;
      r->status = st == YQ_OK ? (r->rel <= s->prm.tol ? YQ_OK : YQ_ENOCONV) : st;
      if (st != YQ_OK) r->err = yq_last_error(r->pb.get());
      s->slots[c] = nullptr;
      s->arena.give(r->off, r->N);
      s->budget.give(r->est_bytes);
      r->pb.reset();
      ++done_now;
      released = true;
    }
    if (released) sync_members(s);
    // ---- FMM lane: collect finished requests ----
    std::vector<Request*> fin;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      fin.swap(s->fmm_done);
    }
    for (Request* r : fin) {
      --s->fmm_inflight;
      s->budget.give(r->est_bytes);
      r->info.seconds = r->t_done - r->t_submit;
      if (r->cancel.load()) {
        r->status = YQ_ESTATE;
        r->err = "cancelled";
      }
      r->phase = (r->status == YQ_OK || r->status == YQ_ENOCONV) ? DONE : FAILED;
      ++done_now;
    }
    s->completed_total += done_now;
    if (completed) *completed = done_now;
    int nbatch = 0;
    for (auto* r : s->slots) nbatch += r ? 1 : 0;
    const int nrun = nbatch + s->fmm_inflight;
    if (nbatch == 0 && s->fmm_inflight > 0 && done_now == 0) {
      // only lane solves in flight: wait a little for one instead of spinning
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_done.wait_for(lk, std::chrono::milliseconds(10), [&] { return !s->fmm_done.empty(); });
    }
    if (running) *running = nrun;
    if (queued) *queued = (int)s->queue.size();
  });
}

int yq_server_result(yq_server* s, int64_t ticket, int32_t* state, int64_t* N, int32_t* n,
                     double* sigma, double* force, double* torque, double* energy,
                     yq_solve_info* info, double* latency_s) {
  return sguard(s, [&] {
    YQ_REQUIRE(s && state, YQ_EINVAL, "null argument");
    auto it = s->reqs.find(ticket);
    YQ_REQUIRE(it != s->reqs.end(), YQ_EINVAL, "unknown ticket");
    Request* r = it->second.get();
    *state = r->phase;
    if (N) *N = r->N;
    if (n) *n = r->n;
    if (r->phase == DONE || r->phase == FAILED) {
      if (sigma && !r->sigma.empty()) std::copy(r->sigma.begin(), r->sigma.end(), sigma);
      if (force && !r->force.empty()) std::copy(r->force.begin(), r->force.end(), force);
      if (torque && !r->torque.empty()) std::copy(r->torque.begin(), r->torque.end(), torque);
      if (energy) *energy = r->energy;
      if (info) *info = r->info;
      if (latency_s) *latency_s = r->t_done - r->t_submit;
    }
  });
}

int yq_server_release(yq_server* s, int64_t ticket) {
  return sguard(s, [&] {
    YQ_REQUIRE(s, YQ_EINVAL, "null server");
    auto it = s->reqs.find(ticket);
    YQ_REQUIRE(it != s->reqs.end(), YQ_EINVAL, "unknown ticket");
    YQ_REQUIRE(it->second->phase == DONE || it->second->phase == FAILED, YQ_ESTATE,
               "request still queued or running");
    s->reqs.erase(it);
  });
}

int yq_server_cancel(yq_server* s, int64_t ticket) {
  return sguard(s, [&] {
    YQ_REQUIRE(s, YQ_EINVAL, "null server");
    auto it = s->reqs.find(ticket);
    YQ_REQUIRE(it != s->reqs.end(), YQ_EINVAL, "unknown ticket");
    Request* r = it->second.get();
    if (r->phase == QUEUED) {
      s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), r), s->queue.end());
    } else if (r->phase == RUNNING && r->fmm_lane) {
      // a worker owns it: it ends, failed, when the server collects it
      r->cancel.store(true);
      return;
    } else if (r->phase == RUNNING) {
      std::vector<int> one(s->max_slots, 0);
      one[r->slot] = 1;
      // drop it from any running cycle before the slot is reused
      s->eng.upload_mask(s->eng.inc, one);
      s->eng.clear_active(s->eng.inc.p);
      s->slots[r->slot] = nullptr;
      s->arena.give(r->off, r->N);
      s->budget.give(r->est_bytes);
      r->pb.reset();
      sync_members(s);
    } else {
      return;
    }
    fail_request(s, r, YQ_ESTATE, "cancelled");
  });
}

}  // extern "C"
