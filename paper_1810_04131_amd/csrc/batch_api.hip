// C ABI of the batch engine (include/yqbx.h, "Batched solves").
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
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

void rebuild_plans(yq_batch* b) {
  for (auto& p : b->probs) {
    yq_problem* pb = p.get();
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
    auto b = std::make_unique<yq_batch>();
    b->prm = *params;
    b->eng.init(*params);
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
    b->offsets.assign(nconf + 1, 0);
    b->poffsets.assign(nconf + 1, 0);
    int64_t pofs = 0;
    for (int c = 0; c < nconf; ++c) {
      YQ_REQUIRE(np[c] >= 1, YQ_EINVAL, "configuration " + std::to_string(c) + " has no particles");
      yq_problem* pb = nullptr;
      int st = yq_create(&b->prm, &pb);
      YQ_REQUIRE(st == YQ_OK, st, "yq_create failed");
      b->probs.emplace_back(pb, yq_destroy);
      pb->batch_member = true;
      pb->far_want = b->far_want;
      pb->stream = b->eng.stream;
      st = yq_set_particles(pb, np[c], center_xy + 2 * pofs, angle + pofs, semi_axes + 2 * pofs,
                            kappa[c]);
      YQ_REQUIRE(st == YQ_OK, st,
                 "configuration " + std::to_string(c) + ": " + yq_last_error(pb));
      b->offsets[c + 1] = b->offsets[c] + pb->N;
      pofs += np[c];
      b->poffsets[c + 1] = pofs;
    }
    b->eng.T = b->offsets[nconf];
    for (int c = 0; c < nconf; ++c) b->eng.members.push_back(Member{b->probs[c].get(), b->offsets[c]});
    b->eng.rebuild();
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
  });
}

int yq_batch_set_boundary_data(yq_batch* b, const double* f) {
  return bguard(b, [&] {
    require(b);
    YQ_REQUIRE(f, YQ_EINVAL, "null f");
    YQ_HIP(hipMemcpyAsync(b->eng.f.p, f, b->eng.T * sizeof(double), hipMemcpyDeviceToDevice,
                          b->eng.stream));
    for (size_t c = 0; c < b->probs.size(); ++c) {
      int st = yq_set_boundary_data(b->probs[c].get(), f + b->offsets[c]);
      YQ_REQUIRE(st == YQ_OK, st, yq_last_error(b->probs[c].get()));
    }
    YQ_HIP(hipStreamSynchronize(b->eng.stream));
    b->have_f = true;
  });
}

int yq_batch_apply_operator(yq_batch* b, const double* sigma, double* out, int32_t precision) {
  return bguard(b, [&] {
    require(b);
    YQ_REQUIRE(sigma && out && sigma != out, YQ_EINVAL, "null or aliased argument");
    YQ_REQUIRE(precision == YQ_FP64 || precision == YQ_MIXED, YQ_EINVAL, "bad precision");
    Engine& e = b->eng;
    std::vector<int> all(e.members.size(), 1);
    e.upload_mask(e.inc, all);
    e.matvec(precision, e.inc.p, sigma, nullptr, out);
    YQ_HIP(hipStreamSynchronize(e.stream));
  });
}

int yq_batch_solve(yq_batch* b, double* sigma, yq_solve_info* info) {
  int status = YQ_OK;
  int rc = bguard(b, [&] {
    require(b);
    YQ_REQUIRE(sigma, YQ_EINVAL, "null sigma");
    YQ_REQUIRE(b->have_f, YQ_ESTATE, "boundary data not set");
    std::vector<yq_solve_info> inf;
    b->eng.solve(inf, sigma);
    YQ_HIP(hipStreamSynchronize(b->eng.stream));
    for (size_t c = 0; c < inf.size(); ++c) {
      if (info) info[c] = inf[c];
      if (!(inf[c].residual <= b->prm.tol)) status = YQ_ENOCONV;
    }
  });
  if (rc != YQ_OK) return rc;
  if (status != YQ_OK) b->err = "at least one configuration did not reach the tolerance";
  return status;
}

int yq_batch_forces(yq_batch* b, const double* sigma, double gamma, double* force, double* torque,
                    double* energy) {
  return bguard(b, [&] {
    require(b);
    YQ_REQUIRE(b->have_f, YQ_ESTATE, "boundary data not set");
    YQ_REQUIRE(sigma && force && torque, YQ_EINVAL, "null argument");
    for (size_t c = 0; c < b->probs.size(); ++c) {
      double e = 0.0;
      int st = yq_forces(b->probs[c].get(), sigma + b->offsets[c], gamma,
                         force + 2 * b->poffsets[c], torque + b->poffsets[c], &e);
      YQ_REQUIRE(st == YQ_OK, st, yq_last_error(b->probs[c].get()));
      if (energy) energy[c] = e;
    }
  });
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
