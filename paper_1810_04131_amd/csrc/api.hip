// The C ABI (include/yqbx.h): problem set-up, operator, GMRES solve with
// optional mixed-precision refinement, surface gradient, forces, potential.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>

#include "common.h"
#include "problem.h"
#include "refine.h"

using namespace yq;

namespace {

thread_local std::string g_last_error;

// Brackets the launches issued in its scope with a pair of events when profiling is on.
struct Timed {
  yq_problem* pb;
  int phase;
  hipEvent_t a = nullptr;
  Timed(yq_problem* p, int ph) : pb(p), phase(ph) {
    if (pb->prof_mask & (1u << ph)) {
      a = pb->event();
      YQ_HIP(hipEventRecord(a, pb->stream));
    }
  }
  ~Timed() {
    if (a) {
      hipEvent_t b = pb->event();
      (void)hipEventRecord(b, pb->stream);
      pb->ev[phase].push_back({a, b});
    }
  }
};

// Like Timed for a single kernel launch that records the two events itself
// (hipExtLaunchKernel), so the timing adds no commands to the stream.
struct LaunchTimed {
  yq_problem* pb;
  int phase;
  hipEvent_t a = nullptr, b = nullptr;
  LaunchTimed(yq_problem* p, int ph) : pb(p), phase(ph) {
    if (pb->prof_mask & (1u << ph)) {
      a = pb->event();
      b = pb->event();
    }
  }
  ~LaunchTimed() {
    if (a) pb->ev[phase].push_back({a, b});
  }
};

int fail(yq_problem* pb, const Error& e) {
  if (pb) pb->err = e.msg;
  g_last_error = e.msg;
  return e.code;
}

template <class F>
int guarded(yq_problem* pb, F&& fn) {
  try {
    fn();
    return YQ_OK;
  } catch (const Error& e) {
    return fail(pb, e);
  } catch (const std::exception& e) {
    return fail(pb, Error{YQ_EDEVICE, e.what()});
  } catch (...) {
    return fail(pb, Error{YQ_EDEVICE, "unknown error"});
  }
}

void check_params(const yq_params& p) {
  YQ_REQUIRE(p.qbx_order >= 1 && p.qbx_order <= MAXP, YQ_EINVAL, "qbx_order out of range 1..30");
  YQ_REQUIRE(p.qbx_window >= 0 && p.qbx_window <= 8, YQ_EINVAL, "qbx_window out of range 0..8");
  YQ_REQUIRE(p.panels_per_particle >= 2 * p.qbx_window + 1 && p.panels_per_particle <= 4096,
             YQ_EINVAL, "panels_per_particle must be in 2*qbx_window+1..4096");
  YQ_REQUIRE(p.qbx_oversample >= 1 && p.qbx_oversample <= MAXSUB, YQ_EINVAL,
             "qbx_oversample out of range 1..16");
  YQ_REQUIRE(p.near_oversample >= 1 && p.near_oversample <= MAXSUB, YQ_EINVAL,
             "near_oversample out of range 1..16");
  YQ_REQUIRE(p.pot_oversample >= 1 && p.pot_oversample <= MAXSUB, YQ_EINVAL,
             "pot_oversample out of range 1..16");
  YQ_REQUIRE(p.qbx_radius > 0.0 && p.qbx_radius < 1.0, YQ_EINVAL, "qbx_radius must be in (0, 1)");
  YQ_REQUIRE(p.near_beta >= 0.0 && p.pot_beta >= 0.0, YQ_EINVAL, "near_beta, pot_beta >= 0");
  YQ_REQUIRE(p.precision == YQ_FP64 || p.precision == YQ_MIXED, YQ_EINVAL, "bad precision");
  YQ_REQUIRE(p.far_mode == YQ_FAR_DIRECT || p.far_mode == YQ_FAR_FMM || p.far_mode == YQ_FAR_AUTO ||
                 p.far_mode == YQ_FAR_CUTOFF,
             YQ_EINVAL, "bad far_mode");
  YQ_REQUIRE(p.far_mode != YQ_FAR_CUTOFF || (p.cutoff_tol > 0.0 && p.cutoff_tol < 1.0), YQ_EINVAL,
             "cutoff_tol must be in (0, 1)");
  YQ_REQUIRE(std::isfinite(p.sl_coupling) && p.sl_coupling >= 0.0, YQ_EINVAL,
             "sl_coupling must be finite and >= 0");
  YQ_REQUIRE(p.sl_coupling == 0.0 || p.far_mode == YQ_FAR_DIRECT, YQ_EINVAL,
             "the combined representation (sl_coupling > 0) needs the direct far field");
  YQ_REQUIRE(p.refine_levels >= 0 && p.refine_levels <= 8, YQ_EINVAL,
             "refine_levels out of range 0..8");
  YQ_REQUIRE(std::isfinite(p.refine_ratio) && p.refine_ratio > 0.0, YQ_EINVAL,
             "refine_ratio must be finite and > 0");
  YQ_REQUIRE(p.fmm_order >= 1 && p.fmm_order <= MAXP_FMM, YQ_EINVAL, "fmm_order out of range 1..48");
  YQ_REQUIRE(p.fmm_resid_order >= 0 && p.fmm_resid_order <= MAXP_FMM, YQ_EINVAL,
             "fmm_resid_order out of range 0..48");
  YQ_REQUIRE(p.fmm_leaf_max >= 1, YQ_EINVAL, "fmm_leaf_max must be >= 1");
  YQ_REQUIRE(p.fmm_m2l == YQ_M2L_MFMA || p.fmm_m2l == YQ_M2L_VALU || p.fmm_m2l == YQ_M2L_MFMA64,
             YQ_EINVAL, "bad fmm_m2l");
  YQ_REQUIRE(p.tol > 0.0 && p.maxiter >= 1 && p.restart >= 1 && p.restart <= 200, YQ_EINVAL,
             "tol > 0, maxiter >= 1, 1 <= restart <= 200");
  YQ_REQUIRE(p.inner_tol > 0.0 && p.inner_tol < 1.0 && p.max_refine >= 1, YQ_EINVAL,
             "inner_tol in (0, 1), max_refine >= 1");
}

void upload(DevBuf<double>& b, const std::vector<double>& h, hipStream_t s) {
  b.fit(h.size());
  YQ_HIP(hipMemcpyAsync(b.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s));
}

void upload_i(DevBuf<int>& b, const std::vector<int>& h, hipStream_t s) {
  b.fit(std::max<size_t>(h.size(), 1));
  if (!h.empty())
    YQ_HIP(hipMemcpyAsync(b.p, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice, s));
}

std::vector<double> interp_for(const Consts& c, int nsub) {
  std::vector<double> xi(nsub * Q), L(nsub * Q * Q);
  sub_panel_coords(c.xg, Q, nsub, xi.data());
  lagrange_matrix(c.xg, Q, xi.data(), nsub * Q, L.data());
  return L;
}

// ---- operator ------------------------------------------------------------------------------

// The far field of the FP32-class (inner) operator comes from the FMM when it is
// enabled; the FP64 operator is always the exact direct sum.
void far_fmm(yq_problem* pb, const double* sigma) {
  Timed t(pb, 1);
  pb->fmm->apply(sigma, pb->partial.p, true, pb->tab.p, pb->stream, pb->stop_dev);
}

void apply_op(yq_problem* pb, const double* sigma, double* out, int prec) {
  GeomView g = pb->view();
  const int win = pb->prm.qbx_window;
  if (prec == YQ_MIXED && pb->fmm) {
    far_fmm(pb, sigma);
    FarPlan one{pb->fp.tblocks, 1, (int)pb->N};
    Timed t(pb, 2);
    launch_finish(g, win, one, pb->partial.p, nullptr, pb->W.p, pb->xrow.p, pb->xpan.p,
                  pb->xvals.p, sigma, out, pb->stream);
    return;
  }
  if (prec == YQ_MIXED) {
    if (g.eta > 0.0) {
      // combined representation: both layers in one pass (FP32 arithmetic)
      LaunchTimed t(pb, 1);
      launch_far_sd(g, sigma, pb->fp, nullptr, pb->partial32.p, pb->stream, pb->stop_dev, t.a, t.b);
    } else {
      if (pb->src_for != sigma) pb->pack32(sigma);   // else packed by the Arnoldi step
      pb->src_for = nullptr;
      LaunchTimed t(pb, 1);
      launch_far32(pb->far32(), pb->fp, pb->partial32.p, pb->stream, pb->stop_dev, t.a, t.b);
    }
    Timed t(pb, 2);
    launch_finish(g, win, pb->fp, nullptr, pb->partial32.p, pb->W.p, pb->xrow.p, pb->xpan.p,
                  pb->xvals.p, sigma, out, pb->stream);
  } else {
    {
      LaunchTimed t(pb, 0);
      if (g.eta > 0.0)
        launch_far_sd(g, sigma, pb->fp, pb->partial.p, nullptr, pb->stream, pb->stop_dev, t.a, t.b);
      else
        launch_far64(g, sigma, pb->fp, pb->partial.p, pb->stream, pb->stop_dev, t.a, t.b);
    }
    Timed t(pb, 2);
    launch_finish(g, win, pb->fp, pb->partial.p, nullptr, pb->W.p, pb->xrow.p, pb->xpan.p,
                  pb->xvals.p, sigma, out, pb->stream);
  }
}

// The operator of refinement residuals, FP64 solves and reported residuals: the
// higher-order FP64 FMM when it is enabled, otherwise the exact direct sum.
constexpr int OP_RESID = 2;
void apply_resid(yq_problem* pb, const double* sigma, double* out) {
  if (!pb->fmm_hi) {
    apply_op(pb, sigma, out, YQ_FP64);
    return;
  }
  {
    Timed t(pb, 0);
    pb->fmm_hi->apply(sigma, pb->partial.p, false, pb->tab.p, pb->stream, pb->stop_dev);
  }
  FarPlan one{pb->fp.tblocks, 1, (int)pb->N};
  Timed t(pb, 2);
  launch_finish(pb->view(), pb->prm.qbx_window, one, pb->partial.p, nullptr, pb->W.p, pb->xrow.p,
                pb->xpan.p, pb->xvals.p, sigma, out, pb->stream);
}

// The FP64 residual operator fused with the gradient far field of the same sigma
// (direct far field only): out = A sigma, and pb->gpartial ready for the forces.
void apply_resid_fused(yq_problem* pb, const double* sigma, double* out) {
  {
    Timed t(pb, 6);
    pb->gpartial.reserve((size_t)pb->fp.chunks * 2 * pb->N);
    launch_far_fused64(pb->view(), sigma, pb->fp, pb->partial.p, pb->gpartial.p, pb->stream);
  }
  Timed t(pb, 2);
  launch_finish(pb->view(), pb->prm.qbx_window, pb->fp, pb->partial.p, nullptr, pb->W.p,
                pb->xrow.p, pb->xpan.p, pb->xvals.p, sigma, out, pb->stream);
  pb->grad_ready = true;
}

void apply_any(yq_problem* pb, const double* sigma, double* out, int prec) {
  if (prec == OP_RESID)
    apply_resid(pb, sigma, out);
  else
    apply_op(pb, sigma, out, prec);
}

// ---- GMRES -----------------------------------------------------------------------------------

// Per-block partial dot products, summed on the host in block order.
double dot_host(yq_problem* pb, const double* a, const double* b) {
  const int nb = krylov_blocks(pb->N);
  launch_multidot(a, 0, 1, b, pb->N, pb->kpart.p, nb, pb->stream);
  pb->hpart.fit(nb * sizeof(double));
  double* hp = (double*)pb->hpart.p;
  YQ_HIP(hipMemcpyAsync(hp, pb->kpart.p, nb * sizeof(double), hipMemcpyDeviceToHost, pb->stream));
  YQ_HIP(hipStreamSynchronize(pb->stream));
  return sum_partials(hp, nb);
}

struct GmresResult {
  int iterations = 0;
  int cycles = 0;
  int matvecs = 0;
  bool converged = false;
  double rel = 0.0;  // residual estimate relative to ||b||
};

// Arnoldi of one GMRES cycle with the bookkeeping on the device (arnoldi
// kernel): the host queues step j + 1 before it waits for step j's status, so
// the GPU does not idle while the host reads it.  When step j stops the cycle,
// the already queued step j + 1 finds the device stop flag set: its far-field
// launch and its Arnoldi kernel do nothing, and its cheap vector kernels write
// only into unused Krylov storage.  Also applies the cycle's update
// x += V H^-1 g.  Every far-field path (direct kernels, both FMMs) honours the
// stop flag.
int arnoldi_pipelined(yq_problem* pb, int prec, int maxsteps, double beta, double bnorm,
                      double rtol, double* x, bool& done, GmresResult& R) {
  const int64_t N = pb->N;
  const int m = pb->prm.restart;
  const int ldh = m + 1;
  const int nb = krylov_blocks(N);
  hipStream_t s = pb->stream;
  double* V = pb->V.p;
  double* w = pb->kw.p;
  double* dH = pb->gm.p;                         // [(m + 1) * m]
  double* dcs = dH + (size_t)ldh * m;            // [m]
  double* dsn = dcs + m;                         // [m]
  double* dg = dsn + m;                          // [m + 1]
  double* dst = dg + m + 1 + 1;                  // [4 m] per-step status
  int* stop = pb->gstop.p;
  double* hst = (double*)pb->hstat.p;            // host copy of the status [4 m]
  launch_gmres_init(dg, m, beta, stop, s);
  pb->stop_dev = stop;
  // the next matvec packs FP32 sources (the combined representation reads sigma itself)
  const bool pack = prec == YQ_MIXED && !pb->fmm && pb->prm.sl_coupling == 0.0;
  int queued = 0, stopped = -1;
  for (int j = 0; j < maxsteps; ++j) {
    double* vj = V + (int64_t)j * N;
    double* vn = V + (int64_t)(j + 1) * N;
    apply_any(pb, vj, w, prec);
    const int64_t pc = (int64_t)(j + 1) * nb;
    double* kp = pb->kpart.p;
    // CGS2; the second update also leaves the partials of |w|^2, and the Arnoldi
    // step normalises the new basis vector (and packs its FP32 source records
    // when the next application is the direct FP32 far field)
    launch_multidot(V, N, j + 1, w, N, kp, nb, s);
    launch_update_partial(w, V, N, j + 1, kp, nb, -1.0, N, s);
    launch_multidot(V, N, j + 1, w, N, kp + pc, nb, s);
    launch_update_norm(w, V, N, j + 1, kp + pc, nb, -1.0, N, kp + 2 * pc, s);
    launch_arnoldi_scale(kp, nb, kp + 2 * pc, j, ldh, dH, dcs, dsn, dg, stop, bnorm, rtol,
                         dst + 4 * j, w, vn, N, pb->frel.p, pb->wnx.p, pb->wny.p,
                         SQRT_LOG2E / pb->kappa, pack ? pb->fsrc.p : nullptr, s);
    pb->src_for = pack ? vn : nullptr;
    YQ_HIP(hipMemcpyAsync(hst + 4 * j, dst + 4 * j, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    YQ_HIP(hipEventRecord(pb->step_ev[j & 1], s));
    ++queued;
    if (j >= 1) {
      YQ_HIP(hipEventSynchronize(pb->step_ev[(j - 1) & 1]));
      if (hst[4 * (j - 1) + 2] != 0.0) {
        stopped = j - 1;
        break;
      }
    }
  }
  pb->stop_dev = nullptr;
  pb->src_for = nullptr;
  YQ_HIP(hipStreamSynchronize(s));
  if (stopped < 0 && queued > 0 && hst[4 * (queued - 1) + 2] != 0.0) stopped = queued - 1;
  const int k = stopped >= 0 ? stopped + 1 : queued;
  // the far-field launches of the steps queued after the stop did nothing: their
  // timing records (the phase's last ones) are dropped
  const int ph = prec == YQ_MIXED ? 1 : 0;
  for (int t = k; t < queued && (pb->prof_mask & (1u << ph)) && !pb->ev[ph].empty(); ++t) {
    pb->pool.push_back(pb->ev[ph].back().first);
    pb->pool.push_back(pb->ev[ph].back().second);
    pb->ev[ph].pop_back();
  }
  R.iterations += k;
  R.matvecs += k;
  if (k > 0) {
    R.rel = hst[4 * (k - 1)];
    // y = H^-1 g and x += V y on the device (queued; no host round trip)
    launch_trisolve(dH, ldh, dg, k, pb->kred.p, s);
    launch_update(x, V, N, k, pb->kred.p, 1.0, N, s);
  }
  done = stopped >= 0;
  return k;
}

// Solves A x = b with restarted GMRES; x holds the initial guess (x_zero: 0).
// The operator is applied with precision prec; Arnoldi is FP64 (CGS2).
// bnorm_known: |b| when the caller has it (else negative).
GmresResult gmres(yq_problem* pb, int prec, const double* b, double* x, bool x_zero, double rtol,
                  int maxit, double bnorm_known = -1.0) {
  GmresResult R;
  const int64_t N = pb->N;
  const int m = pb->prm.restart;
  hipStream_t s = pb->stream;
  double* V = pb->V.p;
  double* w = pb->kw.p;
  double* r = pb->kr.p;

  const double bnorm = bnorm_known >= 0.0 ? bnorm_known : std::sqrt(dot_host(pb, b, b));
  if (bnorm == 0.0) {
    YQ_HIP(hipMemsetAsync(x, 0, N * sizeof(double), s));
    R.converged = true;
    return R;
  }
  if (x_zero) YQ_HIP(hipMemsetAsync(x, 0, N * sizeof(double), s));

  bool first = true;
  while (true) {
    // r = b - A x (b itself for a zero initial guess)
    double beta;
    if (first && x_zero) {
      r = const_cast<double*>(b);   // read only
      beta = bnorm;
    } else {
      r = pb->kr.p;
      apply_any(pb, x, w, prec);
      ++R.matvecs;
      launch_axpby(-1.0, w, 1.0, b, r, N, s);
      beta = std::sqrt(dot_host(pb, r, r));
    }
    first = false;
    R.rel = beta / bnorm;
    if (R.rel <= rtol) {
      R.converged = true;
      return R;
    }
    if (R.iterations >= maxit) return R;
    ++R.cycles;
    launch_axpby(1.0 / beta, r, 0.0, nullptr, V, N, s);
    const int steps = std::min(m, maxit - R.iterations);
    bool done = false;
    arnoldi_pipelined(pb, prec, steps, beta, bnorm, rtol, x, done, R);
    if (done) {
      R.converged = true;
      return R;
    }
    if (R.iterations >= maxit) return R;
  }
}

void ensure_krylov(yq_problem* pb) {
  const int64_t N = pb->N;
  const int m = pb->prm.restart;
  pb->V.reserve((size_t)(m + 1) * N);
  pb->kw.reserve(N);
  pb->kr.reserve(N);
  pb->kd.reserve(N);
  pb->kpart.reserve((size_t)krylov_blocks(N) * (2 * (m + 1) + 1) + krylov_norm_blocks(N));
  pb->kred.reserve(2 * (m + 1) + 8);
  pb->gm.reserve((size_t)(m + 1) * m + 2 * m + (m + 1) + 1 + 4 * m);
  pb->gstop.reserve(1);
  pb->hstat.fit((size_t)4 * m * sizeof(double));
  pb->hpart.fit((size_t)krylov_blocks(N) * sizeof(double));
  pb->delta.fit(N);   // refinement correction (mixed solves)
  for (auto& e : pb->step_ev)
    if (!e) YQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

void require_ready(const yq_problem* pb) {
  YQ_REQUIRE(pb != nullptr, YQ_EINVAL, "null problem");
  YQ_REQUIRE(pb->ready, YQ_ESTATE, "yq_set_particles has not been called");
}

}  // namespace

// =============================================================================================
extern "C" {

void yq_default_params(yq_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->panels_per_particle = 32;
  p->qbx_order = 10;
  p->qbx_window = 2;
  p->qbx_oversample = 4;
  p->qbx_radius = 0.25;
  p->near_beta = 0.5;
  p->near_oversample = 4;
  p->pot_oversample = 8;
  p->pot_beta = 0.5;
  p->precision = YQ_FP64;
  p->far_mode = YQ_FAR_DIRECT;
  p->fmm_order = 20;
  p->fmm_leaf_max = 64;
  p->tol = 1e-10;
  p->maxiter = 200;
  p->restart = 100;
  p->inner_tol = 1e-6;
  p->max_refine = 8;
  p->fmm_resid_order = 40;
  p->fmm_m2l = YQ_M2L_MFMA;
  p->cutoff_tol = 1e-12;
  p->sl_coupling = 0.0;
  p->refine_levels = 0;
  p->refine_ratio = 2.0;
}

const char* yq_error_string(int status) {
  switch (status) {
    case YQ_OK: return "ok";
    case YQ_EINVAL: return "invalid argument";
    case YQ_EGEOM: return "geometry rejected";
    case YQ_ENOCONV: return "GMRES did not converge";
    case YQ_ENOMEM: return "device memory allocation failed";
    case YQ_EDEVICE: return "HIP runtime error";
    case YQ_ESTATE: return "call out of order";
    case YQ_EADMIT: return "request refused by admission";
    default: return "unknown status";
  }
}

const char* yq_last_error(const yq_problem* pb) {
  return pb ? pb->err.c_str() : g_last_error.c_str();
}

int yq_create(const yq_params* params, yq_problem** out) {
  return guarded(nullptr, [&] {
    YQ_REQUIRE(params && out, YQ_EINVAL, "null argument");
    check_params(*params);
    auto pb = std::make_unique<yq_problem>();
    pb->prm = *params;
    gauss_legendre16(pb->consts.xg, pb->consts.wg);
    std::vector<double> t(T_SIZE_HOST);
    fill_tab64(t.data());
    upload(pb->tab, t, nullptr);
    YQ_HIP(hipStreamSynchronize(nullptr));
    *out = pb.release();
  });
}

void yq_destroy(yq_problem* pb) {
  if (!pb) return;
  (void)hipStreamSynchronize(pb->stream);
  delete pb;
}

int yq_set_stream(yq_problem* pb, void* stream) {
  return guarded(pb, [&] {
    YQ_REQUIRE(pb, YQ_EINVAL, "null problem");
    pb->stream = (hipStream_t)stream;
  });
}

}  // extern "C"

namespace {

// Cutoff far field: the smallest z with kappa/(2 pi) sqrt(pi/(2z)) e^-z (1 + 3/(8z)) L
// (times 1 + 3/z for the gradient) <= eps.  The left side bounds kappa K1(z) L / (2 pi)
// (DLMF 10.40.10: the remainder after the 3/(8z) term is negative for z > 0) and
// decreases in z, so bisection finds it.
double cutoff_z(double kappa, double L, double eps, bool grad) {
  auto bound = [&](double z) {
    double b = kappa / (2.0 * PI) * std::sqrt(PI / (2.0 * z)) * std::exp(-z) *
               (1.0 + 3.0 / (8.0 * z)) * L;
    return grad ? b * (1.0 + 3.0 / z) : b;
  };
  double lo = 1e-3, hi = 2000.0;
  if (bound(lo) <= eps) return lo;
  for (int it = 0; it < 200 && hi - lo > 1e-12 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    (bound(mid) <= eps ? hi : lo) = mid;
  }
  return hi;
}

// The set-up of yq_set_particles (throws yq::Error).  The boundary data buffer
// keeps its contents when the node count does not change.  rot (host [n] or null):
// the particles are those of the current set-up moved rigidly, particle i turned
// by rot[i].  The window part of the QBX correction only involves a particle's own
// panels, and the kernel depends on distances and on normals relative to the
// difference vector, so its values stay and its gradient rows turn with the
// particle: the QBX build is replaced by that rotation.
void setup_particles(yq_problem* pb, int32_t n, const double* center_xy, const double* angle,
                     const double* semi_axes, double kappa, const double* rot = nullptr) {
  YQ_REQUIRE(pb && center_xy && angle && semi_axes, YQ_EINVAL, "null argument");
  YQ_REQUIRE(n >= 1, YQ_EINVAL, "need at least one particle");
  YQ_REQUIRE(std::isfinite(kappa) && kappa > 0.0, YQ_EINVAL, "kappa must be finite and > 0");
  const int P = pb->prm.panels_per_particle;
  const int levels = pb->batch_member ? 0 : pb->prm.refine_levels;
  YQ_REQUIRE((int64_t)n * P * Q < (int64_t)INT32_MAX, YQ_EINVAL, "too many nodes for one problem");
  YQ_REQUIRE(!(rot && levels > 0), YQ_EINVAL, "rigid motion set-up with adaptive refinement");
  double amax = 0.0;
  pb->h_pc.assign((size_t)n * 5, 0.0);
  for (int i = 0; i < n; ++i) {
    const double cx = center_xy[2 * i], cy = center_xy[2 * i + 1], th = angle[i];
    const double A = semi_axes[2 * i], B = semi_axes[2 * i + 1];
    YQ_REQUIRE(std::isfinite(cx) && std::isfinite(cy) && std::isfinite(th) &&
                   std::isfinite(A) && std::isfinite(B),
               YQ_EINVAL, "non-finite particle data");
    YQ_REQUIRE(B > 0.0 && A >= B, YQ_EINVAL, "semi-axes must satisfy A >= B > 0");
    double* q = &pb->h_pc[5 * (size_t)i];
    q[0] = cx;
    q[1] = cy;
    q[2] = th;
    q[3] = A;
    q[4] = B;
    amax = std::max(amax, A);
  }
  pb->ready = false;
  pb->pot_fine_ready = false;
  pb->have_f = false;
  const bool had_qbx = pb->qbx_valid;   // W, WGx, WGy hold the current set-up's correction
  pb->qbx_valid = false;
  hipStream_t s = pb->stream;

  // particle neighbour lists (host): every particle whose ellipse could hold
  // a near panel of, or overlap, particle p, or (with refinement) come closer
  // than the longest panel / refine_ratio to it; p itself is included.  A panel's
  // arclength is at most 2 pi A / P.
  double reach = std::max(pb->prm.near_beta, pb->prm.pot_beta);
  if (levels > 0) reach = std::max(reach, 1.0 / pb->prm.refine_ratio);
  const double margin = reach * 2.0 * PI * amax / P * 1.01 + 1e-9;
  // Candidates come from a uniform grid of cell side 2 amax + margin (no pair
  // closer than that can be missed); each list is ascending in q.
  std::vector<int> nbp(n + 1, 0), nbi;
  {
    double xlo = pb->h_pc[0], ylo = pb->h_pc[1], xhi = xlo, yhi = ylo;
    for (int p = 0; p < n; ++p) {
      xlo = std::min(xlo, pb->h_pc[5 * (size_t)p]);
      xhi = std::max(xhi, pb->h_pc[5 * (size_t)p]);
      ylo = std::min(ylo, pb->h_pc[5 * (size_t)p + 1]);
      yhi = std::max(yhi, pb->h_pc[5 * (size_t)p + 1]);
    }
    // at most 1024 cells per side (larger cells only add candidates)
    const double cell = std::max(2.0 * amax + margin, std::max(xhi - xlo, yhi - ylo) / 1024.0);
    const int64_t gx = std::min<int64_t>((int64_t)((xhi - xlo) / cell) + 1, 1025);
    const int64_t gy = std::min<int64_t>((int64_t)((yhi - ylo) / cell) + 1, 1025);
    auto cell_of = [&](double v, double lo, int64_t g) {
      return std::min<int64_t>(std::max<int64_t>((int64_t)((v - lo) / cell), 0), g - 1);
    };
    std::vector<int> head(gx * gy + 1, 0), members(n);
    std::vector<int64_t> cid(n);
    for (int p = 0; p < n; ++p) {
      cid[p] = cell_of(pb->h_pc[5 * (size_t)p], xlo, gx) * gy +
               cell_of(pb->h_pc[5 * (size_t)p + 1], ylo, gy);
      ++head[cid[p] + 1];
    }
    for (int64_t c = 0; c < gx * gy; ++c) head[c + 1] += head[c];
    {
      std::vector<int> fill(head.begin(), head.end() - 1);
      for (int p = 0; p < n; ++p) members[fill[cid[p]]++] = p;
    }
    std::vector<int> cand;
    for (int p = 0; p < n; ++p) {
      const double* a = &pb->h_pc[5 * (size_t)p];
      const int64_t cx = cid[p] / gy, cy = cid[p] % gy;
      cand.clear();
      for (int64_t ix = std::max<int64_t>(cx - 1, 0); ix <= std::min(cx + 1, gx - 1); ++ix)
        for (int64_t iy = std::max<int64_t>(cy - 1, 0); iy <= std::min(cy + 1, gy - 1); ++iy)
          for (int e = head[ix * gy + iy]; e < head[ix * gy + iy + 1]; ++e) {
            const int q = members[e];
            const double* b = &pb->h_pc[5 * (size_t)q];
            const double d = std::hypot(a[0] - b[0], a[1] - b[1]);
            if (q == p || d < a[3] + b[3] + margin) cand.push_back(q);
          }
      std::sort(cand.begin(), cand.end());
      nbi.insert(nbi.end(), cand.begin(), cand.end());
      nbp[p + 1] = (int)nbi.size();
    }
  }
  // adaptive panels near contact (host, FP64): the panel table (particle, base
  // panel, level, index) in node order and every particle's first panel
  std::vector<int4> ptab;
  std::vector<int> poff;
  if (levels > 0) {
    const auto pans = refine_panels(pb->h_pc.data(), n, P, levels, pb->prm.refine_ratio,
                                    pb->prm.qbx_window, pb->consts.xg, pb->consts.wg, Q, nbp, nbi);
    poff.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
      YQ_REQUIRE((int64_t)poff[i] + (int64_t)pans[i].size() < (int64_t)INT32_MAX / Q, YQ_EINVAL,
                 "too many refined panels for one problem");
      poff[i + 1] = poff[i] + (int)pans[i].size();
      for (const PanelDesc& d : pans[i]) ptab.push_back(make_int4(i, d.k, d.lev, d.idx));
    }
  }
  const int64_t npan = levels > 0 ? (int64_t)poff[n] : (int64_t)n * P;
  const int64_t N = npan * Q;
  pb->n = n;
  pb->N = N;
  pb->npan = npan;
  pb->refined = levels > 0;
  pb->kappa = kappa;

  // host inputs go through pinned staging, so their copies are asynchronous; all
  // of them complete before the geometry check below returns
  {
    const size_t b_pc = pb->h_pc.size() * sizeof(double);
    const size_t b_np = nbp.size() * sizeof(int), b_ni = nbi.size() * sizeof(int);
    const size_t b_pt = ptab.size() * sizeof(int4), b_po = poff.size() * sizeof(int);
    // the panel table starts on a 16-byte boundary
    const size_t o_pt = (b_pc + b_np + b_ni + 15) / 16 * 16, o_po = o_pt + b_pt;
    pb->stage.fit(o_po + b_po + 16);
    char* st = pb->stage.p;
    std::memcpy(st, pb->h_pc.data(), b_pc);
    std::memcpy(st + b_pc, nbp.data(), b_np);
    if (b_ni) std::memcpy(st + b_pc + b_np, nbi.data(), b_ni);
    if (b_pt) std::memcpy(st + o_pt, ptab.data(), b_pt);
    if (b_po) std::memcpy(st + o_po, poff.data(), b_po);
    pb->pc.fit(pb->h_pc.size());
    pb->nb_ptr.fit(nbp.size());
    pb->nb_idx.fit(std::max<size_t>(nbi.size(), 1));
    YQ_HIP(hipMemcpyAsync(pb->pc.p, st, b_pc, hipMemcpyHostToDevice, s));
    YQ_HIP(hipMemcpyAsync(pb->nb_ptr.p, st + b_pc, b_np, hipMemcpyHostToDevice, s));
    if (b_ni) YQ_HIP(hipMemcpyAsync(pb->nb_idx.p, st + b_pc + b_np, b_ni, hipMemcpyHostToDevice, s));
    if (levels > 0) {
      pb->pan.fit(ptab.size());
      pb->poff.fit(poff.size());
      YQ_HIP(hipMemcpyAsync(pb->pan.p, st + o_pt, b_pt, hipMemcpyHostToDevice, s));
      YQ_HIP(hipMemcpyAsync(pb->poff.p, st + o_po, b_po, hipMemcpyHostToDevice, s));
    }
  }

  // a1: nodes, normals, weights; panel arclengths and bounding circles
  pb->x.alloc(N);
  pb->y.alloc(N);
  pb->nx.alloc(N);
  pb->ny.alloc(N);
  pb->w.alloc(N);
  pb->wnx.alloc(N);
  pb->wny.alloc(N);
  pb->panel_h.alloc((size_t)npan);
  pb->pcx.alloc((size_t)npan);
  pb->pcy.alloc((size_t)npan);
  pb->pr.alloc((size_t)npan);
  GeomView g = pb->view();
  launch_geometry(g, pb->consts, pb->x.p, pb->y.p, pb->nx.p, pb->ny.p, pb->w.p, pb->wnx.p,
                  pb->wny.p, s);
  launch_panel_stats(g, pb->panel_h.p, pb->pcx.p, pb->pcy.p, pb->pr.p, s);

  // geometry check, and a3: extra near panels per node (count, then their row
  // offsets by a device scan); one round trip brings back the check and the total
  pb->bad.alloc(1);
  YQ_HIP(hipMemsetAsync(pb->bad.p, 0, sizeof(int), s));
  launch_geom_check(g, pb->nb_ptr.p, pb->nb_idx.p, pb->bad.p, s);
  pb->xrow.alloc(N + 1);
  DevBuf<int>& cnt = pb->ncnt;
  cnt.fit(N);
  launch_near_count(g, pb->prm.qbx_window, pb->prm.near_beta, pb->nb_ptr.p, pb->nb_idx.p,
                    pb->pcx.p, pb->pcy.p, pb->pr.p, cnt.p, nullptr, nullptr, s);
  launch_row_scan(cnt.p, N, pb->xrow.p, pb->scan_tmp, s);
  pb->hflags.fit(2 * sizeof(int));
  int* hfl = (int*)pb->hflags.p;
  YQ_HIP(hipMemcpyAsync(hfl, pb->bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  YQ_HIP(hipMemcpyAsync(hfl + 1, pb->xrow.p + N, sizeof(int), hipMemcpyDeviceToHost, s));
  YQ_HIP(hipStreamSynchronize(s));
  YQ_REQUIRE(hfl[0] == 0, YQ_EGEOM, "a node of one particle lies inside another particle");
  pb->x_total = hfl[1];

  // the FMM tree is built on the host from the node positions; their copy is
  // queued now so that the QBX build below runs while the tree is built
  // (a batch member takes the FMM only when its batch asks for it: its far field is
  // then one tree of the batch engine's forest)
  const bool use_fmm = pb->prm.far_mode == YQ_FAR_FMM ||
                       (!pb->batch_member && pb->prm.far_mode == YQ_FAR_AUTO && N >= kFmmAutoNodes);
  if (use_fmm) {
    // the FMM objects of the previous geometry are rebuilt in place: their
    // device buffers only grow, so a new geometry frees nothing
    if (!pb->fmm) pb->fmm = std::make_unique<Fmm>();
    pb->fmm->download(pb->x.p, pb->y.p, pb->wnx.p, pb->wny.p, N, s);
  }

  // a3: fill the extra near panel lists
  pb->xpan.fit(std::max<int64_t>(pb->x_total, 1));
  pb->xvals.fit(std::max<int64_t>(pb->x_total, 1) * Q);
  pb->xgvals.fit(std::max<int64_t>(pb->x_total, 1) * 2 * Q);
  if (pb->x_total > 0)
    launch_near_count(g, pb->prm.qbx_window, pb->prm.near_beta, pb->nb_ptr.p, pb->nb_idx.p,
                      pb->pcx.p, pb->pcy.p, pb->pr.p, nullptr, pb->xpan.p, pb->xrow.p, s);

  // a4: QBX correction (window) and oversampled rows (extra near panels)
  if (!pb->interp_ready) {   // depend on the parameters only
    upload(pb->Lqbx, interp_for(pb->consts, pb->prm.qbx_oversample), s);
    upload(pb->Lnear, interp_for(pb->consts, pb->prm.near_oversample), s);
    upload(pb->Lpot, interp_for(pb->consts, pb->prm.pot_oversample), s);
    pb->interp_ready = true;
  }
  const size_t wsz = (size_t)(2 * pb->prm.qbx_window + 1) * Q * N;
  const bool reuse = rot && had_qbx && pb->W.p && pb->W.n == wsz;
  pb->W.alloc(wsz);
  pb->WGx.alloc(wsz);
  pb->WGy.alloc(wsz);
  if (reuse) {
    Timed t(pb, 4);
    pb->wrot.fit((size_t)2 * n);
    pb->rstage.fit((size_t)2 * n * sizeof(double));
    double* cs = (double*)pb->rstage.p;
    for (int i = 0; i < n; ++i) {
      cs[2 * i] = std::cos(rot[i]);
      cs[2 * i + 1] = std::sin(rot[i]);
    }
    YQ_HIP(hipMemcpyAsync(pb->wrot.p, cs, 2 * (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
    // (the next set-up writes rstage only after its geometry check has synchronised
    // the stream, so this copy has completed by then)
    launch_rotate_grad_rows(pb->WGx.p, pb->WGy.p, (int64_t)(2 * pb->prm.qbx_window + 1) * Q, N,
                            (int64_t)P * Q, pb->wrot.p, s);
  } else {
    Timed t(pb, 4);
    const int qs = pb->prm.qbx_oversample;
    const size_t nq = (size_t)N * qs;
    pb->qfx.fit(nq);
    pb->qfy.fit(nq);
    pb->qfwx.fit(nq);
    pb->qfwy.fit(nq);
    launch_pot_fine(g, pb->consts, qs,
                    PotFine{qs, pb->qfx.p, pb->qfy.p, pb->qfwx.p, pb->qfwy.p, nullptr}, s);
    launch_qbx_build(g, pb->prm.qbx_order, pb->prm.qbx_window, qs, pb->prm.qbx_radius,
                     pb->Lqbx.p, pb->qfx.p, pb->qfy.p, pb->qfwx.p, pb->qfwy.p, pb->W.p,
                     pb->WGx.p, pb->WGy.p, s);
  }
  pb->qbx_valid = true;
  if (pb->x_total > 0)
    launch_near_rows(g, pb->consts, pb->prm.near_oversample, pb->Lnear.p, pb->xrow.p,
                     pb->xpan.p, pb->xvals.p, pb->xgvals.p, s);

  // FP32 far field: bounding circles, relative positions, source records
  pb->ftile.alloc((N + FT - 1) / FT);
  pb->fgrp.alloc((N + FG - 1) / FG);
  pb->fpan.alloc(N / Q);
  pb->frel.alloc(N);
  pb->fsrc.alloc(N);
  launch_far32_geom(pb->x.p, pb->y.p, N, kappa, pb->ftile.p, pb->fgrp.p, pb->fpan.p, pb->frel.p,
                    s);

  pb->fp = far_plan(N, N, 256, pb->far_want);
  if (pb->prm.far_mode == YQ_FAR_CUTOFF) {
    double L = 0.0;   // >= the total perimeter (each ellipse lies in its circle of radius A)
    for (int i = 0; i < n; ++i) L += 2.0 * PI * pb->h_pc[5 * (size_t)i + 3];
    const double eps = pb->prm.cutoff_tol;
    pb->zcut64 = cutoff_z(kappa, L, eps, false);
    pb->zcut64g = cutoff_z(kappa, L, eps, true);
    pb->zcut32 = cutoff_z(kappa, L, std::max(eps, 0.1 * pb->prm.inner_tol), false);
  } else {
    pb->zcut64 = pb->zcut64g = pb->zcut32 = HUGE_VAL;
  }
  if (use_fmm) {
    pb->fmm->use_mfma = pb->prm.fmm_m2l != YQ_M2L_VALU;
    pb->fmm->want_m2l32 = pb->prm.fmm_m2l == YQ_M2L_MFMA;
    pb->fmm->build(N, kappa, pb->prm.fmm_order, pb->prm.fmm_leaf_max, pb->tab.p, s);
    if (pb->prm.fmm_resid_order > 0) {
      if (!pb->fmm_hi) pb->fmm_hi = std::make_unique<Fmm>();
      pb->fmm_hi->use_mfma = pb->prm.fmm_m2l != YQ_M2L_VALU;
      pb->fmm_hi->want_m2l32 = false;
      pb->fmm_hi->copy_tree(*pb->fmm, pb->prm.fmm_resid_order, pb->tab.p, s);
    } else {
      pb->fmm_hi.reset();
    }
  } else {
    pb->fmm.reset();
    pb->fmm_hi.reset();
  }
  pb->partial.alloc((size_t)pb->fp.chunks * N);
  pb->partial32.alloc((size_t)pb->fp.chunks * N);
  pb->f.alloc(N);
  pb->en.alloc(n);
  if (!pb->batch_member) {
    pb->gpartial.alloc((size_t)pb->fp.chunks * 2 * N);
    pb->gx.alloc(N);
    pb->gy.alloc(N);
    ensure_krylov(pb);
  }
  // the rest of the set-up stays queued on the problem's stream, ahead of any
  // later work of the problem; batch members are read from the batch's stream
  if (pb->batch_member) YQ_HIP(hipStreamSynchronize(s));
  pb->ready = true;
}

}  // namespace

extern "C" {

int yq_set_particles(yq_problem* pb, int32_t n, const double* center_xy, const double* angle,
                     const double* semi_axes, double kappa) {
  return guarded(pb, [&] { setup_particles(pb, n, center_xy, angle, semi_axes, kappa); });
}

int yq_num_nodes(const yq_problem* pb, int64_t* N) {
  if (!pb || !N) return YQ_EINVAL;
  *N = pb->N;
  return YQ_OK;
}

int yq_num_particles(const yq_problem* pb, int32_t* n) {
  if (!pb || !n) return YQ_EINVAL;
  *n = pb->n;
  return YQ_OK;
}

int yq_get_nodes(const yq_problem* cpb, double* x, double* y, double* nx, double* ny, double* w) {
  yq_problem* pb = const_cast<yq_problem*>(cpb);
  return guarded(pb, [&] {
    require_ready(pb);
    const size_t b = pb->N * sizeof(double);
    hipStream_t s = pb->stream;
    if (x) YQ_HIP(hipMemcpyAsync(x, pb->x.p, b, hipMemcpyDeviceToDevice, s));
    if (y) YQ_HIP(hipMemcpyAsync(y, pb->y.p, b, hipMemcpyDeviceToDevice, s));
    if (nx) YQ_HIP(hipMemcpyAsync(nx, pb->nx.p, b, hipMemcpyDeviceToDevice, s));
    if (ny) YQ_HIP(hipMemcpyAsync(ny, pb->ny.p, b, hipMemcpyDeviceToDevice, s));
    if (w) YQ_HIP(hipMemcpyAsync(w, pb->w.p, b, hipMemcpyDeviceToDevice, s));
    YQ_HIP(hipStreamSynchronize(s));
  });
}

int yq_near_count(const yq_problem* pb, int64_t* total) {
  if (!pb || !total) return YQ_EINVAL;
  if (!pb->ready) return YQ_ESTATE;
  *total = pb->x_total;
  return YQ_OK;
}

int yq_get_near(const yq_problem* cpb, int32_t* row_ptr, int32_t* panels) {
  yq_problem* pb = const_cast<yq_problem*>(cpb);
  return guarded(pb, [&] {
    require_ready(pb);
    YQ_REQUIRE(row_ptr, YQ_EINVAL, "null row_ptr");
    hipStream_t s = pb->stream;
    YQ_HIP(hipMemcpyAsync(row_ptr, pb->xrow.p, (pb->N + 1) * sizeof(int), hipMemcpyDeviceToDevice, s));
    if (pb->x_total > 0) {
      YQ_REQUIRE(panels, YQ_EINVAL, "null panels");
      YQ_HIP(hipMemcpyAsync(panels, pb->xpan.p, pb->x_total * sizeof(int), hipMemcpyDeviceToDevice, s));
    }
    YQ_HIP(hipStreamSynchronize(s));
  });
}

int yq_boundary_label(yq_problem* pb, int32_t kind, double a, double b, double* f) {
  return guarded(pb, [&] {
    require_ready(pb);
    YQ_REQUIRE(f, YQ_EINVAL, "null f");
    YQ_REQUIRE(kind == YQ_LABEL_ARC || kind == YQ_LABEL_JANUS, YQ_EINVAL, "unknown label kind");
    YQ_REQUIRE(kind != YQ_LABEL_ARC || b > 0.0, YQ_EINVAL, "arc edge width must be > 0");
    launch_label(pb->view(), kind, a, b, f, pb->stream);
    YQ_HIP(hipStreamSynchronize(pb->stream));
  });
}

int yq_set_boundary_data(yq_problem* pb, const double* f) {
  return guarded(pb, [&] {
    require_ready(pb);
    YQ_REQUIRE(f, YQ_EINVAL, "null f");
    YQ_HIP(hipMemcpyAsync(pb->f.p, f, pb->N * sizeof(double), hipMemcpyDeviceToDevice, pb->stream));
    pb->have_f = true;
  });
}

int yq_apply_far(yq_problem* pb, const double* sigma, double* out, int32_t precision) {
  return guarded(pb, [&] {
    require_ready(pb);
    YQ_REQUIRE(sigma && out, YQ_EINVAL, "null argument");
    YQ_REQUIRE(precision == YQ_FP64 || precision == YQ_MIXED ||
                   (precision == YQ_FMM64 && pb->fmm),
               YQ_EINVAL, "bad precision");
    GeomView g = pb->view();
    if ((precision == YQ_MIXED || precision == YQ_FMM64) && pb->fmm) {
      pb->fmm->apply(sigma, pb->partial.p, precision == YQ_MIXED, pb->tab.p, pb->stream);
      FarPlan one{pb->fp.tblocks, 1, (int)pb->N};
      launch_finish(g, -1, one, pb->partial.p, nullptr, pb->W.p, pb->xrow.p, pb->xpan.p, nullptr,
                    sigma, out, pb->stream);
      return;
    }
    // far field with a zero near correction: reuse finish with window 0 rows skipped
    if (g.eta > 0.0) {
      launch_far_sd(g, sigma, pb->fp, precision == YQ_MIXED ? nullptr : pb->partial.p,
                    precision == YQ_MIXED ? pb->partial32.p : nullptr, pb->stream);
    } else if (precision == YQ_MIXED) {
      pb->pack32(sigma);
      launch_far32(pb->far32(), pb->fp, pb->partial32.p, pb->stream);
    } else {
      launch_far64(g, sigma, pb->fp, pb->partial.p, pb->stream);
    }
    launch_finish(g, -1, pb->fp, precision == YQ_MIXED ? nullptr : pb->partial.p,
                  precision == YQ_MIXED ? pb->partial32.p : nullptr, pb->W.p, pb->xrow.p,
                  pb->xpan.p, nullptr, sigma, out, pb->stream);
  });
}

int yq_apply_operator(yq_problem* pb, const double* sigma, double* out, int32_t precision) {
  return guarded(pb, [&] {
    require_ready(pb);
    YQ_REQUIRE(sigma && out && sigma != out, YQ_EINVAL, "null or aliased argument");
    YQ_REQUIRE(precision == YQ_FP64 || precision == YQ_MIXED, YQ_EINVAL, "bad precision");
    apply_op(pb, sigma, out, precision);
  });
}

}  // extern "C"

namespace {

// The solve of yq_solve.  fuse: the mixed-precision residual that is expected to
// be the last one (the inner tolerance was set from tol / residual, so the
// inner solve aims straight at the outer tolerance) also leaves the gradient far
// field of sigma in pb->gpartial (pb->grad_ready), for yq_solve_forces.
int solve_impl(yq_problem* pb, const double* sigma0, double* sigma, yq_solve_info* info,
               bool fuse) {
  int status = YQ_OK;
  int rc = guarded(pb, [&] {
    require_ready(pb);
    YQ_REQUIRE(sigma, YQ_EINVAL, "null sigma");
    YQ_REQUIRE(pb->have_f, YQ_ESTATE, "boundary data not set");
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = pb->stream;
    const int64_t N = pb->N;
    yq_solve_info inf{};
    if (sigma0 && sigma0 != sigma)
      YQ_HIP(hipMemcpyAsync(sigma, sigma0, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    bool zero = sigma0 == nullptr;
    bool conv = false;
    bool r_current = false;  // r holds f - A sigma (FP64 operator) for the current sigma
    double* r = pb->kd.p;    // refinement residual
    pb->grad_ready = false;
    fuse = fuse && pb->prm.precision == YQ_MIXED && !pb->fmm && !pb->fmm_hi &&
           pb->prm.sl_coupling == 0.0;
    bool expect_last = false;  // the next residual is expected to meet the tolerance
    double last_rel = -1.0;    // mixed: |f - A sigma| / |f| of the current residual r
    if (pb->prm.precision == YQ_FP64) {
      GmresResult R = gmres(pb, OP_RESID, pb->f.p, sigma, zero, pb->prm.tol, pb->prm.maxiter);
      inf.iterations = R.iterations;
      inf.outer_steps = R.cycles;
      inf.matvecs_fp64 = R.matvecs;
      conv = R.converged;
    } else {
      // mixed precision: FP64 residual, FP32-far-field inner GMRES, sigma += delta
      if (zero) YQ_HIP(hipMemsetAsync(sigma, 0, N * sizeof(double), s));
      DevBuf<double>& delta = pb->delta;
      delta.fit(N);
      const double fnorm = std::sqrt(dot_host(pb, pb->f.p, pb->f.p));
      int budget = pb->prm.maxiter;
      for (int outer = 0; outer < pb->prm.max_refine; ++outer) {
        double rel, rn;   // |r| / |f|, |r|
        if (outer == 0 && zero) {
          YQ_HIP(hipMemcpyAsync(r, pb->f.p, N * sizeof(double), hipMemcpyDeviceToDevice, s));
          rel = 1.0;
          rn = fnorm;
        } else {
          if (fuse && expect_last)
            apply_resid_fused(pb, sigma, pb->kw.p);
          else
            apply_resid(pb, sigma, pb->kw.p);
          ++inf.matvecs_fp64;
          launch_axpby(-1.0, pb->kw.p, 1.0, pb->f.p, r, N, s);
          rn = std::sqrt(dot_host(pb, r, r));
          rel = fnorm > 0.0 ? rn / fnorm : 0.0;
          last_rel = rel;
        }
        r_current = true;
        if (rel <= pb->prm.tol) {
          conv = true;
          break;
        }
        if (budget <= 0) break;
        ++inf.outer_steps;
        const double itol = std::max(pb->prm.inner_tol, 0.5 * pb->prm.tol / std::max(rel, 1e-300));
        GmresResult R = gmres(pb, YQ_MIXED, r, delta.p, true, std::min(itol, 0.5), budget, rn);
        inf.iterations += R.iterations;
        inf.matvecs_fp32 += R.matvecs;
        budget -= R.iterations;
        launch_axpby(1.0, delta.p, 1.0, sigma, sigma, N, s);
        r_current = false;
        last_rel = -1.0;
        pb->grad_ready = false;
        expect_last = rel * std::min(itol, 0.5) <= pb->prm.tol;
      }
    }
    // final FP64 residual (the refinement loop's last one when sigma has not moved since)
    if (r_current && last_rel >= 0.0) {
      inf.residual = last_rel;
    } else {
      if (!r_current) {
        if (fuse)
          apply_resid_fused(pb, sigma, pb->kw.p);
        else
          apply_resid(pb, sigma, pb->kw.p);
        ++inf.matvecs_fp64;
        launch_axpby(-1.0, pb->kw.p, 1.0, pb->f.p, r, N, s);
      }
      const double fn = std::sqrt(dot_host(pb, pb->f.p, pb->f.p));
      inf.residual = fn > 0.0 ? std::sqrt(dot_host(pb, r, r)) / fn : 0.0;
    }
    if (pb->prm.precision == YQ_MIXED) conv = inf.residual <= pb->prm.tol;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    if (!conv) status = YQ_ENOCONV;
  });
  if (rc != YQ_OK) return rc;
  if (status != YQ_OK && pb) pb->err = "GMRES did not reach the tolerance";
  return status;
}

}  // namespace

extern "C" {

int yq_solve(yq_problem* pb, const double* sigma0, double* sigma, yq_solve_info* info) {
  return solve_impl(pb, sigma0, sigma, info, false);
}

namespace {

// Gradient far field of sigma into pb->gpartial: the FMM (its FP64 residual
// instance when there is one) when the FMM is enabled, else the direct sum.
// Returns the chunk plan the finishing kernel reads it with.
FarPlan far_grad(yq_problem* pb, const double* sigma) {
  Timed t(pb, 3);
  Fmm* fmm = pb->fmm_hi ? pb->fmm_hi.get() : pb->fmm.get();
  if (fmm) {
    pb->gpartial.reserve((size_t)2 * pb->N);
    fmm->apply_grad(sigma, pb->gpartial.p, pb->tab.p, pb->stream);
    FarPlan one = pb->fp;
    one.chunks = 1;
    return one;
  }
  pb->gpartial.reserve((size_t)pb->fp.chunks * 2 * pb->N);
  if (pb->prm.sl_coupling > 0.0)
    launch_far_sd_grad64(pb->view(), sigma, pb->fp, pb->gpartial.p, pb->stream);
  else
    launch_far_grad64(pb->view(), sigma, pb->fp, pb->gpartial.p, pb->stream);
  return pb->fp;
}

}  // namespace

int yq_surface_gradient(yq_problem* pb, const double* sigma, double* gx, double* gy) {
  return guarded(pb, [&] {
    require_ready(pb);
    YQ_REQUIRE(sigma && gx && gy, YQ_EINVAL, "null argument");
    const FarPlan fp = far_grad(pb, sigma);
    launch_finish_grad(pb->view(), pb->prm.qbx_window, fp, pb->gpartial.p, pb->WGx.p, pb->WGy.p,
                       pb->xrow.p, pb->xpan.p, pb->xgvals.p, sigma, gx, gy, pb->stream);
  });
}

}  // extern "C"

namespace {

// Forces, torques and energy of eqs. (force) and (torque) from sigma: the
// surface gradient (its far field from pb->gpartial when the solve left it
// there for this sigma, else computed now), then the per-particle sums.
void forces_of(yq_problem* pb, const double* sigma, double gamma, double* force, double* torque,
               double* energy) {
  pb->gx.reserve(pb->N);
  pb->gy.reserve(pb->N);
  GeomView g = pb->view();
  const FarPlan fp = pb->grad_ready ? pb->fp : far_grad(pb, sigma);
  pb->grad_ready = false;
  launch_finish_grad(g, pb->prm.qbx_window, fp, pb->gpartial.p, pb->WGx.p, pb->WGy.p, pb->xrow.p,
                     pb->xpan.p, pb->xgvals.p, sigma, pb->gx.p, pb->gy.p, pb->stream);
  launch_forces(g, pb->f.p, pb->gx.p, pb->gy.p, gamma, force, torque, pb->en.p, pb->stream);
  std::vector<double> e(pb->n);
  YQ_HIP(hipMemcpyAsync(e.data(), pb->en.p, pb->n * sizeof(double), hipMemcpyDeviceToHost,
                        pb->stream));
  YQ_HIP(hipStreamSynchronize(pb->stream));
  if (energy) {
    double t = 0.0;
    for (double v : e) t += v;
    *energy = t;
  }
}

}  // namespace

extern "C" {

int yq_forces(yq_problem* pb, const double* sigma, double gamma, double* force, double* torque,
              double* energy) {
  return guarded(pb, [&] {
    require_ready(pb);
    YQ_REQUIRE(sigma && force && torque, YQ_EINVAL, "null argument");
    YQ_REQUIRE(pb->have_f, YQ_ESTATE, "boundary data not set");
    pb->grad_ready = false;
    forces_of(pb, sigma, gamma, force, torque, energy);
  });
}

int yq_solve_forces(yq_problem* pb, const double* sigma0, double* sigma, yq_solve_info* info,
                    double gamma, double* force, double* torque, double* energy) {
  if (pb && !(force && torque)) {
    pb->err = "null argument";
    return YQ_EINVAL;
  }
  const int st = solve_impl(pb, sigma0, sigma, info, true);
  if (st != YQ_OK && st != YQ_ENOCONV) return st;
  const int rc = guarded(pb, [&] { forces_of(pb, sigma, gamma, force, torque, energy); });
  if (rc != YQ_OK) return rc;
  if (st != YQ_OK) pb->err = "GMRES did not reach the tolerance";
  return st;
}

int yq_eval_potential(yq_problem* pb, const double* sigma, int64_t M, const double* tx,
                      const double* ty, double* u) {
  return guarded(pb, [&] {
    require_ready(pb);
    YQ_REQUIRE(M >= 0, YQ_EINVAL, "M < 0");
    if (M == 0) return;
    YQ_REQUIRE(sigma && tx && ty && u, YQ_EINVAL, "null argument");
    const int64_t npan = pb->npan;
    PotPlan pp = pot_plan(M, npan);
    pb->pot_partial.reserve((size_t)pp.chunks * M);
    const int nsub = pb->prm.pot_oversample;
    const size_t nf = (size_t)npan * nsub * Q;
    GeomView g = pb->view();
    PotFine pf{nsub, nullptr, nullptr, nullptr, nullptr, nullptr};
    pb->pfs.reserve(nf);
    if (!pb->pot_fine_ready) {
      pb->pfx.reserve(nf);
      pb->pfy.reserve(nf);
      pb->pfwx.reserve(nf);
      pb->pfwy.reserve(nf);
    }
    pf.x = pb->pfx.p;
    pf.y = pb->pfy.p;
    pf.wx = pb->pfwx.p;
    pf.wy = pb->pfwy.p;
    pf.s = pb->pfs.p;
    if (!pb->pot_fine_ready) {
      launch_pot_fine(g, pb->consts, nsub, pf, pb->stream);
      pb->pot_fine_ready = true;
    }
    launch_potential(g, pf, pb->Lpot.p, pb->prm.pot_beta, sigma, M, tx, ty, pp,
                     pb->pot_partial.p, u, pb->stream);
  });
}

}  // extern "C"

namespace {

void check_repulsion(double c0, int32_t q) {
  YQ_REQUIRE(std::isfinite(c0) && c0 >= 0.0, YQ_EINVAL, "c0 must be finite and >= 0");
  YQ_REQUIRE(q >= 1 && q <= 16, YQ_EINVAL, "repulsion order q out of range 1..16");
}

// Repulsion of the current particles (eq. repul, three circles per ellipse);
// with update, also the Euler update of eq. euler from the hydrophobic force
// and torque fh, th into pb->dpnew, which is then on the host in
// pb->dstage after the n potential partials.  Returns Phi_rep.
double repulsion_of(yq_problem* pb, double c0, int32_t q, const double* fh, const double* th,
                    double dtx, double dtt, double* force, double* torque, bool update) {
  const int n = pb->n;
  hipStream_t s = pb->stream;
  pb->dcc.fit(n);
  pb->drad.fit(n);
  pb->dphi.fit(n);
  pb->dbad.fit(1);
  if (update) pb->dpnew.fit((size_t)3 * n);
  YQ_HIP(hipMemsetAsync(pb->dbad.p, 0, sizeof(int), s));
  {
    Timed t(pb, 7);
    launch_circles3(pb->pc.p, n, pb->dcc.p, pb->drad.p, s);
    DynArgs a{};
    a.pc = pb->pc.p;
    a.cc = pb->dcc.p;
    a.rad = pb->drad.p;
    a.n = n;
    a.q = q;
    a.c3 = c0 / 3.0;
    a.fh = fh;
    a.th = th;
    a.dtx = dtx;
    a.dtt = dtt;
    a.force = force;
    a.torque = torque;
    a.phi = pb->dphi.p;
    a.pnew = update ? pb->dpnew.p : nullptr;
    a.bad = pb->dbad.p;
    launch_repulsion(a, s);
  }
  // one round trip: the potential partials, the new configuration, the flag
  const size_t nd = (size_t)n * (update ? 4 : 1);
  pb->dstage.fit(nd * sizeof(double) + sizeof(double));
  double* h = (double*)pb->dstage.p;
  YQ_HIP(hipMemcpyAsync(h, pb->dphi.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
  if (update)
    YQ_HIP(hipMemcpyAsync(h + n, pb->dpnew.p, 3 * (size_t)n * sizeof(double),
                          hipMemcpyDeviceToHost, s));
  int* hb = (int*)(h + nd);
  YQ_HIP(hipMemcpyAsync(hb, pb->dbad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  YQ_HIP(hipStreamSynchronize(s));
  YQ_REQUIRE(*hb == 0, YQ_EGEOM, "two circles of the repulsion model touch or overlap");
  double t = 0.0;
  for (int i = 0; i < n; ++i) t += h[i];
  return 0.5 * t;
}

}  // namespace

extern "C" {

int yq_repulsion(yq_problem* pb, double c0, int32_t q, double* force, double* torque,
                 double* energy) {
  return guarded(pb, [&] {
    require_ready(pb);
    YQ_REQUIRE(force && torque, YQ_EINVAL, "null argument");
    check_repulsion(c0, q);
    const double e = repulsion_of(pb, c0, q, nullptr, nullptr, 0.0, 0.0, force, torque, false);
    if (energy) *energy = e;
  });
}

int yq_get_particles(const yq_problem* pb, double* center_xy, double* angle) {
  if (!pb) return YQ_EINVAL;
  if (pb->h_pc.empty()) return YQ_ESTATE;
  for (int i = 0; i < pb->n; ++i) {
    if (center_xy) {
      center_xy[2 * i] = pb->h_pc[5 * (size_t)i];
      center_xy[2 * i + 1] = pb->h_pc[5 * (size_t)i + 1];
    }
    if (angle) angle[i] = pb->h_pc[5 * (size_t)i + 2];
  }
  return YQ_OK;
}

int yq_step(yq_problem* pb, const yq_dynamics* dyn, double* sigma, double* sigma_prev,
            yq_solve_info* info, double* force, double* torque, double* energy) {
  int rc = guarded(pb, [&] {
    require_ready(pb);
    YQ_REQUIRE(dyn && sigma, YQ_EINVAL, "null argument");
    YQ_REQUIRE(sigma_prev != sigma, YQ_EINVAL, "sigma_prev aliases sigma");
    YQ_REQUIRE(pb->prm.refine_levels == 0, YQ_EINVAL,
               "time steps keep the nodes in each particle's frame: no adaptive refinement");
    YQ_REQUIRE(pb->have_f, YQ_ESTATE, "boundary data not set");
    YQ_REQUIRE(std::isfinite(dyn->dt) && dyn->dt >= 0.0, YQ_EINVAL, "dt must be finite and >= 0");
    YQ_REQUIRE(std::isfinite(dyn->xi_x) && dyn->xi_x > 0.0 && std::isfinite(dyn->xi_theta) &&
                   dyn->xi_theta > 0.0,
               YQ_EINVAL, "drag coefficients must be finite and > 0");
    YQ_REQUIRE(std::isfinite(dyn->gamma), YQ_EINVAL, "gamma must be finite");
    check_repulsion(dyn->c0, dyn->q);
    pb->dfh.fit((size_t)2 * pb->n);
    pb->dth.fit(pb->n);
    if (sigma_prev) launch_predict(sigma, sigma_prev, pb->N, pb->stream);
  });
  if (rc != YQ_OK) return rc;
  // solve at the current configuration, warm-started from sigma, and its forces
  double e_h = 0.0;
  const int st = yq_solve_forces(pb, sigma, sigma, info, dyn->gamma, pb->dfh.p, pb->dth.p, &e_h);
  if (st != YQ_OK && st != YQ_ENOCONV) return st;
  rc = guarded(pb, [&] {
    const bool move = st == YQ_OK;
    const int n = pb->n;
    const double e_r = repulsion_of(pb, dyn->c0, dyn->q, pb->dfh.p, pb->dth.p,
                                    dyn->dt / dyn->xi_x, dyn->dt / dyn->xi_theta, force, torque,
                                    move);
    if (energy) {
      energy[0] = e_h;
      energy[1] = e_r;
    }
    if (!move) return;
    // the new configuration; the boundary data stay, node k keeping its value
    const double* h = (const double*)pb->dstage.p + n;
    std::vector<double> cxy(2 * (size_t)n), ang(n), ax(2 * (size_t)n), ocxy(2 * (size_t)n),
        oang(n);
    for (int i = 0; i < n; ++i) {
      const double* o = &pb->h_pc[5 * (size_t)i];
      cxy[2 * i] = h[3 * i];
      cxy[2 * i + 1] = h[3 * i + 1];
      ang[i] = h[3 * i + 2];
      ax[2 * i] = o[3];
      ax[2 * i + 1] = o[4];
      ocxy[2 * i] = o[0];
      ocxy[2 * i + 1] = o[1];
      oang[i] = o[2];
    }
    const double kappa = pb->kappa;
    std::vector<double> rot(n);
    for (int i = 0; i < n; ++i) rot[i] = ang[i] - oang[i];
    try {
      setup_particles(pb, n, cxy.data(), ang.data(), ax.data(), kappa, rot.data());
    } catch (const Error& e) {
      if (e.code != YQ_EGEOM) throw;
      // rejected: rebuild the configuration the step started from
      setup_particles(pb, n, ocxy.data(), oang.data(), ax.data(), kappa);
      pb->have_f = true;
      throw Error{YQ_EGEOM, "the updated configuration was rejected (" + e.msg +
                                "); the particles did not move"};
    }
    pb->have_f = true;
  });
  if (rc != YQ_OK) return rc;
  if (st != YQ_OK) pb->err = "GMRES did not reach the tolerance; the particles did not move";
  return st;
}

int yq_profile_enable(yq_problem* pb, int32_t phase_mask) {
  return guarded(pb, [&] {
    YQ_REQUIRE(pb, YQ_EINVAL, "null problem");
    pb->prof_mask = (uint32_t)phase_mask;
  });
}

int yq_profile_read(yq_problem* pb, int32_t phase, int64_t* launches, double* total_ms,
                    int32_t reset) {
  return guarded(pb, [&] {
    YQ_REQUIRE(pb && launches && total_ms, YQ_EINVAL, "null argument");
    YQ_REQUIRE(phase >= 0 && phase < yq_problem::NPHASE, YQ_EINVAL, "bad phase");
    YQ_HIP(hipStreamSynchronize(pb->stream));
    double tot = 0.0;
    for (auto& p : pb->ev[phase]) {
      float ms = 0.0f;
      YQ_HIP(hipEventElapsedTime(&ms, p.first, p.second));
      tot += ms;
    }
    *launches = (int64_t)pb->ev[phase].size();
    *total_ms = tot;
    if (reset) {
      for (auto& p : pb->ev[phase]) {
        pb->pool.push_back(p.first);
        pb->pool.push_back(p.second);
      }
      pb->ev[phase].clear();
    }
  });
}

int yq_fmm_stats(const yq_problem* pb, int32_t* depth, int32_t* leaves, int32_t* max_leaf,
                 double* p2p_pairs, double* m2l_pairs) {
  return guarded(const_cast<yq_problem*>(pb), [&] {
    require_ready(pb);
    YQ_REQUIRE(pb->fmm != nullptr, YQ_ESTATE, "the problem has no FMM far field");
    const Fmm& f = *pb->fmm;
    if (depth) *depth = f.depth;
    if (leaves) *leaves = f.nleaf;
    if (max_leaf) *max_leaf = f.max_leaf;
    if (p2p_pairs) *p2p_pairs = (double)f.p2p_pairs;
    if (m2l_pairs) *m2l_pairs = (double)f.m2l_pairs;
  });
}

int yq_bessel(int32_t kind, int32_t order, int32_t precision, int64_t n, const double* z,
              double* out) {
  return guarded(nullptr, [&] {
    YQ_REQUIRE(kind >= 0 && kind <= 3, YQ_EINVAL, "kind must be 0..3");
    YQ_REQUIRE(order >= 0 && order <= MAXP + 1, YQ_EINVAL, "order out of range");
    YQ_REQUIRE(n >= 0 && (n == 0 || (z && out)), YQ_EINVAL, "null argument");
    std::vector<double> t(T_SIZE_HOST);
    fill_tab64(t.data());
    DevBuf<double> tab;
    upload(tab, t, nullptr);
    launch_bessel(kind, order, precision, n, z, out, tab.p, nullptr);
    YQ_HIP(hipStreamSynchronize(nullptr));
  });
}

}  // extern "C"
