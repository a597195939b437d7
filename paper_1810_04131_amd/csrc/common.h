// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <pthread.h>

#include <cstdint>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "yqbx.h"

namespace yq {

constexpr int Q = 16;            // Gauss-Legendre nodes per panel
constexpr int MAXP = 30;         // largest QBX order
constexpr int MAXP_FMM = 48;     // largest FMM order
// YQ_FAR_AUTO switches the inner operator (and the server lane) to the FMM from
// this many nodes on (the measured crossover of the fused direct sum and the
// FMM on mixed-size request streams).
constexpr int64_t kFmmAutoNodes = 20000;
constexpr int MAXSUB = 16;       // largest oversampling factor
constexpr double PI = 3.14159265358979323846264338327950288;
constexpr int T_SIZE_HOST = 160;  // doubles in the FP64 coefficient table (bessel.h T_SIZE)

struct Error {
  int code;
  std::string msg;
};

#define YQ_HIP(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess)                                                                  \
      throw ::yq::Error{YQ_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)};        \
  } while (0)

#define YQ_REQUIRE(cond, code, msg)                                                        \
  do {                                                                                     \
    if (!(cond)) throw ::yq::Error{(code), (msg)};                                         \
  } while (0)

// Owning device buffer (hipMalloc / hipFree).  alloc() gives exactly the
// requested size; fit() only grows (the logical size n may be below the
// capacity), so buffers rebuilt for every geometry stop calling hipFree, which
// waits for the device.
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  size_t cap = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), cap(o.cap) {
    o.p = nullptr;
    o.n = o.cap = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      cap = o.cap;
      o.p = nullptr;
      o.n = o.cap = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = cap = 0;
  }
  void alloc(size_t count) {
    if (count == n && p) return;
    release();
    if (count == 0) return;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{YQ_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) +
                                 " bytes failed: " + hipGetErrorString(e)};
    }
    n = cap = count;
  }
  // grows, never shrinks; n = count
  void fit(size_t count) {
    if (p && count <= cap) {
      n = count;
      return;
    }
    alloc(count);
  }
  // grows, never shrinks (n becomes the new capacity)
  void reserve(size_t count) {
    if (count > n) alloc(count);
  }
  size_t bytes() const { return n * sizeof(T); }
};

// Grow-only pinned host buffer (hipHostMalloc), for staging set-up transfers.
struct PinnedBuf {
  char* p = nullptr;
  size_t cap = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  void fit(size_t bytes) {
    if (p && bytes <= cap) return;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipHostMalloc((void**)&p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{YQ_ENOMEM, "hipHostMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                 hipGetErrorString(e)};
    }
    cap = bytes;
  }
};

// A host thread with a stack of a stated size (std::thread takes the process
// default, which can be small where a profiler's callbacks run on the same stack).
// The constructor starts fn; join() (or the destructor) waits for it.
class HostThread {
 public:
  static constexpr size_t kStack = size_t(64) << 20;
  explicit HostThread(std::function<void()> fn) : fn_(new std::function<void()>(std::move(fn))) {
    pthread_attr_t a;
    pthread_attr_init(&a);
    pthread_attr_setstacksize(&a, kStack);
    const int rc = pthread_create(&t_, &a, &HostThread::run, fn_.get());
    pthread_attr_destroy(&a);
    if (rc != 0) throw Error{YQ_EDEVICE, "pthread_create failed"};
    live_ = true;
  }
  HostThread(const HostThread&) = delete;
  HostThread& operator=(const HostThread&) = delete;
  ~HostThread() { join(); }
  void join() {
    if (live_) (void)pthread_join(t_, nullptr);
    live_ = false;
  }

 private:
  static void* run(void* f) {
    try {
      (*static_cast<std::function<void()>*>(f))();
    } catch (...) {   // the callers' functions report errors through their own state
    }
    return nullptr;
  }
  std::unique_ptr<std::function<void()>> fn_;
  pthread_t t_{};
  bool live_ = false;
};

// Uniform loads through a constant-address-space pointer become scalar loads.
template <class T>
using kptr = const __attribute__((address_space(4))) T*;
template <class T>
__device__ __forceinline__ kptr<T> as_k(const T* p) {
  return (kptr<T>)p;
}

// A pointer known to address global memory (vector loads with a scalar base and a
// 32-bit offset instead of generic loads), for pointers read from memory.
template <class T>
using gptr = const __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> as_g(const T* p) {
  return (gptr<T>)p;
}
template <class T>
using gmut = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gmut<T> as_gm(T* p) {
  return (gmut<T>)p;
}

// Geometry of one problem as the kernels see it (all device pointers).
struct GeomView {
  int n;                 // particles
  int P;                 // panels per particle
  int64_t N;             // nodes
  double kappa;
  const double* pc;      // particles: [n*5] (cx, cy, angle, A, B)
  const double* x;       // nodes [N]
  const double* y;
  const double* nx;
  const double* ny;
  const double* w;
  const double* wnx;     // w * nx
  const double* wny;     // w * ny
  const double* panel_h; // [n*P]
  const double* tab;     // FP64 special-function coefficients (bessel.h, T_SIZE doubles)
  const double4* ftile;  // bounding circles of 256-node source tiles
  const double4* fgrp;   // bounding circles of 64-node target groups
  const double4* fpan;   // bounding circles of 16-node panels
  // cutoff far field: (group, tile) pairs with kappa x gap >= zcut are skipped in
  // the value sums, >= zcut_g in the gradient sums (HUGE_VAL: exact sums)
  double zcut = HUGE_VAL;
  double zcut_g = HUGE_VAL;
  // combined representation D + eta S (eq. bwform): coupling of the single layer,
  // 0 for the double layer alone
  double eta = 0.0;
  // adaptive panels (null: P equal-parameter panels per particle, panel J =
  // particle * P + k): per panel (particle, base panel k, level, index at that
  // level), and the first panel of every particle [n + 1]; npan panels in all
  const int4* pan = nullptr;
  const int* poff = nullptr;
  int64_t npan = 0;
};

// ---- panels of a geometry (uniform or adaptively refined) -----------------------------

__device__ __forceinline__ int panel_particle(const GeomView& g, int64_t J) {
  return g.pan ? g.pan[J].x : (int)(J / g.P);
}

// The panels of particle p: [first, first + cnt), in increasing parameter.
__device__ __forceinline__ void particle_panels(const GeomView& g, int p, int64_t& first,
                                                int& cnt) {
  if (g.poff) {
    first = g.poff[p];
    cnt = g.poff[p + 1] - g.poff[p];
  } else {
    first = (int64_t)p * g.P;
    cnt = g.P;
  }
}

// Panel J's place on its particle's ring: the ring's first panel, its length,
// and J - first.
struct Ring {
  int64_t first;
  int cnt, k;
};

__device__ __forceinline__ Ring ring_of(const GeomView& g, int64_t J) {
  Ring r;
  particle_panels(g, panel_particle(g, J), r.first, r.cnt);
  r.k = (int)(J - r.first);
  return r;
}

// The panel o places from the ring position r (|o| < r.cnt).
__device__ __forceinline__ int64_t ring_step(const Ring& r, int o) {
  int kj = (r.k + o) % r.cnt;
  if (kj < 0) kj += r.cnt;
  return r.first + kj;
}

// Parameter t of panel J at coordinate xi in [-1, 1], and dt / dxi: panel J is
// 2 pi / P (k + [idx, idx + 1] 2^-lev) of base panel k of its ellipse.
__device__ __forceinline__ double panel_param(const GeomView& g, int64_t J, double xi,
                                              double& dt) {
  int k, lev = 0, idx = 0;
  if (g.pan) {
    const int4 d = g.pan[J];
    k = d.y;
    lev = d.z;
    idx = d.w;
  } else {
    k = (int)(J % g.P);
  }
  dt = ldexp(PI / g.P, -lev);
  return 2.0 * PI / g.P * (k + ldexp(idx + 0.5 * (xi + 1.0), -lev));
}

// Discretisation constants, passed to kernels by value.
struct Consts {
  double xg[Q];                 // Gauss-Legendre nodes on [-1, 1], ascending
  double wg[Q];                 // weights
};

// ---------------------------------------------------------------------------------------
// Host launchers (implemented in the .hip files)
// ---------------------------------------------------------------------------------------

// gauss.cpp-like host helpers (geometry.hip)
void gauss_legendre16(double* x, double* w);
void lagrange_matrix(const double* src, int q, const double* dst, int nd, double* L);
void sub_panel_coords(const double* xg, int q, int nsub, double* xi);

void launch_geometry(const GeomView& g, const Consts& c, double* x, double* y, double* nx, double* ny, double* w,
                     double* wnx, double* wny, hipStream_t s);
void launch_panel_stats(const GeomView& g, double* panel_h, double* pcx, double* pcy, double* pr,
                        hipStream_t s);
void launch_label(const GeomView& g, int kind, double a, double b, double* f, hipStream_t s);
void launch_geom_check(const GeomView& g, const int* nb_ptr, const int* nb_idx, int* bad,
                       hipStream_t s);
void launch_near_count(const GeomView& g, int win, double beta, const int* nb_ptr,
                       const int* nb_idx, const double* pcx, const double* pcy, const double* pr,
                       int* count, int* list, const int* offs, hipStream_t s);
// row[0] = 0, row[i + 1] = count[0] + ... + count[i] (device; tmp: scan scratch)
void launch_row_scan(const int* count, int64_t N, int* row, DevBuf<char>& tmp, hipStream_t s);

// fx, fy, fwx, fwy: the oversampled points of every panel (nsub sub-panels), as
// built by launch_pot_fine
void launch_qbx_build(const GeomView& g, int p, int win, int nsub, double radius, const double* L,
                      const double* fx, const double* fy, const double* fwx, const double* fwy,
                      double* W, double* WGx, double* WGy, hipStream_t s);
void launch_near_rows(const GeomView& g, const Consts& c, int nsub, const double* L,
                      const int* row_ptr, const int* panels, double* vals, double* gvals,
                      hipStream_t s);

struct FarPlan {
  int tblocks;   // target blocks
  int chunks;    // source chunks
  int chunk;     // sources per chunk (multiple of the block size)
};
FarPlan far_plan(int64_t nt, int64_t ns, int block, int want = 4096);

// FP32 far field (farfield_core.h): 256-node source tiles, 64-node target groups.
constexpr int FT = 256;   // source tile (nodes)
constexpr int FG = 64;    // target group (nodes)
constexpr double LOG2E = 1.44269504088896340736;
constexpr double SQRT_LOG2E = 1.20112240878644981;

struct Far32View {
  const double* x;     // FP64 node positions [N]
  const double* y;
  const double4* tile; // per 256-node tile: centre x, y, radius
  const double4* grp;  // per 64-node group: centre x, y, radius
  const double4* pan;  // per 16-node panel: centre x, y, radius
  const float4* src;   // per node, packed per matvec
  int64_t N;
  double s;            // kappa log2(e)
  double kappa;        // pairs are far when kappa x the gap between circles is >= 2
  double qc;           // sqrt(log2 e) / kappa: source strength scaling of the records
  float kap2;          // kappa^2 (general path)
  float nscale;        // kappa / sqrt(log2 e): general-path sum -> far-path scaling
  double zcut = HUGE_VAL;  // tiles with kappa x gap >= zcut are skipped (cutoff far field)
};

void launch_far32_geom(const double* x, const double* y, int64_t N, double kappa, double4* tile,
                       double4* grp, double4* pan, float2* rel, hipStream_t s);
void launch_pack32(const float2* rel, const double* wnx, const double* wny, const double* sigma,
                   int64_t N, double qc, float4* src, hipStream_t s);
// stop: optional device flag; the launch does nothing when it is set.  e0, e1:
// optional events that the launch itself records at the kernel's start and end.
void launch_far64(const GeomView& g, const double* sigma, const FarPlan& fp, double* partial,
                  hipStream_t s, const int* stop = nullptr, hipEvent_t e0 = nullptr,
                  hipEvent_t e1 = nullptr);
void launch_far32(const Far32View& v, const FarPlan& fp, float* partial, hipStream_t s,
                  const int* stop = nullptr, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_finish(const GeomView& g, int win, const FarPlan& fp, const double* partial64,
                   const float* partial32, const double* W, const int* xrow, const int* xpan,
                   const double* xvals, const double* sigma, double* out, hipStream_t s);
void launch_far_grad64(const GeomView& g, const double* sigma, const FarPlan& fp, double* partial,
                       hipStream_t s);
// Combined representation D + g.eta S (g.eta > 0): the far field in FP64 (p64) or
// FP32 arithmetic (p32; exactly one of the two is non-null), partials in the
// scaling of the double-layer kernels; and its FP64 gradient.
void launch_far_sd(const GeomView& g, const double* sigma, const FarPlan& fp, double* p64,
                   float* p32, hipStream_t s, const int* stop = nullptr, hipEvent_t e0 = nullptr,
                   hipEvent_t e1 = nullptr);
void launch_far_sd_grad64(const GeomView& g, const double* sigma, const FarPlan& fp,
                          double* partial, hipStream_t s);
void launch_far_fused64(const GeomView& g, const double* sigma, const FarPlan& fp,
                        double* partial, double* gpartial, hipStream_t s);
void launch_finish_grad(const GeomView& g, int win, const FarPlan& fp, const double* partial,
                        const double* WGx, const double* WGy, const int* xrow, const int* xpan,
                        const double* xgvals, const double* sigma, double* gx, double* gy,
                        hipStream_t s);

// Krylov helpers (krylov.hip)
int krylov_blocks(int64_t n);
void launch_multidot(const double* V, int64_t ld, int k, const double* w, int64_t n, double* partial,
                     int nb, hipStream_t s);
// w += alpha V h with h[k] the in-order sum of partial[k * nb .. k * nb + nb)
void launch_update_partial(double* w, const double* V, int64_t ld, int k, const double* partial,
                           int nb, double alpha, int64_t n, hipStream_t s);
// p[0] + p[1] + ... + p[nb - 1] in that order, on the host (the update kernel's order)
double sum_partials(const double* p, int nb);
// Blocks of the update_norm kernel (= the number of |w|^2 partials it writes)
int krylov_norm_blocks(int64_t n);
// launch_update_partial, and npart[b] = block b's sum of the new w_i^2
void launch_update_norm(double* w, const double* V, int64_t ld, int k, const double* partial,
                        int nb, double alpha, int64_t n, double* npart, hipStream_t s);
// One Arnoldi step on the device: Hessenberg column j (leading dimension ldh)
// from the partials of the two Gram-Schmidt passes at part (nb per column),
// h_{j+1,j} = |w| from npart (krylov_norm_blocks(n) partials), the earlier Givens
// rotations (cs, sn) applied, the new rotation, g updated, *stop set when
// |g_{j+1}| / bnorm <= rtol or at a breakdown, status = (|g_{j+1}| / bnorm,
// h_{j+1,j}, stop); fused with vn = w / h_{j+1,j} (0 at a breakdown) and, when src
// is given, vn's FP32 source records (rel, wnx, wny, qc as for launch_pack32).
// Nothing happens when *stop is already set.
void launch_arnoldi_scale(const double* part, int nb, const double* npart, int j, int ldh,
                          double* H, double* cs, double* sn, double* g, int* stop, double bnorm,
                          double rtol, double* status, const double* w, double* vn, int64_t n,
                          const float2* rel, const double* wnx, const double* wny, double qc,
                          float4* src, hipStream_t s);
// y[0..k) = R^-1 g, R the leading k x k upper triangle of H (device arrays)
void launch_trisolve(const double* H, int ldh, const double* g, int k, double* y, hipStream_t s);
// g[0] = beta, g[1..m] = 0, *stop = 0 (start of a GMRES cycle)
void launch_gmres_init(double* g, int m, double beta, int* stop, hipStream_t s);
void launch_update(double* w, const double* V, int64_t ld, int k, const double* h, double alpha,
                   int64_t n, hipStream_t s);
void launch_axpby(double a, const double* x, double b, const double* y, double* out, int64_t n,
                  hipStream_t s);

// excluded-volume repulsion and the Euler update (dynamics.hip)
struct DynArgs {
  const double* pc;    // [5n] particles (cx, cy, theta, A, B)
  const double4* cc;   // [n] centre and h d of the three circles (launch_circles3)
  const double* rad;   // [n] circle radius B
  int n;
  int q;               // repulsion order
  double c3;           // c0 / 3, the strength of one circle pair
  const double* fh;    // [2n] hydrophobic force added before the update, or null
  const double* th;    // [n] hydrophobic torque, with fh
  double dtx, dtt;     // dt / xi_x and dt / xi_theta
  double* force;       // [2n] out: total force (F^rep + fh), or null
  double* torque;      // [n] out: total torque, or null
  double* phi;         // [n] out: sum over the circle pairs of particle i of (c0/3) g^-q
  double* pnew;        // [3n] out: updated (cx, cy, theta), or null
  int* bad;            // set to 1 when two circles touch or overlap
};
void launch_circles3(const double* pc, int n, double4* cc, double* rad, hipStream_t s);
void launch_repulsion(const DynArgs& a, hipStream_t s);
// (gx, gy) <- R (gx, gy) for entries k * N + i (k < K), R the turn of node i's
// particle (i / npp): cs [2n] holds its (cos, sin)
void launch_rotate_grad_rows(double* gx, double* gy, int64_t K, int64_t N, int64_t npp,
                             const double* cs, hipStream_t s);
// sigma <- 2 sigma - sigma_prev, sigma_prev <- the old sigma
void launch_predict(double* sigma, double* sigma_prev, int64_t N, hipStream_t s);

// post-processing (post.hip)
void launch_forces(const GeomView& g, const double* f, const double* gx, const double* gy,
                   double gamma, double* force, double* torque, double* energy_part,
                   hipStream_t s);
struct PotPlan {
  int tblocks;   // target blocks of 64
  int chunks;    // panel chunks
  int per;       // panels per chunk
};
PotPlan pot_plan(int64_t M, int64_t npan);
// Oversampled panel rule of the off-surface potential: points, (weight) * (unit
// normal) and the interpolated density, [panel * nsub * Q + k] each.
struct PotFine {
  int nsub;
  double *x, *y, *wx, *wy, *s;
};
void launch_pot_fine(const GeomView& g, const Consts& c, int nsub, const PotFine& pf,
                     hipStream_t s);
void launch_potential(const GeomView& g, const PotFine& pf, const double* L, double beta,
                      const double* sigma, int64_t M, const double* tx, const double* ty,
                      const PotPlan& pp, double* partial, double* u, hipStream_t s);

// special functions (bessel_test.hip)
void launch_bessel(int kind, int order, int prec, int64_t n, const double* z, double* out,
                   const double* tab, hipStream_t s);
void fill_tab64(double* host_tab);   // writes the T_SIZE FP64 coefficients

}  // namespace yq
