// Excluded-volume repulsion and the constant-drag Euler update.
//
// Repulsion (eq. repul, with the three-circle model of ellipses of supplementary
// section S1): particle i is three circles of radius B_i centred at
// a_i + k h_i d_i, k = -1, 0, +1, h_i = A_i - B_i, d_i = (cos th_i, sin th_i).
// Two circles with centre distance r and gap g = r - (B_i + B_j) > 0 repel with
// (c0/3) q g^-(q+1) along the line of centres and carry the pair potential
// (c0/3) g^-q.  F_i^rep sums the nine circle pairs over every other particle;
// tau_i^rep is the torque about a_i of the forces on the end circles.
//
// Update (eq. euler): a_i += dt/xi_x (F_i + F_i^rep), th_i += dt/xi_th (tau_i + tau_i^rep).
//
// Layout: one wavefront per particle i, its 64 lanes striding over the other
// particles j; a fixed butterfly sums the lanes, so results do not depend on
// timing.  All arithmetic is FP64: the sum is O(n^2) circle-pair evaluations of
// about 40 FP64 operations each, VALU-bound and negligible next to the solve
// for the particle counts of one configuration.
#include "common.h"

namespace yq {
namespace {

constexpr int DB = 256;             // threads per block: four particles
constexpr int DW = 64;              // wavefront

// Per particle: centre, h d (the offset of the end circles) and radius B.
__global__ __launch_bounds__(DB) void circles3_kernel(const double* __restrict__ pc, int n,
                                                      double4* __restrict__ cc,
                                                      double* __restrict__ rad) {
  const int i = blockIdx.x * DB + threadIdx.x;
  if (i >= n) return;
  const double* p = pc + 5 * (size_t)i;
  const double h = p[3] - p[4];
  double s, c;
  sincos(p[2], &s, &c);
  cc[i] = make_double4(p[0], p[1], h * c, h * s);
  rad[i] = p[4];
}

__device__ __forceinline__ double wsum(double v) {
  for (int o = DW / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, DW);
  return v;
}

__device__ __forceinline__ double ipow(double x, int q) {
  double r = x;
  for (int k = 1; k < q; ++k) r *= x;
  return r;
}

__global__ __launch_bounds__(DB) void repulsion_kernel(DynArgs a) {
  const int lane = threadIdx.x % DW;
  const int i = blockIdx.x * (DB / DW) + threadIdx.x / DW;
  if (i >= a.n) return;   // whole wavefronts leave together
  const double4 ci = a.cc[i];
  const double bi = a.rad[i];
  const double cq = a.c3 * a.q;
  double fx[3] = {0.0, 0.0, 0.0}, fy[3] = {0.0, 0.0, 0.0}, ph = 0.0;
  int bad = 0;
  for (int j = lane; j < a.n; j += DW) {
    if (j == i) continue;
    const double4 cj = a.cc[j];
    const double rr = bi + a.rad[j];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double xk = ci.x + (k - 1) * ci.z, yk = ci.y + (k - 1) * ci.w;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const double rx = xk - (cj.x + (l - 1) * cj.z);
        const double ry = yk - (cj.y + (l - 1) * cj.w);
        const double r = sqrt(rx * rx + ry * ry);
        const double g = r - rr;
        if (!(g > 0.0)) {
          bad = 1;
          continue;
        }
        const double ig = 1.0 / g;
        const double pw = ipow(ig, a.q);
        ph += pw;
        const double m = cq * pw * ig / r;
        fx[k] += m * rx;
        fy[k] += m * ry;
      }
    }
  }
  // the end circles' torque about a_i: (k h d_i) x f_k for k = -1, +1
  const double Fx = wsum(fx[0] + fx[1] + fx[2]);
  const double Fy = wsum(fy[0] + fy[1] + fy[2]);
  const double dfx = fx[2] - fx[0], dfy = fy[2] - fy[0];
  const double T = wsum(ci.z * dfy - ci.w * dfx);
  const double P = wsum(ph) * a.c3;
  const bool anybad = __any(bad);
  if (lane != 0) return;
  if (anybad) a.bad[0] = 1;
  double gx = Fx, gy = Fy, gt = T;
  if (a.fh) {
    gx += a.fh[2 * i];
    gy += a.fh[2 * i + 1];
    gt += a.th[i];
  }
  if (a.force) {
    a.force[2 * i] = gx;
    a.force[2 * i + 1] = gy;
  }
  if (a.torque) a.torque[i] = gt;
  a.phi[i] = P;
  if (a.pnew) {
    const double* p = a.pc + 5 * (size_t)i;
    a.pnew[3 * i] = p[0] + a.dtx * gx;
    a.pnew[3 * i + 1] = p[1] + a.dtx * gy;
    a.pnew[3 * i + 2] = p[2] + a.dtt * gt;
  }
}

// Initial guess of a time step from the densities of the last two steps:
// g = 2 s - p (linear extrapolation in time); p takes s's old value, s takes g.
__global__ __launch_bounds__(DB) void predict_kernel(double* __restrict__ s, double* __restrict__ p,
                                                     int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * DB + threadIdx.x;
  if (i >= N) return;
  const double si = s[i];
  s[i] = 2.0 * si - p[i];
  p[i] = si;
}

// The gradient rows of the window QBX correction turned with their particle.
__global__ __launch_bounds__(DB) void rotate_grad_rows_kernel(double* __restrict__ gx,
                                                              double* __restrict__ gy, int64_t N,
                                                              int64_t npp,
                                                              const double* __restrict__ cs) {
  const int64_t i = (int64_t)blockIdx.x * DB + threadIdx.x;
  if (i >= N) return;
  const int64_t o = (int64_t)blockIdx.y * N + i;
  const int64_t p = i / npp;
  const double c = cs[2 * p], s = cs[2 * p + 1];
  const double a = gx[o], b = gy[o];
  gx[o] = c * a - s * b;
  gy[o] = s * a + c * b;
}

}  // namespace

void launch_rotate_grad_rows(double* gx, double* gy, int64_t K, int64_t N, int64_t npp,
                             const double* cs, hipStream_t s) {
  if (N <= 0 || K <= 0) return;
  YQ_REQUIRE(K <= 65535 && npp > 0 && N % npp == 0, YQ_EINVAL, "rotate_grad_rows: bad shape");
  rotate_grad_rows_kernel<<<dim3((unsigned)((N + DB - 1) / DB), (unsigned)K), DB, 0, s>>>(
      gx, gy, N, npp, cs);
  YQ_HIP(hipGetLastError());
}

void launch_predict(double* sigma, double* sigma_prev, int64_t N, hipStream_t s) {
  if (N <= 0) return;
  predict_kernel<<<(unsigned)((N + DB - 1) / DB), DB, 0, s>>>(sigma, sigma_prev, N);
  YQ_HIP(hipGetLastError());
}

void launch_circles3(const double* pc, int n, double4* cc, double* rad, hipStream_t s) {
  if (n <= 0) return;
  circles3_kernel<<<(n + DB - 1) / DB, DB, 0, s>>>(pc, n, cc, rad);
  YQ_HIP(hipGetLastError());
}

void launch_repulsion(const DynArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  const int per = DB / DW;
  repulsion_kernel<<<(a.n + per - 1) / per, DB, 0, s>>>(a);
  YQ_HIP(hipGetLastError());
}

}  // namespace yq
