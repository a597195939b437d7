// Steps a11 (stress, forces, torques, energy), a12 (off-surface potential)
// and the special-function test entry.
//
// Stress (eq. stress) with rho = 1/kappa and nu the unit normal into the water:
//   T.nu = gamma [kappa u^2 + |grad u|^2 / kappa] nu - (2 gamma / kappa) (grad u . nu) grad u,
// u = f on Sigma.  F_i = int T.nu dS, tau_i = int (x - a_i) x T.nu dS
// (eqs. force_torque, scalar-torque); the energy of eq. main follows from
// Green's first identity: Phi = -(gamma/kappa) int f du/dnu dS.
#include "bessel.h"
#include "common.h"

namespace yq {

constexpr int FB = 256;

__device__ __forceinline__ double bsum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = FB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// One block per particle.
__global__ __launch_bounds__(FB) void forces_kernel(GeomView g, const double* __restrict__ f,
                                                    const double* __restrict__ gx,
                                                    const double* __restrict__ gy, double gamma,
                                                    double* __restrict__ force,
                                                    double* __restrict__ torque,
                                                    double* __restrict__ energy) {
  __shared__ double sh[FB];
  const int p = blockIdx.x;
  const int64_t b = (int64_t)p * g.P * Q;
  const int64_t e = b + (int64_t)g.P * Q;
  const double cx = g.pc[5 * p], cy = g.pc[5 * p + 1];
  const double kap = g.kappa;
  double fx = 0.0, fy = 0.0, tq = 0.0, en = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += FB) {
    const double ux = gx[i], uy = gy[i];
    const double nx = g.nx[i], ny = g.ny[i];
    const double un = ux * nx + uy * ny;
    const double iso = gamma * (kap * f[i] * f[i] + (ux * ux + uy * uy) / kap);
    const double c2 = 2.0 * gamma / kap * un;
    const double tx = iso * nx - c2 * ux;
    const double ty = iso * ny - c2 * uy;
    const double w = g.w[i];
    fx += w * tx;
    fy += w * ty;
    tq += w * ((g.x[i] - cx) * ty - (g.y[i] - cy) * tx);
    en += -gamma / kap * w * f[i] * un;
  }
  fx = bsum(fx, sh);
  fy = bsum(fy, sh);
  tq = bsum(tq, sh);
  en = bsum(en, sh);
  if (threadIdx.x == 0) {
    force[2 * p] = fx;
    force[2 * p + 1] = fy;
    torque[p] = tq;
    energy[p] = en;
  }
}

// u(z) = sum over panels of the 16-point rule, or of an nsub-fold oversampled
// rule (sigma interpolated) for panels whose nearest node is closer than beta*h.
// Grid: (target blocks of 64) x (panel chunks); chunk partials are summed in a
// fixed order by potential_finish_kernel.
PotPlan pot_plan(int64_t M, int64_t npan) {
  PotPlan pp;
  pp.tblocks = (int)((M + 63) / 64);
  int64_t chunks = (4096 + pp.tblocks - 1) / pp.tblocks;
  if (chunks > npan) chunks = npan;
  if (chunks < 1) chunks = 1;
  pp.per = (int)((npan + chunks - 1) / chunks);
  pp.chunks = (int)((npan + pp.per - 1) / pp.per);
  return pp;
}

__global__ __launch_bounds__(64) void potential_kernel(GeomView g, Consts c, int nsub,
                                                       const double* __restrict__ L, double beta,
                                                       const double* __restrict__ sigma,
                                                       int64_t M, const double* __restrict__ tx,
                                                       const double* __restrict__ ty, int per,
                                                       double* __restrict__ partial) {
  const int64_t a0 = blockIdx.x * (int64_t)64 + threadIdx.x;
  const bool active = a0 < M;
  const int64_t a = active ? a0 : 0;
  const double zx = tx[a], zy = ty[a];
  const double kap2 = g.kappa * g.kappa;
  const int64_t npan = (int64_t)g.n * g.P;
  const int64_t J0 = (int64_t)blockIdx.y * per;
  const int64_t J1 = min(npan, J0 + per);
  double acc = 0.0;
  for (int64_t J = J0; J < J1; ++J) {
    const int64_t b = J * Q;
    double d2 = 1e300, part = 0.0;
    for (int m = 0; m < Q; ++m) {
      const double dx = zx - g.x[b + m], dy = zy - g.y[b + m];
      const double r2 = dx * dx + dy * dy;
      d2 = fmin(d2, r2);
      part += k1z_64(kap2 * r2, g.tab) * (dx * g.wnx[b + m] + dy * g.wny[b + m]) * sigma[b + m];
    }
    const double bh = beta * g.panel_h[J];
    if (d2 >= bh * bh) {
      acc += part;
      continue;
    }
    // oversampled: sub-panel nodes from the exact parametrisation
    const int pid = (int)(J / g.P), kj = (int)(J % g.P);
    const double* pp = g.pc + 5 * pid;
    double sa, ca;
    sincos(pp[2], &sa, &ca);
    for (int sub = 0; sub < nsub; ++sub) {
      for (int gq = 0; gq < Q; ++gq) {
        const double xl = -1.0 + (2.0 * sub + c.xg[gq] + 1.0) / nsub;
        const double t = 2.0 * PI / g.P * (kj + 0.5 * (xl + 1.0));
        double st, ct;
        sincos(t, &st, &ct);
        const double ex = pp[3] * ct, ey = pp[4] * st;
        const double ddx = -pp[3] * st, ddy = pp[4] * ct;
        const double yx = pp[0] + ca * ex - sa * ey;
        const double yy = pp[1] + sa * ex + ca * ey;
        const double gx = ca * ddx - sa * ddy, gy = sa * ddx + ca * ddy;
        const double sp = sqrt(gx * gx + gy * gy);
        const double wf = (PI / g.P / nsub) * c.wg[gq] * sp;
        const double* Lr = L + (sub * Q + gq) * Q;
        double sf = 0.0;
        for (int m = 0; m < Q; ++m) sf = fma(Lr[m], sigma[b + m], sf);
        const double dx = zx - yx, dy = zy - yy;
        const double r2 = dx * dx + dy * dy;
        acc += k1z_64(kap2 * r2, g.tab) * (dx * gy - dy * gx) / sp * wf * sf;
      }
    }
  }
  if (active) partial[(int64_t)blockIdx.y * M + a] = acc;
}

__global__ void potential_finish_kernel(const double* __restrict__ partial, int chunks, int64_t M,
                                        double scale, double* __restrict__ u) {
  const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= M) return;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += partial[(int64_t)c * M + a];
  u[a] = s * scale;
}

__global__ void bessel_kernel(int kind, int order, int prec, int64_t n, const double* __restrict__ z,
                              double* __restrict__ out, const double* __restrict__ tab) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = z[i];
  double v = 0.0;
  if (prec == YQ_MIXED && kind <= 1) {
    float k0, k1z;
    float xf = (float)x;
    k0_k1z_32(xf * xf, k0, k1z);
    // K1 through k1z_32, the evaluation of the FP32 pair kernels
    v = kind == 0 ? (double)k0 : (double)(k1z_32(xf * xf) * xf);
  } else if (kind == 0 || kind == 1 || kind == 2) {
    double k0, k1;
    k01_64(x, k0, k1, tab);
    if (kind == 0) {
      v = k0;
    } else if (kind == 1) {
      v = k1;
    } else {
      if (order == 0) {
        v = k0;
      } else {
        double km = k0, kc = k1;
        for (int l = 1; l < order; ++l) {
          double kp = km + (2.0 * l / x) * kc;
          km = kc;
          kc = kp;
        }
        v = kc;
      }
    }
  } else {
    double I[MAXP + 2];
    bessel_i_series64(x, order < MAXP + 1 ? order : MAXP + 1, I);
    v = I[order < MAXP + 1 ? order : MAXP + 1];
  }
  out[i] = v;
}

void launch_forces(const GeomView& g, const double* f, const double* gx, const double* gy,
                   double gamma, double* force, double* torque, double* energy_part,
                   hipStream_t s) {
  forces_kernel<<<g.n, FB, 0, s>>>(g, f, gx, gy, gamma, force, torque, energy_part);
  YQ_HIP(hipGetLastError());
}

void launch_potential(const GeomView& g, const Consts& c, int nsub, const double* L, double beta,
                      const double* sigma, int64_t M, const double* tx, const double* ty,
                      const PotPlan& pp, double* partial, double* u, hipStream_t s) {
  if (M == 0) return;
  dim3 grid(pp.tblocks, pp.chunks);
  potential_kernel<<<grid, 64, 0, s>>>(g, c, nsub, L, beta, sigma, M, tx, ty, pp.per, partial);
  YQ_HIP(hipGetLastError());
  potential_finish_kernel<<<(unsigned)((M + 255) / 256), 256, 0, s>>>(
      partial, pp.chunks, M, g.kappa * g.kappa / (2.0 * PI), u);
  YQ_HIP(hipGetLastError());
}

void fill_tab64(double* t) { build_tab64(t); }

void launch_bessel(int kind, int order, int prec, int64_t n, const double* z, double* out,
                   const double* tab, hipStream_t s) {
  if (n == 0) return;
  bessel_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(kind, order, prec, n, z, out, tab);
  YQ_HIP(hipGetLastError());
}

}  // namespace yq
