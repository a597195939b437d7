// Stress, forces, torques and energy; the off-surface potential;
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
  int64_t first;
  int cnt;
  particle_panels(g, p, first, cnt);
  const int64_t b = first * Q;
  const int64_t e = b + (int64_t)cnt * Q;
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
// Grid: (target blocks of 64) x (panel chunks); the chunk partials,
// [target * chunks + chunk], are summed in a fixed order by potential_finish_kernel.
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

// Oversampled source points of every panel for targets near it: point
// k = sub * Q + gq of panel J lies at the exact parametrisation of sub-panel sub
// (Gauss-Legendre node gq), with (fwx, fwy) = (weight) * (unit normal) of the
// oversampled rule.  Per geometry; layout [J * nsub * Q + k].
__global__ void pot_fine_kernel(GeomView g, Consts c, int nsub, double* __restrict__ fx,
                                double* __restrict__ fy, double* __restrict__ fwx,
                                double* __restrict__ fwy) {
  const int F = nsub * Q;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= g.npan * F) return;
  const int64_t J = idx / F;
  const int k = (int)(idx - J * F);
  const int sub = k / Q, gq = k - sub * Q;
  const int pid = panel_particle(g, J);
  const double* pp = g.pc + 5 * pid;
  double sa, ca;
  sincos(pp[2], &sa, &ca);
  const double xl = -1.0 + (2.0 * sub + c.xg[gq] + 1.0) / nsub;
  double dt;
  const double t = panel_param(g, J, xl, dt);
  double st, ct;
  sincos(t, &st, &ct);
  const double ex = pp[3] * ct, ey = pp[4] * st;
  const double ddx = -pp[3] * st, ddy = pp[4] * ct;
  const double gx = ca * ddx - sa * ddy, gy = sa * ddx + ca * ddy;
  // w / |gamma'| = (dt / nsub) wg, so (w nu) = (dt / nsub) wg (gy, -gx)
  const double wq = (dt / nsub) * c.wg[gq];
  fx[idx] = pp[0] + ca * ex - sa * ey;
  fy[idx] = pp[1] + sa * ex + ca * ey;
  fwx[idx] = wq * gy;
  fwy[idx] = -wq * gx;
}

// sigma interpolated to the oversampled points: fs[J * F + k] = sum_m L[k][m] sigma[J * Q + m].
__global__ void pot_fine_sigma_kernel(int64_t npan, int nsub, const double* __restrict__ L,
                                      const double* __restrict__ sigma, double* __restrict__ fs) {
  const int F = nsub * Q;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= npan * F) return;
  const int64_t J = idx / F;
  const int k = (int)(idx - J * F);
  const double* Lr = L + (int64_t)k * Q;
  const double* sg = sigma + J * Q;
  double t = 0.0;
#pragma unroll
  for (int m = 0; m < Q; ++m) t = fma(Lr[m], sg[m], t);
  fs[idx] = t;
}

__global__ __launch_bounds__(64) void potential_kernel(GeomView g, PotFine pf, double beta,
                                                       const double* __restrict__ sigma,
                                                       int64_t M, const double* __restrict__ tx,
                                                       const double* __restrict__ ty, int per,
                                                       double* __restrict__ partial) {
  const int lane = threadIdx.x;
  const int64_t a0 = blockIdx.x * (int64_t)64 + lane;
  const bool active = a0 < M;
  const int64_t a = active ? a0 : 0;
  const double zx = tx[a], zy = ty[a];
  const double kap2 = g.kappa * g.kappa;
  const int64_t npan = g.npan;
  const int64_t J0 = (int64_t)blockIdx.y * per;
  const int64_t J1 = min(npan, J0 + per);
  const int F = pf.nsub * Q;
  kptr<double> sx = as_k(g.x), sy = as_k(g.y), swx = as_k(g.wnx), swy = as_k(g.wny);
  kptr<double> ssg = as_k(sigma), sww = as_k(g.w);
  // combined representation D + eta S: the single layer's eta w G, in the same
  // kappa^2 / 2pi scaling (G = (kappa^2 / 2pi) K0 / kappa^2)
  const double ek = g.eta / kap2;
  double acc = 0.0;
  for (int64_t J = J0; J < J1; ++J) {
    const int64_t b = J * Q;
    double d2 = 1e300, part = 0.0;
    for (int m = 0; m < Q; ++m) {
      const double dx = zx - sx[b + m], dy = zy - sy[b + m];
      const double r2 = dx * dx + dy * dy;
      d2 = fmin(d2, r2);
      if (g.eta > 0.0) {
        double k0, k1z;
        k0_k1z_64(kap2 * r2, k0, k1z, g.tab);
        part += (k1z * (dx * swx[b + m] + dy * swy[b + m]) + ek * k0 * sww[b + m]) * ssg[b + m];
      } else {
        part += k1z_64(kap2 * r2, g.tab) * (dx * swx[b + m] + dy * swy[b + m]) * ssg[b + m];
      }
    }
    const double bh = beta * g.panel_h[J];
    const bool near = active && d2 < bh * bh;
    if (!near) acc += part;
    // oversampled rule for the lanes near this panel, one lane at a time: the
    // whole wavefront evaluates its points for that lane's target and sums them
    uint64_t nm = __ballot(near);
    const double* fx = pf.x + J * F;
    const double* fy = pf.y + J * F;
    const double* fwx = pf.wx + J * F;
    const double* fwy = pf.wy + J * F;
    const double* fs = pf.s + J * F;
    while (nm) {
      const int t = __ffsll((unsigned long long)nm) - 1;
      nm &= nm - 1;
      const double ux = __shfl(zx, t, 64), uy = __shfl(zy, t, 64);
      double sum = 0.0;
      for (int k = lane; k < F; k += 64) {
        const double dx = ux - fx[k], dy = uy - fy[k];
        if (g.eta > 0.0) {
          double k0, k1z;
          k0_k1z_64(kap2 * (dx * dx + dy * dy), k0, k1z, g.tab);
          const double wk = sqrt(fwx[k] * fwx[k] + fwy[k] * fwy[k]);   // the normal is a unit vector
          sum += (k1z * (dx * fwx[k] + dy * fwy[k]) + ek * k0 * wk) * fs[k];
        } else {
          sum += k1z_64(kap2 * (dx * dx + dy * dy), g.tab) * (dx * fwx[k] + dy * fwy[k]) * fs[k];
        }
      }
      for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
      if (lane == t) acc += sum;
    }
  }
  if (active) partial[a * gridDim.y + blockIdx.y] = acc;
}

// u[a] = scale * sum_c partial[a * chunks + c]: one wavefront per target, each
// lane summing every 64th chunk in order, then a fixed butterfly.
__global__ __launch_bounds__(256) void potential_finish_kernel(const double* __restrict__ partial,
                                                               int chunks, int64_t M, double scale,
                                                               double* __restrict__ u) {
  const int64_t a = blockIdx.x * (int64_t)4 + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (a >= M) return;   // uniform over the wavefront
  double s = 0.0;
  for (int c = lane; c < chunks; c += 64) s += partial[a * chunks + c];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) u[a] = s * scale;
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

void launch_pot_fine(const GeomView& g, const Consts& c, int nsub, const PotFine& pf,
                     hipStream_t s) {
  const int64_t n = g.npan * nsub * Q;
  if (n == 0) return;
  pot_fine_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g, c, nsub, pf.x, pf.y, pf.wx, pf.wy);
  YQ_HIP(hipGetLastError());
}

void launch_potential(const GeomView& g, const PotFine& pf, const double* L, double beta,
                      const double* sigma, int64_t M, const double* tx, const double* ty,
                      const PotPlan& pp, double* partial, double* u, hipStream_t s) {
  if (M == 0) return;
  const int64_t npan = g.npan;
  const int64_t nf = npan * pf.nsub * Q;
  pot_fine_sigma_kernel<<<(unsigned)((nf + 255) / 256), 256, 0, s>>>(npan, pf.nsub, L, sigma,
                                                                      pf.s);
  YQ_HIP(hipGetLastError());
  dim3 grid(pp.tblocks, pp.chunks);
  potential_kernel<<<grid, 64, 0, s>>>(g, pf, beta, sigma, M, tx, ty, pp.per, partial);
  YQ_HIP(hipGetLastError());
  potential_finish_kernel<<<(unsigned)((M + 3) / 4), 256, 0, s>>>(
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
