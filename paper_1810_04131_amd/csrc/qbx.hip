// The FP64 QBX near correction of the operator and of its surface gradient.
//
// For target x_i on panel k the contribution of the window panels k-win..k+win
// goes through local expansions about c = x_i +/- r nu_i, r = radius * h_k
// (section 5, eqs. local-exp, graf-coefficient, graf-addition written for the
// Yukawa kernel k = i kappa):
//
//   u(x) = sum_{l=-p..p} alpha_l I_l(kappa r_x) e^{-i l th_x},
//   alpha_l = (1/2pi) int d/dnu [K_l(kappa r_y) e^{i l th_y}] sigma ds.
//
// Pairing l with -l (K_{-l} = K_l, I_{-l} = I_l) gives, per unit sigma at a
// sub-panel node y with weight w, Delta = th_y - th_x,
//   a_l = kappa K_l'(kappa r_y) (rhat . nu_y),  b_l = K_l(kappa r_y) (thhat . nu_y) / r_y,
//   P_l = a_l cos(l Delta) - l b_l sin(l Delta),  Q_l = a_l sin(l Delta) + l b_l cos(l Delta),
//   value    (w/2pi) [ I_0 a_0 + 2 sum_l I_l P_l ],
//   gradient (w/2pi) [ a_0 kappa I_0' rhat_x + 2 sum_l (P_l kappa I_l' rhat_x + Q_l (l/r) I_l thhat_x) ].
// The single layer (eq. single-layer-def) has the coefficients (1/2pi) int K_l(kappa
// r_y) e^{i l th_y} sigma ds, so the combined representation D + eta S (eq. bwform)
// adds eta K_l(kappa r_y) to a_l.
// sigma on the sub-panels is the Lagrange interpolant of the 16 coarse values.
// The operator row is the mean of the exterior (+) and interior (-) expansions
// plus 1/2 at the self node (1/2 sigma + p.v. D sigma, eq. djump / eq. bie);
// the gradient row is the exterior expansion (the exterior limit).  The plain
// 16-point far-field terms of the window nodes are subtracted, because the
// far-field kernel sums every pair j != i.
//
// Layout: W[(slot*16 + m) * N + i] for window slot 0..2*win, coarse node m.
#include "bessel.h"
#include "common.h"

namespace yq {

// Plain far-field coefficient and gradient of source j at target i (same
// formulas as the far-field kernels, scaled by kappa^2 / 2pi; with g.eta > 0 the
// single layer's eta w G and eta w grad G are included).
__device__ __forceinline__ void smooth_pair(const GeomView& g, double xi, double yi, int64_t j,
                                            double& s, double& sgx, double& sgy) {
  double dx = xi - g.x[j], dy = yi - g.y[j];
  double r2 = dx * dx + dy * dy;
  double kap2 = g.kappa * g.kappa;
  double k0, k1z;
  k0_k1z_64(kap2 * r2, k0, k1z, g.tab);
  double c = kap2 / (2.0 * PI);
  double qx = g.wnx[j], qy = g.wny[j];
  double dq = dx * qx + dy * qy;
  const double ew = g.eta * g.w[j];
  s = c * (k1z * dq + ew * k0 / kap2);
  double b = dq * (k0 + 2.0 * k1z) * rcp64(r2) + ew * k1z;
  sgx = c * (k1z * qx - b * dx);
  sgy = c * (k1z * qy - b * dy);
}

// The oversampled points of the window panels come from a per-geometry table
// (fx, fy, and (fwx, fwy) = weight x unit normal, [panel * nsub * 16 + k]); the
// normal and the weight enter the sums only through their product.
template <int BS>
__global__ __launch_bounds__(BS) void qbx_build_kernel(GeomView g, int p, int win, int nsub,
                                                       double radius, const double* __restrict__ L,
                                                       const double* __restrict__ fx,
                                                       const double* __restrict__ fy,
                                                       const double* __restrict__ fwx,
                                                       const double* __restrict__ fwy,
                                                       double* __restrict__ W,
                                                       double* __restrict__ WGx,
                                                       double* __restrict__ WGy) {
  __shared__ double sI[MAXP + 2][BS];
  const int tid = threadIdx.x;
  const int64_t i0 = blockIdx.x * (int64_t)BS + tid;
  const bool active = i0 < g.N;
  const int64_t i = active ? i0 : 0;
  const int slot = blockIdx.y;
  const double kap = g.kappa;

  const int64_t pan = i / Q;
  const double xi = g.x[i], yi = g.y[i], nxi = g.nx[i], nyi = g.ny[i];
  const double r = radius * g.panel_h[pan];
  const double ir = rcp64(r);

  // I_l(kappa r), l = 0..p+1, by the ascending series
  {
    const double xr = kap * r;
    const double t = 0.25 * xr * xr;
    double pref = 1.0;
    for (int l = 0; l <= p + 1; ++l) {
      double term = pref, sum = pref;
      for (int kk = 1; kk < 200; ++kk) {
        term *= t / (double(kk) * double(l + kk));
        sum += term;
        if (term <= 1e-18 * sum) break;
      }
      sI[l][tid] = sum;
      pref *= 0.5 * xr / double(l + 1);
    }
  }

  const int64_t J = ring_step(ring_of(g, pan), slot - win);
  const int F = nsub * Q;
  const int64_t fbase = J * F;

  double acc[Q], agx[Q], agy[Q];
#pragma unroll
  for (int m = 0; m < Q; ++m) acc[m] = agx[m] = agy[m] = 0.0;

  for (int sub = 0; sub < nsub; ++sub) {
    for (int gq = 0; gq < Q; ++gq) {
      const int64_t fo = fbase + sub * Q + gq;
      const double yfx = fx[fo], yfy = fy[fo];
      const double nfx = fwx[fo], nfy = fwy[fo];   // weight x normal
      // eta x weight (the normal is a unit vector) for the single layer's coefficients
      const double ew = g.eta > 0.0 ? g.eta * sqrt(nfx * nfx + nfy * nfy) : 0.0;

      double cval = 0.0, gr = 0.0, gt = 0.0;
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const double side = sd == 0 ? 1.0 : -1.0;
        const double dx = yfx - (xi + side * r * nxi);
        const double dy = yfy - (yi + side * r * nyi);
        const double rf2 = dx * dx + dy * dy;
        const double irf = rsqrt64(rf2);
        const double rf = rf2 * irf;
        const double rhx = dx * irf, rhy = dy * irf;
        const double txh = -side * nxi, tyh = -side * nyi;  // direction of x_i - c
        const double cosD = rhx * txh + rhy * tyh;
        const double sinD = txh * rhy - tyh * rhx;
        const double rn = rhx * nfx + rhy * nfy;
        const double tn = -rhy * nfx + rhx * nfy;
        const double z = kap * rf;
        double K0, K1;
        k01_64(z, K0, K1, g.tab);
        const double iz2 = 2.0 * rcp64(z);
        const double a0 = -kap * K1 * rn + ew * K0;
        double sum = sI[0][tid] * a0;
        double g_r = a0 * kap * sI[1][tid];
        double g_t = 0.0;
        double Km = K0, Kc = K1, cl = cosD, sl = sinD;
        for (int l = 1; l <= p; ++l) {
          const double Kp = fma(l * iz2, Kc, Km);
          const double a = -0.5 * kap * (Km + Kp) * rn + ew * Kc;
          const double b = Kc * tn * irf;
          const double Pl = a * cl - l * b * sl;
          const double Il = sI[l][tid];
          sum += 2.0 * Il * Pl;
          if (sd == 0) {
            const double Ql = a * sl + l * b * cl;
            const double Ild = 0.5 * (sI[l - 1][tid] + sI[l + 1][tid]);
            g_r += 2.0 * Pl * kap * Ild;
            g_t += 2.0 * Ql * l * Il * ir;
          }
          const double cn = cl * cosD - sl * sinD;
          sl = sl * cosD + cl * sinD;
          cl = cn;
          Km = Kc;
          Kc = Kp;
        }
        cval += 0.5 * sum;
        if (sd == 0) {
          gr = g_r;
          gt = g_t;
        }
      }
      // rhat_x = -nu_i, thhat_x = (nu_iy, -nu_ix) for the exterior centre
      const double w2 = 1.0 / (2.0 * PI);
      const double cv = w2 * cval;
      const double gvx = w2 * (-gr * nxi + gt * nyi);
      const double gvy = w2 * (-gr * nyi - gt * nxi);
      const double* Lr = L + (sub * Q + gq) * Q;
#pragma unroll
      for (int m = 0; m < Q; ++m) {
        const double lm = Lr[m];
        acc[m] = fma(cv, lm, acc[m]);
        agx[m] = fma(gvx, lm, agx[m]);
        agy[m] = fma(gvy, lm, agy[m]);
      }
    }
  }

  const int64_t jb = J * Q;
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    const int64_t j = jb + m;
    if (j == i) {
      acc[m] += 0.5;
    } else {
      double s, sgx, sgy;
      smooth_pair(g, xi, yi, j, s, sgx, sgy);
      acc[m] -= s;
      agx[m] -= sgx;
      agy[m] -= sgy;
    }
  }
  if (!active) return;
  const int64_t N = g.N;
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    const int64_t o = ((int64_t)slot * Q + m) * N + i;
    W[o] = acc[m];
    WGx[o] = agx[m];
    WGy[o] = agy[m];
  }
}

// Oversampled direct rows for the extra near panels of each target
// (nsub sub-panels, interpolated sigma), minus the plain far-field terms (both
// layers of the combined representation when g.eta > 0).
// vals[e*16 + m]; gvals[(e*2 + c)*16 + m].
__global__ void near_rows_kernel(GeomView g, Consts c, int nsub, const double* __restrict__ L,
                                 const int* __restrict__ row_ptr, const int* __restrict__ panels,
                                 double* __restrict__ vals, double* __restrict__ gvals) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  const double xi = g.x[i], yi = g.y[i];
  const double kap2 = g.kappa * g.kappa;
  const double cst = kap2 / (2.0 * PI);
  for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    const int J = panels[e];
    const int pid = panel_particle(g, J);
    const double* pp = g.pc + 5 * pid;
    double acc[Q], agx[Q], agy[Q];
    for (int m = 0; m < Q; ++m) acc[m] = agx[m] = agy[m] = 0.0;
    for (int sub = 0; sub < nsub; ++sub) {
      for (int gq = 0; gq < Q; ++gq) {
        const double xl = -1.0 + (2.0 * sub + c.xg[gq] + 1.0) / nsub;
        double dt;
        const double t = panel_param(g, J, xl, dt);
        double st, ct, sa, ca;
        sincos(t, &st, &ct);
        sincos(pp[2], &sa, &ca);
        const double ex = pp[3] * ct, ey = pp[4] * st;
        const double ddx = -pp[3] * st, ddy = pp[4] * ct;
        const double yfx = pp[0] + ca * ex - sa * ey;
        const double yfy = pp[1] + sa * ex + ca * ey;
        const double gx = ca * ddx - sa * ddy, gy = sa * ddx + ca * ddy;
        const double sp = sqrt(gx * gx + gy * gy);
        const double wf = (dt / nsub) * c.wg[gq] * sp;
        const double qx = wf * gy / sp, qy = -wf * gx / sp;
        const double dx = xi - yfx, dy = yi - yfy;
        const double r2 = dx * dx + dy * dy;
        double k0, k1z;
        k0_k1z_64(kap2 * r2, k0, k1z, g.tab);
        const double dq = dx * qx + dy * qy;
        const double ew = g.eta * wf;   // single layer of the combined representation
        const double v = cst * (k1z * dq + ew * k0 / kap2);
        const double b = dq * (k0 + 2.0 * k1z) * rcp64(r2) + ew * k1z;
        const double vx = cst * (k1z * qx - b * dx);
        const double vy = cst * (k1z * qy - b * dy);
        const double* Lr = L + (sub * Q + gq) * Q;
        for (int m = 0; m < Q; ++m) {
          acc[m] = fma(v, Lr[m], acc[m]);
          agx[m] = fma(vx, Lr[m], agx[m]);
          agy[m] = fma(vy, Lr[m], agy[m]);
        }
      }
    }
    for (int m = 0; m < Q; ++m) {
      double s, sgx, sgy;
      smooth_pair(g, xi, yi, (int64_t)J * Q + m, s, sgx, sgy);
      vals[(int64_t)e * Q + m] = acc[m] - s;
      gvals[((int64_t)e * 2 + 0) * Q + m] = agx[m] - sgx;
      gvals[((int64_t)e * 2 + 1) * Q + m] = agy[m] - sgy;
    }
  }
}

void launch_qbx_build(const GeomView& g, int p, int win, int nsub, double radius, const double* L,
                      const double* fx, const double* fy, const double* fwx, const double* fwy,
                      double* W, double* WGx, double* WGy, hipStream_t s) {
  constexpr int BS = 64;
  dim3 grid((unsigned)((g.N + BS - 1) / BS), (unsigned)(2 * win + 1));
  qbx_build_kernel<BS><<<grid, BS, 0, s>>>(g, p, win, nsub, radius, L, fx, fy, fwx, fwy, W, WGx,
                                           WGy);
  YQ_HIP(hipGetLastError());
}

void launch_near_rows(const GeomView& g, const Consts& c, int nsub, const double* L,
                      const int* row_ptr, const int* panels, double* vals, double* gvals,
                      hipStream_t s) {
  near_rows_kernel<<<(unsigned)((g.N + 127) / 128), 128, 0, s>>>(g, c, nsub, L, row_ptr, panels,
                                                                 vals, gvals);
  YQ_HIP(hipGetLastError());
}

}  // namespace yq
