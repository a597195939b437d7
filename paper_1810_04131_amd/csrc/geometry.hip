// Nodes, normals and weights, boundary labels, and near lists (with the
// geometry check) of the solve.  Particles are the ellipses of section 2.1;
// panels are the composite Gauss-Legendre panels of section 5.
#include <cmath>

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace yq {

// ---- host: Gauss-Legendre rule and Lagrange interpolation -----------------------------

// 16-point Gauss-Legendre nodes (ascending) and weights by Newton's method on
// P_16, evaluated with the three-term recurrence; P_16' from the standard
// derivative identity (1 - x^2) P_n' = n (P_{n-1} - x P_n).
void gauss_legendre16(double* x, double* w) {
  const int n = Q;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (p0 - z * p1) / (1.0 - z * z);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    // recompute the derivative at the converged root for the weight
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (p0 - z * p1) / (1.0 - z * z);
    x[n - 1 - i] = z;  // cos decreases with i: store ascending
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// L[f*q + m] = l_m(dst_f), the Lagrange basis of the q source nodes, in
// barycentric form l_m(x) = (b_m / (x - s_m)) / sum_j (b_j / (x - s_j)).
void lagrange_matrix(const double* src, int q, const double* dst, int nd, double* L) {
  std::vector<double> b(q);
  for (int m = 0; m < q; ++m) {
    double prod = 1.0;
    for (int j = 0; j < q; ++j)
      if (j != m) prod *= (src[m] - src[j]);
    b[m] = 1.0 / prod;
  }
  for (int f = 0; f < nd; ++f) {
    int hit = -1;
    for (int m = 0; m < q; ++m)
      if (dst[f] == src[m]) hit = m;
    if (hit >= 0) {
      for (int m = 0; m < q; ++m) L[f * q + m] = (m == hit) ? 1.0 : 0.0;
      continue;
    }
    double den = 0.0;
    for (int j = 0; j < q; ++j) den += b[j] / (dst[f] - src[j]);
    for (int m = 0; m < q; ++m) L[f * q + m] = (b[m] / (dst[f] - src[m])) / den;
  }
}

// Coordinates in the coarse panel's [-1, 1] of the nodes of nsub equal sub-panels.
void sub_panel_coords(const double* xg, int q, int nsub, double* xi) {
  for (int s = 0; s < nsub; ++s)
    for (int m = 0; m < q; ++m) xi[s * q + m] = -1.0 + (2.0 * s + (xg[m] + 1.0)) / nsub;
}

// ---- device ------------------------------------------------------------------------------

__device__ __forceinline__ void ellipse_point(const double* pp, double t, double& px, double& py,
                                              double& nxo, double& nyo, double& speed) {
  double st, ct, sa, ca;
  sincos(t, &st, &ct);
  sincos(pp[2], &sa, &ca);
  double A = pp[3], B = pp[4];
  double ex = A * ct, ey = B * st;
  double dx = -A * st, dy = B * ct;
  px = pp[0] + ca * ex - sa * ey;
  py = pp[1] + sa * ex + ca * ey;
  double gx = ca * dx - sa * dy, gy = sa * dx + ca * dy;
  speed = sqrt(gx * gx + gy * gy);
  nxo = gy / speed;
  nyo = -gx / speed;
}

__global__ void geometry_kernel(GeomView g, Consts c, double* __restrict__ x, double* __restrict__ y,
                                double* __restrict__ nx, double* __restrict__ ny,
                                double* __restrict__ w, double* __restrict__ wnx,
                                double* __restrict__ wny) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  int m = (int)(i % Q);
  int64_t pan = i / Q;
  int p = panel_particle(g, pan);
  double dt;
  double t = panel_param(g, pan, c.xg[m], dt);
  double px, py, nxo, nyo, sp;
  ellipse_point(g.pc + 5 * p, t, px, py, nxo, nyo, sp);
  double ww = dt * c.wg[m] * sp;
  x[i] = px;
  y[i] = py;
  nx[i] = nxo;
  ny[i] = nyo;
  w[i] = ww;
  wnx[i] = ww * nxo;
  wny[i] = ww * nyo;
}

// Panel arclength h (sum of its weights in node order) and a bounding circle
// (centre = node mean, radius = largest node distance, slightly inflated).
__global__ void panel_stats_kernel(GeomView g, double* __restrict__ h, double* __restrict__ pcx,
                                   double* __restrict__ pcy, double* __restrict__ pr) {
  int64_t J = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (J >= g.npan) return;
  const int64_t b = J * Q;
  double s = 0.0, mx = 0.0, my = 0.0;
  for (int m = 0; m < Q; ++m) {
    s += g.w[b + m];
    mx += g.x[b + m];
    my += g.y[b + m];
  }
  mx *= 1.0 / Q;
  my *= 1.0 / Q;
  double r2 = 0.0;
  for (int m = 0; m < Q; ++m) {
    double dx = g.x[b + m] - mx, dy = g.y[b + m] - my;
    r2 = fmax(r2, dx * dx + dy * dy);
  }
  h[J] = s;
  pcx[J] = mx;
  pcy[J] = my;
  pr[J] = sqrt(r2) * (1.0 + 1e-12) + 1e-300;
}

__global__ void label_kernel(GeomView g, int kind, double a, double b, double* __restrict__ f) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  int p = panel_particle(g, i / Q);
  const double* pp = g.pc + 5 * p;
  double sa, ca;
  sincos(pp[2], &sa, &ca);
  double dx = g.x[i] - pp[0], dy = g.y[i] - pp[1];
  double phi = atan2(ca * dy - sa * dx, ca * dx + sa * dy);
  double v;
  if (kind == YQ_LABEL_ARC)
    v = 0.5 * (tanh((phi + a) / b) - tanh((phi - a) / b));
  else
    v = 1.0 - pow(sin(0.5 * phi), a);
  f[i] = v;
}

// Inside test for ellipse q (implicit form in its frame).
__device__ __forceinline__ double ellipse_level(const double* pp, double x, double y) {
  double sa, ca;
  sincos(pp[2], &sa, &ca);
  double dx = x - pp[0], dy = y - pp[1];
  double u = ca * dx + sa * dy, v = -sa * dx + ca * dy;
  return (u / pp[3]) * (u / pp[3]) + (v / pp[4]) * (v / pp[4]);
}

// Flags a node that lies inside (or on) another particle.
__global__ void geom_check_kernel(GeomView g, const int* __restrict__ nb_ptr,
                                  const int* __restrict__ nb_idx, int* bad) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  int p = panel_particle(g, i / Q);
  double xi = g.x[i], yi = g.y[i];
  for (int e = nb_ptr[p]; e < nb_ptr[p + 1]; ++e) {
    int q = nb_idx[e];
    if (q == p) continue;
    if (ellipse_level(g.pc + 5 * q, xi, yi) <= 1.0) {
      atomicMax(bad, 1);
      return;
    }
  }
}

// Extra near panels of every target: panels outside its QBX window whose
// nearest node is closer than beta * h.  Pass 1 (offs == nullptr) counts,
// pass 2 writes the panel indices in ascending order.
__global__ void near_kernel(GeomView g, int win, double beta, const int* __restrict__ nb_ptr,
                            const int* __restrict__ nb_idx, const double* __restrict__ pcx,
                            const double* __restrict__ pcy, const double* __restrict__ pr,
                            int* __restrict__ count, int* __restrict__ list,
                            const int* __restrict__ offs) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  int64_t pan = i / Q;
  int p = panel_particle(g, pan);
  int64_t pfirst;
  int pcnt;
  particle_panels(g, p, pfirst, pcnt);
  int k = (int)(pan - pfirst);
  double xi = g.x[i], yi = g.y[i];
  int cnt = 0;
  int base = offs ? offs[i] : 0;
  for (int e = nb_ptr[p]; e < nb_ptr[p + 1]; ++e) {
    int q = nb_idx[e];
    int64_t qfirst;
    int qcnt;
    particle_panels(g, q, qfirst, qcnt);
    for (int kk = 0; kk < qcnt; ++kk) {
      if (q == p) {
        int dk = kk - k;
        if (dk < 0) dk = -dk;
        if (dk > qcnt - dk) dk = qcnt - dk;  // circular distance along the ring
        if (dk <= win) continue;
      }
      int64_t J = qfirst + kk;
      double bh = beta * g.panel_h[J];
      double dx = xi - pcx[J], dy = yi - pcy[J];
      double dc = sqrt(dx * dx + dy * dy) - pr[J];
      if (dc > bh * (1.0 + 1e-9)) continue;
      double d2 = 1e300;
      for (int m = 0; m < Q; ++m) {
        double ex = xi - g.x[J * Q + m], ey = yi - g.y[J * Q + m];
        d2 = fmin(d2, ex * ex + ey * ey);
      }
      if (d2 < bh * bh) {
        if (offs) list[base + cnt] = (int)J;
        ++cnt;
      }
    }
  }
  if (!offs) count[i] = cnt;
}

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

void launch_geometry(const GeomView& g, const Consts& c, double* x, double* y, double* nx,
                     double* ny, double* w, double* wnx, double* wny, hipStream_t s) {
  geometry_kernel<<<nblk(g.N, 256), 256, 0, s>>>(g, c, x, y, nx, ny, w, wnx, wny);
  YQ_HIP(hipGetLastError());
}

void launch_panel_stats(const GeomView& g, double* panel_h, double* pcx, double* pcy, double* pr,
                        hipStream_t s) {
  panel_stats_kernel<<<nblk(g.npan, 256), 256, 0, s>>>(g, panel_h, pcx, pcy, pr);
  YQ_HIP(hipGetLastError());
}

void launch_label(const GeomView& g, int kind, double a, double b, double* f, hipStream_t s) {
  label_kernel<<<nblk(g.N, 256), 256, 0, s>>>(g, kind, a, b, f);
  YQ_HIP(hipGetLastError());
}

void launch_geom_check(const GeomView& g, const int* nb_ptr, const int* nb_idx, int* bad,
                       hipStream_t s) {
  geom_check_kernel<<<nblk(g.N, 256), 256, 0, s>>>(g, nb_ptr, nb_idx, bad);
  YQ_HIP(hipGetLastError());
}

void launch_near_count(const GeomView& g, int win, double beta, const int* nb_ptr,
                       const int* nb_idx, const double* pcx, const double* pcy, const double* pr,
                       int* count, int* list, const int* offs, hipStream_t s) {
  near_kernel<<<nblk(g.N, 128), 128, 0, s>>>(g, win, beta, nb_ptr, nb_idx, pcx, pcy, pr, count,
                                             list, offs);
  YQ_HIP(hipGetLastError());
}

void launch_row_scan(const int* count, int64_t N, int* row, DevBuf<char>& tmp, hipStream_t s) {
  YQ_HIP(hipMemsetAsync(row, 0, sizeof(int), s));
  if (N == 0) return;
  size_t bytes = 0;
  YQ_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, bytes, count, row + 1, (int)N, s));
  tmp.fit(std::max<size_t>(bytes, 1));
  YQ_HIP(hipcub::DeviceScan::InclusiveSum(tmp.p, bytes, count, row + 1, (int)N, s));
}

}  // namespace yq
