// Inner loops of the far field and of the correction apply, shared by the
// single-problem kernels (farfield.hip) and the fused batch kernels
// (batch.hip) so that a configuration gives bit-identical sums either way.
#pragma once

#include "bessel.h"
#include "common.h"

namespace yq {

// acc += sum over the staged tile of K1(z)/z ((x_i - y_j) . q_j), FP64.
__device__ __forceinline__ double far64_tile(double xi, double yi, const double2* sxy,
                                             const double2* sq, int nb, double kap2,
                                             const double* __restrict__ tab, double acc) {
  for (int k = 0; k < nb; ++k) {
    const double2 p = sxy[k];
    const double2 q = sq[k];
    const double dx = xi - p.x, dy = yi - p.y;
    const double r2 = fma(dx, dx, dy * dy);
    const double v = k1z_64(kap2 * r2, tab) * fma(dx, q.x, dy * q.y);
    acc += r2 > 0.0 ? v : 0.0;
  }
  return acc;
}

// ---- FP64 far field: tile classes -------------------------------------------------------
//
// The smallest z of a (target group, source tile) pair, from their bounding
// circles, picks the evaluation of all its pairs: z >= 8 and z >= 4 take short
// fits of h_n (s <= 1/4 and 1/2), z >= 2 the full large-argument fit, and only
// pairs whose z may be smaller (the self pair included) take the general form
// with both branches.  The class is the same for every lane of a wavefront.
constexpr int C64_GENERAL = 0, C64_Z2 = 1, C64_Z4 = 2, C64_Z8 = 3;

__device__ __forceinline__ int far64_class(const double4* grp, const double4* tile, int64_t g,
                                           int64_t t, double kappa);

template <int NC, int H1>
__device__ __forceinline__ double far64_far_tile(double xi, double yi, const double2* sxy,
                                                 const double2* sq, int nb, double kap2,
                                                 const double* __restrict__ tab, double acc) {
  for (int k = 0; k < nb; ++k) {
    const double2 p = sxy[k];
    const double2 q = sq[k];
    const double dx = xi - p.x, dy = yi - p.y;
    const double r2 = fma(dx, dx, dy * dy);
    acc += k1z_64_large<NC, H1>(kap2 * r2, tab) * fma(dx, q.x, dy * q.y);
  }
  return acc;
}

__device__ __forceinline__ double far64_class_tile(int cls, double xi, double yi,
                                                   const double2* sxy, const double2* sq, int nb,
                                                   double kap2, const double* __restrict__ tab,
                                                   double acc) {
  switch (cls) {
    case C64_Z8: return far64_far_tile<12, T_H1_Z8>(xi, yi, sxy, sq, nb, kap2, tab, acc);
    case C64_Z4: return far64_far_tile<16, T_H1_Z4>(xi, yi, sxy, sq, nb, kap2, tab, acc);
    case C64_Z2: return far64_far_tile<21, T_H1>(xi, yi, sxy, sq, nb, kap2, tab, acc);
    default: return far64_tile(xi, yi, sxy, sq, nb, kap2, tab, acc);
  }
}

// FP32 over an LDS-staged tile (FMM neighbour interactions); positions stay
// FP64 and the difference is rounded to FP32.
__device__ __forceinline__ float far32_tile(double xi, double yi, const double2* sxy,
                                           const float2* sq, int nb, float kap2, float acc) {
#pragma unroll 4
  for (int k = 0; k < nb; ++k) {
    const double2 p = sxy[k];
    const float2 q = sq[k];
    const float dx = (float)(xi - p.x), dy = (float)(yi - p.y);
    const float z2 = fmaxf(kap2 * fmaf(dx, dx, dy * dy), 1e-30f);
    acc = fmaf(k1z_32(z2), fmaf(dx, q.x, dy * q.y), acc);
  }
  return acc;
}

// ---- FP32 far field ----------------------------------------------------------------------
//
// Sources are visited in tiles of 256 consecutive nodes, targets in groups of
// 64 (one wavefront); each has a bounding circle computed once per geometry.
// A (group, tile) pair is "far" when kappa times the gap between the circles is
// at least 2, so every pair in it has z >= 2: those pairs take a branch-free
// path in coordinates scaled by kappa log2(e) and taken relative to the tile
// centre (no FP64 arithmetic per pair).  Other pairs take the general path:
// FP64 differences rounded to FP32 (adjacent nodes stay accurate) and both
// branches of K1(z)/z.  Sources are packed per matvec into
// (rel x, rel y, q'x, q'y), q' = w nu sigma sqrt(log2 e) / kappa, and read
// through scalar loads: every lane of a wavefront needs the same source.


// Far pairs: with D = s (x_i - y_j), Z2 = |D|^2 = (z log2 e)^2, Y = 1/sqrt(Z2),
// K1(z)/z ((x_i - y_j) . q) = 2^-Z Z^-3/2 h1(2 log2(e) Y) (D . q').  H is the fit
// of h1 for the tile's range of z (z >= 2, 4 or 8), as a polynomial in Y.  The
// factor 2^-Z Z^-3/2 is one exp2 of -(Z + 1.5 log2 Z): its rounding adds little to
// that of -Z itself, which already sets the factor's relative error.
template <int NH, const float (&H)[NH]>
__device__ __forceinline__ float far32_pair(float tx, float ty, float4 p, float acc) {
  const float dx = tx - p.x, dy = ty - p.y;
  const float z2 = fmaf(dx, dx, dy * dy);
  const float yv = __builtin_amdgcn_rsqf(z2);
  const float z = z2 * yv;
  const float e = __builtin_amdgcn_exp2f(fmaf(-1.5f, __builtin_amdgcn_logf(z), -z));
  const float h = horner(H, yv);
  return fmaf(e * h, fmaf(dx, p.z, dy * p.w), acc);
}

__device__ __forceinline__ float4 ld_rec(kptr<float> p) {
  return make_float4(p[0], p[1], p[2], p[3]);
}

// sp: the tile's records as 4 floats each; nb a multiple of 16 (panels hold 16
// nodes).  The next 4 records are loaded (scalar) before the current 4 are used.
template <int NH, const float (&H)[NH]>
__device__ __forceinline__ float far32_far_tile(float tx, float ty, kptr<float> sp, int nb,
                                                float acc) {
  float4 a0 = ld_rec(sp), a1 = ld_rec(sp + 4), a2 = ld_rec(sp + 8), a3 = ld_rec(sp + 12);
  for (int k = 0; k < nb; k += 4) {
    kptr<float> pn = sp + 4 * (k + 4 < nb ? k + 4 : k);
    const float4 b0 = ld_rec(pn), b1 = ld_rec(pn + 4), b2 = ld_rec(pn + 8), b3 = ld_rec(pn + 12);
    acc = far32_pair<NH, H>(tx, ty, a0, acc);
    acc = far32_pair<NH, H>(tx, ty, a1, acc);
    acc = far32_pair<NH, H>(tx, ty, a2, acc);
    acc = far32_pair<NH, H>(tx, ty, a3, acc);
    a0 = b0;
    a1 = b1;
    a2 = b2;
    a3 = b3;
  }
  return acc;
}

// General pairs (any z, including the self pair, whose z^2 is clamped away from
// 0 while (x_i - y_j) . q = 0).  Sums K1(z)/z ((x_i - y_j) . q') with unscaled
// differences.
__device__ __forceinline__ float far32_near_tile(double xi, double yi, kptr<double> sx,
                                                 kptr<double> sy, kptr<float> sp, int nb,
                                                 float kap2, float acc) {
  // four sources at a time; the next four are loaded (scalar) before these are used
  double ax[4], ay[4];
  float aqx[4], aqy[4];
  auto load = [&](int k, double* x, double* y, float* qx, float* qy) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = sx[k + u];
      y[u] = sy[k + u];
      qx[u] = sp[4 * (k + u) + 2];
      qy[u] = sp[4 * (k + u) + 3];
    }
  };
  load(0, ax, ay, aqx, aqy);
  for (int k = 0; k < nb; k += 4) {
    double bx[4], by[4];
    float bqx[4], bqy[4];
    load(k + 4 < nb ? k + 4 : k, bx, by, bqx, bqy);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float dx = (float)(xi - ax[u]), dy = (float)(yi - ay[u]);
      const float z2 = fmaxf(kap2 * fmaf(dx, dx, dy * dy), 1e-30f);
      acc = fmaf(k1z_32(z2), fmaf(dx, aqx[u], dy * aqy[u]), acc);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ax[u] = bx[u];
      ay[u] = by[u];
      aqx[u] = bqx[u];
      aqy[u] = bqy[u];
    }
  }
  return acc;
}

// Sum over sources [j0, j1) (j0 a multiple of 256, j1 - j0 a multiple of 16) for
// target i of target group g (wavefront-uniform), in the scaling of far64_tile.
// A source tile whose circle is far from the group's (kappa x gap >= 2) is one
// segment of the class of that gap; a tile with close pairs is split into its
// panels (16 sources), each classified by its own circle, so that only panels
// near the group take the general path.
__device__ __forceinline__ float far32_range(const Far32View& v, int64_t i, int64_t g,
                                             int64_t j0, int64_t j1) {
  const double xi = i < v.N ? v.x[i] : 0.0;
  const double yi = i < v.N ? v.y[i] : 0.0;
  kptr<double> gc = as_k((const double*)v.grp) + 4 * g;
  const double gx = gc[0], gy = gc[1], gr = gc[2];
  kptr<float> src = as_k((const float*)v.src);
  float accf = 0.0f, accn = 0.0f;
  int64_t jb = j0;
  while (jb < j1) {
    const int64_t t = jb / FT;
    kptr<double> tc = as_k((const double*)v.tile) + 4 * t;
    const double tcx = tc[0], tcy = tc[1];
    const int64_t te = min(j1, (t + 1) * FT);   // end of this tile within the range
    const double cx = gx - tcx, cy = gy - tcy;
    const double zt = v.kappa * (sqrt(cx * cx + cy * cy) - gr - tc[2]);
    if (zt >= v.zcut) {   // cutoff far field: every pair of the tile is beyond the cutoff
      jb = te;
      continue;
    }
    const float tx = (float)((xi - tcx) * v.s), ty = (float)((yi - tcy) * v.s);
    for (int64_t js = jb; js < te;) {
      double z;
      int len;
      if (zt >= 2.0) {
        z = zt;
        len = (int)(te - js);
      } else {
        kptr<double> pc = as_k((const double*)v.pan) + 4 * (js / Q);
        const double px = gx - pc[0], py = gy - pc[1];
        z = v.kappa * (sqrt(px * px + py * py) - gr - pc[2]);
        len = Q;
      }
      kptr<float> sp = src + 4 * js;
      if (z >= 8.0)
        accf = far32_far_tile<4, kH1Y_32_z8>(tx, ty, sp, len, accf);
      else if (z >= 4.0)
        accf = far32_far_tile<5, kH1Y_32_z4>(tx, ty, sp, len, accf);
      else if (z >= 2.0)
        accf = far32_far_tile<7, kH1Y_32>(tx, ty, sp, len, accf);
      else
        accn = far32_near_tile(xi, yi, as_k(v.x) + js, as_k(v.y) + js, sp, len, v.kap2, accn);
      js += len;
    }
    jb = te;
  }
  return fmaf(accn, v.nscale, accf);
}

// kappa x the gap between the bounding circles of target group g and source tile t
__device__ __forceinline__ double far64_zmin(const double4* grp, const double4* tile, int64_t g,
                                             int64_t t, double kappa) {
  kptr<double> gc = as_k((const double*)grp) + 4 * g;
  kptr<double> tc = as_k((const double*)tile) + 4 * t;
  const double cx = gc[0] - tc[0], cy = gc[1] - tc[1];
  return kappa * (sqrt(cx * cx + cy * cy) - gc[2] - tc[2]);
}

__device__ __forceinline__ int far64_class(const double4* grp, const double4* tile, int64_t g,
                                           int64_t t, double kappa) {
  const double zmin = far64_zmin(grp, tile, g, t, kappa);
  return zmin >= 8.0 ? C64_Z8 : zmin >= 4.0 ? C64_Z4 : zmin >= 2.0 ? C64_Z2 : C64_GENERAL;
}

// Gradient of the double layer over a staged source tile, accumulated into
// (ax, ay) in the scaling of far64_tile:
// (K1(z)/z) q - ((x-y).q) (x-y) (K0(z) + 2 K1(z)/z) / r^2, self pair skipped.
__device__ __forceinline__ void far_grad64_tile(double xi, double yi, const double2* sxy,
                                                const double2* sq, int nb, double kap2,
                                                const double* __restrict__ tab, double& ax,
                                                double& ay) {
  for (int k = 0; k < nb; ++k) {
    const double2 p = sxy[k];
    const double2 q = sq[k];
    const double dx = xi - p.x, dy = yi - p.y;
    const double r2 = fma(dx, dx, dy * dy);
    if (r2 > 0.0) {
      double k0, k1z;
      k0_k1z_64(kap2 * r2, k0, k1z, tab);
      const double dq = fma(dx, q.x, dy * q.y);
      const double b = dq * (k0 + 2.0 * k1z) * rcp64(r2);
      ax += k1z * q.x - b * dx;
      ay += k1z * q.y - b * dy;
    }
  }
}

// Gradient pairs of a tile whose z is at least 2 (4, 8): no self pair, large branch only.
template <int NC, int H0, int H1>
__device__ __forceinline__ void far_grad64_far_tile(double xi, double yi, const double2* sxy,
                                                    const double2* sq, int nb, double kap2,
                                                    const double* __restrict__ tab, double& ax,
                                                    double& ay) {
  for (int k = 0; k < nb; ++k) {
    const double2 p = sxy[k];
    const double2 q = sq[k];
    const double dx = xi - p.x, dy = yi - p.y;
    const double r2 = fma(dx, dx, dy * dy);
    double k0, k1z;
    k0_k1z_64_large<NC, H0, H1>(kap2 * r2, k0, k1z, tab);
    const double dq = fma(dx, q.x, dy * q.y);
    const double b = dq * (k0 + 2.0 * k1z) * rcp64(r2);
    ax += k1z * q.x - b * dx;
    ay += k1z * q.y - b * dy;
  }
}

__device__ __forceinline__ void far_grad64_class_tile(int cls, double xi, double yi,
                                                      const double2* sxy, const double2* sq,
                                                      int nb, double kap2,
                                                      const double* __restrict__ tab, double& ax,
                                                      double& ay) {
  switch (cls) {
    case C64_Z8:
      far_grad64_far_tile<12, T_H0_Z8, T_H1_Z8>(xi, yi, sxy, sq, nb, kap2, tab, ax, ay);
      break;
    case C64_Z4:
      far_grad64_far_tile<16, T_H0_Z4, T_H1_Z4>(xi, yi, sxy, sq, nb, kap2, tab, ax, ay);
      break;
    case C64_Z2:
      far_grad64_far_tile<21, T_H0, T_H1>(xi, yi, sxy, sq, nb, kap2, tab, ax, ay);
      break;
    default:
      far_grad64_tile(xi, yi, sxy, sq, nb, kap2, tab, ax, ay);
  }
}

// Double-layer value and gradient over a staged tile in one pass (the final
// refinement residual and the surface gradient of the same density):
// acc += K1(z)/z ((x-y).q) as far64_tile, (ax, ay) as far_grad64_tile.
template <int NC, int H0, int H1>
__device__ __forceinline__ void far_fused64_far_tile(double xi, double yi, const double2* sxy,
                                                     const double2* sq, int nb, double kap2,
                                                     const double* __restrict__ tab, double& acc,
                                                     double& ax, double& ay) {
  for (int k = 0; k < nb; ++k) {
    const double2 p = sxy[k];
    const double2 q = sq[k];
    const double dx = xi - p.x, dy = yi - p.y;
    const double r2 = fma(dx, dx, dy * dy);
    double k0, k1z;
    k0_k1z_64_large<NC, H0, H1>(kap2 * r2, k0, k1z, tab);
    const double dq = fma(dx, q.x, dy * q.y);
    acc += k1z * dq;
    const double b = dq * (k0 + 2.0 * k1z) * rcp64(r2);
    ax += k1z * q.x - b * dx;
    ay += k1z * q.y - b * dy;
  }
}

__device__ __forceinline__ void far_fused64_general_tile(double xi, double yi, const double2* sxy,
                                                         const double2* sq, int nb, double kap2,
                                                         const double* __restrict__ tab,
                                                         double& acc, double& ax, double& ay) {
  for (int k = 0; k < nb; ++k) {
    const double2 p = sxy[k];
    const double2 q = sq[k];
    const double dx = xi - p.x, dy = yi - p.y;
    const double r2 = fma(dx, dx, dy * dy);
    if (r2 > 0.0) {
      double k0, k1z;
      k0_k1z_64(kap2 * r2, k0, k1z, tab);
      const double dq = fma(dx, q.x, dy * q.y);
      acc += k1z * dq;
      const double b = dq * (k0 + 2.0 * k1z) * rcp64(r2);
      ax += k1z * q.x - b * dx;
      ay += k1z * q.y - b * dy;
    }
  }
}

__device__ __forceinline__ void far_fused64_class_tile(int cls, double xi, double yi,
                                                       const double2* sxy, const double2* sq,
                                                       int nb, double kap2,
                                                       const double* __restrict__ tab,
                                                       double& acc, double& ax, double& ay) {
  switch (cls) {
    case C64_Z8:
      far_fused64_far_tile<12, T_H0_Z8, T_H1_Z8>(xi, yi, sxy, sq, nb, kap2, tab, acc, ax, ay);
      break;
    case C64_Z4:
      far_fused64_far_tile<16, T_H0_Z4, T_H1_Z4>(xi, yi, sxy, sq, nb, kap2, tab, acc, ax, ay);
      break;
    case C64_Z2:
      far_fused64_far_tile<21, T_H0, T_H1>(xi, yi, sxy, sq, nb, kap2, tab, acc, ax, ay);
      break;
    default:
      far_fused64_general_tile(xi, yi, sxy, sq, nb, kap2, tab, acc, ax, ay);
  }
}

// Window + extra-near correction of target i (local index) for density sg.
template <class TW>
__device__ __forceinline__ double correction_row(int64_t i, int64_t N, int P, int win,
                                                 const TW* __restrict__ W,
                                                 const int* __restrict__ xrow,
                                                 const int* __restrict__ xpan,
                                                 const double* __restrict__ xvals,
                                                 const double* __restrict__ sigma) {
  const int64_t pan = i / Q;
  const int64_t pid = pan / P;
  const int k = (int)(pan % P);
  double corr = 0.0;
  for (int sl = 0; sl <= 2 * win; ++sl) {
    int kj = (k + sl - win) % P;
    if (kj < 0) kj += P;
    const double* sg = sigma + (pid * P + kj) * Q;
    const TW* wr = W + (int64_t)sl * Q * N + i;
#pragma unroll
    for (int m = 0; m < Q; ++m) corr = fma((double)wr[(int64_t)m * N], sg[m], corr);
  }
  if (xvals)
    for (int e = xrow[i]; e < xrow[i + 1]; ++e) {
      const double* sg = sigma + (int64_t)xpan[e] * Q;
      const double* vr = xvals + (int64_t)e * Q;
      for (int m = 0; m < Q; ++m) corr = fma(vr[m], sg[m], corr);
    }
  return corr;
}

}  // namespace yq
