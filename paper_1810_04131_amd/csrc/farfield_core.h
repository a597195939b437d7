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

// FP32 version; positions stay FP64 and the difference is rounded to FP32.
__device__ __forceinline__ float far32_tile(double xi, double yi, const double2* sxy,
                                           const float2* sq, int nb, float kap2, float acc) {
  for (int k = 0; k < nb; ++k) {
    const double2 p = sxy[k];
    const float2 q = sq[k];
    const float dx = (float)(xi - p.x), dy = (float)(yi - p.y);
    const float z2 = fmaxf(kap2 * fmaf(dx, dx, dy * dy), 1e-30f);
    acc = fmaf(k1z_32(z2), fmaf(dx, q.x, dy * q.y), acc);
  }
  return acc;
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

// Window + extra-near correction of target i (local index) for density sg.
__device__ __forceinline__ double correction_row(int64_t i, int64_t N, int P, int win,
                                                 const double* __restrict__ W,
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
    const double* wr = W + (int64_t)sl * Q * N + i;
#pragma unroll
    for (int m = 0; m < Q; ++m) corr = fma(wr[(int64_t)m * N], sg[m], corr);
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
