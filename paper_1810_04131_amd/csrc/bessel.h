// Device modified Bessel functions K0, K1, K_l, I_l in FP64 and FP32.
//
// K0(z) and K1(z)/z are evaluated from the ascending series for z < 2 and
// from h_n(s) = sqrt(z) e^z K_n(z), s = 2/z, for z >= 2 (coefficients and their
// derivation in gen_bessel_tables.py).  Both are written as functions of
// z^2 so that the double-layer kernel, which needs K1(kappa r)/r, takes no
// square root on the small-argument branch.  Higher orders use the upward
// recurrence K_{l+1} = K_{l-1} + (2l/z) K_l (stable for K); I_l uses its
// ascending series.
#pragma once

#include <hip/hip_runtime.h>

#include "bessel_tables.h"
#include "common.h"

namespace yq {

// FP64 coefficient tables live in one small device buffer (build_tab64) that
// kernels receive as a pointer: the loads are uniform, so the compiler keeps
// the coefficients in scalar registers and every Horner step is a single FMA
// with a scalar operand.  (Literal 64-bit constants cannot be FMA operands
// and cost a vector move per use.)
constexpr int T_E = 0, T_F = 12, T_I0 = 24, T_P0 = 36, T_H0 = 48, T_H1 = 69, T_EX = 90,
              T_H0_Z8 = 104, T_H1_Z8 = 116, T_H0_Z4 = 128, T_H1_Z4 = 144, T_SIZE = 160;
static_assert(T_SIZE == T_SIZE_HOST, "table size");

// T + T_EX: e^-r on |r| <= ln2/2, the degree-11 interpolant at Chebyshev points
// (kEXP64, relative error about 2e-17)
inline void build_tab64(double* t) {
  for (int k = 0; k < 12; ++k) {
    t[T_E + k] = kE64[k];
    t[T_F + k] = kF64[k];
    t[T_I0 + k] = kI064[k];
    t[T_P0 + k] = kP064[k];
  }
  for (int k = 0; k < 21; ++k) {
    t[T_H0 + k] = kH0_64[k];
    t[T_H1 + k] = kH1_64[k];
  }
  for (int k = 0; k < 12; ++k) {
    t[T_H0_Z8 + k] = kH0_64_z8[k];
    t[T_H1_Z8 + k] = kH1_64_z8[k];
  }
  for (int k = 0; k < 16; ++k) {
    t[T_H0_Z4 + k] = kH0_64_z4[k];
    t[T_H1_Z4 + k] = kH1_64_z4[k];
  }
  for (int k = 0; k < 14; ++k) t[T_EX + k] = k < 12 ? kEXP64[k] : 0.0;
}

// r * x + c with the uniform coefficient c taken from a scalar register.  Written
// as a single VOP3 FMA: left to itself the compiler emits the two-address
// v_fmac_f64 form, which needs two extra moves per step to bring c into the
// destination register.  Register-only arithmetic, no memory access.
__device__ __forceinline__ double fma_sc(double r, double x, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(r), "v"(x), "s"(c));
  return d;
}

template <int N>
__device__ __forceinline__ double hornerT(const double* __restrict__ c, double x) {
  double r = c[N - 1];
#pragma unroll
  for (int k = N - 2; k >= 0; --k) r = fma_sc(r, x, c[k]);
  return r;
}

template <int N, class T>
__device__ __forceinline__ T horner(const T (&c)[N], T x) {
  T r = c[N - 1];
#pragma unroll
  for (int k = N - 2; k >= 0; --k) r = fma(r, x, c[k]);
  return r;
}

// 1/x to full double precision: hardware reciprocal estimate + two Newton steps.
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/sqrt(x) to full double precision: estimate + two Newton steps.
__device__ __forceinline__ double rsqrt64(double x) {
  double r = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  double e = fma(-h * r, r, 0.5);
  r = fma(r, e, r);
  e = fma(-h * r, r, 0.5);
  return fma(r, e, r);
}

// ---- FP64 ------------------------------------------------------------------------------

// e^-z for z >= 0: z = k ln2 + r (Cody-Waite split of ln2 into a 32-bit head
// and a tail, so k*ln2_hi is exact for |k| < 2^20), e^-z = 2^-k e^-r.
__device__ __forceinline__ double expm64(double z, const double* __restrict__ T) {
  const double k = rint(z * 1.4426950408889634074);
  double r = fma(-k, 6.93147180369123816490e-01, z);
  r = fma(-k, 1.90821492927058770002e-10, r);
  return ldexp(hornerT<12>(T + T_EX, r), -(int)k);
}

// Natural logarithm of a positive normal x, within about one ulp.  x = 2^e m with
// m in [1/sqrt 2, sqrt 2); f = m - 1 is exact and, with s = f / (2 + f),
//   log m = 2 atanh s = f - s (f - s^2 P(s^2)),  P(w) = sum_{k>=0} 2 w^k / (2k + 3),
// the Taylor series of atanh, here through w^10 (|s| <= 0.1716, so the first omitted
// term is below 1e-19 of the result).  e ln 2 is a 42-bit head of ln 2 (its product
// with |e| < 2^11 is exact) plus the tail.  About 30 instructions against the
// library's correctly rounded logarithm's 65.
__device__ __forceinline__ double log64(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);    // [1/2, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  const bool lo = m < 0.70710678118654752440;
  m = lo ? 2.0 * m : m;
  e = lo ? e - 1 : e;
  const double f = m - 1.0;
  const double s = f * rcp64(2.0 + f);
  const double w = s * s;
  double P = 2.0 / 23.0;
#pragma unroll
  for (int k = 9; k >= 0; --k) P = fma(P, w, 2.0 / (2 * k + 3));
  const double r = fma(-s, fma(-w, P, f), f);
  const double de = (double)e;
  return fma(de, 0x1.62e42fefa3800p-1, fma(de, 0x1.ef35793c76730p-45, r));
}

// K1(z)/z for z^2 = z2 < 4 (the ascending series).
__device__ __forceinline__ double k1z_64_small(double z2, const double* __restrict__ T) {
  double t = 0.25 * z2;
  double lt = log64(t);
  return 0.25 * rcp64(t) + 0.25 * (lt * hornerT<12>(T + T_E, t) - hornerT<12>(T + T_F, t));
}

// K1(z)/z for z^2 = z2.
__device__ __forceinline__ double k1z_64(double z2, const double* __restrict__ T) {
  if (z2 < 4.0) return k1z_64_small(z2, T);
  double y = rsqrt64(z2);  // 1/z
  double z = z2 * y;
  double q = rsqrt64(z);   // z^(-1/2)
  return hornerT<21>(T + T_H1, 2.0 * y) * expm64(z, T) * q * y;
}

// Large-argument forms for pairs whose z is known to be at least 2, 4 or 8: h_n
// from the degree-(NC - 1) fit stored at T + H0 / T + H1 (a fit for that range).
template <int NC, int H1>
__device__ __forceinline__ double k1z_64_large(double z2, const double* __restrict__ T) {
  double y = rsqrt64(z2);  // 1/z
  double z = z2 * y;
  double q = rsqrt64(z);   // z^(-1/2)
  return hornerT<NC>(T + H1, 2.0 * y) * expm64(z, T) * q * y;
}

template <int NC, int H0, int H1>
__device__ __forceinline__ void k0_k1z_64_large(double z2, double& k0, double& k1z,
                                                const double* __restrict__ T) {
  double y = rsqrt64(z2);
  double z = z2 * y;
  double q = rsqrt64(z);
  double e = expm64(z, T) * q;
  double s = 2.0 * y;
  k0 = hornerT<NC>(T + H0, s) * e;
  k1z = hornerT<NC>(T + H1, s) * e * y;
}

// K0(z) and K1(z)/z for z^2 = z2 < 4 (the ascending series).
__device__ __forceinline__ void k0_k1z_64_small(double z2, double& k0, double& k1z,
                                                const double* __restrict__ T) {
  double t = 0.25 * z2;
  double lt = log64(t);
  k0 = -0.5 * lt * hornerT<12>(T + T_I0, t) + hornerT<12>(T + T_P0, t);
  k1z = 0.25 * rcp64(t) + 0.25 * (lt * hornerT<12>(T + T_E, t) - hornerT<12>(T + T_F, t));
}

// K0(z) and K1(z)/z together for z^2 = z2.
__device__ __forceinline__ void k0_k1z_64(double z2, double& k0, double& k1z,
                                          const double* __restrict__ T) {
  if (z2 < 4.0) {
    k0_k1z_64_small(z2, k0, k1z, T);
    return;
  }
  double y = rsqrt64(z2);
  double z = z2 * y;
  double q = rsqrt64(z);
  double e = expm64(z, T) * q;
  double s = 2.0 * y;
  k0 = hornerT<21>(T + T_H0, s) * e;
  k1z = hornerT<21>(T + T_H1, s) * e * y;
}

// K0(z), K1(z) for z > 0 given z itself (no square / square-root round trip,
// which would cost a relative error of about z * eps through e^-z).
__device__ __forceinline__ void k01_64(double z, double& k0, double& k1,
                                       const double* __restrict__ T) {
  if (z < 2.0) {
    double k1z;
    k0_k1z_64(z * z, k0, k1z, T);
    k1 = k1z * z;
    return;
  }
  double y = rcp64(z);
  double e = expm64(z, T) * rsqrt64(z);
  double s = 2.0 * y;
  k0 = hornerT<21>(T + T_H0, s) * e;
  k1 = hornerT<21>(T + T_H1, s) * e;
}

// I_l(x), l = 0..lmax, by the ascending series (x >= 0, moderate).
__device__ inline void bessel_i_series64(double x, int lmax, double* I) {
  double t = 0.25 * x * x;
  double pref = 1.0;  // (x/2)^l / l!
  for (int l = 0; l <= lmax; ++l) {
    double term = pref, sum = pref;
    for (int k = 1; k < 200; ++k) {
      term *= t / (double(k) * double(l + k));
      sum += term;
      if (term <= 1e-18 * sum) break;
    }
    I[l] = sum;
    pref *= 0.5 * x / double(l + 1);
  }
}

// ---- FP32 ------------------------------------------------------------------------------

// K1(z)/z for z^2 = z2 (> 0, normal).  z < 2: the ascending series with the raw
// base-2 logarithm (log2 t folded into the coefficients); z >= 2: e^-z z^-3/2
// h1(2/z) with h1 as a degree-6 polynomial in 1/z.
// The two branches on their own (the small-z one for z < 2, the other for z >= 2).
__device__ __forceinline__ float k1z_32_small(float z2) {
  const float t = 0.25f * z2;
  const float l2 = __builtin_amdgcn_logf(t);
  return fmaf(0.25f, __builtin_amdgcn_rcpf(t), fmaf(l2, horner(kE2_32, t), -horner(kF4_32, t)));
}

__device__ __forceinline__ float k1z_32_large(float z2) {
  const float y = __builtin_amdgcn_rsqf(z2);
  const float z = z2 * y;
  const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * z);
  const float q = __builtin_amdgcn_rsqf(z);
  return (e * horner(kH1Z_32, y)) * (q * y);
}

__device__ __forceinline__ float k1z_32(float z2) {
  if (z2 < 4.0f) return k1z_32_small(z2);
  return k1z_32_large(z2);
}

__device__ __forceinline__ void k0_k1z_32(float z2, float& k0, float& k1z) {
  if (z2 < 4.0f) {
    float t = 0.25f * z2;
    float lt = __logf(t);
    k0 = -0.5f * lt * horner(kI032, t) + horner(kP032, t);
    k1z = 0.25f * __builtin_amdgcn_rcpf(t) + 0.25f * (lt * horner(kE32, t) - horner(kF32, t));
    return;
  }
  float y = __builtin_amdgcn_rsqf(z2);
  float z = z2 * y;
  float q = __builtin_amdgcn_rsqf(z);
  float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * z) * q;
  float s = 2.0f * y;
  k0 = horner(kH0_32, s) * e;
  k1z = horner(kH1_32, s) * e * y;
}

}  // namespace yq
