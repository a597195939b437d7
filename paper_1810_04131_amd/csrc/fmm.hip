// Quadtree Yukawa FMM for the double-layer far field.
//
// Expansions follow Graf's addition theorem for the modified Bessel functions
// (the Yukawa case of section 5's eq. graf-addition).  With
//   g_n(z) = I_n(kappa|z|) e^{i n arg z}   (regular),
//   S_n(z) = K_n(kappa|z|) e^{i n arg z}   (singular),
// K0(kappa|x - y|) = sum_n g_{-n}(y - c) S_n(x - c) for |y - c| < |x - c|, and the
// double-layer source of strength q = w sigma at y with unit normal nu
// (complex nu = nu_x + i nu_y) gives, using
// (d_x + i d_y) g_m = kappa g_{m+1} and (d_x - i d_y) g_m = kappa g_{m-1},
//   P2M  M_n = (kappa / 4 pi) sum q [ conj(nu) g_{1-n}(y - c) + nu g_{-1-n}(y - c) ],
//   M2M  M_n(c) = sum_k M_k(c') g_{k-n}(c' - c),
//   M2L  L_m(t) = (-1)^m sum_n M_n(s) S_{n-m}(c_t - c_s),
//   L2L  L_m(c') = sum_n L_n(c) g_{n-m}(c' - c),
//   L2P  u(x) = sum_n L_n g_n(x - c),
// n, m = -p..p, with M_{-n} = conj(M_n), L_{-n} = conj(L_n) (real potential), so
// only n = 0..p is stored.  Quadtree over the bounding square, uniform down to the
// level where occupied boxes average leaf_max nodes and adaptive below it (a box
// over leaf_max is split further), so leaves sit on different levels and hold at
// most leaf_max nodes (quadtree.h); interaction lists are the children of the parent's
// neighbours that are not adjacent; a leaf interacts directly with every leaf
// whose ancestor at the coarser of the two levels is adjacent to its own (P2P
// uses the far-field kernels' pair formula, so the QBX correction still cancels
// the plain terms of window pairs).  Tree and lists are built on the host once
// per geometry; translation tables (per level, child position or offset) on the
// device.  The expansions of all levels live in one array each (Mall, Lall), so
// a leaf's coefficients are addressed by its box index there.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <type_traits>
#include <unordered_map>

#include <hipcub/hipcub.hpp>

#include "bessel.h"
#include "common.h"
#include "farfield_core.h"
#include "fmm.h"
#include "quadtree.h"

namespace yq {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmad(double2 a, double2 b, double2 c) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// 1/m for m = 1..kRecipN-1, correctly rounded, for the integer reciprocals of the
// Bessel series and recurrences below (a constant-memory lookup in place of a
// refined FP64 reciprocal).
constexpr int kRecipN = 512;
struct RecipTable {
  double v[kRecipN];
  constexpr RecipTable() : v() {
    for (int m = 1; m < kRecipN; ++m) v[m] = 1.0 / m;
  }
};
__constant__ RecipTable kRecip = RecipTable();
__device__ __forceinline__ double recip(int m) { return kRecip.v[m]; }

// I_k(x) for one order k by the ascending series, from pref = (x/2)^k / k! and
// t = x^2 / 4 (all terms positive; reciprocals instead of divisions).
__device__ __forceinline__ double iorder(double t, double pref, int k) {
  double term = pref, sum = pref;
  for (int j = 1; j < 400; ++j) {
    term *= t * (recip(j) * recip(k + j));
    sum += term;
    if (term <= 1e-17 * sum) break;
  }
  return sum;
}

// I_k(x), k = 0..n; I[k * stride].
__device__ inline void iseries(double x, int n, double* I, int stride) {
  const double t = 0.25 * x * x;
  double pref = 1.0;
  for (int k = 0; k <= n; ++k) {
    I[(int64_t)k * stride] = iorder(t, pref, k);
    pref *= 0.5 * x * recip(k + 1);
  }
}

// Orders up to this keep the scaled I_n of each lane in LDS (iscaled_col); above
// it the column would cut the leaf kernels' occupancy by more than the recurrence
// saves, and each I_n comes from its own series (iorder).
constexpr int kColMaxOrder = 24;

// Scaled modified Bessel functions of this lane, It_n = I_n(x) n! / (x/2)^n with
// t = x^2/4, for n = 0..nmax, into col[n * 64] (the lane's LDS column): the two
// highest orders by their ascending series, the others by the backward
// recurrence It_{n-1} = It_n + t It_{n+1} / (n (n+1)), which follows from
// I_{n-1} = I_{n+1} + (2n/x) I_n and adds positive terms only.
__device__ inline void iscaled_col(double t, int nmax, double* col) {
  auto ser = [t](int n) {
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 200; ++k) {
      term *= t * (recip(k) * recip(n + k));
      sum += term;
      if (term <= 1e-17 * sum) break;
    }
    return sum;
  };
  double hi = ser(nmax + 1), cur = ser(nmax);
  col[nmax * 64] = cur;
  for (int n = nmax; n >= 1; --n) {
    const double prev = fma(t * hi, recip(n) * recip(n + 1), cur);
    col[(n - 1) * 64] = prev;
    hi = cur;
    cur = prev;
  }
}

// It_n(x) = I_n(x) n! / (x/2)^n by its ascending series in t = x^2/4, for n = p
// and p + 1 together: term k of It_n's series is t^k / (k! (n+1)...(n+k)),
// both summed in one loop to a relative 1e-17.
__device__ __forceinline__ void iscaled_pair(double t, int p, double& ip, double& ip1) {
  double a = 1.0, b = 1.0, sa = 1.0, sb = 1.0;
  for (int k = 1; k < 200; ++k) {
    const double tk = t * recip(k);
    a *= tk * recip(p + k);
    b *= tk * recip(p + 1 + k);
    sa += a;
    sb += b;
    if (a <= 1e-17 * sa && b <= 1e-17 * sb) break;
  }
  ip = sa;
  ip1 = sb;
}

// The local expansion L_0..L_p of a box with centre (cx, cy) at (xi, yi):
//   u = L_0 I_0 + 2 Re sum_{n>=1} L_n I_n(x) e^{i n theta},  x = kappa rho,
// as 2 Re S - L_0 It_0 with S = sum_n L_n It_n z^n / n!, z = (x/2) e^{i theta}: the
// scaled It_n come down the recurrence of iscaled_col from the series of It_{p+1}
// and It_p, and S is summed by Horner's rule in the same descending order
// (registers only, no LDS column).  z = (kappa / 2)(dx + i dy) and t = |z|^2 need no
// square root or division.
__device__ __forceinline__ double l2p_value(double xi, double yi, double cx, double cy,
                                            double kappa, int p, const double2* __restrict__ lb) {
  const double dx = xi - cx, dy = yi - cy;
  const double hk = 0.5 * kappa;
  const double2 z = make_double2(hk * dx, hk * dy);
  const double t = fma(z.x, z.x, z.y * z.y);
  double cur, hi;
  iscaled_pair(t, p, cur, hi);
  const gptr<double> lg = as_g(reinterpret_cast<const double*>(lb));   // (re, im) pairs
  double2 R = make_double2(lg[2 * p] * cur, lg[2 * p + 1] * cur);
  for (int n = p; n >= 1; --n) {
    const double prev = fma(t * hi, recip(n) * recip(n + 1), cur);   // It_{n-1}
    const double2 Rz = cmul(R, z);
    const double2 L = make_double2(lg[2 * n - 2], lg[2 * n - 1]);
    R = make_double2(fma(L.x, prev, Rz.x * recip(n)), fma(L.y, prev, Rz.y * recip(n)));
    hi = cur;
    cur = prev;
  }
  return 2.0 * R.x - lg[0] * cur;
}

// Sum over the 64 lanes of a wave (fixed butterfly order: the same bits on every run).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---- translation tables ------------------------------------------------------------------

// One block per table; the threads share the 4p + 1 entries.
constexpr int TAB_BS = 128;

// tg[((l * 4 + pos) * (4p + 1)) + k + 2p] = g_k(c_child - c_parent), child level l >= 1
__global__ __launch_bounds__(TAB_BS) void tab_g_kernel(int p, double W, double kappa,
                                                       double2* __restrict__ tg) {
  __shared__ double I[2 * MAXP_FMM + 1];
  const int t = blockIdx.x;                 // l * 4 + pos
  const int l = t / 4, pos = t % 4;
  const int K = 4 * p + 1;
  double2* out = tg + (int64_t)t * K;
  if (l == 0) {
    for (int k = threadIdx.x; k < K; k += TAB_BS) out[k] = make_double2(0.0, 0.0);
    return;
  }
  const double w = W / (double)(1 << l);
  const double dx = (pos & 1 ? 0.5 : -0.5) * w, dy = (pos & 2 ? 0.5 : -0.5) * w;
  const double r = sqrt(dx * dx + dy * dy), ph = atan2(dy, dx);
  const double x = kappa * r, tq = 0.25 * x * x;
  for (int k = threadIdx.x; k <= 2 * p; k += TAB_BS) {
    double pref = 1.0;                      // (x/2)^k / k!, built as in iseries
    for (int j = 0; j < k; ++j) pref *= 0.5 * x * recip(j + 1);
    I[k] = iorder(tq, pref, k);
  }
  __syncthreads();
  for (int k = threadIdx.x - 2 * p; k <= 2 * p; k += TAB_BS) {
    double s, c;
    sincos(k * ph, &s, &c);
    const double v = I[k < 0 ? -k : k];
    out[k + 2 * p] = make_double2(v * c, v * s);
  }
}

// ts[((l * 49 + o) * (4p + 1)) + k + 2p] = S_k(c_t - c_s), offset o = (ox + 3) * 7 + (oy + 3)
// of the source box relative to the target box, levels l >= 2.
__global__ __launch_bounds__(TAB_BS) void tab_s_kernel(int p, double W, double kappa,
                                                       const double* __restrict__ tab,
                                                       double2* __restrict__ ts) {
  __shared__ double Kn[2 * MAXP_FMM + 1];
  const int t = blockIdx.x;                 // l * 49 + o
  const int l = t / 49, o = t % 49;
  const int K = 4 * p + 1;
  double2* out = ts + (int64_t)t * K;
  const int ox = o / 7 - 3, oy = o % 7 - 3;
  if (l < 2 || (abs(ox) <= 1 && abs(oy) <= 1)) {
    for (int k = threadIdx.x; k < K; k += TAB_BS) out[k] = make_double2(0.0, 0.0);
    return;
  }
  const double w = W / (double)(1 << l);
  const double dx = -ox * w, dy = -oy * w;
  const double r = sqrt(dx * dx + dy * dy), ph = atan2(dy, dx);
  const double z = kappa * r;
  if (threadIdx.x == 0) {
    // K_n by the upward recurrence (stable for K)
    double k0, k1;
    k01_64(z, k0, k1, tab);
    Kn[0] = k0;
    Kn[1] = k1;
    for (int n = 1; n < 2 * p; ++n) Kn[n + 1] = Kn[n - 1] + (2.0 * n / z) * Kn[n];
  }
  __syncthreads();
  for (int k = threadIdx.x - 2 * p; k <= 2 * p; k += TAB_BS) {
    double s, c;
    sincos(k * ph, &s, &c);
    const double v = Kn[k < 0 ? -k : k];
    out[k + 2 * p] = make_double2(v * c, v * s);
  }
}

// ---- per-application kernels -----------------------------------------------------------------

// Sorted node k's source strength w nu sigma (the kernels' q).
// ss (may be null): the density itself in sorted order (near-field cache passes)
__device__ __forceinline__ void gather_one(int64_t k, const int* __restrict__ perm,
                                           const double* __restrict__ sigma,
                                           const double* __restrict__ wnxs,
                                           const double* __restrict__ wnys, double* __restrict__ qx,
                                           double* __restrict__ qy, double* __restrict__ ss) {
  const double s = as_g(sigma)[as_g(perm)[k]];
  as_gm(qx)[k] = as_g(wnxs)[k] * s;
  as_gm(qy)[k] = as_g(wnys)[k] * s;
  if (ss) as_gm(ss)[k] = s;
}

__global__ void gather_kernel(int64_t N, const int* __restrict__ perm, const double* __restrict__ sigma,
                              const double* __restrict__ wnxs, const double* __restrict__ wnys,
                              double* __restrict__ qx, double* __restrict__ qy,
                              double* __restrict__ ss) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= N) return;
  gather_one(k, perm, sigma, wnxs, wnys, qx, qy, ss);
}

constexpr int FB = 64;

// One wave per leaf: multipole coefficients M_n, n = 0..p.  A lane takes one
// node at a time, rolls I_{n-1}, I_n, I_{n+1} and e^{i(n +- 1) phi} along n, and
// the wave sums each coefficient; lane n keeps M_n.  Leaf b's coefficients go to
// box gid[b] of M.
// itab: [(p + 2) * 64] doubles of LDS (scaled I_n, one column per lane) when use_col.
// COEF: instead of the sums, write each node's terms for unit density (qx, qy = the
// nodes' w nu) times kappa / 4 pi to coef[k 2 (p + 1) + 2 n + (re, im)] (FP32), the
// P2M coefficients of the cached pass.
template <bool COEF = false>
__device__ __forceinline__ void p2m_leaf(int b, int p, int use_col, double kappa,
                                         const int* __restrict__ ls, const int* __restrict__ lc,
                                         const int* __restrict__ gid,
                                         const double* __restrict__ ccx,
                                         const double* __restrict__ ccy,
                                         const double* __restrict__ xs,
                                         const double* __restrict__ ys,
                                         const double* __restrict__ qx,
                                         const double* __restrict__ qy, double2* __restrict__ M,
                                         double* itab, float* __restrict__ coef = nullptr) {
  const int lane = threadIdx.x;
  const int s0 = as_k(ls)[b], cnt = as_k(lc)[b];
  const double cx = as_k(ccx)[b], cy = as_k(ccy)[b];
  double* col = itab + lane;
  double2 mine = make_double2(0.0, 0.0);
  for (int r0 = 0; r0 < cnt; r0 += 64) {
    const int j = r0 + lane;
    double dx = 0.0, dy = 0.0;
    double2 Q = make_double2(0.0, 0.0);
    if (j < cnt) {
      dx = as_g(xs)[s0 + j] - cx;
      dy = as_g(ys)[s0 + j] - cy;
      Q = make_double2(as_g(qx)[s0 + j], as_g(qy)[s0 + j]);
    }
    const double rho = sqrt(dx * dx + dy * dy);
    const double x = kappa * rho, t = 0.25 * x * x, hx = 0.5 * x;
    const double2 e1 = rho > 0.0 ? make_double2(dx / rho, dy / rho) : make_double2(1.0, 0.0);
    const double2 Qc = cconj(Q);
    if (use_col) iscaled_col(t, p + 1, col);
    double pref = hx;                               // (x/2)^{n+1} / (n+1)!
    double Im = 0.0, I0 = use_col ? col[0] : iorder(t, 1.0, 0);
    double Ip = use_col ? pref * col[64] : iorder(t, pref, 1);
    double2 Em = cconj(e1), Ep = e1;                // e^{i(n-1)phi}, e^{i(n+1)phi}
    for (int n = 0; n <= p; ++n) {
      const double2 gm = n == 0 ? make_double2(Ip * e1.x, Ip * e1.y)     // g_1
                                : make_double2(Im * Em.x, -Im * Em.y);   // conj(g_{n-1})
      const double2 gp = make_double2(Ip * Ep.x, -Ip * Ep.y);            // conj(g_{n+1})
      double2 c = cmul(Qc, gm);
      c = cmad(Q, gp, c);
      if (COEF) {
        if (j < cnt) {
          const double sc = kappa / (4.0 * PI);
          const int64_t a = (int64_t)(s0 + j) * 2 * (p + 1) + 2 * n;
          as_gm(coef)[a] = (float)(c.x * sc);
          as_gm(coef)[a + 1] = (float)(c.y * sc);
        }
      } else {
        c.x = wave_sum(c.x);
        c.y = wave_sum(c.y);
        if (lane == n) {
          mine.x += c.x;
          mine.y += c.y;
        }
      }
      pref *= hx * recip(n + 2);
      Im = I0;
      I0 = Ip;
      Ip = n + 2 > p + 1 ? 0.0                                 // I_{p+2} is never used
                         : (use_col ? pref * col[(n + 2) * 64] : iorder(t, pref, n + 2));
      Em = (n == 0) ? make_double2(1.0, 0.0) : cmul(Em, e1);
      Ep = cmul(Ep, e1);
    }
  }
  if (!COEF && lane <= p) {
    const double sc = kappa / (4.0 * PI);
    M[(int64_t)gid[b] * (p + 1) + lane] = make_double2(mine.x * sc, mine.y * sc);
  }
}

// One halving step of the exchange that sums 2 H values over the lanes: a lane keeps
// the half of V[0, 2 H) that its lane bit H selects, sends the other half to the lane
// that differs in that bit and adds what it receives, into V[0, H).
template <int H>
__device__ __forceinline__ void halve_sum(double* V, int lane) {
  const bool up = (lane & H) != 0;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double keep = up ? V[H + i] : V[i];
    const double send = up ? V[i] : V[H + i];
    V[i] = keep + __shfl_xor(send, H, 64);
  }
}

// p2m_leaf for an order P with 2 (P + 1) <= 64 without a wave sum per coefficient:
// each lane adds the terms of its nodes for every n in registers (values
// v = 2 n + (re, im), zero from 2 (P + 1) on), then six halving steps (H = 32 .. 1)
// leave the sum of value l in lane l.  The terms use I_k(x) e^{i k phi} = It_k W_k with
// W_k = z^k / k!, z = (kappa / 2)(dx + i dy), and It_k down the recurrence of
// iscaled_col from the series of It_{P+1}, It_{P+2}: no square root or division.
template <int P>
__device__ __forceinline__ void p2m_leaf_halving(int b, double kappa, const int* __restrict__ ls,
                                                 const int* __restrict__ lc,
                                                 const int* __restrict__ gid,
                                                 const double* __restrict__ ccx,
                                                 const double* __restrict__ ccy,
                                                 const double* __restrict__ xs,
                                                 const double* __restrict__ ys,
                                                 const double* __restrict__ qx,
                                                 const double* __restrict__ qy,
                                                 double2* __restrict__ M) {
  static_assert(2 * (P + 1) <= 64, "one value per lane");
  const int lane = threadIdx.x % FB;
  const int s0 = as_k(ls)[b], cnt = as_k(lc)[b];
  const double cx = as_k(ccx)[b], cy = as_k(ccy)[b];
  const double hk = 0.5 * kappa;
  double V[64];
#pragma unroll
  for (int v = 0; v < 64; ++v) V[v] = 0.0;
  for (int r0 = 0; r0 < cnt; r0 += FB) {
    const int j = r0 + lane;
    double dx = 0.0, dy = 0.0;
    double2 Q = make_double2(0.0, 0.0);
    if (j < cnt) {
      dx = as_g(xs)[s0 + j] - cx;
      dy = as_g(ys)[s0 + j] - cy;
      Q = make_double2(as_g(qx)[s0 + j], as_g(qy)[s0 + j]);
    }
    const double2 z = make_double2(hk * dx, hk * dy);
    const double t = fma(z.x, z.x, z.y * z.y);
    double It[P + 2], top;
    iscaled_pair(t, P + 1, It[P + 1], top);
    It[P] = fma(t * top, recip(P + 1) * recip(P + 2), It[P + 1]);
#pragma unroll
    for (int n = P; n >= 1; --n) It[n - 1] = fma(t * It[n + 1], recip(n) * recip(n + 1), It[n]);
    const double2 Qc = cconj(Q);
    double2 Wm = make_double2(0.0, 0.0), W0 = make_double2(1.0, 0.0), Wp = z;   // W_{n-1,n,n+1}
#pragma unroll
    for (int n = 0; n <= P; ++n) {
      const double2 gp = make_double2(It[n + 1] * Wp.x, -It[n + 1] * Wp.y);   // conj(g_{n+1})
      const double2 gm = n == 0 ? make_double2(It[1] * Wp.x, It[1] * Wp.y)   // g_1
                                : make_double2(It[n - 1] * Wm.x, -It[n - 1] * Wm.y);
      const double2 c = cmad(Q, gp, cmul(Qc, gm));
      V[2 * n] += c.x;
      V[2 * n + 1] += c.y;
      Wm = W0;
      W0 = Wp;
      const double2 zw = cmul(Wp, z);
      Wp = make_double2(zw.x * recip(n + 2), zw.y * recip(n + 2));
    }
  }
  halve_sum<32>(V, lane);
  halve_sum<16>(V, lane);
  halve_sum<8>(V, lane);
  halve_sum<4>(V, lane);
  halve_sum<2>(V, lane);
  halve_sum<1>(V, lane);
  if (lane < 2 * (P + 1))
    as_gm(reinterpret_cast<double*>(M))[(int64_t)as_k(gid)[b] * 2 * (P + 1) + lane] =
        V[0] * (kappa / (4.0 * PI));
}

// p2m_leaf, by p2m_leaf_halving for the orders it is instantiated for.
__device__ __forceinline__ void p2m_leaf_any(int b, int p, int use_col, double kappa,
                                             const int* __restrict__ ls, const int* __restrict__ lc,
                                             const int* __restrict__ gid,
                                             const double* __restrict__ ccx,
                                             const double* __restrict__ ccy,
                                             const double* __restrict__ xs,
                                             const double* __restrict__ ys,
                                             const double* __restrict__ qx,
                                             const double* __restrict__ qy,
                                             double2* __restrict__ M, double* itab) {
  if (p == 31)
    p2m_leaf_halving<31>(b, kappa, ls, lc, gid, ccx, ccy, xs, ys, qx, qy, M);
  else if (p == 20)
    p2m_leaf_halving<20>(b, kappa, ls, lc, gid, ccx, ccy, xs, ys, qx, qy, M);
  else if (p == 15)
    p2m_leaf_halving<15>(b, kappa, ls, lc, gid, ccx, ccy, xs, ys, qx, qy, M);
  else
    p2m_leaf(b, p, use_col, kappa, ls, lc, gid, ccx, ccy, xs, ys, qx, qy, M, itab);
}

// M_n of leaf b from the P2M coefficients and the sorted densities: one wave, lane m
// < 2 (p + 1) sums component m over the leaf's nodes in order (FP32 products and sums,
// the inner operator's precision).
__device__ __forceinline__ void p2m_cached_leaf(int b, int p, const int* __restrict__ ls,
                                                const int* __restrict__ lc,
                                                const int* __restrict__ gid,
                                                const float* __restrict__ coef,
                                                const double* __restrict__ ssd,
                                                double2* __restrict__ M) {
  constexpr int CB = 8;
  const int lane = threadIdx.x % FB;
  const int s0 = as_k(ls)[b], cnt = as_k(lc)[b];
  const int R = 2 * (p + 1);
  const int m = lane < R ? lane : 0;
  const gptr<float> cb = as_g(coef + (int64_t)s0 * R + m);
  float acc = 0.0f;
  for (int j0 = 0; j0 < cnt; j0 += CB) {
    float c[CB], sv[CB];
#pragma unroll
    for (int v = 0; v < CB; ++v) {
      const int jc = min(j0 + v, cnt - 1);
      c[v] = cb[(int64_t)jc * R];
      sv[v] = (float)as_k(ssd)[s0 + jc];
    }
#pragma unroll
    for (int v = 0; v < CB; ++v) acc = fmaf(j0 + v < cnt ? c[v] : 0.0f, sv[v], acc);
  }
  if (lane < R) as_gm(reinterpret_cast<double*>(M))[(int64_t)as_k(gid)[b] * R + lane] = (double)acc;
}

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2v __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// p2m_cached_leaf for one wavefront of a multi-wave block.  The leaf's coefficients
// are one contiguous block of cnt R floats (R = 2 (p + 1)); lane l reads its float4
// chunks l, l + 64, ..., so when R divides 256 (and 4 divides R) the lane's four
// components m = 4 l mod R, ..., m + 3 stay fixed while its node advances by 256 / R
// per load.  All of a leaf's loads are issued before their first use; lanes with the
// same m (l mod R / 4) are summed by cross-lane exchanges.  Other orders take
// p2m_cached_leaf's lane-per-component loop.
__device__ __forceinline__ void p2m_cached_wave(int b, int p, const int* __restrict__ ls,
                                                const int* __restrict__ lc,
                                                const int* __restrict__ gid,
                                                const float* __restrict__ coef,
                                                const double* __restrict__ ssd,
                                                double2* __restrict__ M) {
  const int R = 2 * (p + 1);
  if (R % 4 != 0 || 256 % R != 0) {
    p2m_cached_leaf(b, p, ls, lc, gid, coef, ssd, M);
    return;
  }
  constexpr int U = 8;
  const int lane = threadIdx.x % FB;
  const int s0 = as_k(ls)[b], cnt = as_k(lc)[b];
  const int npl = 256 / R;                  // nodes per wave load
  const int jl = (4 * lane) / R, m = (4 * lane) % R;
  const int nld = (cnt + npl - 1) / npl;    // wave loads of the leaf
  const gptr<f32x4> cb = as_g(reinterpret_cast<const f32x4*>(coef + (int64_t)s0 * R));
  const gptr<double> sb = as_g(ssd + s0);
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < nld; k0 += U) {
    f32x4 c[U];
    double sv[U];
#pragma unroll
    for (int v = 0; v < U; ++v) {
      // past the leaf's last node: re-read that node (in bounds), weight zero below
      const int j = min((k0 + v) * npl + jl, cnt - 1);
      c[v] = cb[(j * R + m) >> 2];
      sv[v] = sb[j];
    }
#pragma unroll
    for (int v = 0; v < U; ++v) {
      const float w = (k0 + v) * npl + jl < cnt ? (float)sv[v] : 0.0f;
      acc.x = fmaf(c[v].x, w, acc.x);
      acc.y = fmaf(c[v].y, w, acc.y);
      acc.z = fmaf(c[v].z, w, acc.z);
      acc.w = fmaf(c[v].w, w, acc.w);
    }
  }
  for (int off = R / 4; off < FB; off *= 2) {
    acc.x += __shfl_xor(acc.x, off);
    acc.y += __shfl_xor(acc.y, off);
    acc.z += __shfl_xor(acc.z, off);
    acc.w += __shfl_xor(acc.w, off);
  }
  if (lane < R / 4) {
    const gmut<dbl2v> o = as_gm(reinterpret_cast<dbl2v*>(reinterpret_cast<double*>(M) +
                                                         (int64_t)as_k(gid)[b] * R + m));
    o[0] = dbl2v{(double)acc.x, (double)acc.y};
    o[1] = dbl2v{(double)acc.z, (double)acc.w};
  }
}

__global__ __launch_bounds__(64) void p2m_kernel(int p, int use_col, double kappa,
                                                 const int* __restrict__ ls,
                                                 const int* __restrict__ lc,
                                                 const int* __restrict__ gid,
                                                 const double* __restrict__ ccx,
                                                 const double* __restrict__ ccy,
                                                 const double* __restrict__ xs,
                                                 const double* __restrict__ ys,
                                                 const double* __restrict__ qx,
                                                 const double* __restrict__ qy,
                                                 double2* __restrict__ M,
                                                 const int* __restrict__ stop) {
  if (stop && *stop) return;   // a GMRES step queued after the stop
  extern __shared__ double itab[];
  p2m_leaf_any(blockIdx.x, p, use_col, kappa, ls, lc, gid, ccx, ccy, xs, ys, qx, qy, M, itab);
}

// M2M: parent level lp from children at level lp + 1 (table level lp + 1).
__global__ void m2m_kernel(int p, int nbox, const int* __restrict__ ch, const double2* __restrict__ Mc,
                           const double2* __restrict__ tgl, double2* __restrict__ Mp) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)nbox * (p + 1)) return;
  const int P = (int)(t / (p + 1)), n = (int)(t % (p + 1));
  const int K = 4 * p + 1;
  // a leaf keeps the coefficients of its own nodes (P2M)
  if (ch[4 * P] < 0 && ch[4 * P + 1] < 0 && ch[4 * P + 2] < 0 && ch[4 * P + 3] < 0) return;
  double2 sum = make_double2(0.0, 0.0);
  for (int pos = 0; pos < 4; ++pos) {
    const int c = ch[4 * P + pos];
    if (c < 0) continue;
    const double2* T = tgl + pos * K + 2 * p;
    const double2* m = Mc + (int64_t)c * (p + 1);
    for (int k = -p; k <= p; ++k) {
      const double2 mk = k >= 0 ? m[k] : cconj(m[-k]);
      sum = cmad(mk, T[k - n], sum);
    }
  }
  Mp[t] = sum;
}

// M2L at one level: L_m(t) = (-1)^m sum_s sum_n M_n(s) S_{n-m}(c_t - c_s).
__global__ void m2l_kernel(int p, int nbox, const int* __restrict__ ilp, const int* __restrict__ ils,
                           const int* __restrict__ ilo, const double2* __restrict__ M,
                           const double2* __restrict__ tsl, double2* __restrict__ L) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)nbox * (p + 1)) return;
  const int b = (int)(t / (p + 1)), m = (int)(t % (p + 1));
  const int K = 4 * p + 1;
  double2 sum = make_double2(0.0, 0.0);
  for (int e = ilp[b]; e < ilp[b + 1]; ++e) {
    const double2* T = tsl + ilo[e] * K + 2 * p;
    const double2* ms = M + (int64_t)ils[e] * (p + 1);
    for (int n = -p; n <= p; ++n) {
      const double2 mn = n >= 0 ? ms[n] : cconj(ms[-n]);
      sum = cmad(mn, T[n - m], sum);
    }
  }
  if (m & 1) sum = make_double2(-sum.x, -sum.y);
  L[t] = sum;
}

// ---- M2L as batched dense products on the matrix cores --------------------------------------
//
// With x = (Re M_0..Re M_p, Im M_0..Im M_p) and y likewise for L, one M2L term
// is y += A_o x, A_o a real 2(p+1) x 2(p+1) matrix per (level, offset) that
// carries (-1)^m and the M_{-n} = conj(M_n) fold (rows and columns padded to
// R, a multiple of 16).  A wave owns one 16 x 16 output tile: 16 rows of y
// for 16 consecutive target boxes of one level.  For every far offset it
// gathers the 16 source vectors (zero where a target has none there) and
// accumulates A_o B with v_mfma_f64_16x16x4f64 (FP64, so the FMM keeps its
// accuracy).  All levels go in one launch: their M2L terms are independent.

// Translation matrices in the operand order of the 16x16x4 product: lane =
// i + 16 kk holds A[16 rt + i][4 ks + kk].  Row order (packed = 0, the M2M and
// L2L matrices): for (level, slot, row tile rt, k step ks) the 64 values lane by
// lane, so that a wave's operand load is one coalesced row.  Lane order (packed =
// 1, the M2L matrices): for (level, slot, rt) the KS = R / 4 values of each lane
// in a row, [(rt * 64 + lane) * KS + ks], so that a lane loads its KS operands
// with a few wide loads.  A slot is an M2L offset (49 per level, table ts, sign
// (-1)^m) or a child position (4 per level, table tg, no sign).
__global__ void trans_amat_kernel(int nlev, int nslot, int p, int R, int alt_sign, int packed,
                                  const double2* __restrict__ tab, double* __restrict__ amat) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)R * R;        // values per (level, slot)
  if (t >= (int64_t)nlev * nslot * per) return;
  const int64_t lo = t / per;                // level * nslot + slot
  const int rem = (int)(t % per);
  int lane, rt, ks;
  if (packed) {
    const int KS = R / 4, q = rem / KS;
    ks = rem % KS;
    lane = q & 63;
    rt = q >> 6;
  } else {
    const int tile = rem >> 6;                           // tile = rt * (R / 4) + ks
    lane = rem & 63;
    rt = tile / (R / 4);
    ks = tile % (R / 4);
  }
  const int r = 16 * rt + (lane & 15), k = 4 * ks + (lane >> 4);
  const int P1 = p + 1;
  double v = 0.0;
  if (r < 2 * P1 && k < 2 * P1) {
    const double2* T = tab + lo * (4 * p + 1) + 2 * p;
    const int m = r < P1 ? r : r - P1;
    const int n = k < P1 ? k : k - P1;
    const double2 t1 = T[n - m];
    const double2 t2 = n > 0 ? T[-n - m] : make_double2(0.0, 0.0);
    if (r < P1)   // Re y_m
      v = k < P1 ? t1.x + t2.x : -t1.y + t2.y;
    else          // Im y_m
      v = k < P1 ? t1.y + t2.y : t1.x - t2.x;
    if (alt_sign && (m & 1)) v = -v;
  }
  amat[t] = v;
}

// Operands of one 16x16 result tile (A rows, source columns) for KS k steps.
template <int KS>
struct TileOps {
  double a[KS], b[KS];
};

// Loads the operands: A from its operand-ordered rows, B from the source box's
// coefficients (ms == nullptr: a zero column).
template <int KS>
__device__ __forceinline__ void tile_load(TileOps<KS>& op, const double* __restrict__ A,
                                          const double2* __restrict__ ms, int P1, int kk) {
  // (global loads: the pointers may come from the trees' descriptors)
  const gptr<double> Ag = as_g(A);
  const gptr<double> mg = as_g(reinterpret_cast<const double*>(ms));
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    op.a[ks] = Ag[ks * 64];
    const int k = 4 * ks + kk;
    double b = 0.0;
    if (ms != nullptr && k < 2 * P1) b = k < P1 ? mg[2 * k] : mg[2 * (k - P1) + 1];
    op.b[ks] = b;
  }
}

template <int KS>
__device__ __forceinline__ dbl4 tile_mfma(const TileOps<KS>& op, dbl4 acc) {
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(op.a[ks], op.b[ks], acc, 0, 0, 0);
  return acc;
}

// Writes (or adds) a result tile to box rows 16 rt .. 16 rt + 15 of y.
// FP64 16x16 result layout: lane l holds column l % 16, its register j row 4 j + l / 16.
template <bool ADD>
__device__ __forceinline__ void tile_store(double2* __restrict__ y, int rt, int kk, int P1, dbl4 acc) {
  const gmut<double> yg = as_gm(reinterpret_cast<double*>(y));   // (re, im) pairs
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r = rt * 16 + 4 * j + kk;
    const int a = r < P1 ? 2 * r : 2 * (r - P1) + 1;
    if (r < 2 * P1) yg[a] = ADD ? yg[a] + acc[j] : acc[j];
  }
}

// i-th of the 40 offsets (ox, oy) outside the 3 x 3 neighbourhood, as o = (ox+3) 7 + (oy+3).
__host__ __device__ __forceinline__ int far_offset(int i) {
  if (i < 14) return i;                                   // ox = -3, -2
  if (i < 26) {                                           // ox = -1, 0, 1: oy = -3, -2, 2, 3
    const int k = i - 14, c = k & 3;
    return (2 + (k >> 2)) * 7 + (c < 2 ? c : c + 3);
  }
  return i + 9;                                           // ox = 2, 3
}

// Scaled FP32 copy of the M2L matrices (the lane order of trans_amat_kernel with
// packed = 1): amat32 = A_mn / (s_m s_n), s = msc of the matrix's level.
__global__ void trans_amat32_kernel(int nlev, int p, int R, const double* __restrict__ amat,
                                    const double* __restrict__ msc, float* __restrict__ amat32) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)R * R;
  if (t >= (int64_t)nlev * 49 * per) return;
  const int l = (int)(t / (49 * per));
  const int rem = (int)(t % per);
  const int KS = R / 4, q = rem / KS, ks = rem % KS;
  const int lane = q & 63, rt = q >> 6;
  const int r = 16 * rt + (lane & 15), k = 4 * ks + (lane >> 4);
  const int P1 = p + 1;
  float v = 0.0f;
  if (r < 2 * P1 && k < 2 * P1) {
    const double* sc = msc + (int64_t)l * P1;
    v = (float)(amat[t] / (sc[r < P1 ? r : r - P1] * sc[k < P1 ? k : k - P1]));
  }
  amat32[t] = v;
}

// Multipole coefficients of the boxes [g0, g1) (levels >= 2) as the B operands of
// the M2L products: box g's row x = (Re M_0..Re M_p, Im M_0..Im M_p, zero padding
// to R) stored lane by lane, Mp[g R + kk KS + ks] = x[4 ks + kk], so that the lane
// with kk = lane / 16 loads its KS operands with a few wide loads.  T = float
// scales by s_n of the box's level (msc) for the FP32 products.
template <typename T>
__device__ __forceinline__ void m2l_pack_one(int64_t t, int p, int R, int64_t g0,
                                             const M2LLevels& lv,
                                             const double2* __restrict__ Mall,
                                             const double* __restrict__ msc, T* __restrict__ Mp) {
  const int64_t g = g0 + t / R;
  const int e = (int)(t % R);
  const int KS = R / 4, kk = e / KS, ks = e % KS;
  const int k = 4 * ks + kk;
  const int P1 = p + 1;
  double v = 0.0;
  if (k < 2 * P1) {
    const int n = k < P1 ? k : k - P1;
    v = as_g(reinterpret_cast<const double*>(Mall))[2 * (g * P1 + n) + (k < P1 ? 0 : 1)];
    if (sizeof(T) == 4) {
      int l = 2;
      while (g >= lv.off[l + 1]) ++l;
      v *= as_g(msc)[(int64_t)l * P1 + n];
    }
  }
  as_gm(Mp)[g * R + e] = (T)v;
}

template <typename T>
__global__ void m2l_pack_kernel(int p, int R, int64_t g0, int64_t g1, M2LLevels lv,
                                const double2* __restrict__ Mall, const double* __restrict__ msc,
                                T* __restrict__ Mp) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (g1 - g0) * R) return;
  m2l_pack_one<T>(t, p, R, g0, lv, Mall, msc, Mp);
}

// M2L on the matrix cores: L_m(t) = sum over the 40 far offsets o of A_o M(source at
// o), for one 16-box tile of one level per block (4 waves; the offsets that hold a
// source of some box of the tile, known from the tile, go to the waves in turn).  A
// wave loads each of its offsets' 16 source vectors once (zero where a target has no
// source there) and multiplies them with all RT row tiles of A_o.  T = double: FP64 products
// (v_mfma_f64_16x16x4f64); T = float: FP32 products (v_mfma_f32_16x16x4f32) on the
// scaled operands M_n s_n and A_mn / (s_m s_n), which keeps entries O(1) inside the
// FP32 range, and L_m = (sum) s_m.  The four waves' tiles are summed in FP64 in a
// fixed order.  Result layouts: FP64, lane l holds column l % 16, register j row
// 4 j + l / 16; FP32, column l % 16, register j row 4 (l / 16) + j.
// One tile tl = (level, first position in the level's M2L order: the 16 boxes are
// ord[tl.y ..], their list rows ild[tl.y ..]; the union of their offset sets, bit i
// the i-th far offset, low and high halves); red: 3 RT 64 dbl4 of LDS.
template <typename T, int RT>
__device__ __forceinline__ void m2l_tile(int4 tl, int p, const M2LLevels& lv,
                                         const T* __restrict__ amat, const T* __restrict__ Mp,
                                         const double* __restrict__ msc, dbl4* red) {
  constexpr int R = RT * 16, KS = R / 4;
  constexpr bool F32 = sizeof(T) == 4;
  using acc_t = typename std::conditional<F32, f32x4, dbl4>::type;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int l = tl.x, nbox = lv.nbox[l];
  const gptr<int> ild = as_g(lv.ild[l]);
  const int P1 = p + 1;
  const int col = lane & 15, kk = lane >> 4;
  const int q = tl.y + col;                                 // position in the M2L order
  const int tb = q < nbox ? as_g(lv.ord[l])[q] : nbox;      // the box
  const gptr<T> Ml = as_g(Mp + lv.off[l] * R + kk * KS);
  const gptr<T> Al = as_g(amat + (int64_t)l * 49 * RT * 64 * KS + (int64_t)lane * KS);
  acc_t acc[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) acc[rt] = acc_t{0, 0, 0, 0};
  // the offsets used by the tile's boxes, dealt to the waves in turn
  uint64_t um = ((uint64_t)(uint32_t)tl.w << 32) | (uint32_t)tl.z;
  for (int r = 0; um != 0; ++r) {
    const int i = __builtin_ctzll(um);
    um &= um - 1;
    if ((r & 3) != wave) continue;
    const int o = far_offset(i);
    const int src = q < nbox ? ild[(int64_t)q * 49 + o] : -1;
    T b[KS];
    const gptr<T> mb = Ml + (int64_t)(src >= 0 ? src : 0) * R;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) b[ks] = src >= 0 ? mb[ks] : T(0);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const gptr<T> A = Al + ((int64_t)o * RT + rt) * 64 * KS;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if constexpr (F32)
          acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[ks], b[ks], acc[rt], 0, 0, 0);
        else
          acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[ks], b[ks], acc[rt], 0, 0, 0);
      }
    }
  }
  if (wave > 0)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
      red[((wave - 1) * RT + rt) * 64 + lane] =
          dbl4{(double)acc[rt][0], (double)acc[rt][1], (double)acc[rt][2], (double)acc[rt][3]};
  __syncthreads();
  if (wave != 0 || tb >= nbox) return;
  const gmut<double> y = as_gm(reinterpret_cast<double*>(lv.L[l] + (int64_t)tb * P1));
  const gptr<double> sc = as_g(F32 ? msc + (int64_t)l * P1 : msc);
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    dbl4 v = {(double)acc[rt][0], (double)acc[rt][1], (double)acc[rt][2], (double)acc[rt][3]};
    for (int w = 0; w < 3; ++w) v += red[(w * RT + rt) * 64 + lane];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = F32 ? rt * 16 + 4 * kk + j : rt * 16 + 4 * j + kk;
      if (r < P1)
        y[2 * r] = F32 ? v[j] * sc[r] : v[j];
      else if (r < 2 * P1)
        y[2 * (r - P1) + 1] = F32 ? v[j] * sc[r - P1] : v[j];
    }
  }
}

template <typename T, int RT>
__global__ __launch_bounds__(256) void m2l_mfma_kernel(int p, const int4* __restrict__ tiles,
                                                       M2LLevels lv, const T* __restrict__ amat,
                                                       const T* __restrict__ Mp,
                                                       const double* __restrict__ msc,
                                                       const int* __restrict__ stop) {
  if (stop && *stop) return;
  __shared__ dbl4 red[3 * RT * 64];
  m2l_tile<T, RT>(tiles[blockIdx.x], p, lv, amat, Mp, msc, red);
}

// M2M (GATHER: parent tiles at level l, y = sum over the 4 children of A_pos x_child)
// and L2L (scatter: parent tiles, child_pos += A_pos x_parent), one level per
// launch, one wavefront per item bx = (16-box tile, row tile) = (bx / RT, bx % RT) of
// the level's boxes in the order ord (sorted by which children they have): the child
// positions' products chain into one accumulator (M2M) or run as independent chains
// (L2L), a position that no box of the tile has skipped, with no exchange between
// wavefronts; A points at the child level's 4 matrices, ch is the children table.
template <int RT, bool GATHER>
__device__ __forceinline__ void tree_tile(int bx, int p, int nbox, const int* __restrict__ ch,
                                          const int* __restrict__ ord,
                                          const double2* __restrict__ X,
                                          const double* __restrict__ amat,
                                          double2* __restrict__ Y) {
  constexpr int R = RT * 16, KS = R / 4;
  const int lane = threadIdx.x & 63;
  const int rt = bx % RT;
  const int P1 = p + 1;
  const int col = lane & 15, kk = lane >> 4;
  const int q = (bx / RT) * 16 + col;
  const int tb = q < nbox ? as_g(ord)[q] : nbox;
  const double* A = amat + (int64_t)rt * KS * 64 + lane;
  const gptr<int> chg = as_g(ch);
  int c[4];
#pragma unroll
  for (int pos = 0; pos < 4; ++pos) c[pos] = tb < nbox ? chg[4 * (int64_t)tb + pos] : -1;
  if (GATHER) {
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int pos = 0; pos < 4; ++pos) {
      if (__ballot(c[pos] >= 0) == 0) continue;
      TileOps<KS> op;
      tile_load<KS>(op, A + (int64_t)pos * R * R, c[pos] >= 0 ? X + (int64_t)c[pos] * P1 : nullptr,
                    P1, kk);
      acc = tile_mfma<KS>(op, acc);
    }
    // a leaf keeps the coefficients of its own nodes (P2M)
    if (c[0] >= 0 || c[1] >= 0 || c[2] >= 0 || c[3] >= 0)
      tile_store<false>(Y + (int64_t)tb * P1, rt, kk, P1, acc);
  } else {
    bool any[4];
#pragma unroll
    for (int pos = 0; pos < 4; ++pos) any[pos] = __ballot(c[pos] >= 0) != 0;
    if (!(any[0] || any[1] || any[2] || any[3])) return;
    TileOps<KS> op;   // B: the parent's coefficients, shared by the positions
    tile_load<KS>(op, A, tb < nbox ? X + (int64_t)tb * P1 : nullptr, P1, kk);
#pragma unroll
    for (int pos = 0; pos < 4; ++pos) {
      if (!any[pos]) continue;
      const gptr<double> Ag = as_g(A + (int64_t)pos * R * R);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) op.a[ks] = Ag[ks * 64];
      const dbl4 acc = tile_mfma<KS>(op, dbl4{0.0, 0.0, 0.0, 0.0});
      if (c[pos] >= 0) tile_store<true>(Y + (int64_t)c[pos] * P1, rt, kk, P1, acc);
    }
  }
}

// nitems (tile, row tile) items of one level, four per block.
template <int RT, bool GATHER>
__global__ __launch_bounds__(256) void tree_mfma_kernel(int p, int nbox, int nitems,
                                                        const int* __restrict__ ch,
                                                        const int* __restrict__ ord,
                                                        const double2* __restrict__ X,
                                                        const double* __restrict__ amat,
                                                        double2* __restrict__ Y) {
  const int i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (i >= nitems) return;
  tree_tile<RT, GATHER>(i, p, nbox, ch, ord, X, amat, Y);
}

// L2L: child level lc from parents (table level lc), accumulated.
__global__ void l2l_kernel(int p, int nbox, const int* __restrict__ parent, const int* __restrict__ cpos,
                           const double2* __restrict__ Lp, const double2* __restrict__ tgl,
                           double2* __restrict__ Lc) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)nbox * (p + 1)) return;
  const int c = (int)(t / (p + 1)), m = (int)(t % (p + 1));
  const int K = 4 * p + 1;
  const double2* T = tgl + cpos[c] * K + 2 * p;
  const double2* lp = Lp + (int64_t)parent[c] * (p + 1);
  double2 sum = Lc[t];
  for (int n = -p; n <= p; ++n) {
    const double2 ln = n >= 0 ? lp[n] : cconj(lp[-n]);
    sum = cmad(ln, T[n - m], sum);
  }
  Lc[t] = sum;
}

// Waves per leaf in l2p_p2p_grad_kernel (and p2p_kernel below kLeavesFor2): wave
// w takes every PW-th leaf of the leaf's P2P list (a leaf holds at most leaf_max
// targets, 64 by default, so one wave per leaf left most SIMDs with a single wave to
// hide latency); the waves' partial sums are combined in a fixed order by wave 0
// (which in the gradient pass also evaluates the local expansion's gradient).  From
// kLeavesFor2 leaves on the leaves
// alone fill the SIMDs and p2p_kernel takes two waves per leaf (measured on the
// uniform tree this replaced: 4 waves best at 800 leaves, 2 at 4,000; 8 slower at
// both).
constexpr int PW = 4;
constexpr int kLeavesFor2 = 2048;

// Orders this wave's LDS writes before its later reads (wave-local exchange).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane groups of the leaf passes: a round of rem <= 64 targets takes rem lanes per
// group and G = 64 / rem groups split the sources of every staged tile, so that a
// leaf of few nodes still keeps most lanes busy.  Lane l serves target l % rem for
// group l / rem; lanes past G rem read group 0's sources and are not used.
struct LaneGroups {
  int rem, G, t, g, ga;
};

__device__ __forceinline__ LaneGroups lane_groups(int lane, int rem) {
  LaneGroups r;
  r.rem = rem;
  r.G = FB / rem;
  r.t = lane % rem;
  r.g = lane / rem;
  r.ga = r.g < r.G ? r.g : 0;
  return r;
}

// Tile slot of the source k of a staged tile of nbk sources for G groups of S =
// ceil(nbk / G) sources each: group g reads the S consecutive slots from g S.  Slots
// of k in [nbk, G S) hold padding (zero strength); G S <= nbk + G - 1 < 2 FB.
__device__ __forceinline__ int group_slot(int k, int G, int S) { return (k % G) * S + k / G; }

// Pair classes of a (target leaf, source leaf) pair from the circles about their box
// centres that hold their nodes: every z < 2 (the small-z branch of K1(z)/z alone),
// every z >= 2 (the large-z branch alone), or both kinds (both branches, selected per
// pair without a branch).  The selection rule is that of k1z_32 / k1z_64 (z^2 < 4).
constexpr int LC_NEAR = 0, LC_FAR = 1, LC_MIXED = 2;

__device__ __forceinline__ int leaf_class(double kappa, double cx, double cy, double r,
                                          double sx, double sy, double rs) {
  const double ex = cx - sx, ey = cy - sy;
  const double d = sqrt(ex * ex + ey * ey), rr = r + rs;
  return kappa * (d - rr) >= 2.0 ? LC_FAR : kappa * (d + rr) < 2.0 ? LC_NEAR : LC_MIXED;
}

template <int CLS>
__device__ __forceinline__ float leaf_k1z_32(float z2) {
  if (CLS == LC_NEAR) return k1z_32_small(z2);
  if (CLS == LC_FAR) return k1z_32_large(z2);
  const float a = k1z_32_small(z2), b = k1z_32_large(z2);
  return z2 < 4.0f ? a : b;
}

template <int CLS>
__device__ __forceinline__ double leaf_k1z_64(double z2, const double* __restrict__ T) {
  if (CLS == LC_NEAR) return k1z_64_small(z2, T);
  if (CLS == LC_FAR) return k1z_64_large<21, T_H1>(z2, T);
  const double a = k1z_64_small(z2, T), b = k1z_64_large<21, T_H1>(z2, T);
  return z2 < 4.0 ? a : b;
}

template <int CLS>
__device__ __forceinline__ void leaf_k0_k1z_64(double z2, double& k0, double& k1z,
                                               const double* __restrict__ T) {
  if (CLS == LC_NEAR) {
    k0_k1z_64_small(z2, k0, k1z, T);
  } else if (CLS == LC_FAR) {
    k0_k1z_64_large<21, T_H0, T_H1>(z2, k0, k1z, T);
  } else {
    double a0, a1, b0, b1;
    k0_k1z_64_small(z2, a0, a1, T);
    k0_k1z_64_large<21, T_H0, T_H1>(z2, b0, b1, T);
    const bool sm = z2 < 4.0;
    k0 = sm ? a0 : b0;
    k1z = sm ? a1 : b1;
  }
}

// The pair sums of far32_tile / far64_tile / far_grad64_tile over nb staged sources
// for one pair class, with the next source read before the current one is used (the
// tile has room for one entry past its sources).
template <int CLS>
__device__ __forceinline__ float leaf_tile32(double xi, double yi, const double2* sxy,
                                             const float2* sq, int nb, float kap2, float acc) {
  double2 p = sxy[0];
  float2 q = sq[0];
  for (int k = 0; k < nb; ++k) {
    const double2 pn = sxy[k + 1];
    const float2 qn = sq[k + 1];
    const float dx = (float)(xi - p.x), dy = (float)(yi - p.y);
    const float z2 = fmaxf(kap2 * fmaf(dx, dx, dy * dy), 1e-30f);
    acc = fmaf(leaf_k1z_32<CLS>(z2), fmaf(dx, q.x, dy * q.y), acc);
    p = pn;
    q = qn;
  }
  return acc;
}

template <int CLS>
__device__ __forceinline__ double leaf_tile64(double xi, double yi, const double2* sxy,
                                              const double2* sq, int nb, double kap2,
                                              const double* __restrict__ tab, double acc) {
  double2 p = sxy[0], q = sq[0];
  for (int k = 0; k < nb; ++k) {
    const double2 pn = sxy[k + 1], qn = sq[k + 1];
    const double dx = xi - p.x, dy = yi - p.y;
    const double r2 = fma(dx, dx, dy * dy);
    const double v = leaf_k1z_64<CLS>(kap2 * r2, tab) * fma(dx, q.x, dy * q.y);
    acc += r2 > 0.0 ? v : 0.0;
    p = pn;
    q = qn;
  }
  return acc;
}

// (the self pair, r = 0, adds nothing; others add exactly far_grad64_tile's terms)
template <int CLS>
__device__ __forceinline__ void leaf_grad_tile64(double xi, double yi, const double2* sxy,
                                                 const double2* sq, int nb, double kap2,
                                                 const double* __restrict__ tab, double& ax,
                                                 double& ay) {
  double2 p = sxy[0], q = sq[0];
  for (int k = 0; k < nb; ++k) {
    const double2 pn = sxy[k + 1], qn = sq[k + 1];
    const double dx = xi - p.x, dy = yi - p.y;
    const double r2 = fma(dx, dx, dy * dy);
    const bool self = !(r2 > 0.0);
    const double r2s = self ? 1.0 : r2;
    double k0, k1z;
    leaf_k0_k1z_64<CLS>(kap2 * r2s, k0, k1z, tab);
    const double dq = fma(dx, q.x, dy * q.y);
    const double b = dq * (k0 + 2.0 * k1z) * rcp64(r2s);
    const double gx = k1z * q.x - b * dx, gy = k1z * q.y - b * dy;
    ax += self ? 0.0 : gx;
    ay += self ? 0.0 : gy;
    p = pn;
    q = qn;
  }
}

// LDS of leaf_pass for nw wavefronts: per wavefront a tile of 2 FB positions and
// 2 FB strengths (FP64, or FP32 in the same space) and FB partial sums.
static size_t leaf_lds_bytes(int nw) {
  return (size_t)nw * FB * (4 * sizeof(double2) + sizeof(double));
}

// LDS of leaf_grad_pass: tiles as above, FB partial gradients per wavefront, columns
// up to I_{p+1}.
static size_t leaf_grad_lds_bytes(int p, int use_col) {
  return (size_t)PW * FB * (4 * sizeof(double2) + sizeof(double2)) +
         (use_col ? (size_t)(p + 2) * 64 * sizeof(double) : 0);
}

// One block per leaf: the direct interactions of the leaf's targets with the leaves of
// its P2P list, added to partial[node] (which holds the local expansion's value from
// l2p_kernel) in the far-field kernels' scaling (far field * 2 pi / kappa^2).
// Leaf b; sh: the kernel's dynamic LDS (leaf_lds_bytes).
template <bool F32, int NW>
__device__ __forceinline__ void leaf_pass(int b, double kappa, const int* __restrict__ ls,
                                          const int* __restrict__ lc,
                                          const int* __restrict__ nbp,
                                          const int* __restrict__ nbi,
                                          const double* __restrict__ ccx,
                                          const double* __restrict__ ccy,
                                          const double* __restrict__ lr,
                                          const double* __restrict__ xs,
                                          const double* __restrict__ ys,
                                          const double* __restrict__ qx,
                                          const double* __restrict__ qy,
                                          const int* __restrict__ perm,
                                          const double* __restrict__ tab,
                                          double* __restrict__ partial, double* sh) {
  // the wave index is uniform over the wave: in a scalar register, the neighbour-leaf
  // and source loops below run on scalar counters (the LDS tiles are addressed from a
  // vector register, so the unrolled pair loop reads them with immediate offsets)
  const int lane = threadIdx.x % FB, w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FB));
  const int wv = threadIdx.x / FB;
  double2* sbase = reinterpret_cast<double2*>(sh);
  double2* sxy = sbase + wv * 2 * FB;                                  // [NW][2 FB]
  double2* sq = sbase + (NW + wv) * 2 * FB;                            // [NW][2 FB] (FP64)
  float2* sq32 = reinterpret_cast<float2*>(sq);                        // (FP32, same space)
  double* red = reinterpret_cast<double*>(sbase + 4 * NW * FB);        // [NW][FB] wave sums
  // leaf and list data through scalar loads (uniform over the wave)
  const int s0 = as_k(ls)[b], cnt = as_k(lc)[b];
  const double kap2 = kappa * kappa;
  const double cx = as_k(ccx)[b], cy = as_k(ccy)[b], rb = as_k(lr)[b];
  const int e0 = as_k(nbp)[b], e1 = as_k(nbp)[b + 1];
  for (int r0 = 0; r0 < cnt; r0 += FB) {
    const LaneGroups lg = lane_groups(lane, min(cnt - r0, FB));
    const int j = r0 + lg.t;
    const double xi = as_g(xs)[s0 + j], yi = as_g(ys)[s0 + j];
    const bool act = lg.g == 0;   // one lane per target: the sums of every wave and group
    double acc64 = 0.0;
    float acc32 = 0.0f;
    for (int e = e0 + w; e < e1; e += NW) {
      const int nb = as_k(nbi)[e];
      const int t0 = as_k(ls)[nb];
      const int tc = as_k(lc)[nb];
      const int cls = leaf_class(kappa, cx, cy, rb, as_k(ccx)[nb], as_k(ccy)[nb], as_k(lr)[nb]);
      for (int k0 = 0; k0 < tc; k0 += FB) {
        const int nbk = min(FB, tc - k0);
        const int S = (nbk + lg.G - 1) / lg.G;
        wave_sync();   // this wave's reads of the previous tile are done
        for (int k = lane; k < lg.G * S; k += FB) {
          const int sl = group_slot(k, lg.G, S);
          if (k < nbk) {
            const int ks = t0 + k0 + k;
            sxy[sl] = make_double2(as_g(xs)[ks], as_g(ys)[ks]);
            if (F32)
              sq32[sl] = make_float2((float)as_g(qx)[ks], (float)as_g(qy)[ks]);
            else
              sq[sl] = make_double2(as_g(qx)[ks], as_g(qy)[ks]);
          } else {   // padding: zero strength at a point of no target
            sxy[sl] = make_double2(cx + 1.0, cy);
            if (F32)
              sq32[sl] = make_float2(0.0f, 0.0f);
            else
              sq[sl] = make_double2(0.0, 0.0);
          }
        }
        wave_sync();
        const int g0 = lg.ga * S;
        if (F32) {
          const float k2 = (float)kap2;
          if (cls == LC_NEAR)
            acc32 = leaf_tile32<LC_NEAR>(xi, yi, sxy + g0, sq32 + g0, S, k2, acc32);
          else if (cls == LC_FAR)
            acc32 = leaf_tile32<LC_FAR>(xi, yi, sxy + g0, sq32 + g0, S, k2, acc32);
          else
            acc32 = leaf_tile32<LC_MIXED>(xi, yi, sxy + g0, sq32 + g0, S, k2, acc32);
        } else {
          if (cls == LC_NEAR)
            acc64 = leaf_tile64<LC_NEAR>(xi, yi, sxy + g0, sq + g0, S, kap2, tab, acc64);
          else if (cls == LC_FAR)
            acc64 = leaf_tile64<LC_FAR>(xi, yi, sxy + g0, sq + g0, S, kap2, tab, acc64);
          else
            acc64 = leaf_tile64<LC_MIXED>(xi, yi, sxy + g0, sq + g0, S, kap2, tab, acc64);
        }
      }
    }
    red[w * FB + lane] = F32 ? (double)acc32 : acc64;
    __syncthreads();
    if (w == 0 && act) {
      double direct = 0.0;
      for (int q = 0; q < NW; ++q)
        for (int gg = 0; gg < lg.G; ++gg) direct += red[q * FB + gg * lg.rem + lg.t];
      // the local expansion's value is there already (l2p_kernel)
      const int node = as_g(perm)[s0 + j];
      as_gm(partial)[node] = as_g(partial)[node] + direct;
    }
    __syncthreads();   // red is rewritten by the next group of targets
  }
}

template <bool F32, int NW>
__global__ __launch_bounds__(FB * NW) void p2p_kernel(double kappa, const int* __restrict__ ls,
                                                      const int* __restrict__ lc,
                                                      const int* __restrict__ nbp,
                                                      const int* __restrict__ nbi,
                                                      const double* __restrict__ ccx,
                                                      const double* __restrict__ ccy,
                                                      const double* __restrict__ lr,
                                                      const double* __restrict__ xs,
                                                      const double* __restrict__ ys,
                                                      const double* __restrict__ qx,
                                                      const double* __restrict__ qy,
                                                      const int* __restrict__ perm,
                                                      const double* __restrict__ tab,
                                                      double* __restrict__ partial,
                                                      const int* __restrict__ stop) {
  if (stop && *stop) return;
  extern __shared__ double sh[];
  leaf_pass<F32, NW>(blockIdx.x, kappa, ls, lc, nbp, nbi, ccx, ccy, lr, xs, ys, qx, qy, perm, tab,
                     partial, sh);
}

// The leaf pass from the near-field cache, one wavefront per leaf (CW leaves per
// block, no block barrier): entry e's coefficients, source k, target i at
// boff[e] + k cnt + i, times the density in sorted order.  Lane groups split each
// entry's sources; every load of a batch is issued before the first is used (the
// pass is bound by the loads in flight).  Adds the direct sums to partial[node].
constexpr int CW = 4;
template <bool F32>
__device__ __forceinline__ void leaf_cached_wave(int b, const int* __restrict__ ls,
                                                 const int* __restrict__ lc,
                                                 const int* __restrict__ nbp,
                                                 const int2* __restrict__ ent,
                                                 const int64_t* __restrict__ boff,
                                                 const void* nc, const double* __restrict__ ssd,
                                                 const int* __restrict__ perm,
                                                 double* __restrict__ partial, double* red) {
  constexpr int CB = 16;
  const int lane = threadIdx.x % FB;
  // leaf and list data through scalar loads (uniform over the wave)
  const int s0 = as_k(ls)[b], cnt = as_k(lc)[b];
  const int e0 = as_k(nbp)[b], e1 = as_k(nbp)[b + 1];
  const kptr<int> te = as_k(reinterpret_cast<const int*>(ent));
  for (int r0 = 0; r0 < cnt; r0 += FB) {
    const LaneGroups lg = lane_groups(lane, min(cnt - r0, FB));
    const int j = r0 + lg.t;
    // the target's output and its current value (the local expansion's), early
    const int node = lg.g == 0 ? as_g(perm)[s0 + j] : 0;
    const double prev = lg.g == 0 ? as_g(partial)[node] : 0.0;
    double acc64 = 0.0;
    float acc32 = 0.0f;
    for (int e = e0; e < e1; ++e) {
      const int t0 = te[2 * e], tc = te[2 * e + 1];
      const int64_t bo = as_k(boff)[e];
      const gptr<float> cb32 = as_g(static_cast<const float*>(nc) + bo);
      const gptr<double> cb64 = as_g(static_cast<const double*>(nc) + bo);
      // the source leaf's densities, one per lane, handed to the lanes that need them
      // through the cross-lane permute (tc <= 64: a leaf holds at most 64 nodes)
      const double sl = lane < tc ? as_g(ssd)[t0 + lane] : 0.0;
      const float sl32 = (float)sl;
      const int S = (tc + lg.G - 1) / lg.G, k0 = lg.ga * S;
      const int kend = min(k0 + S, tc);   // this group's sources end here
      for (int u = 0; u < S; u += CB) {
        float c32[CB];
        double c64[CB];
#pragma unroll
        for (int v = 0; v < CB; ++v) {
          const int kc = min(k0 + u + v, tc - 1);
          const int a = kc * cnt + j;   // within the block (< 2^31)
          if (F32)
            c32[v] = cb32[a];
          else
            c64[v] = cb64[a];
        }
#pragma unroll
        for (int v = 0; v < CB; ++v) {
          const int k = k0 + u + v;
          const bool ok = k < kend;
          const int kc = min(k, tc - 1);
          if (F32) {
            const float sv = __shfl(sl32, kc, FB);
            acc32 = fmaf(ok ? c32[v] : 0.0f, sv, acc32);
          } else {
            const double sv = __shfl(sl, kc, FB);
            acc64 = fma(ok ? c64[v] : 0.0, sv, acc64);
          }
        }
      }
    }
    wave_sync();   // the previous round's reads of red are done
    red[lane] = F32 ? (double)acc32 : acc64;
    wave_sync();
    if (lg.g == 0) {
      double direct = 0.0;
      for (int gg = 0; gg < lg.G; ++gg) direct += red[gg * lg.rem + lg.t];
      as_gm(partial)[node] = prev + direct;
    }
  }
}

template <bool F32>
__global__ __launch_bounds__(FB * CW) void p2p_cached_kernel(int nleaf, const int* __restrict__ ls,
                                                             const int* __restrict__ lc,
                                                             const int* __restrict__ nbp,
                                                             const int2* __restrict__ ent,
                                                             const int64_t* __restrict__ boff,
                                                             const void* nc,
                                                             const double* __restrict__ ssd,
                                                             const int* __restrict__ perm,
                                                             double* __restrict__ partial,
                                                             const int* __restrict__ stop) {
  __shared__ double red[CW][FB];
  if (stop && *stop) return;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FB));
  const int b = blockIdx.x * CW + w;
  if (b >= nleaf) return;
  leaf_cached_wave<F32>(b, ls, lc, nbp, ent, boff, nc, ssd, perm, partial, red[w]);
}

// The local expansion's value at sorted node k of a tree (leaf leaf_of[k]):
// partial[perm[k]] = (2 pi / kappa^2) u_local, one node per thread.
__device__ __forceinline__ void l2p_node(int64_t k, int p, double kappa,
                                         const int* __restrict__ leaf_of,
                                         const int* __restrict__ gid,
                                         const double* __restrict__ ccx,
                                         const double* __restrict__ ccy,
                                         const double* __restrict__ xs,
                                         const double* __restrict__ ys,
                                         const int* __restrict__ perm,
                                         const double2* __restrict__ L,
                                         double* __restrict__ partial) {
  const int b = as_g(leaf_of)[k];
  const double u = l2p_value(as_g(xs)[k], as_g(ys)[k], as_g(ccx)[b], as_g(ccy)[b], kappa, p,
                             L + (int64_t)as_g(gid)[b] * (p + 1));
  as_gm(partial)[as_g(perm)[k]] = u * (2.0 * PI / (kappa * kappa));
}

__global__ __launch_bounds__(256) void l2p_kernel(int64_t N, int p, double kappa,
                                                  const int* __restrict__ leaf_of,
                                                  const int* __restrict__ gid,
                                                  const double* __restrict__ ccx,
                                                  const double* __restrict__ ccy,
                                                  const double* __restrict__ xs,
                                                  const double* __restrict__ ys,
                                                  const int* __restrict__ perm,
                                                  const double2* __restrict__ L,
                                                  double* __restrict__ partial,
                                                  const int* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= N) return;
  l2p_node(k, p, kappa, leaf_of, gid, ccx, ccy, xs, ys, perm, L, partial);
}

// Gradient counterpart of l2p_kernel + p2p_kernel (FP64): the direct gradient from the
// leaves of the P2P list plus the local expansion's gradient
//   u_x + i u_y = kappa [ L_0 I_1 e^{i theta}
//                 + sum_{n>=1} (L_n I_{n+1} e^{i(n+1) theta} + conj(L_n) I_{n-1} e^{-i(n-1) theta}) ],
// since (d/dx + i d/dy) I_n(kappa rho) e^{i n theta} = kappa I_{n+1} e^{i(n+1) theta} for
// every integer n (I_{-n} = I_n).  Writes gpart[node] (x) and gpart[N + node] (y) in
// the gradient far-field kernels' scaling.
// Leaf b; sh: the kernel's dynamic LDS (leaf_grad_lds_bytes).
__device__ __forceinline__ void leaf_grad_pass(int b, int p, int use_col, double kappa,
                                               const int* __restrict__ ls,
                                               const int* __restrict__ lc,
                                               const int* __restrict__ gid,
                                               const int* __restrict__ nbp,
                                               const int* __restrict__ nbi,
                                               const double* __restrict__ ccx,
                                               const double* __restrict__ ccy,
                                               const double* __restrict__ lr,
                                               const double2* __restrict__ L,
                                               const double* __restrict__ xs,
                                               const double* __restrict__ ys,
                                               const double* __restrict__ qx,
                                               const double* __restrict__ qy,
                                               const int* __restrict__ perm, int64_t N,
                                               const double* __restrict__ tab,
                                               double* __restrict__ gpart, double* sh) {
  // the neighbour leaves are split over PW wavefronts as in p2p_kernel
  // the wave index is uniform over the wave: in a scalar register, the neighbour-leaf
  // and source loops below run on scalar counters
  const int lane = threadIdx.x % FB, w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FB));
  const int wv = threadIdx.x / FB;
  double2* sbase = reinterpret_cast<double2*>(sh);
  double2* sxy = sbase + wv * 2 * FB;                          // [PW][2 FB]
  double2* sq = sbase + (PW + wv) * 2 * FB;                    // [PW][2 FB]
  double2* red = sbase + 4 * PW * FB;                          // [PW][FB] wave sums (x, y)
  double* col = reinterpret_cast<double*>(red + PW * FB) + lane;   // [(p + 2) * 64] scaled I_n
  const int s0 = as_k(ls)[b], cnt = as_k(lc)[b];
  const double kap2 = kappa * kappa;
  const double cx = as_k(ccx)[b], cy = as_k(ccy)[b], rb = as_k(lr)[b];
  const int e0 = as_k(nbp)[b], e1 = as_k(nbp)[b + 1];
  for (int r0 = 0; r0 < cnt; r0 += FB) {
    const LaneGroups lg = lane_groups(lane, min(cnt - r0, FB));
    const int j = r0 + lg.t;
    const double xi = as_g(xs)[s0 + j], yi = as_g(ys)[s0 + j];
    double ax = 0.0, ay = 0.0;
    for (int e = e0 + w; e < e1; e += PW) {
      const int nb = as_k(nbi)[e];
      const int t0 = as_k(ls)[nb];
      const int tc = as_k(lc)[nb];
      const int cls = leaf_class(kappa, cx, cy, rb, as_k(ccx)[nb], as_k(ccy)[nb], as_k(lr)[nb]);
      for (int k0 = 0; k0 < tc; k0 += FB) {
        const int nbk = min(FB, tc - k0);
        const int S = (nbk + lg.G - 1) / lg.G;
        wave_sync();   // this wave's reads of the previous tile are done
        for (int k = lane; k < lg.G * S; k += FB) {
          const int sl = group_slot(k, lg.G, S);
          if (k < nbk) {
            const int ks = t0 + k0 + k;
            sxy[sl] = make_double2(as_g(xs)[ks], as_g(ys)[ks]);
            sq[sl] = make_double2(as_g(qx)[ks], as_g(qy)[ks]);
          } else {   // padding: zero strength at a point of no target
            sxy[sl] = make_double2(cx + 1.0, cy);
            sq[sl] = make_double2(0.0, 0.0);
          }
        }
        wave_sync();
        const int g0 = lg.ga * S;
        if (cls == LC_NEAR)
          leaf_grad_tile64<LC_NEAR>(xi, yi, sxy + g0, sq + g0, S, kap2, tab, ax, ay);
        else if (cls == LC_FAR)
          leaf_grad_tile64<LC_FAR>(xi, yi, sxy + g0, sq + g0, S, kap2, tab, ax, ay);
        else
          leaf_grad_tile64<LC_MIXED>(xi, yi, sxy + g0, sq + g0, S, kap2, tab, ax, ay);
      }
    }
    red[w * FB + lane] = make_double2(ax, ay);
    __syncthreads();
    const bool act = lg.g == 0;   // one lane per target: the sums of every wave and group
    if (w == 0 && act) {
      ax = 0.0;
      ay = 0.0;
      for (int q = 0; q < PW; ++q)
        for (int gg = 0; gg < lg.G; ++gg) {
          ax += red[q * FB + gg * lg.rem + lg.t].x;
          ay += red[q * FB + gg * lg.rem + lg.t].y;
        }
    }
    if (w == 0 && act) {
      const double dx = xi - cx, dy = yi - cy;
      const double rho = sqrt(dx * dx + dy * dy);
      const double x = kappa * rho, t = 0.25 * x * x, hx = 0.5 * x;
      const double2 e1 = rho > 0.0 ? make_double2(dx / rho, dy / rho) : make_double2(1.0, 0.0);
      const double2* lb = L + (int64_t)as_k(gid)[b] * (p + 1);
      if (use_col) iscaled_col(t, p + 1, col);
      double pref = hx;                                   // (x/2)^{n+1} / (n+1)!
      double Iprev = use_col ? col[0] : iorder(t, 1.0, 0);        // I_{n-1}
      double Icur = use_col ? pref * col[64] : iorder(t, pref, 1);  // I_n
      double2 G = make_double2(lb[0].x * Icur * e1.x, lb[0].x * Icur * e1.y);
      double2 Eprev = make_double2(1.0, 0.0);             // e^{i(n-1) theta}
      double2 Enext = e1;                                 // e^{i(n+1) theta} after the update
      for (int n = 1; n <= p; ++n) {
        pref *= hx * recip(n + 1);
        const double Inext = use_col ? pref * col[(n + 1) * 64] : iorder(t, pref, n + 1);
        Enext = cmul(Enext, e1);
        const double2 a = cmul(lb[n], Enext);
        const double2 c = cconj(cmul(lb[n], Eprev));
        G.x += a.x * Inext + c.x * Iprev;
        G.y += a.y * Inext + c.y * Iprev;
        Eprev = cmul(Eprev, e1);
        Iprev = Icur;
        Icur = Inext;
      }
      const double sc = kappa * 2.0 * PI / kap2;
      const int node = perm[s0 + j];
      gpart[node] = ax + G.x * sc;
      gpart[N + node] = ay + G.y * sc;
    }
    __syncthreads();   // red is rewritten by the next group of targets
  }
}

__global__ __launch_bounds__(FB * PW) void l2p_p2p_grad_kernel(int p, int use_col, double kappa,
                                                          const int* __restrict__ ls,
                                                          const int* __restrict__ lc,
                                                          const int* __restrict__ gid,
                                                          const int* __restrict__ nbp,
                                                          const int* __restrict__ nbi,
                                                          const double* __restrict__ ccx,
                                                          const double* __restrict__ ccy,
                                                          const double* __restrict__ lr,
                                                          const double2* __restrict__ L,
                                                          const double* __restrict__ xs,
                                                          const double* __restrict__ ys,
                                                          const double* __restrict__ qx,
                                                          const double* __restrict__ qy,
                                                          const int* __restrict__ perm, int64_t N,
                                                          const double* __restrict__ tab,
                                                          double* __restrict__ gpart) {
  extern __shared__ double sh[];
  leaf_grad_pass(blockIdx.x, p, use_col, kappa, ls, lc, gid, nbp, nbi, ccx, ccy, lr, L, xs, ys, qx,
                 qy, perm, N, tab, gpart, sh);
}

// ---- tree keys (device) ------------------------------------------------------------------

// Bounding box of the nodes, out = (xmin, xmax, ymin, ymax); one block (min and
// max are exact, so the order of the reduction does not matter).
constexpr int BBOX_BS = 1024;
__global__ __launch_bounds__(BBOX_BS) void bbox_kernel(const double* __restrict__ x,
                                                       const double* __restrict__ y, int64_t n,
                                                       double* __restrict__ out) {
  __shared__ double sh[4][BBOX_BS];
  double a = x[0], b = x[0], c = y[0], d = y[0];
  for (int64_t i = threadIdx.x; i < n; i += BBOX_BS) {
    a = fmin(a, x[i]);
    b = fmax(b, x[i]);
    c = fmin(c, y[i]);
    d = fmax(d, y[i]);
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  sh[2][threadIdx.x] = c;
  sh[3][threadIdx.x] = d;
  __syncthreads();
  for (int o = BBOX_BS / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sh[0][threadIdx.x] = fmin(sh[0][threadIdx.x], sh[0][threadIdx.x + o]);
      sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + o]);
      sh[2][threadIdx.x] = fmin(sh[2][threadIdx.x], sh[2][threadIdx.x + o]);
      sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = sh[threadIdx.x][0];
}

// The root box: side W and lower-left corner (x0, y0), from the bounding box.
__host__ __device__ inline void root_box(const double* bb, double& W, double& x0, double& y0) {
  W = fmax(bb[1] - bb[0], bb[3] - bb[2]) * (1.0 + 1e-9) + 1e-12;
  x0 = 0.5 * (bb[0] + bb[1]) - 0.5 * W;
  y0 = 0.5 * (bb[2] + bb[3]) - 0.5 * W;
}

__device__ __forceinline__ uint32_t spread16(uint32_t v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

// Morton key of every node on the 2^DMAX x 2^DMAX grid of the root box (x in
// the even bits), and the sort payload i.
__global__ void keys_kernel(const double* __restrict__ x, const double* __restrict__ y, int64_t n,
                            const double* __restrict__ bb, int dmax, uint32_t* __restrict__ key,
                            int* __restrict__ iota) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double W, x0, y0;
  root_box(bb, W, x0, y0);
  const int64_t m = 1LL << dmax;
  int64_t ix = (int64_t)((x[i] - x0) / W * m), iy = (int64_t)((y[i] - y0) / W * m);
  ix = min(max(ix, (int64_t)0), m - 1);
  iy = min(max(iy, (int64_t)0), m - 1);
  key[i] = spread16((uint32_t)ix) | (spread16((uint32_t)iy) << 1);
  iota[i] = (int)i;
}

// Sorted copies of positions and w nu (perm: sorted position -> node).
// r[b] = the largest distance of leaf b's nodes from its box centre (with a relative
// margin far above rounding), for the leaf passes' pair classes.
__global__ void leaf_radius_kernel(int nleaf, const int* __restrict__ ls,
                                   const int* __restrict__ lc, const double* __restrict__ ccx,
                                   const double* __restrict__ ccy, const double* __restrict__ xs,
                                   const double* __restrict__ ys, double* __restrict__ r) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  double m = 0.0;
  for (int k = ls[b]; k < ls[b] + lc[b]; ++k) {
    const double dx = xs[k] - ccx[b], dy = ys[k] - ccy[b];
    m = fmax(m, sqrt(dx * dx + dy * dy));
  }
  r[b] = m * (1.0 + 1e-12);
}

__global__ void sort_gather_kernel(int64_t n, const int* __restrict__ perm,
                                   const double* __restrict__ x, const double* __restrict__ y,
                                   const double* __restrict__ wx, const double* __restrict__ wy,
                                   double* __restrict__ xs, double* __restrict__ ys,
                                   double* __restrict__ wxs, double* __restrict__ wys) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = perm[k];
  xs[k] = x[i];
  ys[k] = y[i];
  wxs[k] = wx[i];
  wys[k] = wy[i];
}

// ---- host --------------------------------------------------------------------------------

// Host-to-device uploads during set-up: each array is kept until finish(), which
// packs them into the pinned staging buffer, issues one asynchronous copy per
// array and waits for the stream.  Device buffers only grow (DevBuf::fit).
// Many copies in one launch: block (item, slice) copies 32-bit words of item
// blockIdx.x.  Every item's size is a multiple of 4 bytes (int, double, int2).
struct CopyItem {
  void* dst;
  const void* src;
  int64_t words;
};

constexpr int COPY_SLICES = 32;

__global__ __launch_bounds__(256) void batch_copy_kernel(const CopyItem* __restrict__ items) {
  const CopyItem it = items[blockIdx.x];
  const uint32_t* __restrict__ src = static_cast<const uint32_t*>(it.src);
  uint32_t* __restrict__ dst = static_cast<uint32_t*>(it.dst);
  for (int64_t w = (int64_t)blockIdx.y * 256 + threadIdx.x; w < it.words;
       w += (int64_t)COPY_SLICES * 256)
    dst[w] = src[w];
}

// Collects host arrays for device buffers and sends them in one transfer: the
// arrays and a table of (destination, staged source, size) go through pinned
// memory in one host-to-device copy, and batch_copy_kernel moves each array to
// its buffer.  (A copy call per array costs the host tens of microseconds each.)
struct Uploader {
  hipStream_t s;
  PinnedBuf& stage;
  DevBuf<char>& dstage;
  struct Item {
    void* dst;
    std::shared_ptr<void> keep;
    const void* src;
    size_t bytes;
  };
  std::vector<Item> items;
  Uploader(hipStream_t st, PinnedBuf& sb, DevBuf<char>& db) : s(st), stage(sb), dstage(db) {}
  Uploader(const Uploader&) = delete;
  Uploader& operator=(const Uploader&) = delete;
  template <class T>
  void operator()(DevBuf<T>& d, const std::vector<T>& h) {
    static_assert(sizeof(T) % 4 == 0, "uploads move 32-bit words");
    d.fit(std::max<size_t>(h.size(), 1));
    if (h.empty()) return;
    auto c = std::make_shared<std::vector<T>>(h);
    items.push_back({d.p, c, c->data(), h.size() * sizeof(T)});
  }
  void finish() {
    if (!items.empty()) {
      size_t data = 0;
      for (const Item& it : items) data += (it.bytes + 255) & ~(size_t)255;
      const size_t total = data + items.size() * sizeof(CopyItem);
      stage.fit(total);
      dstage.fit(total);
      CopyItem* tab = reinterpret_cast<CopyItem*>(stage.p + data);
      size_t off = 0;
      for (size_t k = 0; k < items.size(); ++k) {
        const Item& it = items[k];
        std::memcpy(stage.p + off, it.src, it.bytes);
        tab[k] = CopyItem{it.dst, dstage.p + off, (int64_t)(it.bytes / 4)};
        off += (it.bytes + 255) & ~(size_t)255;
      }
      YQ_HIP(hipMemcpyAsync(dstage.p, stage.p, total, hipMemcpyHostToDevice, s));
      batch_copy_kernel<<<dim3((unsigned)items.size(), COPY_SLICES), 256, 0, s>>>(
          reinterpret_cast<const CopyItem*>(dstage.p + data));
      YQ_HIP(hipGetLastError());
    }
    YQ_HIP(hipStreamSynchronize(s));   // the pinned stage is reused by the next upload
    items.clear();
  }
};

Fmm::~Fmm() {
  if (dn_done) (void)hipEventDestroy(dn_done);
}

void Fmm::download(const double* dx, const double* dy, const double* dwnx, const double* dwny,
                   int64_t n, hipStream_t s) {
  YQ_REQUIRE(n >= 1 && n < ((int64_t)1 << 31), YQ_EINVAL, "FMM: node count out of range");
  static_assert(2 * DMAX <= 32, "Morton keys must fit 32 bits");
  const unsigned nb = (unsigned)((n + 255) / 256);
  bbox.fit(4);
  keys.fit(n);
  skeys.fit(n);
  iota.fit(n);
  perm.fit(n);
  bbox_kernel<<<1, BBOX_BS, 0, s>>>(dx, dy, n, bbox.p);
  keys_kernel<<<nb, 256, 0, s>>>(dx, dy, n, bbox.p, DMAX, keys.p, iota.p);
  YQ_HIP(hipGetLastError());
  size_t tmp_bytes = 0;
  YQ_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys.p, skeys.p, iota.p, perm.p,
                                            (int)n, 0, 2 * DMAX, s));
  sort_tmp.fit(std::max<size_t>(tmp_bytes, 1));
  // stable: equal keys keep ascending node order
  YQ_HIP(hipcub::DeviceRadixSort::SortPairs(sort_tmp.p, tmp_bytes, keys.p, skeys.p, iota.p, perm.p,
                                            (int)n, 0, 2 * DMAX, s));
  xs.fit(n);
  ys.fit(n);
  wnxs.fit(n);
  wnys.fit(n);
  sort_gather_kernel<<<nb, 256, 0, s>>>(n, perm.p, dx, dy, dwnx, dwny, xs.p, ys.p, wnxs.p, wnys.p);
  YQ_HIP(hipGetLastError());
  stage_dn.fit((size_t)n * sizeof(uint32_t) + 4 * sizeof(double));
  YQ_HIP(hipMemcpyAsync(stage_dn.p, bbox.p, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  YQ_HIP(hipMemcpyAsync(stage_dn.p + 4 * sizeof(double), skeys.p, n * sizeof(uint32_t),
                        hipMemcpyDeviceToHost, s));
  if (!dn_done) YQ_HIP(hipEventCreateWithFlags(&dn_done, hipEventDisableTiming));
  YQ_HIP(hipEventRecord(dn_done, s));
  N = n;
}

namespace {
// M2L order of one level's boxes from their offset sets occ: a tile multiplies every
// offset that any of its 16 boxes uses, and in Morton order the sparse boxes along
// curves share few.  The boxes are sorted by their sets; each tile then starts at
// the first unplaced box in that order and takes, one at a time, the unplaced box
// among the next 32 that adds the fewest offsets to the tile's union.
std::vector<int> m2l_order(const std::vector<uint64_t>& occ) {
  const int nb = (int)occ.size();
  std::vector<int> srt(nb);
  std::iota(srt.begin(), srt.end(), 0);
  std::stable_sort(srt.begin(), srt.end(), [&](int a, int b) { return occ[a] < occ[b]; });
  std::vector<int> ord;
  ord.reserve(nb);
  std::vector<char> used(nb, 0);
  constexpr int WIN = 32;
  for (int s0 = 0; s0 < nb; ++s0) {
    if (used[srt[s0]]) continue;
    uint64_t u = occ[srt[s0]];
    used[srt[s0]] = 1;
    ord.push_back(srt[s0]);
    for (int c = 1; c < 16; ++c) {
      int best = -1, bgrow = 65;
      for (int q = s0 + 1, seen = 0; q < nb && seen < WIN; ++q) {
        if (used[srt[q]]) continue;
        ++seen;
        const int g = __builtin_popcountll(u | occ[srt[q]]) - __builtin_popcountll(u);
        if (g < bgrow) {
          bgrow = g;
          best = srt[q];
          if (g == 0) break;
        }
      }
      if (best < 0) break;
      used[best] = 1;
      ord.push_back(best);
      u |= occ[best];
    }
  }
  return ord;
}
}  // namespace

void Fmm::build(int64_t n, double kap, int order, int lmax, const double* tab, hipStream_t s) {
  YQ_REQUIRE(order >= 1 && order <= MAXP_FMM, YQ_EINVAL, "FMM order must be in 1..48");
  YQ_REQUIRE(lmax >= 1, YQ_EINVAL, "fmm_leaf_max must be >= 1");
  YQ_REQUIRE(dn_done && n == N && stage_dn.cap >= (size_t)n * sizeof(uint32_t) + 4 * sizeof(double),
             YQ_ESTATE, "FMM: build without a matching download");
  p = order;
  leaf_max = lmax;
  kappa = kap;
  Uploader up(s, stage_up, stage_dev);
  YQ_HIP(hipEventSynchronize(dn_done));
  root_box(reinterpret_cast<const double*>(stage_dn.p), W, x0, y0);
  const uint32_t* skey = reinterpret_cast<const uint32_t*>(stage_dn.p + 4 * sizeof(double));
  // Uniform down to the first level (>= 2) where the occupied boxes hold leaf_max
  // nodes or fewer on average, adaptive below it: boxes still over leaf_max keep
  // splitting.  (Sorted neighbours k-1, k fall in different boxes at level d exactly
  // when the highest differing bit of their keys is at or above bit 2 (DMAX - d).)
  // Splitting top-down from the root alone leaves large sparse leaves beside the
  // particles' boundary curves, whose direct lists then take whole subtrees of
  // their split neighbours: twice the direct pairs of this tree on the
  // 500-ellipse workload.
  int base = DMAX;
  {
    std::vector<int64_t> first(DMAX + 2, 0);
    for (int64_t k = 1; k < n; ++k) {
      const uint32_t x = skey[k] ^ skey[k - 1];
      if (!x) continue;
      ++first[DMAX - (31 - __builtin_clz(x)) / 2];
    }
    int64_t occ = 1;
    for (int d = 0; d <= DMAX; ++d) {
      occ += first[d];
      if (d >= 2 && (double)n / occ <= (double)leaf_max) {
        base = d;
        break;
      }
    }
  }
  const qt::Tree t = qt::build(skey, n, DMAX, leaf_max, base);
  depth = t.depth;
  max_leaf = t.max_leaf;
  p2p_pairs = t.p2p_pairs;
  p2p_srcs = 0;
  for (size_t e = 0; e < t.nbi.size(); ++e) p2p_srcs += t.leaf_cnt[t.nbi[e]];
  lv.resize(depth + 1);   // levels keep their device buffers from earlier builds
  nbox_total = 0;
  m2l_pairs = 0;
  int far_index[49];   // offset (ox+3)*7+(oy+3) -> its rank among the 40 far offsets
  for (int i = 0; i < 40; ++i) far_index[far_offset(i)] = i;
  for (int l = 0; l <= depth; ++l) {
    const qt::Level& T = t.lv[l];
    FmmLevel& L = lv[l];
    L.nbox = T.nbox();
    L.w = W / (double)(1LL << l);
    L.off = nbox_total;
    nbox_total += L.nbox;
    std::vector<double> hcx(L.nbox), hcy(L.nbox);
    for (int b = 0; b < L.nbox; ++b) {
      hcx[b] = x0 + (T.ix[b] + 0.5) * L.w;
      hcy[b] = y0 + (T.iy[b] + 0.5) * L.w;
    }
    std::vector<int> hpar(T.parent), hpos(T.cpos);
    if (l == 0) hpar[0] = -1;
    up(L.cx, hcx);
    up(L.cy, hcy);
    up(L.parent, hpar);
    up(L.cpos, hpos);
    up(L.ch, T.child);
    {
      // M2M / L2L order: boxes sorted by the set of child positions they have, so
      // that a 16-box tile skips the positions none of its boxes has (boxes along
      // curves have about two children; leaves none)
      std::vector<int> to(L.nbox);
      std::iota(to.begin(), to.end(), 0);
      auto pat = [&](int b) {
        int m = 0;
        for (int q = 0; q < 4; ++q) m |= (T.child[4 * (size_t)b + q] >= 0) << q;
        return m;
      };
      std::stable_sort(to.begin(), to.end(), [&](int a, int b) { return pat(a) < pat(b); });
      up(L.tord, to);
    }
    if (l >= 2) {
      up(L.ilp, T.ilp);
      up(L.ils, T.ils);
      up(L.ilo, T.ilo);
      std::vector<uint64_t> occ(L.nbox, 0);
      for (int b = 0; b < L.nbox; ++b)
        for (int e = T.ilp[b]; e < T.ilp[b + 1]; ++e) occ[b] |= 1ull << far_index[T.ilo[e]];
      const std::vector<int> ord = m2l_order(occ);
      std::vector<int> dense((size_t)L.nbox * 49, -1);
      L.occ.resize(L.nbox);
      for (int q = 0; q < L.nbox; ++q) {
        const int b = ord[q];
        L.occ[q] = occ[b];
        for (int e = T.ilp[b]; e < T.ilp[b + 1]; ++e) dense[(size_t)q * 49 + T.ilo[e]] = T.ils[e];
      }
      up(L.ild, dense);
      up(L.ord, ord);
      m2l_pairs += (int64_t)T.ils.size();
    }
  }
  nleaf = (int)t.leaf_level.size();
  std::vector<int> gid(nleaf);
  std::vector<double> lcx(nleaf), lcy(nleaf);
  for (int k = 0; k < nleaf; ++k) {
    const int l = t.leaf_level[k], b = t.leaf_box[k];
    gid[k] = (int)(lv[l].off + b);
    lcx[k] = x0 + (t.lv[l].ix[b] + 0.5) * lv[l].w;
    lcy[k] = y0 + (t.lv[l].iy[b] + 0.5) * lv[l].w;
  }
  up(leaf_start, t.leaf_start);
  up(leaf_cnt, t.leaf_cnt);
  {
    std::vector<int> lo(n);
    for (int k = 0; k < nleaf; ++k)
      for (int q = 0; q < t.leaf_cnt[k]; ++q) lo[t.leaf_start[k] + q] = k;
    up(leaf_of, lo);
  }
  up(leaf_gid, gid);
  up(leaf_cx, lcx);
  up(leaf_cy, lcy);
  up(nbp, t.nbp);
  up(nbi, t.nbi);
  {
    std::vector<int64_t> bo(t.nbi.size());
    int64_t acc = 0;
    for (int k = 0; k < nleaf; ++k)
      for (int e = t.nbp[k]; e < t.nbp[k + 1]; ++e) {
        bo[e] = acc;
        acc += (int64_t)t.leaf_cnt[k] * t.leaf_cnt[t.nbi[e]];
      }
    up(blk_off, bo);
    std::vector<int2> en(t.nbi.size());
    for (size_t e = 0; e < t.nbi.size(); ++e)
      en[e] = make_int2(t.leaf_start[t.nbi[e]], t.leaf_cnt[t.nbi[e]]);
    up(ent, en);
  }
  drop_near_cache();   // coefficients of the previous geometry
  qx.fit(n);
  qy.fit(n);
  up.finish();
  leaf_r.fit(std::max(nleaf, 1));
  leaf_radius_kernel<<<(nleaf + 255) / 256, 256, 0, s>>>(nleaf, leaf_start.p, leaf_cnt.p,
                                                          leaf_cx.p, leaf_cy.p, xs.p, ys.p,
                                                          leaf_r.p);
  YQ_HIP(hipGetLastError());
  set_order(order, tab, s);
}

// (Re)allocates the expansions and builds the translation tables for order q.
void Fmm::set_order(int q, const double* tab, hipStream_t s) {
  YQ_REQUIRE(q >= 1 && q <= MAXP_FMM, YQ_EINVAL, "FMM order must be in 1..48");
  p = q;
  Mall.fit((size_t)std::max<int64_t>(nbox_total, 1) * (p + 1));
  Lall.fit((size_t)std::max<int64_t>(nbox_total, 1) * (p + 1));
  for (auto& L : lv) {
    L.M = Mall.p + L.off * (p + 1);
    L.L = Lall.p + L.off * (p + 1);
  }
  const int K = 4 * p + 1;
  tg.fit((size_t)(depth + 1) * 4 * K);
  ts.fit((size_t)(depth + 1) * 49 * K);
  tab_g_kernel<<<(depth + 1) * 4, TAB_BS, 0, s>>>(p, W, kappa, tg.p);
  tab_s_kernel<<<(depth + 1) * 49, TAB_BS, 0, s>>>(p, W, kappa, tab, ts.p);
  YQ_HIP(hipGetLastError());
  R16 = ((2 * (p + 1) + 15) / 16) * 16;
  if (use_mfma) {
    const int64_t vals = (int64_t)(depth + 1) * 49 * R16 * R16;
    amat.fit((size_t)vals);
    trans_amat_kernel<<<(unsigned)((vals + 255) / 256), 256, 0, s>>>(depth + 1, 49, p, R16, 1, 1, ts.p,
                                                                       amat.p);
    const int64_t gvals = (int64_t)(depth + 1) * 4 * R16 * R16;
    gmat.fit((size_t)gvals);
    trans_amat_kernel<<<(unsigned)((gvals + 255) / 256), 256, 0, s>>>(depth + 1, 4, p, R16, 0, 0, tg.p,
                                                                        gmat.p);
    YQ_HIP(hipGetLastError());
    // 16-box tiles of every level with M2L terms, finest level first
    Uploader up(s, stage_up, stage_dev);
    std::vector<int4> ht;
    for (int l = depth; l >= 2; --l)
      for (int b = 0; b < lv[l].nbox; b += 16) {
        uint64_t u = 0;
        for (int q = b; q < std::min(b + 16, lv[l].nbox); ++q) u |= lv[l].occ[q];
        ht.push_back(make_int4(l, b, (int)(uint32_t)u, (int)(uint32_t)(u >> 32)));
      }
    up(m2l_tiles, ht);
    if (want_m2l32) {
      // s_n = n! (2 / (kappa w_l))^n, in logarithms (the factors themselves span
      // hundreds of decades across levels and orders; each stays within FP64)
      std::vector<double> hs((size_t)(depth + 1) * (p + 1));
      for (int l = 0; l <= depth; ++l)
        for (int n = 0; n <= p; ++n)
          hs[(size_t)l * (p + 1) + n] =
              std::exp(std::lgamma(n + 1.0) + n * std::log(2.0 / (kappa * lv[l].w)));
      up(msc, hs);
      amat32.fit((size_t)vals);
    }
    up.finish();
    n_m2l_tiles = (int)ht.size();
    if (want_m2l32) {
      trans_amat32_kernel<<<(unsigned)((vals + 255) / 256), 256, 0, s>>>(depth + 1, p, R16, amat.p,
                                                                         msc.p, amat32.p);
      YQ_HIP(hipGetLastError());
    }
  }
  YQ_HIP(hipStreamSynchronize(s));
  built = true;
}

// A second expansion order on the same tree: copies the tree (device to device).
void Fmm::copy_tree(const Fmm& o, int q, const double* tab, hipStream_t s) {
  drop_near_cache();   // coefficients of the previous geometry
  // the device-to-device copies go in one batch_copy_kernel launch
  std::vector<CopyItem> cp;
  auto dup = [&](auto& dst, const auto& src) {
    using T = std::remove_pointer_t<decltype(src.p)>;
    static_assert(sizeof(T) % 4 == 0, "copies move 32-bit words");
    dst.fit(std::max<size_t>(src.n, 1));
    if (src.n) cp.push_back(CopyItem{dst.p, src.p, (int64_t)(src.n * sizeof(T) / 4)});
  };
  depth = o.depth;
  leaf_max = o.leaf_max;
  x0 = o.x0;
  y0 = o.y0;
  W = o.W;
  kappa = o.kappa;
  N = o.N;
  max_leaf = o.max_leaf;
  nbox_total = o.nbox_total;
  nleaf = o.nleaf;
  p2p_pairs = o.p2p_pairs;
  p2p_srcs = o.p2p_srcs;
  m2l_pairs = o.m2l_pairs;
  lv.resize(o.lv.size());
  for (size_t l = 0; l < o.lv.size(); ++l) {
    lv[l].nbox = o.lv[l].nbox;
    lv[l].w = o.lv[l].w;
    lv[l].off = o.lv[l].off;
    dup(lv[l].cx, o.lv[l].cx);
    dup(lv[l].cy, o.lv[l].cy);
    dup(lv[l].parent, o.lv[l].parent);
    dup(lv[l].cpos, o.lv[l].cpos);
    dup(lv[l].ch, o.lv[l].ch);
    dup(lv[l].tord, o.lv[l].tord);
    if (l >= 2) {
      dup(lv[l].ilp, o.lv[l].ilp);
      dup(lv[l].ils, o.lv[l].ils);
      dup(lv[l].ilo, o.lv[l].ilo);
      dup(lv[l].ild, o.lv[l].ild);
      dup(lv[l].ord, o.lv[l].ord);
      lv[l].occ = o.lv[l].occ;
    }
  }
  dup(perm, o.perm);
  dup(xs, o.xs);
  dup(ys, o.ys);
  dup(wnxs, o.wnxs);
  dup(wnys, o.wnys);
  dup(leaf_start, o.leaf_start);
  dup(leaf_cnt, o.leaf_cnt);
  dup(leaf_gid, o.leaf_gid);
  dup(leaf_cx, o.leaf_cx);
  dup(leaf_cy, o.leaf_cy);
  dup(leaf_r, o.leaf_r);
  dup(blk_off, o.blk_off);
  dup(ent, o.ent);
  dup(leaf_of, o.leaf_of);
  dup(nbp, o.nbp);
  dup(nbi, o.nbi);
  if (!cp.empty()) {
    const size_t tb = cp.size() * sizeof(CopyItem);
    stage_up.fit(tb);
    stage_dev.fit(tb);
    std::memcpy(stage_up.p, cp.data(), tb);
    YQ_HIP(hipMemcpyAsync(stage_dev.p, stage_up.p, tb, hipMemcpyHostToDevice, s));
    batch_copy_kernel<<<dim3((unsigned)cp.size(), COPY_SLICES), 256, 0, s>>>(
        reinterpret_cast<const CopyItem*>(stage_dev.p));
    YQ_HIP(hipGetLastError());
    YQ_HIP(hipStreamSynchronize(s));   // before the stages are reused
  }
  qx.fit(N);
  qy.fit(N);
  set_order(q, tab, s);
}

M2LLevels Fmm::m2l_levels() const {
  M2LLevels a{};
  for (int l = 0; l <= depth; ++l) {
    a.ild[l] = l >= 2 ? lv[l].ild.p : nullptr;
    a.ord[l] = l >= 2 ? lv[l].ord.p : nullptr;
    a.M[l] = lv[l].M;
    a.L[l] = lv[l].L;
    a.nbox[l] = lv[l].nbox;
    a.off[l] = lv[l].off;
  }
  a.off[depth + 1] = nbox_total;
  return a;
}

// Packs the multipoles of levels >= 2 (m2l_pack_kernel) and runs the M2L of all
// levels in one launch, one block per 16-box tile.
template <typename T>
void Fmm::m2l_run(hipStream_t s, const int* stop, DevBuf<T>& mp, const T* A) {
  if (n_m2l_tiles == 0 || depth < 2) return;
  const M2LLevels a = m2l_levels();
  const int64_t g0 = lv[2].off, g1 = nbox_total;
  mp.fit((size_t)nbox_total * R16);
  const int64_t nt = (g1 - g0) * R16;
  m2l_pack_kernel<T><<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(p, R16, g0, g1, a, Mall.p, msc.p,
                                                                   mp.p);
  YQ_HIP(hipGetLastError());
  const unsigned g = (unsigned)n_m2l_tiles;
#define YQ_M2L(rt) m2l_mfma_kernel<T, rt><<<g, 256, 0, s>>>(p, m2l_tiles.p, a, A, mp.p, msc.p, stop)
  switch (R16 / 16) {
    case 1: YQ_M2L(1); break;
    case 2: YQ_M2L(2); break;
    case 3: YQ_M2L(3); break;
    case 4: YQ_M2L(4); break;
    case 5: YQ_M2L(5); break;
    case 6: YQ_M2L(6); break;
    default: YQ_M2L(7); break;
  }
#undef YQ_M2L
  YQ_HIP(hipGetLastError());
}

void Fmm::m2l_mfma(hipStream_t s, const int* stop) { m2l_run<double>(s, stop, mpk64, amat.p); }

void Fmm::m2l_mfma32(hipStream_t s, const int* stop) { m2l_run<float>(s, stop, mpk32, amat32.p); }

// M2M into parent level l (gather) or L2L from parent level l (scatter), both
// with the child level's position matrices.
void Fmm::tree_mfma(bool gather, int l, hipStream_t s) {
  const int nb = lv[l].nbox;
  if (nb == 0) return;
  const int RT = R16 / 16;
  const int ni = ((nb + 15) / 16) * RT;   // one wave per (tile, row tile)
  const unsigned g = (unsigned)((ni + 3) / 4);
  const double* A = gmat.p + (size_t)(l + 1) * 4 * R16 * R16;
  const double2* X = gather ? lv[l + 1].M : lv[l].L;
  double2* Y = gather ? lv[l].M : lv[l + 1].L;
  const int* ch = lv[l].ch.p;
  const int* od = lv[l].tord.p;
#define YQ_TREE(rt)                                                                  \
  if (gather)                                                                        \
    tree_mfma_kernel<rt, true><<<g, 256, 0, s>>>(p, nb, ni, ch, od, X, A, Y);         \
  else                                                                               \
    tree_mfma_kernel<rt, false><<<g, 256, 0, s>>>(p, nb, ni, ch, od, X, A, Y);
  switch (RT) {
    case 1: YQ_TREE(1) break;
    case 2: YQ_TREE(2) break;
    case 3: YQ_TREE(3) break;
    case 4: YQ_TREE(4) break;
    case 5: YQ_TREE(5) break;
    case 6: YQ_TREE(6) break;
    default: YQ_TREE(7) break;
  }
#undef YQ_TREE
  YQ_HIP(hipGetLastError());
}

// Multipole and local expansions of the leaves for density sigma (upward pass,
// M2L, downward pass).
void Fmm::expansions(const double* sigma, hipStream_t s, bool m2l32, const int* stop) {
  YQ_REQUIRE(built, YQ_ESTATE, "FMM tree not built");
  const int K = 4 * p + 1;
  gather_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(N, perm.p, sigma, wnxs.p, wnys.p, qx.p,
                                                            qy.p, nc_kind ? ss.p : nullptr);
  const int col = p <= kColMaxOrder;
  p2m_kernel<<<nleaf, 64, col ? (size_t)(p + 2) * 64 * sizeof(double) : 0, s>>>(
      p, col, kappa, leaf_start.p, leaf_cnt.p, leaf_gid.p, leaf_cx.p, leaf_cy.p, xs.p, ys.p, qx.p,
      qy.p, Mall.p, stop);
  for (int l = depth - 1; l >= 2; --l) {
    if (use_mfma) {
      tree_mfma(true, l, s);
      continue;
    }
    const int64_t nt = (int64_t)lv[l].nbox * (p + 1);
    m2m_kernel<<<(unsigned)((nt + 127) / 128), 128, 0, s>>>(p, lv[l].nbox, lv[l].ch.p, lv[l + 1].M,
                                                            tg.p + (size_t)(l + 1) * 4 * K,
                                                            lv[l].M);
  }
  if (use_mfma && m2l32) {
    m2l_mfma32(s, stop);
  } else if (use_mfma) {
    m2l_mfma(s, stop);
  } else {
    for (int l = 2; l <= depth; ++l) {
      const int64_t nt = (int64_t)lv[l].nbox * (p + 1);
      m2l_kernel<<<(unsigned)((nt + 127) / 128), 128, 0, s>>>(p, lv[l].nbox, lv[l].ilp.p, lv[l].ils.p,
                                                              lv[l].ilo.p, lv[l].M,
                                                              ts.p + (size_t)l * 49 * K, lv[l].L);
    }
  }
  for (int l = 2; l < depth; ++l) {
    if (use_mfma) {
      tree_mfma(false, l, s);
      continue;
    }
    const int64_t nt = (int64_t)lv[l + 1].nbox * (p + 1);
    l2l_kernel<<<(unsigned)((nt + 127) / 128), 128, 0, s>>>(p, lv[l + 1].nbox, lv[l + 1].parent.p,
                                                            lv[l + 1].cpos.p, lv[l].L,
                                                            tg.p + (size_t)(l + 1) * 4 * K,
                                                            lv[l + 1].L);
  }
}

void Fmm::apply(const double* sigma, double* partial, bool p2p_fp32, const double* tab,
                hipStream_t s, const int* stop) {
  // the FP32-class (inner) operator also takes its M2L in FP32 when that is set up
  expansions(sigma, s, p2p_fp32 && want_m2l32 && use_mfma, stop);
  l2p_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(N, p, kappa, leaf_of.p, leaf_gid.p,
                                                         leaf_cx.p, leaf_cy.p, xs.p, ys.p, perm.p,
                                                         Lall.p, partial, stop);
  const int nw = nleaf >= kLeavesFor2 ? 2 : PW;
  // the near-field cache of the apply's precision, if computed
  // (a cache holding folded QBX corrections serves only the engine, whose finish
  // leaves them out; here the caller's finish adds them)
  const void* cache = nc_folded ? nullptr
                      : p2p_fp32 ? (nc_kind == 1 ? (const void*)nc32.p : nullptr)
                                 : (nc_kind == 2 ? (const void*)nc64.p : nullptr);
  if (cache) {
    auto k = p2p_fp32 ? p2p_cached_kernel<true> : p2p_cached_kernel<false>;
    k<<<(nleaf + CW - 1) / CW, FB * CW, 0, s>>>(nleaf, leaf_start.p, leaf_cnt.p, nbp.p, ent.p,
                                                blk_off.p, cache, ss.p, perm.p, partial, stop);
  } else {
    auto k = p2p_fp32 ? (nw == 2 ? p2p_kernel<true, 2> : p2p_kernel<true, PW>)
                      : (nw == 2 ? p2p_kernel<false, 2> : p2p_kernel<false, PW>);
    k<<<nleaf, FB * nw, leaf_lds_bytes(nw), s>>>(kappa, leaf_start.p, leaf_cnt.p, nbp.p, nbi.p,
                                                 leaf_cx.p, leaf_cy.p, leaf_r.p, xs.p, ys.p, qx.p,
                                                 qy.p, perm.p, tab, partial, stop);
  }
  YQ_HIP(hipGetLastError());
}

// Near-field cache: one wave per leaf computes the coefficients of every pair of its
// P2P list with the leaf passes' arithmetic (FP64: far64_tile's terms, the self
// pair 0; FP32: far32_tile's, positions differenced in FP64) without the density:
// K1(z)/z ((x_i - y_k) . w_k nu_k) at boff[e] + k cnt + i.
template <bool F64>
__global__ __launch_bounds__(64) void near_cache_kernel(
    const int* __restrict__ ls, const int* __restrict__ lc, const int* __restrict__ nbp,
    const int* __restrict__ nbi, const int64_t* __restrict__ boff, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ wnxs,
    const double* __restrict__ wnys, double kappa, const double* __restrict__ tab, void* out) {
  const int b = blockIdx.x, lane = threadIdx.x;
  const int s0 = ls[b], cnt = lc[b];
  const double kap2 = kappa * kappa;
  for (int r0 = 0; r0 < cnt; r0 += 64) {
    const int i = r0 + lane;
    const bool act = i < cnt;
    const double xi = act ? xs[s0 + i] : 0.0, yi = act ? ys[s0 + i] : 0.0;
    for (int e = nbp[b]; e < nbp[b + 1]; ++e) {
      const int nb = nbi[e];
      const int t0 = ls[nb], tc = lc[nb];
      const int64_t bo = boff[e];
      for (int k = 0; k < tc; ++k) {
        const double xk = xs[t0 + k], yk = ys[t0 + k], wx = wnxs[t0 + k], wy = wnys[t0 + k];
        if (F64) {
          const double dx = xi - xk, dy = yi - yk;
          const double r2 = fma(dx, dx, dy * dy);
          const double v = k1z_64(kap2 * r2, tab) * fma(dx, wx, dy * wy);
          if (act) static_cast<double*>(out)[bo + (int64_t)k * cnt + i] = r2 > 0.0 ? v : 0.0;
        } else {
          const float dx = (float)(xi - xk), dy = (float)(yi - yk);
          const float z2 = fmaxf((float)kap2 * fmaf(dx, dx, dy * dy), 1e-30f);
          const float v = k1z_32(z2) * fmaf(dx, (float)wx, dy * (float)wy);
          if (act) static_cast<float*>(out)[bo + (int64_t)k * cnt + i] = v;
        }
      }
    }
  }
}

__global__ __launch_bounds__(64) void p2m_coef_kernel(int p, int use_col, double kappa,
                                                      const int* __restrict__ ls,
                                                      const int* __restrict__ lc,
                                                      const int* __restrict__ gid,
                                                      const double* __restrict__ ccx,
                                                      const double* __restrict__ ccy,
                                                      const double* __restrict__ xs,
                                                      const double* __restrict__ ys,
                                                      const double* __restrict__ wnxs,
                                                      const double* __restrict__ wnys,
                                                      float* __restrict__ coef) {
  extern __shared__ double itab[];
  p2m_leaf<true>(blockIdx.x, p, use_col, kappa, ls, lc, gid, ccx, ccy, xs, ys, wnxs, wnys, nullptr,
                 itab, coef);
}

void Fmm::build_near_cache(bool f64, const double* tab, hipStream_t s) {
  YQ_REQUIRE(nleaf > 0 && blk_off.p, YQ_ESTATE, "FMM tree not built");
  YQ_REQUIRE(max_leaf <= 64, YQ_EINVAL, "near-field cache: leaves of more than 64 nodes");
  drop_near_cache();
  const size_t np = (size_t)std::max<int64_t>(p2p_pairs, 1);
  void* out;
  if (f64) {
    nc64.fit(np);
    out = nc64.p;
  } else {
    nc32.fit(np);
    out = nc32.p;
  }
  ss.fit(std::max<int64_t>(N, 1));
  nc_folded = nullptr;
  auto k = f64 ? near_cache_kernel<true> : near_cache_kernel<false>;
  k<<<nleaf, 64, 0, s>>>(leaf_start.p, leaf_cnt.p, nbp.p, nbi.p, blk_off.p, xs.p, ys.p, wnxs.p,
                         wnys.p, kappa, tab, out);
  YQ_HIP(hipGetLastError());
  if (!f64) {   // the inner operator's P2M coefficients
    pc32.fit((size_t)std::max<int64_t>(N, 1) * 2 * (p + 1));
    const int col = p <= kColMaxOrder;
    p2m_coef_kernel<<<nleaf, 64, col ? (size_t)(p + 2) * 64 * sizeof(double) : 0, s>>>(
        p, col, kappa, leaf_start.p, leaf_cnt.p, leaf_gid.p, leaf_cx.p, leaf_cy.p, xs.p, ys.p,
        wnxs.p, wnys.p, pc32.p);
    YQ_HIP(hipGetLastError());
  }
  nc_kind = f64 ? 2 : 1;
}

void Fmm::drop_near_cache() {
  nc_folded = nullptr;
  nc32.release();
  nc64.release();
  ss.release();
  pc32.release();
  nc_kind = 0;
}

void Fmm::apply_grad(const double* sigma, double* gpart, const double* tab, hipStream_t s) {
  expansions(sigma, s);
  const int col = p <= kColMaxOrder;
  const size_t sh = leaf_grad_lds_bytes(p, col);
  l2p_p2p_grad_kernel<<<nleaf, FB * PW, sh, s>>>(p, col, kappa, leaf_start.p, leaf_cnt.p,
                                                  leaf_gid.p, nbp.p, nbi.p, leaf_cx.p, leaf_cy.p,
                                                  leaf_r.p, Lall.p, xs.p, ys.p, qx.p, qy.p, perm.p,
                                                  N, tab, gpart);
  YQ_HIP(hipGetLastError());
}

// ---- forest: one launch per pass over many trees ------------------------------------------
//
// Every block reads its work item (member, index), skips the member when its batch
// configuration is masked off, and runs the same body as the single-tree kernel's
// block of that index, so each tree's sums are those of Fmm::apply.

__global__ void forest_gather_kernel(const FmmDev* __restrict__ fd, const int2* __restrict__ items,
                                     const int* __restrict__ mask, const double* __restrict__ V,
                                     const int* __restrict__ col, int64_t T) {
  const int2 it = items[blockIdx.x];
  const FmmDev& d = fd[it.x];
  if (!mask[d.cfg]) return;
  const int64_t k = (int64_t)it.y * 256 + threadIdx.x;
  if (k >= d.N) return;
  const double* sigma = V + (col ? (int64_t)col[d.cfg] * T : 0) + d.off;
  if (d.pc32) {   // P2M and the leaf pass both read the cache: only the sorted densities
    as_gm(d.ss)[k] = as_g(sigma)[as_g(d.perm)[k]];
    return;
  }
  gather_one(k, d.perm, sigma, d.wnxs, d.wnys, d.qx, d.qy, d.ss);
}

__global__ __launch_bounds__(64) void forest_p2m_kernel(const FmmDev* __restrict__ fd,
                                                        const int2* __restrict__ items,
                                                        const int* __restrict__ mask, int p,
                                                        int use_col) {
  extern __shared__ double itab[];
  const int2 it = items[blockIdx.x];
  const FmmDev& d = fd[it.x];
  if (!mask[d.cfg]) return;
  p2m_leaf_any(it.y, p, use_col, d.kappa, d.leaf_start, d.leaf_cnt, d.leaf_gid, d.leaf_cx,
               d.leaf_cy, d.xs, d.ys, d.qx, d.qy, d.Mall, itab);
}

// P2M of the trees holding the P2M coefficients: items (member, leaf), CW per block.
__global__ __launch_bounds__(FB * CW) void forest_cp2m_kernel(const FmmDev* __restrict__ fd,
                                                              const int2* __restrict__ items,
                                                              int n, const int* __restrict__ mask,
                                                              int p) {
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FB));
  const int i = blockIdx.x * CW + w;
  if (i >= n) return;
  const int2 it = items[i];
  const FmmDev& d = fd[it.x];
  if (!mask[d.cfg]) return;
  p2m_cached_wave(it.y, p, d.leaf_start, d.leaf_cnt, d.leaf_gid, d.pc32, d.ss, d.Mall);
}

// M2M into parent level l (GATHER) or L2L out of it, for every member deep enough.
template <int RT, bool GATHER>
__global__ __launch_bounds__(256) void forest_tree_kernel(const FmmDev* __restrict__ fd,
                                                          const int2* __restrict__ items, int n,
                                                          const int* __restrict__ mask, int p,
                                                          int l) {
  const int i = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (i >= n) return;
  const int2 it = items[i];
  const FmmDev& d = fd[it.x];
  if (!mask[d.cfg]) return;
  constexpr int R = RT * 16;
  const double* A = d.gmat + (size_t)(l + 1) * 4 * R * R;
  const double2* X = GATHER ? d.lv.M[l + 1] : d.lv.L[l];
  double2* Y = GATHER ? const_cast<double2*>(d.lv.M[l]) : d.lv.L[l + 1];
  tree_tile<RT, GATHER>(it.y, p, d.lv.nbox[l], d.ch[l], d.tord[l], X, A, Y);
}

template <typename T>
__global__ void forest_pack_kernel(const FmmDev* __restrict__ fd, const int2* __restrict__ items,
                                   const int* __restrict__ mask, int p, int R) {
  const int2 it = items[blockIdx.x];
  const FmmDev& d = fd[it.x];
  if (!mask[d.cfg]) return;
  const int64_t g0 = d.lv.off[2], g1 = d.lv.off[d.depth + 1];
  const int64_t t = (int64_t)it.y * 256 + threadIdx.x;
  if (t >= (g1 - g0) * R) return;
  m2l_pack_one<T>(t, p, R, g0, d.lv, d.Mall, d.msc, static_cast<T*>(d.mpk));
}

template <typename T, int RT>
__global__ __launch_bounds__(256) void forest_m2l_kernel(const FmmDev* __restrict__ fd,
                                                         const int2* __restrict__ items,
                                                         const int* __restrict__ mask, int p) {
  __shared__ dbl4 red[3 * RT * 64];
  const int2 it = items[blockIdx.x];
  const FmmDev& d = fd[it.x];
  if (!mask[d.cfg]) return;
  m2l_tile<T, RT>(d.m2l_tiles[it.y], p, d.lv, static_cast<const T*>(d.amat),
                  static_cast<const T*>(d.mpk), d.msc, red);
}

template <bool F32, int NW>
__global__ __launch_bounds__(FB * NW) void forest_leaf_kernel(const FmmDev* __restrict__ fd,
                                                              const int2* __restrict__ items,
                                                              const int* __restrict__ mask) {
  extern __shared__ double sh[];
  const int2 it = items[blockIdx.x];
  const FmmDev& d = fd[it.x];
  if (!mask[d.cfg]) return;
  // (the Bessel table through scalar loads, as from a kernel argument)
  leaf_pass<F32, NW>(it.y, d.kappa, d.leaf_start, d.leaf_cnt, d.nbp, d.nbi, d.leaf_cx, d.leaf_cy,
                     d.leaf_r, d.xs, d.ys, d.qx, d.qy, d.perm, (const double*)as_k(d.tab), d.out,
                     sh);
}

// The cached leaf pass over the forest: items (member, leaf) of trees holding the
// cache of the forest's precision, CW per block.
template <bool F32>
__global__ __launch_bounds__(FB * CW) void forest_cleaf_kernel(const FmmDev* __restrict__ fd,
                                                               const int2* __restrict__ items,
                                                               int n, const int* __restrict__ mask) {
  __shared__ double red[CW][FB];
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FB));
  const int i = blockIdx.x * CW + w;
  if (i >= n) return;
  const int2 it = items[i];
  const FmmDev& d = fd[it.x];
  if (!mask[d.cfg]) return;
  leaf_cached_wave<F32>(it.y, d.leaf_start, d.leaf_cnt, d.nbp, d.ent, d.blk_off, d.nc, d.ss, d.perm,
                        d.out, red[w]);
}

// l2p_kernel over the forest: items (member, 256-node block of its sorted nodes).
__global__ __launch_bounds__(256) void forest_l2p_kernel(const FmmDev* __restrict__ fd,
                                                         const int2* __restrict__ items,
                                                         const int* __restrict__ mask, int p) {
  const int2 it = items[blockIdx.x];
  const FmmDev& d = fd[it.x];
  if (!mask[d.cfg]) return;
  const int64_t k = (int64_t)it.y * 256 + threadIdx.x;
  if (k >= d.N) return;
  l2p_node(k, p, d.kappa, d.leaf_of, d.leaf_gid, d.leaf_cx, d.leaf_cy, d.xs, d.ys, d.perm, d.Lall,
           d.out);
}

// Profiling: adds the source-target pairs of the leaf passes of the trees in mask
// (each tree's count from its build) to pairs[0], and the algorithmic bytes of the
// cached trees' passes to pairs[1]: coefficients (4 or 8 bytes per pair), each
// target's output read and written (16), each entry's source densities (8 per source).
__global__ __launch_bounds__(256) void forest_count_pairs_kernel(const FmmDev* __restrict__ fd,
                                                                 int nmem,
                                                                 const int* __restrict__ mask,
                                                                 int f32,
                                                                 unsigned long long* __restrict__ pairs) {
  __shared__ unsigned long long part[2][256];
  unsigned long long s = 0, by = 0;
  for (int m = threadIdx.x; m < nmem; m += blockDim.x)
    if (mask[fd[m].cfg]) {
      const FmmDev& d = fd[m];
      s += (unsigned long long)d.p2p_pairs;
      if (d.nc)
        by += (unsigned long long)(d.p2p_pairs * (f32 ? 4 : 8) + 16 * d.N + 8 * d.p2p_srcs);
    }
  part[0][threadIdx.x] = s;
  part[1][threadIdx.x] = by;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      part[0][threadIdx.x] += part[0][threadIdx.x + h];
      part[1][threadIdx.x] += part[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(pairs, part[0][0]);
    atomicAdd(pairs + 1, part[1][0]);
  }
}

__global__ __launch_bounds__(FB * PW) void forest_leaf_grad_kernel(const FmmDev* __restrict__ fd,
                                                                  const int2* __restrict__ items,
                                                                  const int* __restrict__ mask,
                                                                  int p, int use_col) {
  extern __shared__ double sh[];
  const int2 it = items[blockIdx.x];
  const FmmDev& d = fd[it.x];
  if (!mask[d.cfg]) return;
  leaf_grad_pass(it.y, p, use_col, d.kappa, d.leaf_start, d.leaf_cnt, d.leaf_gid, d.nbp, d.nbi,
                 d.leaf_cx, d.leaf_cy, d.leaf_r, d.Lall, d.xs, d.ys, d.qx, d.qy, d.perm, d.N,
                 (const double*)as_k(d.tab), d.gout, sh);
}

namespace {


template <class V>
void upload_items(DevBuf<V>& d, const std::vector<V>& h, hipStream_t s) {
  d.fit(std::max<size_t>(h.size(), 1));
  if (!h.empty())
    YQ_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, s));
}

}  // namespace

void FmmForest::build(const std::vector<Tree>& trees, bool p2p32, hipStream_t s) {
  nmem = (int)trees.size();
  f32 = p2p32;
  depth = 0;
  n_gather = n_p2m = n_cp2m = n_pack = n_m2l = n_leaf2 = n_leaf4 = n_cleaf = n_leaves = 0;
  if (nmem == 0) return;
  p = trees[0].fmm->p;
  R16 = trees[0].fmm->R16;
  m2l32 = p2p32 && trees[0].fmm->want_m2l32;
  std::vector<FmmDev> h(nmem);
  std::vector<int2> g, pm, cp, pk, ml, l2, l4, cl, la;
  std::vector<std::vector<int2>> tr(DMAX + 1);
  for (int m = 0; m < nmem; ++m) {
    Fmm& f = *trees[m].fmm;
    YQ_REQUIRE(f.built && f.p == p && f.R16 == R16 && f.use_mfma &&
                   (p2p32 ? f.want_m2l32 == trees[0].fmm->want_m2l32 : true),
               YQ_EINVAL, "FMM forest: trees of different orders or translation modes");
    FmmDev& d = h[m];
    std::memset(&d, 0, sizeof(d));
    d.cfg = trees[m].cfg;
    d.depth = f.depth;
    d.nleaf = f.nleaf;
    d.N = f.N;
    d.off = trees[m].off;
    d.kappa = f.kappa;
    d.perm = f.perm.p;
    d.xs = f.xs.p;
    d.ys = f.ys.p;
    d.wnxs = f.wnxs.p;
    d.wnys = f.wnys.p;
    d.qx = f.qx.p;
    d.qy = f.qy.p;
    d.leaf_start = f.leaf_start.p;
    d.leaf_cnt = f.leaf_cnt.p;
    d.leaf_gid = f.leaf_gid.p;
    d.nbp = f.nbp.p;
    d.nbi = f.nbi.p;
    d.leaf_cx = f.leaf_cx.p;
    d.leaf_cy = f.leaf_cy.p;
    d.leaf_r = f.leaf_r.p;
    d.leaf_of = f.leaf_of.p;
    d.p2p_pairs = f.p2p_pairs;
    d.p2p_srcs = f.p2p_srcs;
    // the tree's near-field cache when it holds this forest's precision
    const bool cached = p2p32 ? f.nc_kind == 1 : f.nc_kind == 2;
    d.blk_off = f.blk_off.p;
    d.ent = f.ent.p;
    d.nc = cached ? (p2p32 ? (const void*)f.nc32.p : (const void*)f.nc64.p) : nullptr;
    d.nc_kind = cached ? f.nc_kind : 0;
    d.ss = cached ? f.ss.p : nullptr;
    d.pc32 = cached && p2p32 && f.pc32.p ? f.pc32.p : nullptr;
    d.Mall = f.Mall.p;
    d.Lall = f.Lall.p;
    d.lv = f.m2l_levels();
    for (int l = 0; l <= f.depth; ++l) {
      d.ch[l] = f.lv[l].ch.p;
      d.tord[l] = f.lv[l].tord.p;
    }
    d.gmat = f.gmat.p;
    d.msc = f.msc.p;
    d.m2l_tiles = f.m2l_tiles.p;
    d.tab = trees[m].tab;
    d.out = trees[m].out;
    d.gout = trees[m].gout;
    if (m2l32) {
      f.mpk32.fit((size_t)f.nbox_total * R16);
      d.amat = f.amat32.p;
      d.mpk = f.mpk32.p;
    } else {
      f.mpk64.fit((size_t)f.nbox_total * R16);
      d.amat = f.amat.p;
      d.mpk = f.mpk64.p;
    }
    depth = std::max(depth, f.depth);
    for (int64_t b = 0; b < (f.N + 255) / 256; ++b) g.push_back(make_int2(m, (int)b));
    for (int b = 0; b < f.nleaf; ++b) (d.pc32 ? cp : pm).push_back(make_int2(m, b));
    const int RT = R16 / 16;
    for (int l = 2; l < f.depth; ++l) {
      const int nb = f.lv[l].nbox;
      for (int bx = 0; bx < ((nb + 15) / 16) * RT; ++bx) tr[l].push_back(make_int2(m, bx));
    }
    if (f.n_m2l_tiles > 0 && f.depth >= 2) {
      const int64_t ne = (f.nbox_total - f.lv[2].off) * R16;
      for (int64_t b = 0; b < (ne + 255) / 256; ++b) pk.push_back(make_int2(m, (int)b));
      for (int t = 0; t < f.n_m2l_tiles; ++t) ml.push_back(make_int2(m, t));
    }
    auto& lst = cached ? cl : f.nleaf >= kLeavesFor2 ? l2 : l4;
    for (int b = 0; b < f.nleaf; ++b) {
      lst.push_back(make_int2(m, b));
      la.push_back(make_int2(m, b));   // every leaf (the gradient pass takes PW waves for all)
    }
  }
  dev.fit(nmem);
  YQ_HIP(hipMemcpyAsync(dev.p, h.data(), nmem * sizeof(FmmDev), hipMemcpyHostToDevice, s));
  upload_items(it_gather, g, s);
  upload_items(it_p2m, pm, s);
  upload_items(it_cp2m, cp, s);
  n_cp2m = (int)cp.size();
  upload_items(it_pack, pk, s);
  upload_items(it_m2l, ml, s);
  upload_items(it_leaf2, l2, s);
  upload_items(it_leaf4, l4, s);
  upload_items(it_leaves, la, s);
  upload_items(it_cleaf, cl, s);
  n_cleaf = (int)cl.size();
  n_leaves = (int)la.size();
  n_gather = (int)g.size();
  n_p2m = (int)pm.size();
  n_pack = (int)pk.size();
  n_m2l = (int)ml.size();
  n_leaf2 = (int)l2.size();
  n_leaf4 = (int)l4.size();
  it_tree.resize(DMAX + 1);
  n_tree.assign(DMAX + 1, 0);
  for (int l = 0; l <= DMAX; ++l) {
    upload_items(it_tree[l], tr[l], s);
    n_tree[l] = (int)tr[l].size();
  }
  YQ_HIP(hipStreamSynchronize(s));   // the host lists above are released on return
}

void FmmForest::apply(const int* mask, const double* V, const int* col, int64_t T,
                      hipStream_t s) const {
  expansions(mask, V, col, T, s);
  l2p(mask, s);
  leaves(mask, s);
}

void FmmForest::l2p(const int* mask, hipStream_t s) const {
  if (nmem == 0 || n_gather == 0) return;
  forest_l2p_kernel<<<n_gather, 256, 0, s>>>(dev.p, it_gather.p, mask, p);
  YQ_HIP(hipGetLastError());
}

void FmmForest::leaves(const int* mask, hipStream_t s, unsigned long long* pairs) const {
  if (nmem == 0) return;
  if (n_leaf2) {
    auto k = f32 ? forest_leaf_kernel<true, 2> : forest_leaf_kernel<false, 2>;
    k<<<n_leaf2, FB * 2, leaf_lds_bytes(2), s>>>(dev.p, it_leaf2.p, mask);
  }
  if (n_leaf4) {
    auto k = f32 ? forest_leaf_kernel<true, PW> : forest_leaf_kernel<false, PW>;
    k<<<n_leaf4, FB * PW, leaf_lds_bytes(PW), s>>>(dev.p, it_leaf4.p, mask);
  }
  if (n_cleaf) {
    auto k = f32 ? forest_cleaf_kernel<true> : forest_cleaf_kernel<false>;
    k<<<(n_cleaf + CW - 1) / CW, FB * CW, 0, s>>>(dev.p, it_cleaf.p, n_cleaf, mask);
  }
  if (pairs) forest_count_pairs_kernel<<<1, 256, 0, s>>>(dev.p, nmem, mask, f32, pairs);
  YQ_HIP(hipGetLastError());
}

void FmmForest::apply_grad(const int* mask, const double* V, const int* col, int64_t T,
                           hipStream_t s) const {
  expansions(mask, V, col, T, s);
  leaves_grad(mask, s);
}

void FmmForest::leaves_grad(const int* mask, hipStream_t s) const {
  YQ_REQUIRE(!f32, YQ_EINVAL, "FMM forest: the gradient is FP64");
  if (nmem == 0) return;
  const int use_col = p <= kColMaxOrder;
  const int nl = n_leaves;
  if (nl)
    forest_leaf_grad_kernel<<<nl, FB * PW, leaf_grad_lds_bytes(p, use_col), s>>>(
        dev.p, it_leaves.p, mask, p, use_col);
  YQ_HIP(hipGetLastError());
}

void FmmForest::expansions(const int* mask, const double* V, const int* col, int64_t T,
                           hipStream_t s) const {
  if (nmem == 0) return;
  const int use_col = p <= kColMaxOrder;
  const int RT = R16 / 16;
  if (n_gather)
    forest_gather_kernel<<<n_gather, 256, 0, s>>>(dev.p, it_gather.p, mask, V, col, T);
  if (n_p2m)
    forest_p2m_kernel<<<n_p2m, 64, use_col ? (size_t)(p + 2) * 64 * sizeof(double) : 0, s>>>(
        dev.p, it_p2m.p, mask, p, use_col);
  if (n_cp2m)
    forest_cp2m_kernel<<<(n_cp2m + CW - 1) / CW, FB * CW, 0, s>>>(dev.p, it_cp2m.p, n_cp2m, mask,
                                                                  p);
  YQ_HIP(hipGetLastError());
#define YQ_FTREE(rt, G) \
  forest_tree_kernel<rt, G><<<(n_tree[l] + 3) / 4, 256, 0, s>>>(dev.p, it_tree[l].p, n_tree[l], \
                                                                mask, p, l)
#define YQ_FTREE_ALL(G)                 \
  switch (RT) {                         \
    case 1: YQ_FTREE(1, G); break;      \
    case 2: YQ_FTREE(2, G); break;      \
    case 3: YQ_FTREE(3, G); break;      \
    case 4: YQ_FTREE(4, G); break;      \
    case 5: YQ_FTREE(5, G); break;      \
    case 6: YQ_FTREE(6, G); break;      \
    default: YQ_FTREE(7, G); break;     \
  }
  for (int l = depth - 1; l >= 2; --l)
    if (n_tree[l]) YQ_FTREE_ALL(true)
  YQ_HIP(hipGetLastError());
  if (n_m2l) {
#define YQ_FM2L(T)                                                                              \
  forest_pack_kernel<T><<<n_pack, 256, 0, s>>>(dev.p, it_pack.p, mask, p, R16);                 \
  switch (RT) {                                                                                 \
    case 1: forest_m2l_kernel<T, 1><<<n_m2l, 256, 0, s>>>(dev.p, it_m2l.p, mask, p); break;     \
    case 2: forest_m2l_kernel<T, 2><<<n_m2l, 256, 0, s>>>(dev.p, it_m2l.p, mask, p); break;     \
    case 3: forest_m2l_kernel<T, 3><<<n_m2l, 256, 0, s>>>(dev.p, it_m2l.p, mask, p); break;     \
    case 4: forest_m2l_kernel<T, 4><<<n_m2l, 256, 0, s>>>(dev.p, it_m2l.p, mask, p); break;     \
    case 5: forest_m2l_kernel<T, 5><<<n_m2l, 256, 0, s>>>(dev.p, it_m2l.p, mask, p); break;     \
    case 6: forest_m2l_kernel<T, 6><<<n_m2l, 256, 0, s>>>(dev.p, it_m2l.p, mask, p); break;     \
    default: forest_m2l_kernel<T, 7><<<n_m2l, 256, 0, s>>>(dev.p, it_m2l.p, mask, p); break;    \
  }
    if (m2l32) {
      YQ_FM2L(float)
    } else {
      YQ_FM2L(double)
    }
#undef YQ_FM2L
    YQ_HIP(hipGetLastError());
  }
  for (int l = 2; l < depth; ++l)
    if (n_tree[l]) YQ_FTREE_ALL(false)
#undef YQ_FTREE_ALL
#undef YQ_FTREE
  YQ_HIP(hipGetLastError());
}

}  // namespace yq
