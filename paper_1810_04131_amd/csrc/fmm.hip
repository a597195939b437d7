// Step a7: quadtree Yukawa FMM for the double-layer far field.
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
// only n = 0..p is stored.  Uniform quadtree over the bounding square, depth
// chosen so that occupied leaves hold about leaf_max nodes on average;
// interaction lists are the children of the parent's neighbours that are not
// adjacent; leaves interact directly with their 3 x 3 neighbourhood (P2P uses
// the far-field kernels' pair formula, so the QBX correction still cancels the
// plain terms of window pairs).  Tree and lists are built on the host once per
// geometry; translation tables (per level, child position or offset) on the
// device.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <type_traits>
#include <unordered_map>

#include "bessel.h"
#include "common.h"
#include "farfield_core.h"
#include "fmm.h"

namespace yq {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmad(double2 a, double2 b, double2 c) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// I_k(x), k = 0..n, by the ascending series; I[k * stride].
__device__ inline void iseries(double x, int n, double* I, int stride) {
  const double t = 0.25 * x * x;
  double pref = 1.0;
  for (int k = 0; k <= n; ++k) {
    double term = pref, sum = pref;
    for (int j = 1; j < 400; ++j) {
      term *= t / (double(j) * double(k + j));
      sum += term;
      if (term <= 1e-17 * sum) break;
    }
    I[(int64_t)k * stride] = sum;
    pref *= 0.5 * x / double(k + 1);
  }
}

// ---- translation tables ------------------------------------------------------------------

// tg[((l * 4 + pos) * (4p + 1)) + k + 2p] = g_k(c_child - c_parent), child level l >= 1
__global__ void tab_g_kernel(int depth, int p, double W, double kappa, double2* __restrict__ tg) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (depth + 1) * 4) return;
  const int l = t / 4, pos = t % 4;
  const int K = 4 * p + 1;
  double2* out = tg + (int64_t)t * K;
  if (l == 0) {
    for (int k = 0; k < K; ++k) out[k] = make_double2(0.0, 0.0);
    return;
  }
  const double w = W / (double)(1 << l);
  const double dx = (pos & 1 ? 0.5 : -0.5) * w, dy = (pos & 2 ? 0.5 : -0.5) * w;
  const double r = sqrt(dx * dx + dy * dy), ph = atan2(dy, dx);
  double I[2 * MAXP_FMM + 1];
  iseries(kappa * r, 2 * p, I, 1);
  for (int k = -2 * p; k <= 2 * p; ++k) {
    double s, c;
    sincos(k * ph, &s, &c);
    const double v = I[k < 0 ? -k : k];
    out[k + 2 * p] = make_double2(v * c, v * s);
  }
}

// ts[((l * 49 + o) * (4p + 1)) + k + 2p] = S_k(c_t - c_s), offset o = (ox + 3) * 7 + (oy + 3)
// of the source box relative to the target box, levels l >= 2.
__global__ void tab_s_kernel(int depth, int p, double W, double kappa, const double* __restrict__ tab,
                             double2* __restrict__ ts) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (depth + 1) * 49) return;
  const int l = t / 49, o = t % 49;
  const int K = 4 * p + 1;
  double2* out = ts + (int64_t)t * K;
  const int ox = o / 7 - 3, oy = o % 7 - 3;
  if (l < 2 || (abs(ox) <= 1 && abs(oy) <= 1)) {
    for (int k = 0; k < K; ++k) out[k] = make_double2(0.0, 0.0);
    return;
  }
  const double w = W / (double)(1 << l);
  const double dx = -ox * w, dy = -oy * w;
  const double r = sqrt(dx * dx + dy * dy), ph = atan2(dy, dx);
  const double z = kappa * r;
  double Kn[2 * MAXP_FMM + 1];
  double k0, k1;
  k01_64(z, k0, k1, tab);
  Kn[0] = k0;
  Kn[1] = k1;
  for (int n = 1; n < 2 * p; ++n) Kn[n + 1] = Kn[n - 1] + (2.0 * n / z) * Kn[n];
  for (int k = -2 * p; k <= 2 * p; ++k) {
    double s, c;
    sincos(k * ph, &s, &c);
    const double v = Kn[k < 0 ? -k : k];
    out[k + 2 * p] = make_double2(v * c, v * s);
  }
}

// ---- per-application kernels -----------------------------------------------------------------

__global__ void gather_kernel(int64_t N, const int* __restrict__ perm, const double* __restrict__ sigma,
                              const double* __restrict__ wnxs, const double* __restrict__ wnys,
                              double* __restrict__ qx, double* __restrict__ qy) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= N) return;
  const double s = sigma[perm[k]];
  qx[k] = wnxs[k] * s;
  qy[k] = wnys[k] * s;
}

constexpr int FB = 64;

// One block per leaf (blockDim.x threads, LDS scaled to it): multipole
// coefficients M_n, n = 0..p.
__global__ __launch_bounds__(FB) void p2m_kernel(int p, double kappa, const int* __restrict__ ls,
                                                 const int* __restrict__ lc,
                                                 const double* __restrict__ ccx,
                                                 const double* __restrict__ ccy,
                                                 const double* __restrict__ xs,
                                                 const double* __restrict__ ys,
                                                 const double* __restrict__ qx,
                                                 const double* __restrict__ qy,
                                                 double2* __restrict__ M) {
  extern __shared__ double sh[];
  const int tid = threadIdx.x;
  const int B = blockDim.x;
  const int b = blockIdx.x;
  double* I = sh;                      // [(p + 2) * B]
  double* acc = sh + (p + 2) * B;      // [2 (p + 1) * B]
  for (int n = 0; n <= p; ++n) {
    acc[(2 * n) * B + tid] = 0.0;
    acc[(2 * n + 1) * B + tid] = 0.0;
  }
  const int s0 = ls[b], cnt = lc[b];
  const double cx = ccx[b], cy = ccy[b];
  for (int j = tid; j < cnt; j += B) {
    const double dx = xs[s0 + j] - cx, dy = ys[s0 + j] - cy;
    const double rho = sqrt(dx * dx + dy * dy);
    iseries(kappa * rho, p + 1, I + tid, B);
    const double2 e1 = rho > 0.0 ? make_double2(dx / rho, dy / rho) : make_double2(1.0, 0.0);
    const double2 Q = make_double2(qx[s0 + j], qy[s0 + j]);
    const double2 Qc = cconj(Q);
    double2 Em = cconj(e1), Ep = e1;  // e^{i(n-1)phi}, e^{i(n+1)phi} at n = 0
    for (int n = 0; n <= p; ++n) {
      double2 gm;
      if (n == 0) {
        const double i1 = I[1 * B + tid];
        gm = make_double2(i1 * e1.x, i1 * e1.y);                    // g_1
      } else {
        const double im = I[(n - 1) * B + tid];
        gm = make_double2(im * Em.x, -im * Em.y);                  // conj(g_{n-1})
      }
      const double ip = I[(n + 1) * B + tid];
      const double2 gp = make_double2(ip * Ep.x, -ip * Ep.y);     // conj(g_{n+1})
      double2 a = make_double2(acc[(2 * n) * B + tid], acc[(2 * n + 1) * B + tid]);
      a = cmad(Qc, gm, a);
      a = cmad(Q, gp, a);
      acc[(2 * n) * B + tid] = a.x;
      acc[(2 * n + 1) * B + tid] = a.y;
      Em = (n == 0) ? make_double2(1.0, 0.0) : cmul(Em, e1);
      Ep = cmul(Ep, e1);
    }
  }
  __syncthreads();
  const double sc = kappa / (4.0 * PI);
  for (int v = tid; v < 2 * (p + 1); v += B) {
    double s = 0.0;
    for (int t = 0; t < B; ++t) s += acc[v * B + t];
    const int n = v >> 1;
    if (v & 1)
      M[(int64_t)b * (p + 1) + n].y = s * sc;
    else
      M[(int64_t)b * (p + 1) + n].x = s * sc;
  }
}

// M2M: parent level lp from children at level lp + 1 (table level lp + 1).
__global__ void m2m_kernel(int p, int nbox, const int* __restrict__ ch, const double2* __restrict__ Mc,
                           const double2* __restrict__ tgl, double2* __restrict__ Mp) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)nbox * (p + 1)) return;
  const int P = (int)(t / (p + 1)), n = (int)(t % (p + 1));
  const int K = 4 * p + 1;
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
// carries (-1)^m and the M_{-n} = conj(M_n) fold.  A wave computes 16 target
// boxes at once: for every offset, B = the 16 gathered source vectors (zero
// where a target has no source at that offset), D += A_o B with
// v_mfma_f64_16x16x4f64 tiles (FP64, so the FMM keeps its accuracy).
typedef double dbl4 __attribute__((ext_vector_type(4)));

// amat[((l * 49 + o) * R + r) * R + k], R = 2(p+1) rounded up to 16.
__global__ void m2l_amat_kernel(int depth, int p, int R, const double2* __restrict__ ts,
                                double* __restrict__ amat) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)(depth + 1) * 49 * R) return;
  const int r = (int)(t % R);
  const int lo = (int)(t / R);   // l * 49 + o
  const int K = 4 * p + 1, P1 = p + 1;
  const double2* T = ts + (int64_t)lo * K + 2 * p;
  double* row = amat + t * R;
  for (int k = 0; k < R; ++k) {
    double v = 0.0;
    if (r < 2 * P1 && k < 2 * P1) {
      const int m = r < P1 ? r : r - P1;
      const int n = k < P1 ? k : k - P1;
      const double sg = (m & 1) ? -1.0 : 1.0;
      const double2 t1 = T[n - m];
      const double2 t2 = n > 0 ? T[-n - m] : make_double2(0.0, 0.0);
      if (r < P1)   // Re L_m
        v = k < P1 ? t1.x + t2.x : -t1.y + t2.y;
      else          // Im L_m
        v = k < P1 ? t1.y + t2.y : t1.x - t2.x;
      v *= sg;
    }
    row[k] = v;
  }
}

template <int RT>
__global__ __launch_bounds__(256) void m2l_mfma_kernel(int p, int nbox, const int* __restrict__ ild,
                                                       const double2* __restrict__ M,
                                                       const double* __restrict__ amat,
                                                       double2* __restrict__ L) {
  constexpr int R = RT * 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t0 = (blockIdx.x * 4 + wave) * 16;
  if (t0 >= nbox) return;                       // whole wave
  const int P1 = p + 1;
  const int col = lane & 15, kk = lane >> 4;
  const int tb = t0 + col;
  dbl4 acc[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) acc[rt] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int o = 0; o < 49; ++o) {
    const int ox = o / 7 - 3, oy = o % 7 - 3;
    if (ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1) continue;
    const int src = tb < nbox ? ild[(int64_t)tb * 49 + o] : -1;
    if (__ballot(src >= 0) == 0) continue;      // no target of this wave has a source here
    const double* A = amat + (int64_t)o * R * R;
    for (int ks = 0; ks < R / 4; ++ks) {
      const int k = ks * 4 + kk;
      double bv = 0.0;
      if (src >= 0 && k < 2 * P1) {
        const double2 mv = M[(int64_t)src * P1 + (k < P1 ? k : k - P1)];
        bv = k < P1 ? mv.x : mv.y;
      }
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const double av = A[(int64_t)(rt * 16 + col) * R + k];
        acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[rt], 0, 0, 0);
      }
    }
  }
  if (tb >= nbox) return;
  // FP64 16x16 result layout: lane l holds column l % 16, its register j row 4 j + l / 16
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = rt * 16 + 4 * j + kk;
      if (r < P1)
        L[(int64_t)tb * P1 + r].x = acc[rt][j];
      else if (r < 2 * P1)
        L[(int64_t)tb * P1 + r - P1].y = acc[rt][j];
    }
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

// One block per leaf: local expansion at the leaf's targets plus the direct
// interactions with the 3 x 3 neighbourhood; writes partial[node] in the far-field
// kernels' scaling (far field * 2 pi / kappa^2).
template <bool F32>
__global__ __launch_bounds__(FB) void l2p_p2p_kernel(int p, double kappa, int use_local,
                                                     const int* __restrict__ ls,
                                                     const int* __restrict__ lc,
                                                     const int* __restrict__ nbp,
                                                     const int* __restrict__ nbi,
                                                     const double* __restrict__ ccx,
                                                     const double* __restrict__ ccy,
                                                     const double2* __restrict__ L,
                                                     const double* __restrict__ xs,
                                                     const double* __restrict__ ys,
                                                     const double* __restrict__ qx,
                                                     const double* __restrict__ qy,
                                                     const int* __restrict__ perm,
                                                     const double* __restrict__ tab,
                                                     double* __restrict__ partial) {
  extern __shared__ double sh[];
  double2* sxy = reinterpret_cast<double2*>(sh);            // [FB]
  double2* sq = sxy + FB;                                   // [FB] (FP64 strengths)
  float2* sq32 = reinterpret_cast<float2*>(sq + FB);        // [FB] (FP32 strengths)
  double* I = reinterpret_cast<double*>(sq32 + FB);         // [(p + 1) * FB]
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  const int s0 = ls[b], cnt = lc[b];
  const double kap2 = kappa * kappa;
  const double cx = ccx[b], cy = ccy[b];
  for (int r0 = 0; r0 < cnt; r0 += FB) {
    const int j = r0 + tid;
    const bool act = j < cnt;
    const double xi = act ? xs[s0 + j] : cx, yi = act ? ys[s0 + j] : cy;
    double acc64 = 0.0;
    float acc32 = 0.0f;
    for (int e = nbp[b]; e < nbp[b + 1]; ++e) {
      const int nb = nbi[e];
      const int t0 = ls[nb], tc = lc[nb];
      for (int k0 = 0; k0 < tc; k0 += FB) {
        __syncthreads();
        if (k0 + tid < tc) {
          const int k = t0 + k0 + tid;
          sxy[tid] = make_double2(xs[k], ys[k]);
          if (F32)
            sq32[tid] = make_float2((float)qx[k], (float)qy[k]);
          else
            sq[tid] = make_double2(qx[k], qy[k]);
        }
        __syncthreads();
        const int nbk = min(FB, tc - k0);
        if (F32)
          acc32 = far32_tile(xi, yi, sxy, sq32, nbk, (float)kap2, acc32);
        else
          acc64 = far64_tile(xi, yi, sxy, sq, nbk, kap2, tab, acc64);
      }
    }
    double loc = 0.0;
    if (use_local && act) {
      const double dx = xi - cx, dy = yi - cy;
      const double rho = sqrt(dx * dx + dy * dy);
      iseries(kappa * rho, p, I + tid, FB);
      const double2 e1 = rho > 0.0 ? make_double2(dx / rho, dy / rho) : make_double2(1.0, 0.0);
      const double2* lb = L + (int64_t)b * (p + 1);
      loc = lb[0].x * I[tid];
      double2 E = e1;
      for (int n = 1; n <= p; ++n) {
        const double2 v = cmul(lb[n], E);
        loc += 2.0 * v.x * I[n * FB + tid];
        E = cmul(E, e1);
      }
    }
    if (act) {
      const double direct = F32 ? (double)acc32 : acc64;
      partial[perm[s0 + j]] = direct + loc * (2.0 * PI / kap2);
    }
  }
}

// ---- host --------------------------------------------------------------------------------

static inline int64_t morton(int64_t ix, int64_t iy) {
  int64_t k = 0;
  for (int b = 0; b < 31; ++b) {
    k |= ((ix >> b) & 1LL) << (2 * b);
    k |= ((iy >> b) & 1LL) << (2 * b + 1);
  }
  return k;
}
static inline void unmorton(int64_t k, int64_t& ix, int64_t& iy) {
  ix = iy = 0;
  for (int b = 0; b < 31; ++b) {
    ix |= ((k >> (2 * b)) & 1LL) << b;
    iy |= ((k >> (2 * b + 1)) & 1LL) << b;
  }
}

template <class T>
static void up(DevBuf<T>& d, const std::vector<T>& h, hipStream_t s) {
  d.alloc(std::max<size_t>(h.size(), 1));
  if (!h.empty()) {
    // the host vector is usually a temporary: wait for the copy
    YQ_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    YQ_HIP(hipStreamSynchronize(s));
  }
}

// Lookup of occupied boxes by grid position at one level: a dense table while the
// level's grid is small, a hash map above that.
struct BoxIndex {
  int l = 0;
  std::vector<int> dense;
  std::unordered_map<int64_t, int> sparse;
  void init(int level, const std::vector<int64_t>& keys) {
    l = level;
    const int64_t cells = 1LL << (2 * level);
    dense.clear();
    sparse.clear();
    if (cells <= (1LL << 24)) {
      dense.assign((size_t)cells, -1);
      for (size_t b = 0; b < keys.size(); ++b) dense[(size_t)keys[b]] = (int)b;
    } else {
      sparse.reserve(keys.size() * 2);
      for (size_t b = 0; b < keys.size(); ++b) sparse[keys[b]] = (int)b;
    }
  }
  int find(int64_t key) const {
    if (!dense.empty()) return key >= 0 && key < (int64_t)dense.size() ? dense[(size_t)key] : -1;
    auto it = sparse.find(key);
    return it == sparse.end() ? -1 : it->second;
  }
};

void Fmm::build(const double* dx, const double* dy, const double* dwnx, const double* dwny, int64_t n,
                double kap, int order, int lmax, const double* tab, hipStream_t s) {
  YQ_REQUIRE(order >= 1 && order <= MAXP_FMM, YQ_EINVAL, "FMM order must be in 1..48");
  YQ_REQUIRE(lmax >= 1, YQ_EINVAL, "fmm_leaf_max must be >= 1");
  p = order;
  leaf_max = lmax;
  kappa = kap;
  N = n;
  std::vector<double> hx(n), hy(n), hwx(n), hwy(n);
  YQ_HIP(hipMemcpyAsync(hx.data(), dx, n * sizeof(double), hipMemcpyDeviceToHost, s));
  YQ_HIP(hipMemcpyAsync(hy.data(), dy, n * sizeof(double), hipMemcpyDeviceToHost, s));
  YQ_HIP(hipMemcpyAsync(hwx.data(), dwnx, n * sizeof(double), hipMemcpyDeviceToHost, s));
  YQ_HIP(hipMemcpyAsync(hwy.data(), dwny, n * sizeof(double), hipMemcpyDeviceToHost, s));
  YQ_HIP(hipStreamSynchronize(s));
  double xmin = hx[0], xmax = hx[0], ymin = hy[0], ymax = hy[0];
  for (int64_t i = 0; i < n; ++i) {
    xmin = std::min(xmin, hx[i]);
    xmax = std::max(xmax, hx[i]);
    ymin = std::min(ymin, hy[i]);
    ymax = std::max(ymax, hy[i]);
  }
  W = std::max(xmax - xmin, ymax - ymin) * (1.0 + 1e-9) + 1e-12;
  x0 = 0.5 * (xmin + xmax) - 0.5 * W;
  y0 = 0.5 * (ymin + ymax) - 0.5 * W;
  // Morton keys at the finest candidate depth, sorted once; a coarser level's key
  // is a right shift, so its occupancy is a linear scan of the sorted keys.
  constexpr int DMAX = 14;
  std::vector<int64_t> kmax(n);
  {
    const int64_t m = 1LL << DMAX;
    for (int64_t i = 0; i < n; ++i) {
      int64_t ix = (int64_t)((hx[i] - x0) / W * m), iy = (int64_t)((hy[i] - y0) / W * m);
      ix = std::min(std::max(ix, (int64_t)0), m - 1);
      iy = std::min(std::max(iy, (int64_t)0), m - 1);
      kmax[i] = morton(ix, iy);
    }
  }
  std::vector<int> order_idx(n);
  std::iota(order_idx.begin(), order_idx.end(), 0);
  std::stable_sort(order_idx.begin(), order_idx.end(),
                   [&](int a, int b) { return kmax[a] < kmax[b]; });
  depth = DMAX;
  for (int d = 2; d <= DMAX; ++d) {
    const int sh = 2 * (DMAX - d);
    int64_t occ = 0, last = -1;
    for (int64_t k = 0; k < n; ++k) {
      const int64_t kk = kmax[order_idx[k]] >> sh;
      if (kk != last) {
        ++occ;
        last = kk;
      }
    }
    if ((double)n / occ <= (double)leaf_max) {
      depth = d;
      break;
    }
  }
  const int shl = 2 * (DMAX - depth);
  lv.clear();
  lv.resize(depth + 1);
  std::vector<int> hls, hlc;
  {
    FmmLevel& L = lv[depth];
    for (int64_t k = 0; k < n; ++k) {
      const int64_t kk = kmax[order_idx[k]] >> shl;
      if (L.key.empty() || L.key.back() != kk) {
        L.key.push_back(kk);
        hls.push_back((int)k);
        hlc.push_back(0);
      }
      ++hlc.back();
    }
  }
  for (int l = depth - 1; l >= 0; --l) {
    std::vector<int64_t>& ck = lv[l + 1].key;
    for (int64_t k : ck) {
      const int64_t pk = k >> 2;
      if (lv[l].key.empty() || lv[l].key.back() != pk) lv[l].key.push_back(pk);
    }
  }
  max_leaf = *std::max_element(hlc.begin(), hlc.end());
  std::vector<BoxIndex> idx(depth + 1);
  for (int l = 0; l <= depth; ++l) {
    FmmLevel& L = lv[l];
    L.nbox = (int)L.key.size();
    L.w = W / (double)(1LL << l);
    idx[l].init(l, L.key);
  }
  std::vector<int> hnbp(1, 0), hnbi;
  for (int l = 0; l <= depth; ++l) {
    FmmLevel& L = lv[l];
    std::vector<double> hcx(L.nbox), hcy(L.nbox);
    std::vector<int> hpar(L.nbox, -1), hpos(L.nbox, 0), hch(4 * (size_t)L.nbox, -1);
    std::vector<int> ilp(1, 0), ils, ilo;
    for (int b = 0; b < L.nbox; ++b) {
      int64_t ix, iy;
      unmorton(L.key[b], ix, iy);
      hcx[b] = x0 + (ix + 0.5) * L.w;
      hcy[b] = y0 + (iy + 0.5) * L.w;
      if (l > 0) {
        hpar[b] = idx[l - 1].find(L.key[b] >> 2);
        hpos[b] = (int)(L.key[b] & 3);
      }
      if (l < depth)
        for (int pos = 0; pos < 4; ++pos) hch[4 * (size_t)b + pos] = idx[l + 1].find((L.key[b] << 2) | pos);
      if (l >= 2) {
        int64_t px, py;
        unmorton(L.key[b] >> 2, px, py);
        const int64_t lim = 1LL << (l - 1);
        for (int ddx = -1; ddx <= 1; ++ddx)
          for (int ddy = -1; ddy <= 1; ++ddy) {
            if (px + ddx < 0 || py + ddy < 0 || px + ddx >= lim || py + ddy >= lim) continue;
            const int pb = idx[l - 1].find(morton(px + ddx, py + ddy));
            if (pb < 0) continue;
            for (int pos = 0; pos < 4; ++pos) {
              const int sb = idx[l].find((lv[l - 1].key[pb] << 2) | pos);
              if (sb < 0) continue;
              int64_t sx, sy;
              unmorton(lv[l].key[sb], sx, sy);
              const int64_t ox = sx - ix, oy = sy - iy;
              if (std::llabs(ox) <= 1 && std::llabs(oy) <= 1) continue;
              ils.push_back(sb);
              ilo.push_back((int)((ox + 3) * 7 + (oy + 3)));
            }
          }
        ilp.push_back((int)ils.size());
      }
      if (l == depth) {
        const int64_t lim = 1LL << l;
        for (int ddx = -1; ddx <= 1; ++ddx)
          for (int ddy = -1; ddy <= 1; ++ddy) {
            if (ix + ddx < 0 || iy + ddy < 0 || ix + ddx >= lim || iy + ddy >= lim) continue;
            const int nb = idx[l].find(morton(ix + ddx, iy + ddy));
            if (nb >= 0) hnbi.push_back(nb);
          }
        hnbp.push_back((int)hnbi.size());
      }
    }
    up(L.cx, hcx, s);
    up(L.cy, hcy, s);
    up(L.parent, hpar, s);
    up(L.cpos, hpos, s);
    up(L.ch, hch, s);
    if (l >= 2) {
      up(L.ilp, ilp, s);
      up(L.ils, ils, s);
      up(L.ilo, ilo, s);
      std::vector<int> dense((size_t)L.nbox * 49, -1);
      for (int b = 0; b < L.nbox; ++b)
        for (int e = ilp[b]; e < ilp[b + 1]; ++e) dense[(size_t)b * 49 + ilo[e]] = ils[e];
      up(L.ild, dense, s);
    }
  }
  up(leaf_start, hls, s);
  up(leaf_cnt, hlc, s);
  up(nbp, hnbp, s);
  up(nbi, hnbi, s);
  std::vector<double> sx(n), sy(n), swx(n), swy(n);
  for (int64_t k = 0; k < n; ++k) {
    const int i = order_idx[k];
    sx[k] = hx[i];
    sy[k] = hy[i];
    swx[k] = hwx[i];
    swy[k] = hwy[i];
  }
  up(perm, order_idx, s);
  up(xs, sx, s);
  up(ys, sy, s);
  up(wnxs, swx, s);
  up(wnys, swy, s);
  qx.alloc(n);
  qy.alloc(n);
  set_order(order, tab, s);
}

// (Re)allocates the expansions and builds the translation tables for order q.
void Fmm::set_order(int q, const double* tab, hipStream_t s) {
  YQ_REQUIRE(q >= 1 && q <= MAXP_FMM, YQ_EINVAL, "FMM order must be in 1..48");
  p = q;
  for (auto& L : lv) {
    L.M.alloc((size_t)std::max(L.nbox, 1) * (p + 1));
    L.L.alloc((size_t)std::max(L.nbox, 1) * (p + 1));
  }
  const int K = 4 * p + 1;
  tg.alloc((size_t)(depth + 1) * 4 * K);
  ts.alloc((size_t)(depth + 1) * 49 * K);
  tab_g_kernel<<<((depth + 1) * 4 + 63) / 64, 64, 0, s>>>(depth, p, W, kappa, tg.p);
  tab_s_kernel<<<((depth + 1) * 49 + 63) / 64, 64, 0, s>>>(depth, p, W, kappa, tab, ts.p);
  YQ_HIP(hipGetLastError());
  R16 = ((2 * (p + 1) + 15) / 16) * 16;
  if (use_mfma) {
    const int64_t rows = (int64_t)(depth + 1) * 49 * R16;
    amat.alloc((size_t)rows * R16);
    m2l_amat_kernel<<<(unsigned)((rows + 127) / 128), 128, 0, s>>>(depth, p, R16, ts.p, amat.p);
    YQ_HIP(hipGetLastError());
  }
  YQ_HIP(hipStreamSynchronize(s));
  built = true;
}

// A second expansion order on the same tree: copies the tree (device to device).
void Fmm::copy_tree(const Fmm& o, int q, const double* tab, hipStream_t s) {
  auto dup = [&](auto& dst, const auto& src) {
    using T = std::remove_pointer_t<decltype(src.p)>;
    dst.alloc(std::max<size_t>(src.n, 1));
    if (src.n) YQ_HIP(hipMemcpyAsync(dst.p, src.p, src.n * sizeof(T), hipMemcpyDeviceToDevice, s));
  };
  depth = o.depth;
  leaf_max = o.leaf_max;
  x0 = o.x0;
  y0 = o.y0;
  W = o.W;
  kappa = o.kappa;
  N = o.N;
  max_leaf = o.max_leaf;
  lv.clear();
  lv.resize(o.lv.size());
  for (size_t l = 0; l < o.lv.size(); ++l) {
    lv[l].nbox = o.lv[l].nbox;
    lv[l].w = o.lv[l].w;
    lv[l].key = o.lv[l].key;
    dup(lv[l].cx, o.lv[l].cx);
    dup(lv[l].cy, o.lv[l].cy);
    dup(lv[l].parent, o.lv[l].parent);
    dup(lv[l].cpos, o.lv[l].cpos);
    dup(lv[l].ch, o.lv[l].ch);
    if (l >= 2) {
      dup(lv[l].ilp, o.lv[l].ilp);
      dup(lv[l].ils, o.lv[l].ils);
      dup(lv[l].ilo, o.lv[l].ilo);
      dup(lv[l].ild, o.lv[l].ild);
    }
  }
  dup(perm, o.perm);
  dup(xs, o.xs);
  dup(ys, o.ys);
  dup(wnxs, o.wnxs);
  dup(wnys, o.wnys);
  dup(leaf_start, o.leaf_start);
  dup(leaf_cnt, o.leaf_cnt);
  dup(nbp, o.nbp);
  dup(nbi, o.nbi);
  qx.alloc(N);
  qy.alloc(N);
  set_order(q, tab, s);
}

void Fmm::apply(const double* sigma, double* partial, bool p2p_fp32, const double* tab,
                hipStream_t s) {
  YQ_REQUIRE(built, YQ_ESTATE, "FMM tree not built");
  const int K = 4 * p + 1;
  gather_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(N, perm.p, sigma, wnxs.p, wnys.p, qx.p,
                                                            qy.p);
  FmmLevel& leaf = lv[depth];
  const int pb = (3 * p + 4) * FB * sizeof(double) <= 48 * 1024 ? FB : FB / 2;
  const size_t sh_p2m = (size_t)(3 * p + 4) * pb * sizeof(double);
  p2m_kernel<<<leaf.nbox, pb, sh_p2m, s>>>(p, kappa, leaf_start.p, leaf_cnt.p, leaf.cx.p, leaf.cy.p,
                                           xs.p, ys.p, qx.p, qy.p, leaf.M.p);
  for (int l = depth - 1; l >= 2; --l) {
    const int64_t nt = (int64_t)lv[l].nbox * (p + 1);
    m2m_kernel<<<(unsigned)((nt + 127) / 128), 128, 0, s>>>(p, lv[l].nbox, lv[l].ch.p, lv[l + 1].M.p,
                                                            tg.p + (size_t)(l + 1) * 4 * K,
                                                            lv[l].M.p);
  }
  for (int l = 2; l <= depth; ++l) {
    const int nb = lv[l].nbox;
    if (use_mfma) {
      const double* A = amat.p + (size_t)l * 49 * R16 * R16;
      const unsigned g = (unsigned)((nb + 63) / 64);
      switch (R16 / 16) {
        case 1: m2l_mfma_kernel<1><<<g, 256, 0, s>>>(p, nb, lv[l].ild.p, lv[l].M.p, A, lv[l].L.p); break;
        case 2: m2l_mfma_kernel<2><<<g, 256, 0, s>>>(p, nb, lv[l].ild.p, lv[l].M.p, A, lv[l].L.p); break;
        case 3: m2l_mfma_kernel<3><<<g, 256, 0, s>>>(p, nb, lv[l].ild.p, lv[l].M.p, A, lv[l].L.p); break;
        case 4: m2l_mfma_kernel<4><<<g, 256, 0, s>>>(p, nb, lv[l].ild.p, lv[l].M.p, A, lv[l].L.p); break;
        case 5: m2l_mfma_kernel<5><<<g, 256, 0, s>>>(p, nb, lv[l].ild.p, lv[l].M.p, A, lv[l].L.p); break;
        case 6: m2l_mfma_kernel<6><<<g, 256, 0, s>>>(p, nb, lv[l].ild.p, lv[l].M.p, A, lv[l].L.p); break;
        default: m2l_mfma_kernel<7><<<g, 256, 0, s>>>(p, nb, lv[l].ild.p, lv[l].M.p, A, lv[l].L.p); break;
      }
    } else {
      const int64_t nt = (int64_t)nb * (p + 1);
      m2l_kernel<<<(unsigned)((nt + 127) / 128), 128, 0, s>>>(p, nb, lv[l].ilp.p, lv[l].ils.p,
                                                              lv[l].ilo.p, lv[l].M.p,
                                                              ts.p + (size_t)l * 49 * K, lv[l].L.p);
    }
  }
  for (int l = 2; l < depth; ++l) {
    const int64_t nt = (int64_t)lv[l + 1].nbox * (p + 1);
    l2l_kernel<<<(unsigned)((nt + 127) / 128), 128, 0, s>>>(p, lv[l + 1].nbox, lv[l + 1].parent.p,
                                                            lv[l + 1].cpos.p, lv[l].L.p,
                                                            tg.p + (size_t)(l + 1) * 4 * K,
                                                            lv[l + 1].L.p);
  }
  const size_t sh_l = (size_t)FB * (2 * sizeof(double2) + sizeof(float2)) +
                      (size_t)(p + 1) * FB * sizeof(double);
  if (p2p_fp32)
    l2p_p2p_kernel<true><<<leaf.nbox, FB, sh_l, s>>>(p, kappa, 1, leaf_start.p, leaf_cnt.p, nbp.p,
                                                     nbi.p, leaf.cx.p, leaf.cy.p, leaf.L.p, xs.p, ys.p,
                                                     qx.p, qy.p, perm.p, tab, partial);
  else
    l2p_p2p_kernel<false><<<leaf.nbox, FB, sh_l, s>>>(p, kappa, 1, leaf_start.p, leaf_cnt.p, nbp.p,
                                                      nbi.p, leaf.cx.p, leaf.cy.p, leaf.L.p, xs.p,
                                                      ys.p, qx.p, qy.p, perm.p, tab, partial);
  YQ_HIP(hipGetLastError());
}

}  // namespace yq
