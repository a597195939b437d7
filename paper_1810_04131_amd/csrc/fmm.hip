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
  if (!h.empty())
    YQ_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

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
  auto keys_at = [&](int d, std::vector<int64_t>& k) {
    const int64_t m = 1LL << d;
    k.resize(n);
    for (int64_t i = 0; i < n; ++i) {
      int64_t ix = (int64_t)((hx[i] - x0) / W * m), iy = (int64_t)((hy[i] - y0) / W * m);
      ix = std::min(std::max(ix, (int64_t)0), m - 1);
      iy = std::min(std::max(iy, (int64_t)0), m - 1);
      k[i] = morton(ix, iy);
    }
  };
  // depth: the shallowest with at most leaf_max nodes per occupied leaf on average
  std::vector<int64_t> key;
  depth = 2;
  for (int d = 2; d <= 14; ++d) {
    keys_at(d, key);
    std::vector<int64_t> u(key);
    std::sort(u.begin(), u.end());
    const int64_t occ = std::unique(u.begin(), u.end()) - u.begin();
    depth = d;
    if ((double)n / occ <= (double)leaf_max) break;
  }
  keys_at(depth, key);
  std::vector<int> order_idx(n);
  std::iota(order_idx.begin(), order_idx.end(), 0);
  std::stable_sort(order_idx.begin(), order_idx.end(),
                   [&](int a, int b) { return key[a] < key[b]; });
  lv.clear();
  lv.resize(depth + 1);
  std::vector<int> hls, hlc;
  {
    FmmLevel& L = lv[depth];
    for (int64_t k = 0; k < n; ++k) {
      const int64_t kk = key[order_idx[k]];
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
  std::vector<std::unordered_map<int64_t, int>> idx(depth + 1);
  for (int l = 0; l <= depth; ++l) {
    FmmLevel& L = lv[l];
    L.nbox = (int)L.key.size();
    L.w = W / (double)(1LL << l);
    for (int b = 0; b < L.nbox; ++b) idx[l][L.key[b]] = b;
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
        hpar[b] = idx[l - 1].at(L.key[b] >> 2);
        hpos[b] = (int)(L.key[b] & 3);
      }
      if (l < depth)
        for (int pos = 0; pos < 4; ++pos) {
          auto it = idx[l + 1].find((L.key[b] << 2) | pos);
          if (it != idx[l + 1].end()) hch[4 * (size_t)b + pos] = it->second;
        }
      if (l >= 2) {
        int64_t px, py;
        unmorton(L.key[b] >> 2, px, py);
        for (int ddx = -1; ddx <= 1; ++ddx)
          for (int ddy = -1; ddy <= 1; ++ddy) {
            if (px + ddx < 0 || py + ddy < 0) continue;
            auto pit = idx[l - 1].find(morton(px + ddx, py + ddy));
            if (pit == idx[l - 1].end()) continue;
            for (int pos = 0; pos < 4; ++pos) {
              auto sit = idx[l].find((lv[l - 1].key[pit->second] << 2) | pos);
              if (sit == idx[l].end()) continue;
              int64_t sx, sy;
              unmorton(lv[l].key[sit->second], sx, sy);
              const int64_t ox = sx - ix, oy = sy - iy;
              if (std::llabs(ox) <= 1 && std::llabs(oy) <= 1) continue;
              ils.push_back(sit->second);
              ilo.push_back((int)((ox + 3) * 7 + (oy + 3)));
            }
          }
        ilp.push_back((int)ils.size());
      }
      if (l == depth) {
        for (int ddx = -1; ddx <= 1; ++ddx)
          for (int ddy = -1; ddy <= 1; ++ddy) {
            if (ix + ddx < 0 || iy + ddy < 0) continue;
            auto nit = idx[l].find(morton(ix + ddx, iy + ddy));
            if (nit != idx[l].end()) hnbi.push_back(nit->second);
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
    }
    L.M.alloc((size_t)L.nbox * (p + 1));
    L.L.alloc((size_t)L.nbox * (p + 1));
  }
  up(leaf_start, hls, s);
  up(leaf_cnt, hlc, s);
  up(nbp, hnbp, s);
  up(nbi, hnbi, s);
  std::vector<int> hperm(order_idx);
  std::vector<double> sx(n), sy(n), swx(n), swy(n);
  for (int64_t k = 0; k < n; ++k) {
    const int i = order_idx[k];
    sx[k] = hx[i];
    sy[k] = hy[i];
    swx[k] = hwx[i];
    swy[k] = hwy[i];
  }
  up(perm, hperm, s);
  up(xs, sx, s);
  up(ys, sy, s);
  up(wnxs, swx, s);
  up(wnys, swy, s);
  qx.alloc(n);
  qy.alloc(n);
  const int K = 4 * p + 1;
  tg.alloc((size_t)(depth + 1) * 4 * K);
  ts.alloc((size_t)(depth + 1) * 49 * K);
  tab_g_kernel<<<((depth + 1) * 4 + 63) / 64, 64, 0, s>>>(depth, p, W, kappa, tg.p);
  tab_s_kernel<<<((depth + 1) * 49 + 63) / 64, 64, 0, s>>>(depth, p, W, kappa, tab, ts.p);
  YQ_HIP(hipGetLastError());
  YQ_HIP(hipStreamSynchronize(s));
  built = true;
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
    const int64_t nt = (int64_t)lv[l].nbox * (p + 1);
    m2l_kernel<<<(unsigned)((nt + 127) / 128), 128, 0, s>>>(p, lv[l].nbox, lv[l].ilp.p, lv[l].ils.p,
                                                            lv[l].ilo.p, lv[l].M.p,
                                                            ts.p + (size_t)l * 49 * K, lv[l].L.p);
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
