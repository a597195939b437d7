// Many independent configurations solved together.
//
// Each configuration is an ordinary problem (geometry, near lists and QBX
// correction built by yq_set_particles).  Its node range lives at a fixed
// offset of an arena of capacity T nodes; the Krylov basis and all batch
// vectors are arena-sized and column-major (V[k * T + g]).
//
// Per GMRES iteration the whole batch runs as one fixed kernel sequence:
//   fused far field   persistent blocks over a static work list of
//                     (configuration, target tile, source chunk) items,
//   fused finish      chunk reduction + QBX window correction for every node,
//   CGS2 Arnoldi      per-configuration multi-dots (fixed row blocks), reduce,
//                     update, twice, then the norm,
//   Givens            one thread per configuration (device-side Hessenberg,
//                     rotations, residual estimate, convergence mask),
//   scale             the next basis vector.
// Every kernel reads the per-configuration column index and active mask from
// device memory, so the sequence is captured once as a hipGraph and replayed
// for every iteration; converged configurations drop out through the mask.
// A configuration's far-field plan and reduction blocks depend only on its own
// size, so its arithmetic -- and result -- is the same alone or in any mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>

#include "bessel.h"
#include "common.h"
#include "farfield_core.h"
#include "problem.h"
#include "batch.h"

namespace yq {

constexpr int BB = 256;    // far-field block
static_assert(BB == FT, "one source tile per staged block");
constexpr int KR = 4096;   // rows per Krylov reduction block
constexpr int KB2 = 256;   // Krylov block size

// ---- fused far field ----------------------------------------------------------------------

// tab: the FP64 Bessel coefficient table (the same constants for every
// configuration), passed as an argument so that it stays in scalar registers.
// Profiling: adds the source-target pairs of one work item (target block tb of a
// configuration of N nodes, sources j0..j1) to the launch's counter.
__device__ __forceinline__ void count_pairs(unsigned long long* pairs, int64_t N, int tb,
                                            int64_t j0, int64_t j1) {
  const int64_t nt = min((int64_t)BB, N - (int64_t)tb * BB);
  atomicAdd(pairs, (unsigned long long)(nt * (j1 - j0)));
}

__global__ __launch_bounds__(BB) void bfar64_kernel(const ConfDev* __restrict__ cf,
                                                    const int4* __restrict__ items, int nitems,
                                                    const int* __restrict__ mask,
                                                    const double* __restrict__ V,
                                                    const int* __restrict__ col, int64_t T,
                                                    const double* __restrict__ tab,
                                                    unsigned long long* __restrict__ pairs) {
  __shared__ double2 sxy[BB];
  __shared__ double2 sq[BB];
  const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FG));
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int4 w = items[it];
    const int c = w.x;
    if (!mask[c]) continue;
    const ConfDev& cd = cf[c];
    const int64_t N = cd.N;
    const double* sg = V + (col ? (int64_t)col[c] * T : 0) + cd.off;
    const int64_t i = (int64_t)w.y * BB + threadIdx.x;
    const double xi = i < N ? cd.x[i] : 0.0;
    const double yi = i < N ? cd.y[i] : 0.0;
    const int64_t j0 = (int64_t)w.z * cd.chunk;
    const int64_t j1 = min(N, j0 + cd.chunk);
    if (pairs && threadIdx.x == 0) count_pairs(pairs, N, w.y, j0, j1);
    const int64_t grp = (int64_t)w.y * (BB / FG) + wib;
    const bool live = grp * FG < N;
    double acc = 0.0;
    for (int64_t jb = j0; jb < j1; jb += BB) {
      const int64_t j = jb + threadIdx.x;
      __syncthreads();
      if (j < j1) {
        const double s = sg[j];
        sxy[threadIdx.x] = make_double2(cd.x[j], cd.y[j]);
        sq[threadIdx.x] = make_double2(cd.wnx[j] * s, cd.wny[j] * s);
      }
      __syncthreads();
      const int nb = (int)min((int64_t)BB, j1 - jb);
      // a tile with close pairs is summed panel by panel, each with its own class
      const int tcls = live ? far64_class(cd.f32.grp, cd.f32.tile, grp, jb / FT, cd.kappa)
                            : C64_GENERAL;
      for (int q = 0; q < nb;) {
        const bool split = tcls == C64_GENERAL && live;
        const int cls = split ? far64_class(cd.f32.grp, cd.f32.pan, grp, (jb + q) / Q, cd.kappa)
                              : tcls;
        const int len = split ? Q : nb - q;
        acc = far64_class_tile(cls, xi, yi, sxy + q, sq + q, len, cd.kap2, tab, acc);
        q += len;
      }
    }
    if (i < N) cd.part64[(int64_t)w.z * N + i] = acc;
  }
}

// Packs the FP32 source records of every active configuration: positions relative
// to the node's 256-node tile centre (bfar32) or, with sym set, to its 64-node
// group centre (bsym32), scaled by kappa log2(e).
__global__ void bpack32_kernel(const ConfDev* __restrict__ cf, const int* __restrict__ node_conf,
                               int64_t T, const int* __restrict__ mask,
                               const double* __restrict__ V, const int* __restrict__ col,
                               int sym) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= T) return;
  const int c = node_conf[g];
  if (c < 0 || !mask[c]) return;
  const ConfDev& cd = cf[c];
  if (cd.fmm) return;   // no FP32 source records: its far field comes from the forest
  const int64_t i = g - cd.off;
  const double sc = V[(col ? (int64_t)col[c] * T : 0) + g] * cd.f32.qc;
  float2 r;
  if (sym) {
    const double4 gc = cd.f32.grp[i / FG];
    r = make_float2((float)((cd.x[i] - gc.x) * cd.f32.s), (float)((cd.y[i] - gc.y) * cd.f32.s));
  } else {
    r = cd.rel[i];
  }
  const_cast<float4*>(cd.f32.src)[i] =
      make_float4(r.x, r.y, (float)(cd.wnx[i] * sc), (float)(cd.wny[i] * sc));
}

// Same arithmetic as far32_kernel for each (configuration, target block, source chunk).
__global__ __launch_bounds__(BB) void bfar32_kernel(const ConfDev* __restrict__ cf,
                                                    const int4* __restrict__ items, int nitems,
                                                    const int* __restrict__ mask,
                                                    unsigned long long* __restrict__ pairs) {
  const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FG));
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int4 w = items[it];
    const int c = w.x;
    if (!mask[c]) continue;
    const ConfDev& cd = cf[c];
    const int64_t N = cd.N;
    const int64_t j0 = (int64_t)w.z * cd.chunk;
    const int64_t j1 = min(N, j0 + cd.chunk);
    if (pairs && threadIdx.x == 0) count_pairs(pairs, N, w.y, j0, j1);
    const int64_t g = (int64_t)w.y * (BB / FG) + wib;
    if (g * FG >= N) continue;
    const int64_t i = (int64_t)w.y * BB + threadIdx.x;
    const float acc = far32_range(cd.f32, i, g, j0, j1);
    if (i < N) cd.part32[(int64_t)w.z * N + i] = acc;
  }
}

// ---- symmetric FP32 far field ------------------------------------------------------------
//
// K1(z)/z depends on the pair only through |x_i - x_j|, so one evaluation serves both
// directions: target i gains K (x_i - x_j).q_j and target j gains -K (x_i - x_j).q_i.
// Work items are pairs p <= q of node chunks (SC nodes) of one configuration, so a
// configuration's items depend only on its size.  Each wavefront of a block takes
// groups of chunk p (64 nodes, one per lane) and visits the groups of chunk q (for p = q
// those at or after its own):
//   far pair of groups (kappa x the gap between their circles >= 2): one evaluation per
//     unordered pair.  The other group's records are staged in LDS twice over so that
//     lane l reads record (l + k) mod 64 at step k through one address and an immediate
//     offset; the reverse partial sum moves with its node by a one-lane rotation of the
//     wavefront per step, so that after 64 steps lane l holds the sum of node l;
//   close pair: bfar32's panel-classified one-directional sums, in both directions;
//   a group with itself: the forward sums only.
// Reverse sums go to a per-wavefront LDS row and are added in a fixed order: the
// result does not depend on timing.  Output: the sums of targets of chunk t over the
// sources of chunk u go to part32[u * N + i] (bfinish adds ceil(N / SC) slots).
constexpr int SW = BB / FG;         // wavefronts per block
static_assert(SW == 4 && SC % FG == 0, "four wavefronts; chunks of whole groups");
constexpr float FAR_AWAY = 1e18f;   // position of padding records (their strength is 0)

__device__ __forceinline__ float rotl1(float v) {   // lane l <- lane (l + 1) mod 64
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x134,
                                                            0xF, 0xF, true));
}

// Orders this wavefront's LDS accesses on either side (LDS executes a wavefront's
// accesses in issue order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One far pair of groups: the lane's node (tx, ty relative to the other group's centre,
// scaled; strength (qx, qy)) against the 64 staged records st[k] = record (lane + k) mod 64.
template <int NH, const float (&H)[NH]>
__device__ __forceinline__ void sym_far_block(float tx, float ty, float qx, float qy,
                                              const float4* st, float& facc, float& racc) {
#pragma unroll 16
  for (int k = 0; k < FG; ++k) {
    const float4 b = st[k];
    const float dx = tx - b.x, dy = ty - b.y;
    const float z2 = fmaf(dx, dx, dy * dy);
    const float yv = __builtin_amdgcn_rsqf(z2);
    const float z = z2 * yv;
    const float e = __builtin_amdgcn_exp2f(fmaf(-1.5f, __builtin_amdgcn_logf(z), -z));
    const float eh = e * horner(H, yv);
    facc = fmaf(eh, fmaf(dx, b.z, dy * b.w), facc);
    racc = rotl1(racc - eh * fmaf(dx, qx, dy * qy));
  }
}

// One-directional sums over the sources [s0, s0 + ns) of one group (ns a multiple of
// 16) for a target at (xt, yt) of a group with circle (gx, gy, gr); (tx, ty) is the
// target relative to the source group's centre, scaled.  Each panel takes the class
// of its own circle, as in far32_range.
__device__ __forceinline__ void sym_panels(const ConfDev& cd, double xt, double yt, float tx,
                                           float ty, double gx, double gy, double gr, int64_t s0,
                                           int ns, float& accf, float& accn) {
  kptr<float> src = as_k((const float*)cd.f32.src);
  for (int64_t js = s0; js < s0 + ns; js += Q) {
    kptr<double> pc = as_k((const double*)cd.f32.pan) + 4 * (js / Q);
    const double px = gx - pc[0], py = gy - pc[1];
    const double z = cd.kappa * (sqrt(px * px + py * py) - gr - pc[2]);
    kptr<float> sp = src + 4 * js;
    if (z >= 8.0)
      accf = far32_far_tile<4, kH1Y_32_z8>(tx, ty, sp, Q, accf);
    else if (z >= 4.0)
      accf = far32_far_tile<5, kH1Y_32_z4>(tx, ty, sp, Q, accf);
    else if (z >= 2.0)
      accf = far32_far_tile<7, kH1Y_32>(tx, ty, sp, Q, accf);
    else
      accn = far32_near_tile(xt, yt, as_k(cd.x) + js, as_k(cd.y) + js, sp, Q, cd.f32.kap2, accn);
  }
}

__global__ __launch_bounds__(BB) void bsym32_kernel(const ConfDev* __restrict__ cf,
                                                    const int4* __restrict__ items, int nitems,
                                                    const int* __restrict__ mask,
                                                    unsigned long long* __restrict__ pairs) {
  __shared__ float rev[SW][SC];
  __shared__ float4 stage[SW][2 * FG];
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FG));
  const int lane = (int)(threadIdx.x % FG);
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int4 w = items[it];
    const int c = w.x;
    if (!mask[c]) continue;
    const ConfDev& cd = cf[c];
    const int64_t N = cd.N;
    const int p = w.y, q = w.z;
    const int64_t a0 = (int64_t)p * SC, b0 = (int64_t)q * SC;
    const int na = (int)min((int64_t)SC, N - a0);
    const int nb = (int)min((int64_t)SC, N - b0);
    if (pairs && threadIdx.x == 0)
      atomicAdd(pairs, (unsigned long long)(p == q ? (int64_t)na * na : 2 * (int64_t)na * nb));
    const int nga = (na + FG - 1) / FG, ngb = (nb + FG - 1) / FG;
    for (int t = lane; t < SC; t += FG) rev[wv][t] = 0.0f;
    kptr<double> grp = as_k((const double*)cd.f32.grp);
    const float4* src = cd.f32.src;
    const double s = cd.f32.s, kappa = cd.kappa;
    const float nscale = cd.f32.nscale;
    // groups of chunk p in snake order over the wavefronts (balances the triangle of p = q)
    for (int r = 0; SW * r < nga; ++r) {
      const int a = SW * r + ((r & 1) ? SW - 1 - wv : wv);
      if (a >= nga) continue;
      const int64_t ga = a0 / FG + a;
      const int64_t ia = ga * FG + lane;
      const bool va = ia < N;
      const int nav = (int)min((int64_t)FG, N - ga * FG);
      const float4 ra = va ? src[ia] : make_float4(FAR_AWAY, FAR_AWAY, 0.0f, 0.0f);
      const double xa = va ? cd.x[ia] : 0.0, ya = va ? cd.y[ia] : 0.0;
      const double cax = grp[4 * ga], cay = grp[4 * ga + 1], car = grp[4 * ga + 2];
      float ff = 0.0f, fn = 0.0f;
      for (int b = (p == q ? a : 0); b < ngb; ++b) {
        const int64_t gb = b0 / FG + b;
        const int64_t jb = gb * FG;
        const int nbv = (int)min((int64_t)FG, N - jb);
        if (p == q && b == a) {
          sym_panels(cd, xa, ya, ra.x, ra.y, cax, cay, car, jb, nbv, ff, fn);
          continue;
        }
        const double cbx = grp[4 * gb], cby = grp[4 * gb + 1], cbr = grp[4 * gb + 2];
        const double ox = cax - cbx, oy = cay - cby;
        const double z = kappa * (sqrt(ox * ox + oy * oy) - car - cbr);
        const float offx = (float)(ox * s), offy = (float)(oy * s);
        const float4 rb =
            lane < nbv ? src[jb + lane] : make_float4(-FAR_AWAY, -FAR_AWAY, 0.0f, 0.0f);
        float racc = 0.0f;
        if (z >= 2.0) {
          wave_lds_order();
          stage[wv][lane] = rb;
          stage[wv][lane + FG] = rb;
          wave_lds_order();
          const float tx = ra.x + offx, ty = ra.y + offy;
          const float4* st = &stage[wv][lane];
          if (z >= 8.0)
            sym_far_block<4, kH1Y_32_z8>(tx, ty, ra.z, ra.w, st, ff, racc);
          else if (z >= 4.0)
            sym_far_block<5, kH1Y_32_z4>(tx, ty, ra.z, ra.w, st, ff, racc);
          else
            sym_far_block<7, kH1Y_32>(tx, ty, ra.z, ra.w, st, ff, racc);
        } else {
          sym_panels(cd, xa, ya, ra.x + offx, ra.y + offy, cax, cay, car, jb, nbv, ff, fn);
          const double xb = lane < nbv ? cd.x[jb + lane] : 0.0;
          const double yb = lane < nbv ? cd.y[jb + lane] : 0.0;
          float rf = 0.0f, rn = 0.0f;
          sym_panels(cd, xb, yb, rb.x - offx, rb.y - offy, cbx, cby, cbr, ga * FG, nav, rf, rn);
          racc = fmaf(rn, nscale, rf);
        }
        rev[wv][b * FG + lane] += racc;
      }
      const float fwd = fmaf(fn, nscale, ff);
      if (p == q)
        rev[wv][a * FG + lane] += fwd;
      else if (va)
        cd.part32[(int64_t)q * N + ia] = fwd;
    }
    __syncthreads();
    const int64_t o0 = p == q ? a0 : b0;
    const int no = p == q ? na : nb;
    for (int t = threadIdx.x; t < no; t += BB)
      cd.part32[(int64_t)p * N + o0 + t] = ((rev[0][t] + rev[1][t]) + rev[2][t]) + rev[3][t];
    __syncthreads();
  }
}

// out[g] = (kappa^2/2pi) sum_chunks partial + correction, for every node of an active config.
// correction_row over the panels that a QBX fold left out: window panel sl where bit
// sl of um is set, extra-panel entry e where xm[e] is (bit 31: some entry is).
template <typename TW>
__device__ double correction_left(int64_t i, int64_t N, int P, int win, const TW* __restrict__ W,
                                  const int* __restrict__ xrow, const int* __restrict__ xpan,
                                  const double* __restrict__ xvals,
                                  const double* __restrict__ sigma, uint32_t um,
                                  const uint8_t* __restrict__ xm) {
  const int64_t pan = i / Q, pid = pan / P;
  const int k = (int)(pan % P);
  double corr = 0.0;
  for (int sl = 0; sl <= 2 * win; ++sl) {
    if (!((um >> sl) & 1u)) continue;
    int kj = (k + sl - win) % P;
    if (kj < 0) kj += P;
    const double* sg = sigma + (pid * P + kj) * Q;
    const TW* wr = W + (int64_t)sl * Q * N + i;
    for (int m = 0; m < Q; ++m) corr = fma((double)wr[(int64_t)m * N], sg[m], corr);
  }
  if (xvals && (um >> 31))
    for (int e = xrow[i]; e < xrow[i + 1]; ++e) {
      if (!xm[e]) continue;
      const double* sg = sigma + (int64_t)xpan[e] * Q;
      const double* vr = xvals + (int64_t)e * Q;
      for (int m = 0; m < Q; ++m) corr = fma(vr[m], sg[m], corr);
    }
  return corr;
}

// Over the kblk items (configuration c, KR rows from lb KR on; a masked-off
// configuration's blocks return after one load): the configuration's descriptor is
// uniform over the block, each thread finishes every KB2-th row.
__global__ __launch_bounds__(KB2) void bfinish_kernel(const ConfDev* __restrict__ cf,
                                                      const int2* __restrict__ blk, int64_t T,
                                                      const int* __restrict__ mask, int f32,
                                                      const double* __restrict__ V,
                                                      const int* __restrict__ col,
                                                      double* __restrict__ out) {
  const int2 b = blk[blockIdx.x];
  const int c = b.x;
  if (!mask[c]) return;
  const ConfDev& cd = cf[c];
  const int64_t N = cd.N;
  const int64_t r0 = (int64_t)b.y * KR;
  const int nr = (int)min((int64_t)KR, N - r0);
  const double* sg = V + (col ? (int64_t)col[c] * T : 0) + cd.off;
  const double scale = cd.kappa * cd.kappa / (2.0 * PI);
  const bool fold = f32 ? cd.qfold32 : cd.qfold64;
  for (int q = threadIdx.x; q < nr; q += KB2) {
    const int64_t i = r0 + q;
    double s = 0.0;
    if (!f32 || cd.fmm) {
      for (int k = 0; k < cd.chunks; ++k) s += cd.part64[(int64_t)k * N + i];
    } else {
      for (int k = 0; k < cd.chunks32; ++k) s += (double)cd.part32[(int64_t)k * N + i];
    }
    s *= scale;
    if (fold) {   // the correction came with the tree's leaf pass (bleft_kernel adds the
      out[cd.off + i] = s;   // panels left out)
      continue;
    }
    // the inner (FP32) operator reads the correction in FP32 when it is there
    const double corr =
        f32 && cd.W32 ? correction_row(i, N, cd.P, cd.win, cd.W32, cd.xrow, cd.xpan, cd.xvals, sg)
                      : correction_row(i, N, cd.P, cd.win, cd.W, cd.xrow, cd.xpan, cd.xvals, sg);
    out[cd.off + i] = s + corr;
  }
}

// The corrections of the panels left out of the QBX folds, after bfinish_kernel: items
// (configuration, node) of the nodes with such panels.
__global__ void bleft_kernel(const ConfDev* __restrict__ cf, const int2* __restrict__ items, int n,
                             int64_t T, const int* __restrict__ mask, int f32,
                             const double* __restrict__ V, const int* __restrict__ col,
                             double* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int2 it = items[q];
  const int c = it.x;
  if (!mask[c]) return;
  const ConfDev& cd = cf[c];
  if (!(f32 ? cd.qfold32 : cd.qfold64)) return;
  const int64_t i = it.y;
  const double* sg = V + (col ? (int64_t)col[c] * T : 0) + cd.off;
  const uint32_t um = cd.qumask[i];
  out[cd.off + i] += f32 && cd.W32 ? correction_left(i, cd.N, cd.P, cd.win, cd.W32, cd.xrow,
                                                     cd.xpan, cd.xvals, sg, um, cd.qxmask)
                                   : correction_left(i, cd.N, cd.P, cd.win, cd.W, cd.xrow,
                                                     cd.xpan, cd.xvals, sg, um, cd.qxmask);
}

__global__ void qbx_left_kernel(int64_t N, const uint32_t* __restrict__ umask,
                                int* __restrict__ left, int* __restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N && umask[i]) left[atomicAdd(cnt, 1)] = (int)i;
}

__global__ void left_items_kernel(int64_t n, int c, const int* __restrict__ left,
                                  int2* __restrict__ items) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) items[k] = make_int2(c, left[k]);
}

// ---- QBX corrections folded into the near-field caches -----------------------------------
//
// The QBX correction of target i, sum_j W_ij sigma_j over the nodes j of its window
// panels and extra near panels (correction_row), involves sources that lie in the
// P2P list of i's leaf, whose pairs the tree's near-field cache holds: the leaf pass
// adds K_ij sigma_j in the far-field scaling (2 pi / kappa^2 times the operator's),
// so adding W_ij 2 pi / kappa^2 to the cached K_ij gives the corrected sum in the same
// pass, and the finish skips the correction's weights and densities.

__global__ void iperm_kernel(int64_t n, const int* __restrict__ perm, int* __restrict__ iperm) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < n) iperm[perm[k]] = k;
}

// Sorted target k (node i = perm[k]): each panel of correction_row's sums (the
// 2 win + 1 window panels, then the extra panels of xrow) whose 16 nodes all lie in
// the P2P list of k's leaf is folded: cache slot (entry e, source position, target
// position, target-fastest) of each node j gets W_ij scale.  Panels with a node
// outside the list are left out and recorded: bit sl of umask[i] for window panel
// sl, xmask[e] = 1 (and bit 31) for extra-panel entry e.
template <typename TC>
__global__ void qbx_fold_kernel(int64_t N, int P, int win, const double* __restrict__ W,
                                const int* __restrict__ xrow, const int* __restrict__ xpan,
                                const double* __restrict__ xvals, const int* __restrict__ perm,
                                const int* __restrict__ iperm, const int* __restrict__ leaf_of,
                                const int* __restrict__ ls, const int* __restrict__ lc,
                                const int* __restrict__ nbp, const int* __restrict__ nbi,
                                const int64_t* __restrict__ boff, double scale, TC* coef,
                                uint32_t* __restrict__ umask, uint8_t* __restrict__ xmask) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int i = perm[k];
  const int b = leaf_of[k];
  const int t = (int)(k - ls[b]), cb = lc[b];
  const int e0 = nbp[b], e1 = nbp[b + 1];
  auto slot = [&](int64_t j) -> int64_t {
    const int sj = iperm[j];
    const int bj = leaf_of[sj];
    for (int e = e0; e < e1; ++e)
      if (nbi[e] == bj) return boff[e] + (int64_t)(sj - ls[bj]) * cb + t;
    return -1;
  };
  // one panel: its 16 sources from j0, weights w[m * ws]
  auto panel = [&](int64_t j0, const double* w, int64_t ws) -> bool {
    int64_t a[Q];
    bool ok = true;
    for (int m = 0; m < Q; ++m) {
      a[m] = slot(j0 + m);
      ok = ok && a[m] >= 0;
    }
    if (ok)
      for (int m = 0; m < Q; ++m) coef[a[m]] = (TC)((double)coef[a[m]] + w[m * ws] * scale);
    return ok;
  };
  uint32_t um = 0;
  const int64_t pan = i / Q, pid = pan / P;
  const int kp = (int)(pan % P);
  for (int sl = 0; sl <= 2 * win; ++sl) {
    int kj = (kp + sl - win) % P;
    if (kj < 0) kj += P;
    if (!panel((pid * P + kj) * Q, W + (int64_t)sl * Q * N + i, N)) um |= 1u << sl;
  }
  if (xvals)
    for (int e = xrow[i]; e < xrow[i + 1]; ++e) {
      const bool ok = panel((int64_t)xpan[e] * Q, xvals + (int64_t)e * Q, 1);
      xmask[e] = ok ? 0 : 1;
      if (!ok) um |= 1u << 31;
    }
  umask[i] = um;
}

// ---- batched forces -----------------------------------------------------------------------

// FP64 gradient far field of the direct members (far_grad64_kernel's sums for each
// (configuration, target block, source chunk) item): gpart[(chunk * 2 + c) * N + i].
__global__ __launch_bounds__(BB) void bgrad64_kernel(const ConfDev* __restrict__ cf,
                                                     const int4* __restrict__ items, int nitems,
                                                     const int* __restrict__ mask,
                                                     const double* __restrict__ sigma,
                                                     const double* __restrict__ tab) {
  __shared__ double2 sxy[BB];
  __shared__ double2 sq[BB];
  const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FG));
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int4 w = items[it];
    const int c = w.x;
    if (!mask[c]) continue;
    const ConfDev& cd = cf[c];
    const int64_t N = cd.N;
    const double* sg = sigma + cd.off;
    const int64_t i = (int64_t)w.y * BB + threadIdx.x;
    const double xi = i < N ? cd.x[i] : 0.0;
    const double yi = i < N ? cd.y[i] : 0.0;
    const int64_t j0 = (int64_t)w.z * cd.chunk;
    const int64_t j1 = min(N, j0 + cd.chunk);
    const int64_t grp = (int64_t)w.y * (BB / FG) + wib;
    const bool live = grp * FG < N;
    double ax = 0.0, ay = 0.0;
    for (int64_t jb = j0; jb < j1; jb += BB) {
      const int64_t j = jb + threadIdx.x;
      __syncthreads();
      if (j < j1) {
        const double s = sg[j];
        sxy[threadIdx.x] = make_double2(cd.x[j], cd.y[j]);
        sq[threadIdx.x] = make_double2(cd.wnx[j] * s, cd.wny[j] * s);
      }
      __syncthreads();
      const int nb = (int)min((int64_t)BB, j1 - jb);
      const int tcls = live ? far64_class(cd.f32.grp, cd.f32.tile, grp, jb / FT, cd.kappa)
                            : C64_GENERAL;
      for (int q = 0; q < nb;) {
        const bool split = tcls == C64_GENERAL && live;
        const int cls = split ? far64_class(cd.f32.grp, cd.f32.pan, grp, (jb + q) / Q, cd.kappa)
                              : tcls;
        const int len = split ? Q : nb - q;
        far_grad64_class_tile(cls, xi, yi, sxy + q, sq + q, len, cd.kap2, tab, ax, ay);
        q += len;
      }
    }
    if (i < N) {
      cd.gpart[((int64_t)w.z * 2 + 0) * N + i] = ax;
      cd.gpart[((int64_t)w.z * 2 + 1) * N + i] = ay;
    }
  }
}

// The FP64 far field and its gradient in one pass over the pairs
// (far_fused64_kernel's sums for each item): part64 and gpart.
__global__ __launch_bounds__(BB) void bfused64_kernel(const ConfDev* __restrict__ cf,
                                                      const int4* __restrict__ items, int nitems,
                                                      const int* __restrict__ mask,
                                                      const double* __restrict__ V,
                                                      const int* __restrict__ col, int64_t T,
                                                      const double* __restrict__ tab) {
  __shared__ double2 sxy[BB];
  __shared__ double2 sq[BB];
  const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FG));
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int4 w = items[it];
    const int c = w.x;
    if (!mask[c]) continue;
    const ConfDev& cd = cf[c];
    const int64_t N = cd.N;
    const double* sg = V + (col ? (int64_t)col[c] * T : 0) + cd.off;
    const int64_t i = (int64_t)w.y * BB + threadIdx.x;
    const double xi = i < N ? cd.x[i] : 0.0;
    const double yi = i < N ? cd.y[i] : 0.0;
    const int64_t j0 = (int64_t)w.z * cd.chunk;
    const int64_t j1 = min(N, j0 + cd.chunk);
    const int64_t grp = (int64_t)w.y * (BB / FG) + wib;
    const bool live = grp * FG < N;
    double acc = 0.0, ax = 0.0, ay = 0.0;
    for (int64_t jb = j0; jb < j1; jb += BB) {
      const int64_t j = jb + threadIdx.x;
      __syncthreads();
      if (j < j1) {
        const double s = sg[j];
        sxy[threadIdx.x] = make_double2(cd.x[j], cd.y[j]);
        sq[threadIdx.x] = make_double2(cd.wnx[j] * s, cd.wny[j] * s);
      }
      __syncthreads();
      const int nb = (int)min((int64_t)BB, j1 - jb);
      const int tcls = live ? far64_class(cd.f32.grp, cd.f32.tile, grp, jb / FT, cd.kappa)
                            : C64_GENERAL;
      for (int q = 0; q < nb;) {
        const bool split = tcls == C64_GENERAL && live;
        const int cls = split ? far64_class(cd.f32.grp, cd.f32.pan, grp, (jb + q) / Q, cd.kappa)
                              : tcls;
        const int len = split ? Q : nb - q;
        far_fused64_class_tile(cls, xi, yi, sxy + q, sq + q, len, cd.kap2, tab, acc, ax, ay);
        q += len;
      }
    }
    if (i < N) {
      cd.part64[(int64_t)w.z * N + i] = acc;
      cd.gpart[((int64_t)w.z * 2 + 0) * N + i] = ax;
      cd.gpart[((int64_t)w.z * 2 + 1) * N + i] = ay;
    }
  }
}

// Surface gradient of every masked node: the chunk sums of the gradient far field
// (one chunk for a forest tree) and the exterior QBX window and extra-row
// corrections, in finish_grad_kernel's order.
__global__ void bfinish_grad_kernel(const ConfDev* __restrict__ cf,
                                    const int* __restrict__ node_conf, int64_t T,
                                    const int* __restrict__ mask, const double* __restrict__ sigma,
                                    double* __restrict__ gx, double* __restrict__ gy) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= T) return;
  const int c = node_conf[g];
  if (c < 0 || !mask[c]) return;
  const ConfDev& cd = cf[c];
  const int64_t N = cd.N;
  const int64_t i = g - cd.off;
  const double* sgc = sigma + cd.off;
  double sx = 0.0, sy = 0.0;
  for (int k = 0; k < cd.chunks; ++k) {
    sx += cd.gpart[((int64_t)k * 2 + 0) * N + i];
    sy += cd.gpart[((int64_t)k * 2 + 1) * N + i];
  }
  const double sc = cd.kappa * cd.kappa / (2.0 * PI);
  sx *= sc;
  sy *= sc;
  const int64_t pan = i / Q;
  const int64_t pid = pan / cd.P;
  const int k = (int)(pan % cd.P);
  for (int sl = 0; sl <= 2 * cd.win; ++sl) {
    int kj = (k + sl - cd.win) % cd.P;
    if (kj < 0) kj += cd.P;
    const double* sg = sgc + (pid * cd.P + kj) * Q;
    const double* wx = cd.WGx + (int64_t)sl * Q * N + i;
    const double* wy = cd.WGy + (int64_t)sl * Q * N + i;
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      sx = fma(wx[(int64_t)m * N], sg[m], sx);
      sy = fma(wy[(int64_t)m * N], sg[m], sy);
    }
  }
  for (int e = cd.xrow[i]; e < cd.xrow[i + 1]; ++e) {
    const double* sg = sgc + (int64_t)cd.xpan[e] * Q;
    for (int m = 0; m < Q; ++m) {
      sx = fma(cd.xgvals[((int64_t)e * 2 + 0) * Q + m], sg[m], sx);
      sy = fma(cd.xgvals[((int64_t)e * 2 + 1) * Q + m], sg[m], sy);
    }
  }
  gx[g] = sx;
  gy[g] = sy;
}

constexpr int FRB = 256;   // forces block (the single-problem forces kernel's)

__device__ __forceinline__ double fsum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = FRB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// Traction (eq. stress) integrated per particle (eqs. force_torque, scalar-torque)
// and the energy of eq. main, one block per (configuration, particle) item, in the
// single-problem forces kernel's order; f: the boundary data (arena layout).
__global__ __launch_bounds__(FRB) void bforces_kernel(const ConfDev* __restrict__ cf,
                                                      const int2* __restrict__ items,
                                                      const double* __restrict__ f,
                                                      const double* __restrict__ gx,
                                                      const double* __restrict__ gy,
                                                      double gamma, double* __restrict__ force,
                                                      double* __restrict__ torque,
                                                      double* __restrict__ energy) {
  __shared__ double sh[FRB];
  const int2 it = items[blockIdx.x];
  const ConfDev& cd = cf[it.x];
  const int p = it.y;
  const int64_t b = (int64_t)p * cd.P * Q;
  const int64_t e = b + (int64_t)cd.P * Q;
  const double cx = cd.pc[5 * p], cy = cd.pc[5 * p + 1];
  const double kap = cd.kappa;
  const double* fc = f + cd.off;
  const double* gxc = gx + cd.off;
  const double* gyc = gy + cd.off;
  double fx = 0.0, fy = 0.0, tq = 0.0, en = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += FRB) {
    const double ux = gxc[i], uy = gyc[i];
    const double nx = cd.nx[i], ny = cd.ny[i];
    const double un = ux * nx + uy * ny;
    const double iso = gamma * (kap * fc[i] * fc[i] + (ux * ux + uy * uy) / kap);
    const double c2 = 2.0 * gamma / kap * un;
    const double tx = iso * nx - c2 * ux;
    const double ty = iso * ny - c2 * uy;
    const double w = cd.w[i];
    fx += w * tx;
    fy += w * ty;
    tq += w * ((cd.x[i] - cx) * ty - (cd.y[i] - cy) * tx);
    en += -gamma / kap * w * fc[i] * un;
  }
  fx = fsum(fx, sh);
  fy = fsum(fy, sh);
  tq = fsum(tq, sh);
  en = fsum(en, sh);
  if (threadIdx.x == 0) {
    const int64_t q = cd.poff + p;
    force[2 * q] = fx;
    force[2 * q + 1] = fy;
    torque[q] = tq;
    energy[q] = en;
  }
}

// ---- batched Krylov kernels -------------------------------------------------------------------

__device__ __forceinline__ double bsum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = KB2 / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// The batched Krylov kernels below run over the kblk items (c, lb): KR rows of
// configuration c from row lb KR on, KB2 threads, KU rows per thread; a block whose
// configuration is masked off returns after one load.
constexpr int KU = KR / KB2;

// One multi-dot pass over NV columns of A: acc[v] = sum over the thread's rows of
// A[(k0 + v) lda + i] w_i, summed over the block into partial[kpoff + k kb + lb].
// sh: [KB2 / 64][8] doubles (the caller alternates two so that one barrier per pass
// separates a pass's reads from the next-but-one pass's writes).
template <int NV, typename TA>
__device__ __forceinline__ void mdot_pass(const TA* __restrict__ ap, int64_t lda, int nr,
                                          const double (&wr)[KU], double (*sh)[8],
                                          double* __restrict__ out, int64_t ostride) {
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll 4
  for (int u = 0; u < KU; ++u) {
    const int i = threadIdx.x + u * KB2;
    const int ic = i < nr ? i : 0;   // a row of the block; its w is zero past nr
    double a[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) a[v] = (double)ap[(int64_t)v * lda + ic];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = fma(a[v], wr[u], acc[v]);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v)
    for (int o = 32; o > 0; o >>= 1) acc[v] += __shfl_xor(acc[v], o);
  const int wv = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) sh[wv][v] = acc[v];
  }
  __syncthreads();
  if ((int)threadIdx.x < NV) {
    double s = 0.0;
    for (int q = 0; q < KB2 / 64; ++q) s += sh[q][threadIdx.x];
    out[(int64_t)threadIdx.x * ostride] = s;
  }
}

// partial[kpoff + k*kb + lb] = sum_{rows of block lb} A[k*lda + off + i] * w[off + i],
// k < (jc ? jc[c] + 1 : 1).  The block's w rows stay in registers; the columns go in
// passes of 8 (then 4, 2, 1 for the rest), each a single block reduction.
template <typename TA>
__global__ __launch_bounds__(KB2) void bmultidot_kernel(const ConfDev* __restrict__ cf,
                                                        const int2* __restrict__ blk,
                                                        const TA* __restrict__ A, int64_t lda,
                                                        const int* __restrict__ jc,
                                                        const double* __restrict__ w,
                                                        const int* __restrict__ mask,
                                                        double* __restrict__ partial) {
  __shared__ double sh[2][KB2 / 64][8];
  const int2 b = blk[blockIdx.x];
  const int c = b.x;
  if (!mask[c]) return;
  const ConfDev& cd = cf[c];
  const int kc = jc ? jc[c] + 1 : 1;
  const int64_t r0 = (int64_t)b.y * KR;
  const int nr = (int)min((int64_t)KR, cd.N - r0);
  const double* wp = w + cd.off + r0;
  double wr[KU];
#pragma unroll
  for (int u = 0; u < KU; ++u) {
    const int i = threadIdx.x + u * KB2;
    wr[u] = i < nr ? wp[i] : 0.0;
  }
  const TA* ap = A + cd.off + r0;
  double* out = partial + cd.kpoff + b.y;
  int k0 = 0, par = 0;
  for (; k0 + 8 <= kc; k0 += 8, par ^= 1)
    mdot_pass<8>(ap + k0 * lda, lda, nr, wr, sh[par], out + (int64_t)k0 * cd.kb, cd.kb);
  if (kc - k0 >= 4) {
    mdot_pass<4>(ap + k0 * lda, lda, nr, wr, sh[par], out + (int64_t)k0 * cd.kb, cd.kb);
    k0 += 4;
    par ^= 1;
  }
  if (kc - k0 >= 2) {
    mdot_pass<2>(ap + k0 * lda, lda, nr, wr, sh[par], out + (int64_t)k0 * cd.kb, cd.kb);
    k0 += 2;
    par ^= 1;
  }
  if (kc - k0 >= 1) mdot_pass<1>(ap + k0 * lda, lda, nr, wr, sh[par], out + (int64_t)k0 * cd.kb, cd.kb);
}

// out[c*stride + off + k] = sum_lb partial[kpoff + k*kb + lb]
__global__ void breduce_kernel(const ConfDev* __restrict__ cf, int nconf, int kmax,
                               const int* __restrict__ jc, const int* __restrict__ mask,
                               const double* __restrict__ partial, double* __restrict__ out,
                               int stride, int off) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = t / kmax, k = t % kmax;
  if (c >= nconf || !mask[c]) return;
  const int kc = jc ? jc[c] + 1 : 1;
  if (k >= kc) return;
  const ConfDev& cd = cf[c];
  double s = 0.0;
  for (int lb = 0; lb < cd.kb; ++lb) s += partial[cd.kpoff + (int64_t)k * cd.kb + lb];
  out[(int64_t)c * stride + off + k] = s;
}

// w[g] += alpha * sum_{k < ncols(c)} V[k*T + g] * h[c*stride + off + k] on the block's
// rows, ncols = jc[c] + 1 (Arnoldi) or kc[c] (solution update).  A thread keeps the sums
// of its KU rows and loads two columns of all of them at once; each row's sum runs in k
// order.
template <typename TV>
__global__ __launch_bounds__(KB2) void bupdate_kernel(const ConfDev* __restrict__ cf,
                                                      const int2* __restrict__ blk, int64_t T,
                                                      const int* __restrict__ mask,
                                                      const int* __restrict__ jc,
                                                      const int* __restrict__ kc,
                                                      const TV* __restrict__ V,
                                                      const double* __restrict__ h, int stride,
                                                      int off, double alpha,
                                                      double* __restrict__ w) {
  const int2 b = blk[blockIdx.x];
  const int c = b.x;
  if (!mask[c]) return;
  const ConfDev& cd = cf[c];
  const int n = jc ? jc[c] + 1 : kc[c];
  const int64_t r0 = (int64_t)b.y * KR;
  const int nr = (int)min((int64_t)KR, cd.N - r0);
  const double* hc = h + (int64_t)c * stride + off;
  const TV* vp = V + cd.off + r0;
  double* wp = w + cd.off + r0;
  int ir[KU];
  double sum[KU];
#pragma unroll
  for (int u = 0; u < KU; ++u) {
    const int i = threadIdx.x + u * KB2;
    ir[u] = i < nr ? i : 0;   // past nr: a row of the block, its sum never stored
    sum[u] = 0.0;
  }
  int k = 0;
  for (; k + 2 <= n; k += 2) {
    double a0[KU], a1[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      a0[u] = (double)vp[(int64_t)k * T + ir[u]];
      a1[u] = (double)vp[(int64_t)(k + 1) * T + ir[u]];
    }
    const double h0 = hc[k], h1 = hc[k + 1];
#pragma unroll
    for (int u = 0; u < KU; ++u) sum[u] = fma(a1[u], h1, fma(a0[u], h0, sum[u]));
  }
  if (k < n) {
    const double h0 = hc[k];
#pragma unroll
    for (int u = 0; u < KU; ++u) sum[u] = fma((double)vp[(int64_t)k * T + ir[u]], h0, sum[u]);
  }
#pragma unroll
  for (int u = 0; u < KU; ++u) {
    const int i = threadIdx.x + u * KB2;
    if (i < nr) wp[i] = fma(alpha, sum[u], wp[i]);
  }
}

// Device-side Arnoldi bookkeeping, one thread per configuration.
__global__ void bgivens_kernel(int nconf, int m, int* __restrict__ active, int* __restrict__ jc,
                               int* __restrict__ kc, const double* __restrict__ hb, int hstride,
                               double* __restrict__ H, double* __restrict__ cs,
                               double* __restrict__ sn, double* __restrict__ gv,
                               double* __restrict__ scale, const double* __restrict__ bnorm,
                               const double* __restrict__ rtol, double* __restrict__ res,
                               int* __restrict__ conv) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nconf || !active[c]) return;
  const int j = jc[c];
  const double* h = hb + (int64_t)c * hstride;
  double* Hc = H + (int64_t)c * (m + 1) * m;
  double* col = Hc + (int64_t)j * (m + 1);
  double* csc = cs + (int64_t)c * m;
  double* snc = sn + (int64_t)c * m;
  double* g = gv + (int64_t)c * (m + 1);
  for (int i = 0; i <= j; ++i) col[i] = h[i] + h[m + 1 + i];
  const double hn = sqrt(fmax(h[2 * (m + 1)], 0.0));
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double t = csc[i] * col[i] + snc[i] * col[i + 1];
    col[i + 1] = -snc[i] * col[i] + csc[i] * col[i + 1];
    col[i] = t;
  }
  const double den = hypot(col[j], col[j + 1]);
  csc[j] = den > 0.0 ? col[j] / den : 1.0;
  snc[j] = den > 0.0 ? col[j + 1] / den : 0.0;
  col[j] = den;
  col[j + 1] = 0.0;
  g[j + 1] = -snc[j] * g[j];
  g[j] = csc[j] * g[j];
  const double r = fabs(g[j + 1]) / bnorm[c];
  res[c] = r;
  jc[c] = j + 1;
  kc[c] = j + 1;
  scale[c] = hn > 0.0 ? 1.0 / hn : 0.0;
  if (r <= rtol[c] || hn == 0.0 || j + 1 >= m) {
    active[c] = 0;
    conv[c] = r <= rtol[c] ? 1 : 0;
  }
}

// V[jc[c]*T + g] = w[g] * scale[c] on the block's rows, and its FP32 copy in V32 when
// given (the mixed solves' Gram-Schmidt passes read the copy).
__global__ __launch_bounds__(KB2) void bscale_kernel(const ConfDev* __restrict__ cf,
                                                     const int2* __restrict__ blk, int64_t T,
                                                     const int* __restrict__ mask,
                                                     const int* __restrict__ jc,
                                                     const double* __restrict__ scale,
                                                     const double* __restrict__ w,
                                                     double* __restrict__ V,
                                                     float* __restrict__ V32) {
  const int2 b = blk[blockIdx.x];
  const int c = b.x;
  if (!mask[c]) return;
  const ConfDev& cd = cf[c];
  const int64_t r0 = (int64_t)b.y * KR;
  const int nr = (int)min((int64_t)KR, cd.N - r0);
  const double sc = scale[c];
  const double* wp = w + cd.off + r0;
  const int64_t o = (int64_t)jc[c] * T + cd.off + r0;
  for (int i = threadIdx.x; i < nr; i += KB2) {
    const double v = wp[i] * sc;
    V[o + i] = v;
    if (V32) V32[o + i] = (float)v;
  }
}

// y = H^-1 g for the kc[c] columns of the finished cycle.
__global__ void bsolve_kernel(int nconf, int m, const int* __restrict__ mask,
                              const int* __restrict__ kc, const double* __restrict__ H,
                              const double* __restrict__ gv, double* __restrict__ y) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nconf || !mask[c]) return;
  const int k = kc[c];
  const double* Hc = H + (int64_t)c * (m + 1) * m;
  const double* g = gv + (int64_t)c * (m + 1);
  double* yc = y + (int64_t)c * m;
  for (int i = k - 1; i >= 0; --i) {
    double t = g[i];
    for (int q = i + 1; q < k; ++q) t -= Hc[(int64_t)q * (m + 1) + i] * yc[q];
    yc[i] = t / Hc[(int64_t)i * (m + 1) + i];
  }
}

// out = a*x + b*y on the nodes of masked configurations (y may be null).
__global__ void baxpby_kernel(const int* __restrict__ node_conf, int64_t T,
                              const int* __restrict__ mask, double a, const double* __restrict__ x,
                              double b, const double* __restrict__ y, double* __restrict__ out) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= T) return;
  const int c = node_conf[g];
  if (c < 0 || !mask[c]) return;
  out[g] = a * x[g] + (y ? b * y[g] : 0.0);
}

__global__ void round_f32_kernel(const double* __restrict__ a, int64_t n, float* __restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

__global__ void fill_int_kernel(int* __restrict__ p, int64_t n, int v) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < n) p[g] = v;
}

static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

// ---- host engine -----------------------------------------------------------------------------

Engine::~Engine() {
  drop_graphs();
  for (auto& pv : prof_ev)
    for (auto& v : pv)
      for (auto& e : v) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
  for (auto e : ev_pool) (void)hipEventDestroy(e);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

void Engine::init(const yq_params& p) {
  prm = p;
  m = p.restart;
  if (!stream) {
    YQ_HIP(hipStreamCreate(&stream));  // default priority
    own_stream = true;
  }
  std::vector<double> t(T_SIZE_HOST);
  fill_tab64(t.data());
  tab64.alloc(t.size());
  YQ_HIP(hipMemcpyAsync(tab64.p, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  YQ_HIP(hipStreamSynchronize(stream));
}

// Rebuilds the descriptors, work lists and per-configuration reduction blocks.
void Engine::rebuild() {
  const int nc = (int)members.size();
  std::vector<ConfDev> h(nc);
  std::vector<int4> it, sit;
  std::vector<int2> kb;
  std::vector<FmmForest::Tree> tin, thi;
  std::vector<int2> fi;
  int64_t npart = 0;
  int64_t kpoff = 0;
  for (int c = 0; c < nc; ++c) {
    Member& mb = members[c];
    yq_problem* pb = mb.pb;
    ConfDev& d = h[c];
    std::memset(&d, 0, sizeof(d));
    if (pb) {
      d.x = pb->x.p;
      d.y = pb->y.p;
      d.wnx = pb->wnx.p;
      d.wny = pb->wny.p;
      d.f32 = pb->far32();
      d.rel = pb->frel.p;
      d.W = pb->W.p;
      if (prm.precision == YQ_MIXED && pb->W.n) {
        if (pb->W32.n != pb->W.n || pb->W32_src != pb->W.p) {
          pb->W32.alloc(pb->W.n);
          round_f32_kernel<<<nb256((int64_t)pb->W.n), 256, 0, stream>>>(pb->W.p, (int64_t)pb->W.n,
                                                                        pb->W32.p);
          YQ_HIP(hipGetLastError());
          pb->W32_src = pb->W.p;
        }
        d.W32 = pb->W32.p;
      }
      d.xrow = pb->xrow.p;
      d.xpan = pb->xpan.p;
      d.xvals = pb->x_total > 0 ? pb->xvals.p : nullptr;
      d.tab = pb->tab.p;
      d.part64 = pb->partial.p;
      d.part32 = pb->partial32.p;
      d.N = pb->N;
      d.off = mb.off;
      d.kappa = pb->kappa;
      d.kap2 = pb->kappa * pb->kappa;
      d.P = pb->prm.panels_per_particle;
      d.win = pb->prm.qbx_window;
      d.tblocks = pb->fp.tblocks;
      d.chunks = pb->fp.chunks;
      d.chunk = pb->fp.chunk;
      d.kb = (int)((pb->N + KR - 1) / KR);
      d.kpoff = kpoff;
      kpoff += (int64_t)(m + 1) * d.kb;
      if (pb->fmm) {
        // FMM member: the forests write its far field to its FP64 partial buffer
        YQ_REQUIRE(pb->fmm_hi, YQ_EINVAL, "an FMM member of the batch engine needs fmm_resid_order > 0");
        d.fmm = 1;
        d.chunks = 1;
        pb->gpartial.reserve((size_t)2 * pb->N);
        tin.push_back(FmmForest::Tree{pb->fmm.get(), c, mb.off, pb->partial.p, nullptr, pb->tab.p});
        thi.push_back(FmmForest::Tree{pb->fmm_hi.get(), c, mb.off, pb->partial.p, pb->gpartial.p,
                                      pb->tab.p});
      } else {
        pb->gpartial.reserve((size_t)d.chunks * 2 * pb->N);
        for (int t = 0; t < d.tblocks; ++t)
          for (int s = 0; s < d.chunks; ++s) it.push_back(make_int4(c, t, s, 0));
        d.chunks32 = d.chunks;
        if (sym32) {
          d.chunks32 = (int)((pb->N + SC - 1) / SC);
          pb->partial32.reserve((size_t)d.chunks32 * pb->N);
          d.part32 = pb->partial32.p;
          for (int p = 0; p < d.chunks32; ++p)
            for (int q = p; q < d.chunks32; ++q) sit.push_back(make_int4(c, p, q, 0));
        }
      }
      for (int b = 0; b < d.kb; ++b) kb.push_back(make_int2(c, b));
      d.nx = pb->nx.p;
      d.ny = pb->ny.p;
      d.w = pb->w.p;
      d.pc = pb->pc.p;
      d.WGx = pb->WGx.p;
      d.WGy = pb->WGy.p;
      d.xgvals = pb->x_total > 0 ? pb->xgvals.p : nullptr;
      d.gpart = pb->gpartial.p;
      d.n = pb->n;
      d.poff = mb.poff;
      for (int q = 0; q < pb->n; ++q) fi.push_back(make_int2(c, q));
      npart = std::max<int64_t>(npart, mb.poff + pb->n);
    }
  }
  nitems = (int)it.size();
  nkblk = (int)kb.size();
  // symmetric items by decreasing pair count (the persistent grid deals them in order;
  // each item's sums do not depend on the order)
  auto spairs = [&](const int4& v) {
    const int64_t N = h[v.x].N;
    const int64_t na = std::min<int64_t>(SC, N - (int64_t)v.y * SC);
    const int64_t nb = std::min<int64_t>(SC, N - (int64_t)v.z * SC);
    return v.y == v.z ? na * na : 2 * na * nb;
  };
  std::stable_sort(sit.begin(), sit.end(),
                   [&](const int4& u, const int4& v) { return spairs(u) > spairs(v); });
  nsitems = (int)sit.size();
  sitems.alloc(std::max(nsitems, 1));
  if (nsitems)
    YQ_HIP(hipMemcpyAsync(sitems.p, sit.data(), nsitems * sizeof(int4), hipMemcpyHostToDevice, stream));
  nfitems = (int)fi.size();
  fitems.alloc(std::max(nfitems, 1));
  if (nfitems)
    YQ_HIP(hipMemcpyAsync(fitems.p, fi.data(), nfitems * sizeof(int2), hipMemcpyHostToDevice, stream));
  pen.alloc(std::max<int64_t>(npart, 1));
  // the Krylov basis and work vectors before the caches, which take what is left
  V.reserve((size_t)(m + 1) * std::max<int64_t>(T, 1));
  w.reserve(std::max<int64_t>(T, 1));
  r.reserve(std::max<int64_t>(T, 1));
  tmp.reserve(std::max<int64_t>(T, 1));
  delta.reserve(std::max<int64_t>(T, 1));
  f.reserve(std::max<int64_t>(T, 1));
  // near-field caches within the budget, FP32 (inner operator, every iteration)
  // first; a tree keeps its cache until its geometry changes
  {
    int64_t held = 0;
    for (auto* tv : {&tin, &thi})
      for (auto& t : *tv)
        if (t.fmm->nc_kind) held += t.fmm->near_cache_bytes(t.fmm->nc_kind == 2);
    int64_t budget = near_budget;
    if (budget < 0) {   // what is free (with the caches held) less a reserve for later work
      size_t fr = 0, tot = 0;
      YQ_HIP(hipMemGetInfo(&fr, &tot));
      const int64_t reserve = std::max<int64_t>((int64_t)8 << 30, (int64_t)tot / 10);
      budget = std::max<int64_t>(0, (int64_t)fr + held - reserve);
    }
    int64_t used = 0;
    near_trees32 = near_trees64 = 0;
    for (int pass = 0; pass < 2; ++pass) {
      const bool f64 = pass == 1;
      for (auto& t : f64 ? thi : tin) {
        const int want = f64 ? 2 : 1;
        const int64_t need = t.fmm->near_cache_bytes(f64);
        if (t.fmm->near_cacheable() && used + need <= budget) {
          if (t.fmm->nc_kind != want) t.fmm->build_near_cache(f64, t.tab, stream);
          used += need;
          (f64 ? near_trees64 : near_trees32) += 1;
        } else if (t.fmm->nc_kind) {
          t.fmm->drop_near_cache();
        }
      }
    }
    near_bytes = used;
  }
  // QBX corrections folded into the caches just built (a kept cache keeps its fold);
  // the panels left out are recorded with the configuration's geometry
  {
    DevBuf<int> ip;
    bool used_ip = false;
    std::vector<yq_problem*> refolded;
    for (int pass = 0; pass < 2; ++pass) {
      const bool f64 = pass == 1;
      for (auto& t : f64 ? thi : tin) {
        Fmm& f = *t.fmm;
        yq_problem* pb = members[t.cfg].pb;
        if (f.nc_kind != (f64 ? 2 : 1) || !pb || !pb->W.n || f.N == 0) continue;
        if (f.nc_folded && f.nc_folded != (const void*)pb->W.p)
          f.build_near_cache(f64, t.tab, stream);   // folded from other weights
        if (!f.nc_folded) {
          const int64_t N = f.N;
          if (ip.n < (size_t)N) {
            if (used_ip) YQ_HIP(hipStreamSynchronize(stream));
            ip.alloc((size_t)N);
          }
          used_ip = true;
          pb->qf_umask.fit((size_t)N);
          pb->qf_xmask.fit((size_t)std::max<int64_t>(pb->x_total, 1));
          iperm_kernel<<<nb256(N), 256, 0, stream>>>(N, f.perm.p, ip.p);
          const double scale = 2.0 * PI / (pb->kappa * pb->kappa);
          const double* xv = pb->x_total > 0 ? pb->xvals.p : nullptr;
#define YQ_FOLD(TC, C)                                                                             \
  qbx_fold_kernel<TC><<<nb256(N), 256, 0, stream>>>(                                               \
      N, pb->prm.panels_per_particle, pb->prm.qbx_window, pb->W.p, pb->xrow.p, pb->xpan.p, xv,     \
      f.perm.p, ip.p, f.leaf_of.p, f.leaf_start.p, f.leaf_cnt.p, f.nbp.p, f.nbi.p, f.blk_off.p,     \
      scale, C, pb->qf_umask.p, pb->qf_xmask.p)
          if (f64)
            YQ_FOLD(double, f.nc64.p);
          else
            YQ_FOLD(float, f.nc32.p);
#undef YQ_FOLD
          YQ_HIP(hipGetLastError());
          f.nc_folded = pb->W.p;
          if (std::find(refolded.begin(), refolded.end(), pb) == refolded.end())
            refolded.push_back(pb);
        }
        ConfDev& d = h[t.cfg];
        (f64 ? d.qfold64 : d.qfold32) = 1;
        d.qumask = pb->qf_umask.p;
        d.qxmask = pb->qf_xmask.p;
      }
    }
    // the nodes with panels left out, per geometry folded now (kept folds keep theirs)
    for (yq_problem* pb : refolded) {
      pb->qf_left.fit((size_t)std::max<int64_t>(pb->N, 1));
      pb->qf_cnt.fit(1);
      fill_int_kernel<<<1, 256, 0, stream>>>(pb->qf_cnt.p, 1, 0);
      qbx_left_kernel<<<nb256(pb->N), 256, 0, stream>>>(pb->N, pb->qf_umask.p, pb->qf_left.p,
                                                        pb->qf_cnt.p);
    }
    std::vector<int> hc(refolded.size());
    for (size_t q = 0; q < refolded.size(); ++q)
      YQ_HIP(hipMemcpyAsync(&hc[q], refolded[q]->qf_cnt.p, sizeof(int), hipMemcpyDeviceToHost,
                            stream));
    YQ_HIP(hipStreamSynchronize(stream));
    for (size_t q = 0; q < refolded.size(); ++q) refolded[q]->qf_nleft = hc[q];
    // one list over the batch, in configuration order
    int64_t nl = 0;
    for (int c = 0; c < nc; ++c)
      if ((h[c].qfold32 || h[c].qfold64) && members[c].pb) nl += members[c].pb->qf_nleft;
    nlitems = (int)nl;
    litems.fit((size_t)std::max<int64_t>(nl, 1));
    nl = 0;
    for (int c = 0; c < nc; ++c) {
      yq_problem* pb = members[c].pb;
      if (!(h[c].qfold32 || h[c].qfold64) || !pb || pb->qf_nleft == 0) continue;
      left_items_kernel<<<nb256(pb->qf_nleft), 256, 0, stream>>>(pb->qf_nleft, c, pb->qf_left.p,
                                                                  litems.p + nl);
      nl += pb->qf_nleft;
    }
    YQ_HIP(hipGetLastError());
    if (used_ip) YQ_HIP(hipStreamSynchronize(stream));   // before the scratch buffer goes
  }
  // the basis's FP32 copy for the mixed solves' Gram-Schmidt passes, out of what the
  // caches left
  if (prm.precision == YQ_MIXED)
    V32.reserve((size_t)(m + 1) * std::max<int64_t>(T, 1));
  else
    V32.release();
  forest_in.build(tin, true, stream);
  forest_hi.build(thi, false, stream);
  conf.alloc(std::max(nc, 1));
  items.alloc(std::max(nitems, 1));
  kblk.alloc(std::max(nkblk, 1));
  node_conf.alloc(std::max<int64_t>(T, 1));
  kpart.alloc(std::max<int64_t>(kpoff, 1));
  if (nc) YQ_HIP(hipMemcpyAsync(conf.p, h.data(), nc * sizeof(ConfDev), hipMemcpyHostToDevice, stream));
  if (nitems) YQ_HIP(hipMemcpyAsync(items.p, it.data(), nitems * sizeof(int4), hipMemcpyHostToDevice, stream));
  if (nkblk) YQ_HIP(hipMemcpyAsync(kblk.p, kb.data(), nkblk * sizeof(int2), hipMemcpyHostToDevice, stream));
  // node -> configuration map (-1 on free arena ranges)
  if (T) {
    fill_int_kernel<<<nb256(T), 256, 0, stream>>>(node_conf.p, T, -1);
    for (int c = 0; c < nc; ++c)
      if (members[c].pb && members[c].pb->N > 0)
        fill_int_kernel<<<nb256(members[c].pb->N), 256, 0, stream>>>(node_conf.p + members[c].off,
                                                                   members[c].pb->N, c);
    YQ_HIP(hipGetLastError());
  }
  // per-configuration state; flags start at zero when (re)allocated and are
  // otherwise kept, so configurations in the middle of a cycle survive a rebuild
  const int hs = 2 * (m + 1) + 2;
  const bool fresh = active.n != (size_t)std::max(nc, 1);
  active.alloc(std::max(nc, 1));
  inc.alloc(std::max(nc, 1));
  pmask.alloc(std::max(nc, 1));
  fmask.alloc(std::max(nc, 1));
  jc.alloc(std::max(nc, 1));
  kc.alloc(std::max(nc, 1));
  conv.alloc(std::max(nc, 1));
  hb.alloc((size_t)std::max(nc, 1) * hs);
  H.alloc((size_t)std::max(nc, 1) * (m + 1) * m);
  cs.alloc((size_t)std::max(nc, 1) * m);
  sn.alloc((size_t)std::max(nc, 1) * m);
  gv.alloc((size_t)std::max(nc, 1) * (m + 1));
  yv.alloc((size_t)std::max(nc, 1) * m);
  scale.alloc(std::max(nc, 1));
  bnorm.alloc(std::max(nc, 1));
  rtol.alloc(std::max(nc, 1));
  res.alloc(std::max(nc, 1));
  nrm.alloc(std::max(nc, 1));
  if (fresh) {
    fill_int_kernel<<<nb256(std::max(nc, 1)), 256, 0, stream>>>(active.p, std::max(nc, 1), 0);
    fill_int_kernel<<<nb256(std::max(nc, 1)), 256, 0, stream>>>(kc.p, std::max(nc, 1), 0);
    fill_int_kernel<<<nb256(std::max(nc, 1)), 256, 0, stream>>>(jc.p, std::max(nc, 1), 0);
    fill_int_kernel<<<nb256(std::max(nc, 1)), 256, 0, stream>>>(conv.p, std::max(nc, 1), 0);
    YQ_HIP(hipGetLastError());
  }
  drop_graphs();
  YQ_HIP(hipStreamSynchronize(stream));
}

int Engine::grid_blocks(int n) const {
  const int want = persist_blocks > 0 ? persist_blocks : 2048;
  return std::max(1, std::min(n, want));
}

unsigned long long* Engine::prof_counter(int prec, int kind) const {
  return prof_on ? prof_pairs.p + 2 * (2 * (prec == YQ_MIXED ? 1 : 0) + kind) : nullptr;
}

void Engine::prof_record(int prec, int kind, hipEvent_t a, hipEvent_t b) {
  prof_ev[prec == YQ_MIXED ? 1 : 0][kind].push_back({a, b});
}

// The parts of out = A sigma (precision prec) for configurations in mask, input
// column from V/col: 0 packs the FP32 source records (mixed only) and computes the
// FMM members' expansions (inner operator, or the FP64 residual operator), 1 their
// leaf pass, 2 the fused far-field kernel of the direct members, 3 the chunk sums
// (or the forest's far field) and near correction.
void Engine::matvec_part(int part, int prec, const int* mask, const double* Vin, const int* col,
                         double* out) {
  const FmmForest& fo = prec == YQ_MIXED ? forest_in : forest_hi;
  if (part == 0) {
    if (prec == YQ_MIXED && nitems > 0)
      bpack32_kernel<<<nb256(T), 256, 0, stream>>>(conf.p, node_conf.p, T, mask, Vin, col,
                                                   sym32 ? 1 : 0);
    fo.expansions(mask, Vin, col, T, stream);
    fo.l2p(mask, stream);
  } else if (part == PART_LEAF) {
    fo.leaves(mask, stream, prof_counter(prec, PK_LEAF));
  } else if (part == PART_DIRECT) {
    if (nitems == 0) return;
    unsigned long long* pc = prof_counter(prec, PK_DIRECT);
    if (prec == YQ_MIXED && sym32)
      bsym32_kernel<<<grid_blocks(nsitems), BB, 0, stream>>>(conf.p, sitems.p, nsitems, mask, pc);
    else if (prec == YQ_MIXED)
      bfar32_kernel<<<grid_blocks(nitems), BB, 0, stream>>>(conf.p, items.p, nitems, mask, pc);
    else
      bfar64_kernel<<<grid_blocks(nitems), BB, 0, stream>>>(conf.p, items.p, nitems, mask, Vin, col, T,
                                                      tab64.p, pc);
  } else {
    if (nkblk)
      bfinish_kernel<<<nkblk, KB2, 0, stream>>>(conf.p, kblk.p, T, mask, prec == YQ_MIXED, Vin,
                                                col, out);
    if (nlitems)
      bleft_kernel<<<nb256(nlitems), 256, 0, stream>>>(conf.p, litems.p, nlitems, T, mask,
                                                       prec == YQ_MIXED, Vin, col, out);
  }
  YQ_HIP(hipGetLastError());
}

// out = A sigma; with the timers on, the leaf pass and the direct far-field launch
// are bracketed by events.
void Engine::matvec(int prec, const int* mask, const double* Vin, const int* col, double* out) {
  for (int part = 0; part < NPART; ++part) {
    const int kind = part == PART_LEAF ? PK_LEAF : part == PART_DIRECT ? PK_DIRECT : -1;
    hipEvent_t a = prof_on && kind >= 0 ? prof_event() : nullptr;
    if (a) YQ_HIP(hipEventRecord(a, stream));
    matvec_part(part, prec, mask, Vin, col, out);
    if (a) {
      hipEvent_t b = prof_event();
      YQ_HIP(hipEventRecord(b, stream));
      prof_record(prec, kind, a, b);
    }
  }
}

// nrm[c] = x_c . y_c for masked configurations (device)
void Engine::dots(const int* mask, const double* x, const double* y) {
  const int nc = (int)members.size();
  if (nkblk == 0) return;
  bmultidot_kernel<<<nkblk, KB2, 0, stream>>>(conf.p, kblk.p, x, 0, nullptr, y, mask, kpart.p);
  YQ_HIP(hipGetLastError());
  breduce_kernel<<<nb256(nc), 256, 0, stream>>>(conf.p, nc, 1, nullptr, mask, kpart.p, nrm.p, 1, 0);
  YQ_HIP(hipGetLastError());
}

void Engine::axpby(const int* mask, double a, const double* x, double b, const double* y,
                   double* out) {
  baxpby_kernel<<<nb256(T), 256, 0, stream>>>(node_conf.p, T, mask, a, x, b, y, out);
  YQ_HIP(hipGetLastError());
}

// One Arnoldi step for every active configuration (the captured sequence).
void Engine::iteration(int prec) {
  for (int part = 0; part < NPART; ++part) iteration_part(prec, part);
}

// The parts of an Arnoldi step are those of its matvec; the last one also holds the
// orthogonalisation, Givens step and normalisation.
void Engine::iteration_part(int prec, int part) {
  if (part < NPART - 1) {
    matvec_part(part, prec, active.p, V.p, jc.p, w.p);
    return;
  }
  const int nc = (int)members.size();
  const int hs = 2 * (m + 1) + 2;
  matvec_part(NPART - 1, prec, active.p, V.p, jc.p, w.p);
  if (nkblk == 0) return;   // no configuration has nodes
  // the mixed solves orthogonalise against the basis's FP32 copy (the Arnoldi relation
  // then holds to FP32 rounding, far below the inner tolerance; the operator's input
  // and the solution update use the FP64 basis)
  const bool k32 = prec == YQ_MIXED && V32.p;
  for (int pass = 0; pass < 2; ++pass) {
    if (k32)
      bmultidot_kernel<<<nkblk, KB2, 0, stream>>>(conf.p, kblk.p, (const float*)V32.p, T, jc.p,
                                                  w.p, active.p, kpart.p);
    else
      bmultidot_kernel<<<nkblk, KB2, 0, stream>>>(conf.p, kblk.p, (const double*)V.p, T, jc.p,
                                                  w.p, active.p, kpart.p);
    breduce_kernel<<<nb256((int64_t)nc * (m + 1)), 256, 0, stream>>>(
        conf.p, nc, m + 1, jc.p, active.p, kpart.p, hb.p, hs, pass * (m + 1));
    if (k32)
      bupdate_kernel<<<nkblk, KB2, 0, stream>>>(conf.p, kblk.p, T, active.p, jc.p, nullptr,
                                                (const float*)V32.p, hb.p, hs, pass * (m + 1),
                                                -1.0, w.p);
    else
      bupdate_kernel<<<nkblk, KB2, 0, stream>>>(conf.p, kblk.p, T, active.p, jc.p, nullptr,
                                                (const double*)V.p, hb.p, hs, pass * (m + 1),
                                                -1.0, w.p);
  }
  bmultidot_kernel<<<nkblk, KB2, 0, stream>>>(conf.p, kblk.p, w.p, 0, nullptr, w.p, active.p,
                                              kpart.p);
  breduce_kernel<<<nb256(nc), 256, 0, stream>>>(conf.p, nc, 1, nullptr, active.p, kpart.p, hb.p, hs,
                                                2 * (m + 1));
  bgivens_kernel<<<nb256(nc), 256, 0, stream>>>(nc, m, active.p, jc.p, kc.p, hb.p, hs, H.p, cs.p,
                                                sn.p, gv.p, scale.p, bnorm.p, rtol.p, res.p,
                                                conv.p);
  bscale_kernel<<<nkblk, KB2, 0, stream>>>(conf.p, kblk.p, T, active.p, jc.p, scale.p, w.p, V.p,
                                           k32 ? V32.p : nullptr);
  YQ_HIP(hipGetLastError());
}

namespace {
// part < 0: the whole iteration; else one of its three parts
void capture_iteration(Engine& e, int prec, int part, hipGraphExec_t& out) {
  hipGraph_t graph;
  YQ_HIP(hipStreamBeginCapture(e.stream, hipStreamCaptureModeThreadLocal));
  if (part < 0)
    e.iteration(prec);
  else
    e.iteration_part(prec, part);
  YQ_HIP(hipStreamEndCapture(e.stream, &graph));
  YQ_HIP(hipGraphInstantiate(&out, graph, nullptr, nullptr, 0));
  YQ_HIP(hipGraphDestroy(graph));
}
}  // namespace

void Engine::drop_graphs() {
  for (auto& g : graph_exec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  for (auto& g : graph_part)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

void Engine::ensure_graphs() {
  if (!use_graphs || members.empty()) return;
  for (int gi = 0; gi < 2; ++gi) {
    const int prec = gi ? YQ_MIXED : YQ_FP64;
    if (!prof_on) {
      if (!graph_exec[gi]) capture_iteration(*this, prec, -1, graph_exec[gi]);
    } else {
      for (int part = 0; part < NPART; ++part)
        if (!graph_part[NPART * gi + part])
          capture_iteration(*this, prec, part, graph_part[NPART * gi + part]);
    }
  }
}

// One iteration: a replay of the captured graph.  With the timers on, the
// iteration is captured as one graph per part, and events recorded between their
// launches bracket the leaf pass and the direct far-field kernel.
void Engine::run_iteration(int prec) {
  const int gi = prec == YQ_MIXED ? 1 : 0;
  if (use_graphs) {
    ensure_graphs();
    if (!prof_on) {
      YQ_HIP(hipGraphLaunch(graph_exec[gi], stream));
      return;
    }
  }
  for (int part = 0; part < NPART; ++part) {
    const int kind = part == PART_LEAF ? PK_LEAF : part == PART_DIRECT ? PK_DIRECT : -1;
    hipEvent_t a = prof_on && kind >= 0 ? prof_event() : nullptr;
    if (a) YQ_HIP(hipEventRecord(a, stream));
    if (use_graphs)
      YQ_HIP(hipGraphLaunch(graph_part[NPART * gi + part], stream));
    else
      iteration_part(prec, part);
    if (a) {
      hipEvent_t b = prof_event();
      YQ_HIP(hipEventRecord(b, stream));
      prof_record(prec, kind, a, b);
    }
  }
}

hipEvent_t Engine::prof_event() {
  if (!ev_pool.empty()) {
    hipEvent_t e = ev_pool.back();
    ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  YQ_HIP(hipEventCreate(&e));
  return e;
}

void Engine::set_profiling(bool on) {
  if (on == prof_on) return;
  YQ_HIP(hipStreamSynchronize(stream));
  drop_graphs();   // the captured sequence changes with the timers
  prof_on = on;
  if (on && !prof_pairs.p) {
    prof_pairs.alloc(8);
    YQ_HIP(hipMemsetAsync(prof_pairs.p, 0, 8 * sizeof(unsigned long long), stream));
    YQ_HIP(hipStreamSynchronize(stream));
  }
}

void Engine::read_profile(int prec, int kind, int64_t& launches, double& ms, double& pairs,
                          double& bytes, bool reset) {
  const int gi = prec == YQ_MIXED ? 1 : 0;
  auto& ev = prof_ev[gi][kind];
  YQ_HIP(hipStreamSynchronize(stream));
  launches = (int64_t)ev.size();
  ms = 0.0;
  for (auto& e : ev) {
    float t = 0.0f;
    YQ_HIP(hipEventElapsedTime(&t, e.first, e.second));
    ms += t;
  }
  unsigned long long pc[8] = {};
  if (prof_pairs.p)
    YQ_HIP(hipMemcpy(pc, prof_pairs.p, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost));
  const int slot = 2 * (2 * gi + kind);
  pairs = (double)pc[slot];
  bytes = (double)pc[slot + 1];
  if (reset) {
    for (auto& e : ev) {
      ev_pool.push_back(e.first);
      ev_pool.push_back(e.second);
    }
    ev.clear();
    if (prof_pairs.p) {
      YQ_HIP(hipMemsetAsync(prof_pairs.p + slot, 0, 2 * sizeof(unsigned long long), stream));
      YQ_HIP(hipStreamSynchronize(stream));
    }
  }
}

// y = H^-1 g and x += V y for the masked configurations' finished cycles.
void Engine::solve_cycle(const int* mask, double* x) {
  const int nc = (int)members.size();
  bsolve_kernel<<<nb256(nc), 256, 0, stream>>>(nc, m, mask, kc.p, H.p, gv.p, yv.p);
  if (nkblk)
    bupdate_kernel<<<nkblk, KB2, 0, stream>>>(conf.p, kblk.p, T, mask, nullptr, kc.p,
                                              (const double*)V.p, yv.p, m, 0, 1.0, x);
  YQ_HIP(hipGetLastError());
}

__global__ void clear_kernel(int n, const int* __restrict__ mask, int* __restrict__ active) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n && mask[c]) active[c] = 0;
}

void Engine::clear_active(const int* mask) {
  const int nc = (int)members.size();
  clear_kernel<<<nb256(nc), 256, 0, stream>>>(nc, mask, active.p);
  YQ_HIP(hipGetLastError());
}

int Engine::count_active(std::vector<int>& h) {
  const int nc = (int)members.size();
  h.resize(nc);
  YQ_HIP(hipMemcpyAsync(h.data(), active.p, nc * sizeof(int), hipMemcpyDeviceToHost, stream));
  YQ_HIP(hipStreamSynchronize(stream));
  int n = 0;
  for (int v : h) n += v;
  return n;
}

std::vector<double> Engine::read_nrm() {
  const int nc = (int)members.size();
  std::vector<double> h(nc);
  YQ_HIP(hipMemcpyAsync(h.data(), nrm.p, nc * sizeof(double), hipMemcpyDeviceToHost, stream));
  YQ_HIP(hipStreamSynchronize(stream));
  return h;
}

void Engine::upload_mask(DevBuf<int>& d, const std::vector<int>& h) {
  YQ_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice, stream));
}

// Batched restarted GMRES: solve A x_c = b_c (x zero on entry) for configurations in incl.
// Per configuration: relative tolerance tolv[c], iteration budget budget[c] (updated).
void Engine::gmres(int prec, const double* b, double* x, const std::vector<int>& incl,
                   const std::vector<double>& tolv, std::vector<int>& iters,
                   std::vector<int>& budget, std::vector<int>& converged, int& matvecs) {
  const int nc = (int)members.size();
  std::vector<int> part(incl);
  converged.assign(nc, 0);
  upload_mask(inc, part);
  axpby(inc.p, 0.0, b, 0.0, nullptr, x);
  axpby(inc.p, 1.0, b, 0.0, nullptr, r.p);
  dots(inc.p, b, b);
  std::vector<double> bn = read_nrm();
  for (double& v : bn) v = std::sqrt(std::max(v, 0.0));
  std::vector<int> hact;
  bool first = true;
  while (true) {
    if (!first) {
      // r = b - A x for configurations still running
      upload_mask(inc, part);
      matvec(prec, inc.p, x, nullptr, tmp.p);
      ++matvecs;
      axpby(inc.p, 1.0, b, -1.0, tmp.p, r.p);
    }
    first = false;
    dots(inc.p, r.p, r.p);
    std::vector<double> beta = read_nrm();
    std::vector<int> act(nc, 0);
    std::vector<double> sc(nc, 0.0), g0((size_t)nc * (m + 1), 0.0), bnv(nc, 1.0), rt(nc, 0.0);
    int nact = 0;
    for (int c = 0; c < nc; ++c) {
      if (!part[c]) continue;
      const double bt = std::sqrt(std::max(beta[c], 0.0));
      if (bn[c] == 0.0 || bt / bn[c] <= tolv[c]) {
        converged[c] = 1;
        part[c] = 0;
        continue;
      }
      if (budget[c] <= 0) {
        part[c] = 0;
        continue;
      }
      act[c] = 1;
      ++nact;
      sc[c] = 1.0 / bt;
      g0[(size_t)c * (m + 1)] = bt;
      bnv[c] = bn[c];
      rt[c] = tolv[c];
    }
    if (nact == 0) break;
    std::vector<int> zeros(nc, 0);
    upload_mask(active, act);
    upload_mask(jc, zeros);
    upload_mask(kc, zeros);
    upload_mask(conv, zeros);
    YQ_HIP(hipMemcpyAsync(scale.p, sc.data(), nc * sizeof(double), hipMemcpyHostToDevice, stream));
    YQ_HIP(hipMemcpyAsync(gv.p, g0.data(), g0.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    YQ_HIP(hipMemcpyAsync(bnorm.p, bnv.data(), nc * sizeof(double), hipMemcpyHostToDevice, stream));
    YQ_HIP(hipMemcpyAsync(rtol.p, rt.data(), nc * sizeof(double), hipMemcpyHostToDevice, stream));
    // V0 = r / beta
    bscale_kernel<<<nkblk, KB2, 0, stream>>>(conf.p, kblk.p, T, active.p, jc.p, scale.p, r.p, V.p,
                                             prec == YQ_MIXED ? V32.p : nullptr);
    YQ_HIP(hipGetLastError());
    // iterate: at most m steps; the mask retires converged configurations
    int left = nact;
    for (int step = 0; step < m && left > 0; step += 2) {
      run_iteration(prec);
      if (step + 1 < m) run_iteration(prec);
      left = count_active(hact);
    }
    // cycle end: y = H^-1 g and x += V y for the cycle's participants
    upload_mask(inc, act);
    bsolve_kernel<<<nb256(nc), 256, 0, stream>>>(nc, m, inc.p, kc.p, H.p, gv.p, yv.p);
    bupdate_kernel<<<nkblk, KB2, 0, stream>>>(conf.p, kblk.p, T, inc.p, nullptr, kc.p,
                                              (const double*)V.p, yv.p, m, 0, 1.0, x);
    YQ_HIP(hipGetLastError());
    std::vector<int> hk(nc), hc(nc);
    YQ_HIP(hipMemcpyAsync(hk.data(), kc.p, nc * sizeof(int), hipMemcpyDeviceToHost, stream));
    YQ_HIP(hipMemcpyAsync(hc.data(), conv.p, nc * sizeof(int), hipMemcpyDeviceToHost, stream));
    YQ_HIP(hipStreamSynchronize(stream));
    for (int c = 0; c < nc; ++c) {
      if (!act[c]) continue;
      iters[c] += hk[c];
      budget[c] -= hk[c];
      if (hc[c]) {
        converged[c] = 1;
        part[c] = 0;
      } else if (budget[c] <= 0) {
        part[c] = 0;
      }
    }
    int any = 0;
    for (int c = 0; c < nc; ++c) any += part[c];
    if (!any) break;
  }
}

// Forces of every member: the gradient far field (direct members' fused FP64 sums,
// the trees' FP64 forest), the surface gradient with its QBX corrections, the
// per-particle traction integrals, then each member's energy summed on the host in
// particle order.
void Engine::forces(const double* sigma, double gamma, double* force, double* torque,
                    std::vector<double>& energy, const std::vector<char>* grad_done) {
  const int nc = (int)members.size();
  energy.assign(nc, 0.0);
  if (nc == 0) return;
  std::vector<int> all(nc, 0), need(nc, 0);
  int nneed = 0;
  for (int c = 0; c < nc; ++c) {
    all[c] = members[c].pb ? 1 : 0;
    need[c] = all[c] && !(grad_done && (*grad_done)[c]);
    nneed += need[c];
  }
  gx.reserve(std::max<int64_t>(T, 1));
  gy.reserve(std::max<int64_t>(T, 1));
  if (nneed) {   // gradient far field of the members whose solve did not leave it
    upload_mask(pmask, need);
    if (nitems)
      bgrad64_kernel<<<grid_blocks(nitems), BB, 0, stream>>>(conf.p, items.p, nitems, pmask.p, sigma,
                                                       tab64.p);
    forest_hi.apply_grad(pmask.p, sigma, nullptr, T, stream);
  }
  upload_mask(inc, all);
  bfinish_grad_kernel<<<nb256(T), 256, 0, stream>>>(conf.p, node_conf.p, T, inc.p, sigma, gx.p, gy.p);
  if (nfitems)
    bforces_kernel<<<nfitems, FRB, 0, stream>>>(conf.p, fitems.p, f.p, gx.p, gy.p, gamma, force,
                                                torque, pen.p);
  YQ_HIP(hipGetLastError());
  std::vector<double> e(pen.n);
  YQ_HIP(hipMemcpyAsync(e.data(), pen.p, pen.n * sizeof(double), hipMemcpyDeviceToHost, stream));
  YQ_HIP(hipStreamSynchronize(stream));
  for (int c = 0; c < nc; ++c) {
    if (!members[c].pb) continue;
    double t = 0.0;
    for (int q = 0; q < members[c].pb->n; ++q) t += e[members[c].poff + q];
    energy[c] = t;
  }
}

// out = A x (FP64 operator: the direct members' fused FP64 sums, the trees' order-40
// forest) for the configurations in plain or fused; for those in fused the same pass
// over the pairs (and the same expansions) also leaves the gradient far field of x in
// the members' gradient partials.
void Engine::resid(const std::vector<int>& plain, const std::vector<int>& fused, const double* x,
                   double* out) {
  const int nc = (int)members.size();
  std::vector<int> uni(nc);
  int nf = 0;
  for (int c = 0; c < nc; ++c) {
    uni[c] = plain[c] || fused[c];
    nf += fused[c];
  }
  if (nf == 0) {
    upload_mask(inc, uni);
    matvec(YQ_FP64, inc.p, x, nullptr, out);
    return;
  }
  upload_mask(inc, uni);
  upload_mask(pmask, plain);
  upload_mask(fmask, fused);
  forest_hi.expansions(inc.p, x, nullptr, T, stream);
  forest_hi.l2p(inc.p, stream);
  {
    hipEvent_t a = prof_on ? prof_event() : nullptr;
    if (a) YQ_HIP(hipEventRecord(a, stream));
    forest_hi.leaves(inc.p, stream, prof_counter(YQ_FP64, PK_LEAF));
    if (a) {
      hipEvent_t b = prof_event();
      YQ_HIP(hipEventRecord(b, stream));
      prof_record(YQ_FP64, PK_LEAF, a, b);
    }
  }
  forest_hi.leaves_grad(fmask.p, stream);
  if (nitems) {
    unsigned long long* pc = prof_counter(YQ_FP64, PK_DIRECT);
    hipEvent_t a = prof_on ? prof_event() : nullptr;
    if (a) YQ_HIP(hipEventRecord(a, stream));
    bfar64_kernel<<<grid_blocks(nitems), BB, 0, stream>>>(conf.p, items.p, nitems, pmask.p, x, nullptr, T,
                                                    tab64.p, pc);
    if (a) {
      hipEvent_t b = prof_event();
      YQ_HIP(hipEventRecord(b, stream));
      prof_record(YQ_FP64, PK_DIRECT, a, b);
    }
    bfused64_kernel<<<grid_blocks(nitems), BB, 0, stream>>>(conf.p, items.p, nitems, fmask.p, x, nullptr,
                                                      T, tab64.p);
  }
  if (nkblk)
    bfinish_kernel<<<nkblk, KB2, 0, stream>>>(conf.p, kblk.p, T, inc.p, 0, x, nullptr, out);
  if (nlitems)
    bleft_kernel<<<nb256(nlitems), 256, 0, stream>>>(conf.p, litems.p, nlitems, T, inc.p, 0, x,
                                                     nullptr, out);
  YQ_HIP(hipGetLastError());
}

// Full solve (FP64 or mixed with refinement) of every member; results in x.
void Engine::solve(std::vector<yq_solve_info>& info, double* x_out, bool fuse) {
  const int nc = (int)members.size();
  auto t0 = std::chrono::steady_clock::now();
  info.assign(nc, yq_solve_info{});
  grad_ok.assign(nc, 0);
  fuse = fuse && prm.precision == YQ_MIXED;
  // per configuration: the next FP64 residual is expected to meet the tolerance (its
  // inner solve aimed straight at it), so it also computes the forces' gradient
  std::vector<int> expect_last(nc, 0);
  std::vector<int> all(nc, 1), iters(nc, 0), budget(nc, prm.maxiter), conv_c(nc, 0);
  for (int c = 0; c < nc; ++c) all[c] = members[c].pb ? 1 : 0;
  int mv = 0;
  // residual of the final iterate, when the refinement loop computed it last (-1: unknown)
  std::vector<double> res_known(nc, -1.0);
  upload_mask(inc, all);
  dots(inc.p, f.p, f.p);
  std::vector<double> fn = read_nrm();
  for (double& v : fn) v = std::sqrt(std::max(v, 0.0));
  if (prm.precision == YQ_FP64) {
    std::vector<double> tolv(nc, prm.tol);
    gmres(YQ_FP64, f.p, x_out, all, tolv, iters, budget, conv_c, mv);
    for (int c = 0; c < nc; ++c) {
      info[c].iterations = iters[c];
      info[c].matvecs_fp64 = iters[c];
      info[c].outer_steps = 1;
    }
  } else {
    std::vector<int> run(all), dummy;
    axpby(inc.p, 0.0, f.p, 0.0, nullptr, x_out);
    for (int outer = 0; outer < prm.max_refine; ++outer) {
      std::vector<double> rel(nc, 1.0);
      upload_mask(inc, run);
      if (outer == 0) {
        axpby(inc.p, 1.0, f.p, 0.0, nullptr, r.p);
      } else {
        std::vector<int> pl(nc, 0), fu(nc, 0);
        for (int c = 0; c < nc; ++c) {
          fu[c] = run[c] && fuse && expect_last[c];
          pl[c] = run[c] && !fu[c];
          if (fu[c]) grad_ok[c] = 1;
        }
        resid(pl, fu, x_out, tmp.p);
        upload_mask(inc, run);
        axpby(inc.p, 1.0, f.p, -1.0, tmp.p, r.p);
        for (int c = 0; c < nc; ++c)
          if (run[c]) ++info[c].matvecs_fp64;
        dots(inc.p, r.p, r.p);
        std::vector<double> rn = read_nrm();
        for (int c = 0; c < nc; ++c)
          if (run[c]) rel[c] = fn[c] > 0.0 ? std::sqrt(std::max(rn[c], 0.0)) / fn[c] : 0.0;
      }
      int nrun = 0;
      std::vector<double> tolv(nc, 0.5);
      for (int c = 0; c < nc; ++c) {
        if (!run[c]) continue;
        if (rel[c] <= prm.tol || budget[c] <= 0) {
          run[c] = 0;
          if (outer > 0) res_known[c] = rel[c];   // x has not moved since
          continue;
        }
        ++nrun;
        ++info[c].outer_steps;
        tolv[c] = std::min(0.5, std::max(prm.inner_tol, 0.5 * prm.tol / std::max(rel[c], 1e-300)));
        grad_ok[c] = 0;   // the inner solve moves x
        expect_last[c] = rel[c] * tolv[c] <= prm.tol;
      }
      if (!nrun) break;
      // the residual r is the right-hand side of the inner solve; delta -> x
      std::vector<int> it0(nc, 0);
      gmres(YQ_MIXED, r.p, delta.p, run, tolv, it0, budget, conv_c, mv);
      for (int c = 0; c < nc; ++c)
        if (run[c]) {
          iters[c] += it0[c];
          info[c].matvecs_fp32 += it0[c];
        }
      upload_mask(inc, run);
      axpby(inc.p, 1.0, delta.p, 1.0, x_out, x_out);
    }
    for (int c = 0; c < nc; ++c) info[c].iterations = iters[c];
  }
  // true FP64 residual of every member whose final iterate has none yet
  std::vector<int> need(nc, 0);
  int nneed = 0;
  for (int c = 0; c < nc; ++c)
    if (all[c] && res_known[c] < 0.0) {
      need[c] = 1;
      ++nneed;
    }
  std::vector<double> rn(nc, 0.0);
  if (nneed) {
    std::vector<int> none(nc, 0);
    if (fuse)
      for (int c = 0; c < nc; ++c) grad_ok[c] = grad_ok[c] || need[c];
    resid(fuse ? none : need, fuse ? need : none, x_out, tmp.p);
    upload_mask(inc, need);
    axpby(inc.p, 1.0, f.p, -1.0, tmp.p, r.p);
    dots(inc.p, r.p, r.p);
    rn = read_nrm();
  }
  const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int c = 0; c < nc; ++c) {
    if (need[c]) {
      info[c].residual = fn[c] > 0.0 ? std::sqrt(std::max(rn[c], 0.0)) / fn[c] : 0.0;
      info[c].matvecs_fp64 += 1;
    } else {
      info[c].residual = res_known[c];
    }
    info[c].seconds = sec;
  }
}

}  // namespace yq
