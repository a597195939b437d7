// The tiled direct far field and the near-correction apply.
//
// Far field: out_i = (kappa^2/2pi) sum_{j != i} [K1(z)/z] ((x_i - y_j) . q_j),
// z = kappa |x_i - y_j|, q_j = w_j sigma_j nu_j -- the 16-point Nystrom rule of
// the double layer dG/dnu_y = (kappa/2pi) K1(kappa r) (x-y).nu / r for every
// pair (section 4, eq. double-layer-def; section 5).
//
// Mapping: one target per lane, 256-lane blocks; the source range is split
// into chunks (grid.y) so that a launch has enough blocks to fill all compute
// units; each block stages 256-source tiles (x, y, qx, qy) through LDS, and
// every lane reads the same source at the same time (LDS broadcast).  Chunk
// partial sums go to partial[chunk * N + i]; the finish kernel adds them in a
// fixed order (deterministic), scales, and applies the near correction.
#include "bessel.h"
#include <hip/hip_ext.h>

#include "common.h"
#include "farfield_core.h"

namespace yq {

constexpr int FAR_BS = 256;
static_assert(FAR_BS == FT, "FP64 kernels stage one source tile per block iteration");

// Source chunks are chosen so that one configuration alone gives about `want`
// blocks (>= 16 per compute unit at 4096); the plan depends only on the sizes.
FarPlan far_plan(int64_t nt, int64_t ns, int block, int want) {
  FarPlan fp;
  fp.tblocks = (int)((nt + block - 1) / block);
  int64_t src_tiles = (ns + block - 1) / block;
  int64_t chunks = (want + fp.tblocks - 1) / fp.tblocks;
  if (chunks > src_tiles) chunks = src_tiles;
  if (chunks < 1) chunks = 1;
  int64_t tiles_per = (src_tiles + chunks - 1) / chunks;
  fp.chunk = (int)(tiles_per * block);
  fp.chunks = (int)((ns + fp.chunk - 1) / fp.chunk);
  if (fp.chunks < 1) fp.chunks = 1;
  return fp;
}

// stop (may be null): when *stop is set the launch does nothing (an operator
// application that a converged GMRES no longer needs).
template <bool CUT>
__global__ __launch_bounds__(FAR_BS) void far64_kernel(GeomView g, const double* __restrict__ sigma,
                                                       int chunk, double* __restrict__ partial,
                                                       const int* __restrict__ stop) {
  __shared__ double2 sxy[FAR_BS];
  __shared__ double2 sq[FAR_BS];
  if (stop && *as_k(stop)) return;   // uniform over the grid
  const int64_t N = g.N;
  const int64_t i = blockIdx.x * (int64_t)FAR_BS + threadIdx.x;
  const double xi = i < N ? g.x[i] : 0.0;
  const double yi = i < N ? g.y[i] : 0.0;
  const double kap2 = g.kappa * g.kappa;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = min(N, j0 + chunk);
  // target group of this wavefront (whole wavefronts past N keep the general form)
  const int64_t grp = blockIdx.x * (int64_t)(FAR_BS / FG) +
                      __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FG));
  const bool live = grp * FG < N;
  double acc = 0.0;
  // cutoff far field: a wavefront skips a tile whose pairs all lie beyond the
  // cutoff (kappa x gap >= zc); a block skips staging a tile all its wavefronts skip
  // (their flags are written before the first barrier and read after it)
  __shared__ int wsk[FAR_BS / FG];
  const double zc = g.zcut;
  constexpr bool cut = CUT;   // zc < HUGE_VAL: the launchers pick the instantiation
  bool wskip = false;
  for (int64_t jb = j0; jb < j1; jb += FAR_BS) {
    if constexpr (cut) {
      wskip = !live || far64_zmin(g.fgrp, g.ftile, grp, jb / FT, g.kappa) >= zc;
      if (threadIdx.x % FG == 0) wsk[threadIdx.x / FG] = wskip;
    }
    const int64_t j = jb + threadIdx.x;
    __syncthreads();
    bool bskip = cut;
    if constexpr (cut)
      for (int w = 0; w < FAR_BS / FG; ++w) bskip = bskip && wsk[w];
    if (!bskip && j < j1) {
      const double s = sigma[j];
      sxy[threadIdx.x] = make_double2(g.x[j], g.y[j]);
      sq[threadIdx.x] = make_double2(g.wnx[j] * s, g.wny[j] * s);
    }
    __syncthreads();
    if (wskip) continue;
    const int nb = (int)min((int64_t)FAR_BS, j1 - jb);
    // a tile with close pairs is summed panel by panel, each with its own class
    const int tcls = live ? far64_class(g.fgrp, g.ftile, grp, jb / FT, g.kappa) : C64_GENERAL;
    for (int q = 0; q < nb;) {
      const bool split = tcls == C64_GENERAL && live;
      const int cls = split ? far64_class(g.fgrp, g.fpan, grp, (jb + q) / Q, g.kappa) : tcls;
      const int len = split ? Q : nb - q;
      acc = far64_class_tile(cls, xi, yi, sxy + q, sq + q, len, kap2, g.tab, acc);
      q += len;
    }
  }
  if (i < N) partial[(int64_t)blockIdx.y * N + i] = acc;
}

// FP32 far field: one target per lane, one 64-target group per wavefront, a
// block = 256 targets x one source chunk (grid.y).  No LDS and no barrier: the
// sources reach every lane through scalar loads (far32_range).
__global__ __launch_bounds__(FAR_BS) void far32_kernel(Far32View v, int chunk,
                                                       float* __restrict__ partial,
                                                       const int* __restrict__ stop) {
  if (stop && *as_k(stop)) return;   // as in far64_kernel
  const int64_t i = blockIdx.x * (int64_t)FAR_BS + threadIdx.x;
  const int64_t g = blockIdx.x * (int64_t)(FAR_BS / FG) +
                    __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FG));
  if (g * FG >= v.N) return;  // whole wavefront past the last node
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = min(v.N, j0 + chunk);
  const float acc = far32_range(v, i, g, j0, j1);
  if (i < v.N) partial[(int64_t)blockIdx.y * v.N + i] = acc;
}

// Bounding circle of nodes [g G, min(N, g G + G)): centre of the bounding box,
// radius = largest distance from it, enlarged by a relative 1e-12 so that
// rounding cannot leave a node outside.
// One wavefront per circle (four per block): lanes take every 64th node, and
// the bounds and the largest distance are wave reductions (min and max do not
// depend on the order, so the circle is the same as from a serial pass).
__global__ __launch_bounds__(256) void circles_kernel(const double* __restrict__ x,
                                                      const double* __restrict__ y, int64_t N,
                                                      int G, int64_t ng,
                                                      double4* __restrict__ out) {
  const int64_t g = blockIdx.x * (int64_t)4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= ng) return;   // uniform over the wavefront
  const int64_t a = g * G, b = min(N, a + G);
  double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
  for (int64_t j = a + lane; j < b; j += 64) {
    x0 = fmin(x0, x[j]);
    x1 = fmax(x1, x[j]);
    y0 = fmin(y0, y[j]);
    y1 = fmax(y1, y[j]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    x0 = fmin(x0, __shfl_xor(x0, o, 64));
    x1 = fmax(x1, __shfl_xor(x1, o, 64));
    y0 = fmin(y0, __shfl_xor(y0, o, 64));
    y1 = fmax(y1, __shfl_xor(y1, o, 64));
  }
  const double cx = 0.5 * (x0 + x1), cy = 0.5 * (y0 + y1);
  double r2 = 0.0;
  for (int64_t j = a + lane; j < b; j += 64) {
    const double dx = x[j] - cx, dy = y[j] - cy;
    r2 = fmax(r2, dx * dx + dy * dy);
  }
  for (int o = 32; o > 0; o >>= 1) r2 = fmax(r2, __shfl_xor(r2, o, 64));
  const double r = sqrt(r2);
  if (lane == 0) out[g] = make_double4(cx, cy, r + 1e-12 * (r + fabs(cx) + fabs(cy)), 0.0);
}

// Node positions relative to their tile centre, scaled by s = kappa log2(e).
__global__ void rel32_kernel(const double* __restrict__ x, const double* __restrict__ y,
                             int64_t N, const double4* __restrict__ tile, double s,
                             float2* __restrict__ rel) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= N) return;
  const double4 t = tile[j / FT];
  rel[j] = make_float2((float)((x[j] - t.x) * s), (float)((y[j] - t.y) * s));
}

// Per-matvec source records (rel x, rel y, q'x, q'y), q' = w nu sigma c.
__global__ void pack32_kernel(const float2* __restrict__ rel, const double* __restrict__ wnx,
                              const double* __restrict__ wny, const double* __restrict__ sigma,
                              int64_t N, double c, float4* __restrict__ src) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= N) return;
  const double sc = sigma[j] * c;
  const float2 r = rel[j];
  src[j] = make_float4(r.x, r.y, (float)(wnx[j] * sc), (float)(wny[j] * sc));
}

// Gradient far field: grad_x of the double layer,
// (kappa^2/2pi) [ (K1(z)/z) q - ((x-y).q) (x-y) (K0(z) + 2 K1(z)/z) / r^2 ].
template <bool CUT>
__global__ __launch_bounds__(FAR_BS) void far_grad64_kernel(GeomView g,
                                                            const double* __restrict__ sigma,
                                                            int chunk,
                                                            double* __restrict__ partial) {
  __shared__ double2 sxy[FAR_BS];
  __shared__ double2 sq[FAR_BS];
  const int64_t N = g.N;
  const int64_t i = blockIdx.x * (int64_t)FAR_BS + threadIdx.x;
  const double xi = i < N ? g.x[i] : 0.0;
  const double yi = i < N ? g.y[i] : 0.0;
  const double kap2 = g.kappa * g.kappa;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = min(N, j0 + chunk);
  const int64_t grp = blockIdx.x * (int64_t)(FAR_BS / FG) +
                      __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FG));
  const bool live = grp * FG < N;
  double ax = 0.0, ay = 0.0;
  // cutoff far field: a wavefront skips a tile whose pairs all lie beyond the
  // cutoff (kappa x gap >= zc); a block skips staging a tile all its wavefronts skip
  // (their flags are written before the first barrier and read after it)
  __shared__ int wsk[FAR_BS / FG];
  const double zc = g.zcut_g;
  constexpr bool cut = CUT;   // zc < HUGE_VAL: the launchers pick the instantiation
  bool wskip = false;
  for (int64_t jb = j0; jb < j1; jb += FAR_BS) {
    if constexpr (cut) {
      wskip = !live || far64_zmin(g.fgrp, g.ftile, grp, jb / FT, g.kappa) >= zc;
      if (threadIdx.x % FG == 0) wsk[threadIdx.x / FG] = wskip;
    }
    const int64_t j = jb + threadIdx.x;
    __syncthreads();
    bool bskip = cut;
    if constexpr (cut)
      for (int w = 0; w < FAR_BS / FG; ++w) bskip = bskip && wsk[w];
    if (!bskip && j < j1) {
      const double s = sigma[j];
      sxy[threadIdx.x] = make_double2(g.x[j], g.y[j]);
      sq[threadIdx.x] = make_double2(g.wnx[j] * s, g.wny[j] * s);
    }
    __syncthreads();
    if (wskip) continue;
    const int nb = (int)min((int64_t)FAR_BS, j1 - jb);
    const int tcls = live ? far64_class(g.fgrp, g.ftile, grp, jb / FT, g.kappa) : C64_GENERAL;
    for (int q = 0; q < nb;) {   // as in far64_kernel
      const bool split = tcls == C64_GENERAL && live;
      const int cls = split ? far64_class(g.fgrp, g.fpan, grp, (jb + q) / Q, g.kappa) : tcls;
      const int len = split ? Q : nb - q;
      far_grad64_class_tile(cls, xi, yi, sxy + q, sq + q, len, kap2, g.tab, ax, ay);
      q += len;
    }
  }
  if (i < N) {
    partial[((int64_t)blockIdx.y * 2 + 0) * N + i] = ax;
    partial[((int64_t)blockIdx.y * 2 + 1) * N + i] = ay;
  }
}

// Far field and its gradient in one pass: partial[chunk * N + i] as far64_kernel,
// gpartial[(chunk * 2 + c) * N + i] as far_grad64_kernel.
template <bool CUT>
__global__ __launch_bounds__(FAR_BS) void far_fused64_kernel(GeomView g,
                                                             const double* __restrict__ sigma,
                                                             int chunk,
                                                             double* __restrict__ partial,
                                                             double* __restrict__ gpartial) {
  __shared__ double2 sxy[FAR_BS];
  __shared__ double2 sq[FAR_BS];
  const int64_t N = g.N;
  const int64_t i = blockIdx.x * (int64_t)FAR_BS + threadIdx.x;
  const double xi = i < N ? g.x[i] : 0.0;
  const double yi = i < N ? g.y[i] : 0.0;
  const double kap2 = g.kappa * g.kappa;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = min(N, j0 + chunk);
  const int64_t grp = blockIdx.x * (int64_t)(FAR_BS / FG) +
                      __builtin_amdgcn_readfirstlane((int)(threadIdx.x / FG));
  const bool live = grp * FG < N;
  double acc = 0.0, ax = 0.0, ay = 0.0;
  // cutoff far field: a wavefront skips a tile whose pairs all lie beyond the
  // cutoff (kappa x gap >= zc); a block skips staging a tile all its wavefronts skip
  // (their flags are written before the first barrier and read after it)
  __shared__ int wsk[FAR_BS / FG];
  const double zc = g.zcut_g;
  constexpr bool cut = CUT;   // zc < HUGE_VAL: the launchers pick the instantiation
  bool wskip = false;
  for (int64_t jb = j0; jb < j1; jb += FAR_BS) {
    if constexpr (cut) {
      wskip = !live || far64_zmin(g.fgrp, g.ftile, grp, jb / FT, g.kappa) >= zc;
      if (threadIdx.x % FG == 0) wsk[threadIdx.x / FG] = wskip;
    }
    const int64_t j = jb + threadIdx.x;
    __syncthreads();
    bool bskip = cut;
    if constexpr (cut)
      for (int w = 0; w < FAR_BS / FG; ++w) bskip = bskip && wsk[w];
    if (!bskip && j < j1) {
      const double s = sigma[j];
      sxy[threadIdx.x] = make_double2(g.x[j], g.y[j]);
      sq[threadIdx.x] = make_double2(g.wnx[j] * s, g.wny[j] * s);
    }
    __syncthreads();
    if (wskip) continue;
    const int nb = (int)min((int64_t)FAR_BS, j1 - jb);
    const int tcls = live ? far64_class(g.fgrp, g.ftile, grp, jb / FT, g.kappa) : C64_GENERAL;
    for (int q = 0; q < nb;) {   // as in far64_kernel
      const bool split = tcls == C64_GENERAL && live;
      const int cls = split ? far64_class(g.fgrp, g.fpan, grp, (jb + q) / Q, g.kappa) : tcls;
      const int len = split ? Q : nb - q;
      far_fused64_class_tile(cls, xi, yi, sxy + q, sq + q, len, kap2, g.tab, acc, ax, ay);
      q += len;
    }
  }
  if (i < N) {
    partial[(int64_t)blockIdx.y * N + i] = acc;
    gpartial[((int64_t)blockIdx.y * 2 + 0) * N + i] = ax;
    gpartial[((int64_t)blockIdx.y * 2 + 1) * N + i] = ay;
  }
}

// out_i = (kappa^2/2pi) sum_chunks partial + sum_window W sigma + sum_extra vals sigma.
// Eight lanes per node (an aligned group of one wavefront): lane q sums chunks
// q, q + 8, ... and the terms m = 2q, 2q + 1 of every window panel and extra
// panel; the group then combines its sums in a fixed order.  A node's group is
// either wholly inside [0, N) or wholly past it.
__global__ __launch_bounds__(256) void finish_kernel(GeomView g, int win, int chunks,
                                                     const double* __restrict__ p64,
                                                     const float* __restrict__ p32,
                                                     const double* __restrict__ W,
                                                     const int* __restrict__ xrow,
                                                     const int* __restrict__ xpan,
                                                     const double* __restrict__ xvals,
                                                     const double* __restrict__ sigma,
                                                     double* __restrict__ out) {
  const int64_t N = g.N;
  const int64_t t = blockIdx.x * (int64_t)256 + threadIdx.x;
  const int64_t i = t >> 3;
  const int q = (int)(t & 7);
  if (i >= N) return;
  double s = 0.0;
  if (p64) {
    for (int c = q; c < chunks; c += 8) s += p64[(int64_t)c * N + i];
  } else {
    for (int c = q; c < chunks; c += 8) s += (double)p32[(int64_t)c * N + i];
  }
  double corr = 0.0;
  if (win >= 0) {
    const Ring rg = ring_of(g, i / Q);
    const int m0 = 2 * q;
    for (int sl = 0; sl <= 2 * win; ++sl) {
      const double* sg = sigma + ring_step(rg, sl - win) * Q + m0;
      const double* wr = W + ((int64_t)sl * Q + m0) * N + i;
      corr = fma(wr[0], sg[0], corr);
      corr = fma(wr[N], sg[1], corr);
    }
    if (xvals)
      for (int e = xrow[i]; e < xrow[i + 1]; ++e) {
        const double* sg = sigma + (int64_t)xpan[e] * Q + m0;
        const double* vr = xvals + (int64_t)e * Q + m0;
        corr = fma(vr[0], sg[0], corr);
        corr = fma(vr[1], sg[1], corr);
      }
  }
  for (int o = 1; o < 8; o <<= 1) {
    s += __shfl_xor(s, o, 64);
    corr += __shfl_xor(corr, o, 64);
  }
  if (q == 0) out[i] = s * (g.kappa * g.kappa / (2.0 * PI)) + corr;
}

__global__ void finish_grad_kernel(GeomView g, int win, int chunks, const double* __restrict__ part,
                                   const double* __restrict__ WGx, const double* __restrict__ WGy,
                                   const int* __restrict__ xrow, const int* __restrict__ xpan,
                                   const double* __restrict__ xg, const double* __restrict__ sigma,
                                   double* __restrict__ gx, double* __restrict__ gy) {
  const int64_t N = g.N;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  double sx = 0.0, sy = 0.0;
  for (int c = 0; c < chunks; ++c) {
    sx += part[((int64_t)c * 2 + 0) * N + i];
    sy += part[((int64_t)c * 2 + 1) * N + i];
  }
  const double sc = g.kappa * g.kappa / (2.0 * PI);
  sx *= sc;
  sy *= sc;
  const Ring rg = ring_of(g, i / Q);
  for (int sl = 0; sl <= 2 * win; ++sl) {
    const double* sg = sigma + ring_step(rg, sl - win) * Q;
    const double* wx = WGx + (int64_t)sl * Q * N + i;
    const double* wy = WGy + (int64_t)sl * Q * N + i;
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      sx = fma(wx[(int64_t)m * N], sg[m], sx);
      sy = fma(wy[(int64_t)m * N], sg[m], sy);
    }
  }
  for (int e = xrow[i]; e < xrow[i + 1]; ++e) {
    const double* sg = sigma + (int64_t)xpan[e] * Q;
    for (int m = 0; m < Q; ++m) {
      sx = fma(xg[((int64_t)e * 2 + 0) * Q + m], sg[m], sx);
      sy = fma(xg[((int64_t)e * 2 + 1) * Q + m], sg[m], sy);
    }
  }
  gx[i] = sx;
  gy[i] = sy;
}

void launch_far64(const GeomView& g, const double* sigma, const FarPlan& fp, double* partial,
                  hipStream_t s, const int* stop, hipEvent_t e0, hipEvent_t e1) {
  dim3 grid(fp.tblocks, fp.chunks);
  auto k = g.zcut < HUGE_VAL ? far64_kernel<true> : far64_kernel<false>;
  if (e0)
    hipExtLaunchKernelGGL(k, grid, dim3(FAR_BS), 0, s, e0, e1, 0, g, sigma, fp.chunk, partial,
                          stop);
  else
    k<<<grid, FAR_BS, 0, s>>>(g, sigma, fp.chunk, partial, stop);
  YQ_HIP(hipGetLastError());
}

void launch_far32_geom(const double* x, const double* y, int64_t N, double kappa, double4* tile,
                       double4* grp, double4* pan, float2* rel, hipStream_t s) {
  YQ_REQUIRE(N % Q == 0 && kappa > 0.0, YQ_EINVAL, "far32 geometry: N % 16 != 0 or kappa <= 0");
  const int64_t nt = (N + FT - 1) / FT, ng = (N + FG - 1) / FG, np = N / Q;
  circles_kernel<<<(unsigned)((nt + 3) / 4), 256, 0, s>>>(x, y, N, FT, nt, tile);
  circles_kernel<<<(unsigned)((ng + 3) / 4), 256, 0, s>>>(x, y, N, FG, ng, grp);
  circles_kernel<<<(unsigned)((np + 3) / 4), 256, 0, s>>>(x, y, N, Q, np, pan);
  rel32_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(x, y, N, tile, kappa * LOG2E, rel);
  YQ_HIP(hipGetLastError());
}

void launch_pack32(const float2* rel, const double* wnx, const double* wny, const double* sigma,
                   int64_t N, double qc, float4* src, hipStream_t s) {
  pack32_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(rel, wnx, wny, sigma, N, qc, src);
  YQ_HIP(hipGetLastError());
}

void launch_far32(const Far32View& v, const FarPlan& fp, float* partial, hipStream_t s,
                  const int* stop, hipEvent_t e0, hipEvent_t e1) {
  YQ_REQUIRE(fp.chunk % FT == 0, YQ_EINVAL, "far32: chunk is not a multiple of the tile");
  dim3 grid(fp.tblocks, fp.chunks);
  if (e0)
    hipExtLaunchKernelGGL(far32_kernel, grid, dim3(FAR_BS), 0, s, e0, e1, 0, v, fp.chunk, partial,
                          stop);
  else
    far32_kernel<<<grid, FAR_BS, 0, s>>>(v, fp.chunk, partial, stop);
  YQ_HIP(hipGetLastError());
}

void launch_far_fused64(const GeomView& g, const double* sigma, const FarPlan& fp,
                        double* partial, double* gpartial, hipStream_t s) {
  dim3 grid(fp.tblocks, fp.chunks);
  auto k = g.zcut_g < HUGE_VAL ? far_fused64_kernel<true> : far_fused64_kernel<false>;
  k<<<grid, FAR_BS, 0, s>>>(g, sigma, fp.chunk, partial, gpartial);
  YQ_HIP(hipGetLastError());
}

// ---- combined representation D + eta S (eq. bwform) ---------------------------------------
//
// Per pair, in the double-layer partials' scaling (finish applies kappa^2 / 2pi):
//   (K1(z)/z) (x_i - y_j).(w nu sigma)_j + (eta / kappa^2) K0(z) (w sigma)_j,   z = kappa r,
// since G = K0 / 2pi = (kappa^2 / 2pi) K0 / kappa^2.  Every pair takes the general
// evaluation of K0 and K1 (both branches of bessel.h); T = float evaluates in FP32 on
// the FP64 differences rounded to FP32.  One target per lane, 256-source tiles in LDS.
template <typename T>
__global__ __launch_bounds__(FAR_BS) void far_sd_kernel(GeomView g, const double* __restrict__ sigma,
                                                        int chunk, T* __restrict__ partial,
                                                        const int* __restrict__ stop) {
  __shared__ double2 sxy[FAR_BS];
  __shared__ double2 sq[FAR_BS];
  __shared__ double sw[FAR_BS];
  if (stop && *as_k(stop)) return;
  const int64_t N = g.N;
  const int64_t i = blockIdx.x * (int64_t)FAR_BS + threadIdx.x;
  const double xi = i < N ? g.x[i] : 0.0;
  const double yi = i < N ? g.y[i] : 0.0;
  const double kap2 = g.kappa * g.kappa;
  const double ek = g.eta / kap2;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = min(N, j0 + chunk);
  T acc = 0;
  for (int64_t jb = j0; jb < j1; jb += FAR_BS) {
    const int64_t j = jb + threadIdx.x;
    __syncthreads();
    if (j < j1) {
      const double s = sigma[j];
      sxy[threadIdx.x] = make_double2(g.x[j], g.y[j]);
      sq[threadIdx.x] = make_double2(g.wnx[j] * s, g.wny[j] * s);
      sw[threadIdx.x] = ek * g.w[j] * s;
    }
    __syncthreads();
    const int nb = (int)min((int64_t)FAR_BS, j1 - jb);
    for (int k = 0; k < nb; ++k) {
      const double2 p = sxy[k];
      const double2 q = sq[k];
      const double dx = xi - p.x, dy = yi - p.y;
      if constexpr (sizeof(T) == 8) {
        const double r2 = fma(dx, dx, dy * dy);
        if (r2 > 0.0) {
          double k0, k1z;
          k0_k1z_64(kap2 * r2, k0, k1z, g.tab);
          acc += fma(k1z, fma(dx, q.x, dy * q.y), k0 * sw[k]);
        }
      } else {
        const float fx = (float)dx, fy = (float)dy;
        const float r2 = fx * fx + fy * fy;
        if (r2 > 0.0f) {
          float k0, k1z;
          k0_k1z_32((float)kap2 * r2, k0, k1z);
          acc += k1z * (fx * (float)q.x + fy * (float)q.y) + k0 * (float)sw[k];
        }
      }
    }
  }
  if (i < N) partial[(int64_t)blockIdx.y * N + i] = acc;
}

// Its gradient (FP64): the double layer's as in far_grad64_kernel plus
// eta (w sigma)_j grad_x G = -(kappa^2 / 2pi) eta (w sigma)_j (K1(z)/z) (x_i - y_j).
__global__ __launch_bounds__(FAR_BS) void far_sd_grad64_kernel(GeomView g,
                                                               const double* __restrict__ sigma,
                                                               int chunk,
                                                               double* __restrict__ partial) {
  __shared__ double2 sxy[FAR_BS];
  __shared__ double2 sq[FAR_BS];
  __shared__ double sw[FAR_BS];
  const int64_t N = g.N;
  const int64_t i = blockIdx.x * (int64_t)FAR_BS + threadIdx.x;
  const double xi = i < N ? g.x[i] : 0.0;
  const double yi = i < N ? g.y[i] : 0.0;
  const double kap2 = g.kappa * g.kappa;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = min(N, j0 + chunk);
  double ax = 0.0, ay = 0.0;
  for (int64_t jb = j0; jb < j1; jb += FAR_BS) {
    const int64_t j = jb + threadIdx.x;
    __syncthreads();
    if (j < j1) {
      const double s = sigma[j];
      sxy[threadIdx.x] = make_double2(g.x[j], g.y[j]);
      sq[threadIdx.x] = make_double2(g.wnx[j] * s, g.wny[j] * s);
      sw[threadIdx.x] = g.eta * g.w[j] * s;
    }
    __syncthreads();
    const int nb = (int)min((int64_t)FAR_BS, j1 - jb);
    for (int k = 0; k < nb; ++k) {
      const double2 p = sxy[k];
      const double2 q = sq[k];
      const double dx = xi - p.x, dy = yi - p.y;
      const double r2 = fma(dx, dx, dy * dy);
      if (r2 > 0.0) {
        double k0, k1z;
        k0_k1z_64(kap2 * r2, k0, k1z, g.tab);
        const double dq = fma(dx, q.x, dy * q.y);
        const double b = dq * (k0 + 2.0 * k1z) * rcp64(r2) + k1z * sw[k];
        ax += k1z * q.x - b * dx;
        ay += k1z * q.y - b * dy;
      }
    }
  }
  if (i < N) {
    partial[((int64_t)blockIdx.y * 2 + 0) * N + i] = ax;
    partial[((int64_t)blockIdx.y * 2 + 1) * N + i] = ay;
  }
}

void launch_far_sd(const GeomView& g, const double* sigma, const FarPlan& fp, double* p64,
                   float* p32, hipStream_t s, const int* stop, hipEvent_t e0, hipEvent_t e1) {
  YQ_REQUIRE((p64 == nullptr) != (p32 == nullptr), YQ_EINVAL, "far_sd: one partial buffer");
  dim3 grid(fp.tblocks, fp.chunks);
  if (p64) {
    if (e0)
      hipExtLaunchKernelGGL(far_sd_kernel<double>, grid, dim3(FAR_BS), 0, s, e0, e1, 0, g, sigma,
                            fp.chunk, p64, stop);
    else
      far_sd_kernel<double><<<grid, FAR_BS, 0, s>>>(g, sigma, fp.chunk, p64, stop);
  } else {
    if (e0)
      hipExtLaunchKernelGGL(far_sd_kernel<float>, grid, dim3(FAR_BS), 0, s, e0, e1, 0, g, sigma,
                            fp.chunk, p32, stop);
    else
      far_sd_kernel<float><<<grid, FAR_BS, 0, s>>>(g, sigma, fp.chunk, p32, stop);
  }
  YQ_HIP(hipGetLastError());
}

void launch_far_sd_grad64(const GeomView& g, const double* sigma, const FarPlan& fp,
                          double* partial, hipStream_t s) {
  dim3 grid(fp.tblocks, fp.chunks);
  far_sd_grad64_kernel<<<grid, FAR_BS, 0, s>>>(g, sigma, fp.chunk, partial);
  YQ_HIP(hipGetLastError());
}

void launch_far_grad64(const GeomView& g, const double* sigma, const FarPlan& fp, double* partial,
                       hipStream_t s) {
  dim3 grid(fp.tblocks, fp.chunks);
  auto k = g.zcut_g < HUGE_VAL ? far_grad64_kernel<true> : far_grad64_kernel<false>;
  k<<<grid, FAR_BS, 0, s>>>(g, sigma, fp.chunk, partial);
  YQ_HIP(hipGetLastError());
}

void launch_finish(const GeomView& g, int win, const FarPlan& fp, const double* partial64,
                   const float* partial32, const double* W, const int* xrow, const int* xpan,
                   const double* xvals, const double* sigma, double* out, hipStream_t s) {
  finish_kernel<<<(unsigned)((8 * g.N + 255) / 256), 256, 0, s>>>(g, win, fp.chunks, partial64,
                                                              partial32, W, xrow, xpan, xvals,
                                                              sigma, out);
  YQ_HIP(hipGetLastError());
}

void launch_finish_grad(const GeomView& g, int win, const FarPlan& fp, const double* partial,
                        const double* WGx, const double* WGy, const int* xrow, const int* xpan,
                        const double* xgvals, const double* sigma, double* gx, double* gy,
                        hipStream_t s) {
  finish_grad_kernel<<<(unsigned)((g.N + 255) / 256), 256, 0, s>>>(
      g, win, fp.chunks, partial, WGx, WGy, xrow, xpan, xgvals, sigma, gx, gy);
  YQ_HIP(hipGetLastError());
}

}  // namespace yq
