// Vector kernels for GMRES (Algorithm 1 solves eq. bie with GMRES).
// Arnoldi uses classical Gram-Schmidt applied twice, so each orthogonalisation
// is two multi-dot products and two updates.  Dot products reduce in a fixed
// order (per-block partials, then one block per column), so results do not
// depend on scheduling.  The Krylov basis V is column-major: V[k * ld + i].
#include "common.h"

namespace yq {

constexpr int KB = 256;

// Row blocks of a multi-dot (the number of partials per column): at most 32, so
// that one thread sums a column's partials with all of its loads in flight.
int krylov_blocks(int64_t n) {
  int64_t nb = (n + 2047) / 2048;
  if (nb < 1) nb = 1;
  if (nb > 32) nb = 32;
  return (int)nb;
}

// Sum over the block in a fixed order: a shuffle tree inside each wavefront, then
// the four wavefront sums in order.  Valid in thread 0.
__device__ __forceinline__ double block_sum_waves(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return threadIdx.x == 0 ? ((sh[0] + sh[1]) + sh[2]) + sh[3] : 0.0;
}

// p[0] + p[1] + ... + p[nb - 1] in that order (nb <= 32 column partials: one
// thread per column keeps every column in flight at once).  The update kernels,
// the Arnoldi step and the host (sum_partials) use this order, so the same
// partials give the same coefficient everywhere.
__device__ __forceinline__ double sum_partials_dev(const double* __restrict__ p, int nb) {
  double t = 0.0;
  for (int b = 0; b < nb; ++b) t += p[b];
  return t;
}

// p[0] + ... + p[nb - 1] by one wavefront (a long list: the |w|^2 partials of
// the update blocks): each lane sums every 64th value in order, then a fixed
// butterfly; every lane ends with the same value.
__device__ __forceinline__ double wave_sum_partials(const double* __restrict__ p, int nb, int lane) {
  double t = 0.0;
  for (int b = lane; b < nb; b += 64) t += p[b];
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  return t;
}

// partial[k * nb + b] = sum over block b's rows of V[k][i] * w[i]; one block per
// (row chunk b = blockIdx.x, column k = blockIdx.y), so small n still fills the GPU.
__global__ __launch_bounds__(KB) void multidot_kernel(const double* __restrict__ V, int64_t ld,
                                                      int kc, const double* __restrict__ w,
                                                      int64_t n, double* __restrict__ partial) {
  __shared__ double sh[KB / 64];
  const int nb = gridDim.x;
  const int k = blockIdx.y;
  const int64_t per = (n + nb - 1) / nb;
  const int64_t r0 = blockIdx.x * per;
  const int64_t r1 = min(n, r0 + per);
  const double* v = V + (int64_t)k * ld;
  double acc = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += KB) acc = fma(v[i], w[i], acc);
  const double s = block_sum_waves(acc, sh);
  if (threadIdx.x == 0) partial[(int64_t)k * nb + blockIdx.x] = s;
}

// w[i] += alpha * sum_{k < kc} V[k][i] h[k], h[k] = sum_{b < nb} partial[k * nb + b]
// summed in order b = 0, 1, ... (the order the host uses for the same sums).
__global__ __launch_bounds__(KB) void update_partial_kernel(double* __restrict__ w,
                                                            const double* __restrict__ V,
                                                            int64_t ld, int kc,
                                                            const double* __restrict__ partial,
                                                            int nb, double alpha, int64_t n) {
  extern __shared__ double h[];
  for (int k = threadIdx.x; k < kc; k += KB) h[k] = sum_partials_dev(partial + (int64_t)k * nb, nb);
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)KB + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < kc; ++k) s = fma(V[(int64_t)k * ld + i], h[k], s);
  w[i] = fma(alpha, s, w[i]);
}

// update_partial_kernel, and npart[block] = the block's sum of the new w_i^2
// (a fixed-order block reduction): the partials of |w|^2 for the Arnoldi step.
__global__ __launch_bounds__(KB) void update_norm_kernel(double* __restrict__ w,
                                                         const double* __restrict__ V, int64_t ld,
                                                         int kc, const double* __restrict__ partial,
                                                         int nb, double alpha, int64_t n,
                                                         double* __restrict__ npart) {
  extern __shared__ double h[];   // [kc] coefficients, then [KB / 64] wavefront sums
  for (int k = threadIdx.x; k < kc; k += KB) h[k] = sum_partials_dev(partial + (int64_t)k * nb, nb);
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)KB + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    double s = 0.0;
    for (int k = 0; k < kc; ++k) s = fma(V[(int64_t)k * ld + i], h[k], s);
    v = fma(alpha, s, w[i]);
    w[i] = v;
  }
  const double t = block_sum_waves(v * v, h + kc);
  if (threadIdx.x == 0) npart[blockIdx.x] = t;
}

// w[i] += alpha * sum_{k < kc} V[k][i] h[k]
__global__ void update_kernel(double* __restrict__ w, const double* __restrict__ V, int64_t ld,
                              int kc, const double* __restrict__ h, double alpha, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < kc; ++k) s = fma(V[(int64_t)k * ld + i], h[k], s);
  w[i] = fma(alpha, s, w[i]);
}

__global__ void axpby_kernel(double a, const double* __restrict__ x, double b,
                             const double* __restrict__ y, double* __restrict__ out, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

constexpr int MAXR = 200;   // largest restart length (checked with the parameters)

// y = R^-1 g for the leading k x k upper triangle R of H (leading dimension
// ldh), by back substitution: one wavefront, each row's dot product split over
// the lanes and summed by a fixed butterfly.
__global__ __launch_bounds__(64) void trisolve_kernel(const double* __restrict__ H, int ldh,
                                                      const double* __restrict__ g, int k,
                                                      double* __restrict__ y) {
  __shared__ double ys[MAXR];
  const int lane = threadIdx.x;
  for (int i = k - 1; i >= 0; --i) {
    double t = 0.0;
    for (int c = i + 1 + lane; c < k; c += 64) t = fma(H[(int64_t)c * ldh + i], ys[c], t);
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) ys[i] = (g[i] - t) / H[(int64_t)i * ldh + i];
    __syncthreads();
  }
  for (int i = lane; i < k; i += 64) y[i] = ys[i];
}

// The Arnoldi step of arnoldi_kernel fused with the normalisation of the new
// basis vector: |w| = h_{j+1,j} comes from the update kernel's block partials
// npart[0..nbu) (every block sums them in the same order, so every block has the
// same value); block 0 does the Hessenberg / Givens bookkeeping; every block
// writes vn = w / h_{j+1,j} (0 at a breakdown) for its rows and, when src is
// given, the FP32 source records of vn (as pack32_kernel).  The stop flag is read
// once per block: a block that starts after block 0 has set it skips its rows,
// which then belong to a basis vector that is never used.
__global__ __launch_bounds__(KB) void arnoldi_scale_kernel(
    const double* __restrict__ part, int nb, const double* __restrict__ npart, int nbu, int j,
    int ldh, double* __restrict__ H, double* __restrict__ cs, double* __restrict__ sn,
    double* __restrict__ g, int* __restrict__ stop, double bnorm, double rtol,
    double* __restrict__ status, const double* __restrict__ w, double* __restrict__ vn, int64_t n,
    const float2* __restrict__ rel, const double* __restrict__ wnx,
    const double* __restrict__ wny, double qc, float4* __restrict__ src) {
  __shared__ double hc[MAXR + 2];
  __shared__ double h2s;
  __shared__ int stopped;
  if (threadIdx.x == 0) stopped = *stop;
  __syncthreads();
  if (stopped) return;   // uniform over the block
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (wave == 0) {
    const double t = wave_sum_partials(npart, nbu, lane);
    if (lane == 0) h2s = t;
  }
  if (blockIdx.x == 0) {
    const int64_t pc = (int64_t)(j + 1) * nb;
    for (int i = threadIdx.x; i <= j; i += KB)
      hc[i] = sum_partials_dev(part + (int64_t)i * nb, nb) +
              sum_partials_dev(part + pc + (int64_t)i * nb, nb);
  }
  __syncthreads();
  const double hn = sqrt(fmax(h2s, 0.0));
  const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hc[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * hc[i] + sn[i] * hc[i + 1];
      hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
      hc[i] = t;
    }
    const double den = hypot(hc[j], hc[j + 1]);
    const double c = den > 0.0 ? hc[j] / den : 1.0;
    const double sv = den > 0.0 ? hc[j + 1] / den : 0.0;
    cs[j] = c;
    sn[j] = sv;
    hc[j] = den;
    hc[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sv * gj;
    g[j] = c * gj;
    const double rel = fabs(sv * gj) / bnorm;
    for (int i = 0; i <= j + 1; ++i) H[(int64_t)j * ldh + i] = hc[i];
    const int st = (rel <= rtol || hn == 0.0) ? 1 : 0;
    status[0] = rel;
    status[1] = hn;
    status[2] = (double)st;
    *stop = st;
  }
  const int64_t i = blockIdx.x * (int64_t)KB + threadIdx.x;
  if (i >= n) return;
  const double v = w[i] * inv;
  vn[i] = v;
  if (src) {
    const double sc = v * qc;
    const float2 r = rel[i];
    src[i] = make_float4(r.x, r.y, (float)(wnx[i] * sc), (float)(wny[i] * sc));
  }
}

__global__ void gmres_init_kernel(double* __restrict__ g, int m, double beta,
                                  int* __restrict__ stop) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= m) g[i] = i == 0 ? beta : 0.0;
  if (i == 0) *stop = 0;
}

void launch_trisolve(const double* H, int ldh, const double* g, int k, double* y, hipStream_t s) {
  if (k < 1) return;
  YQ_REQUIRE(k <= MAXR && k < ldh, YQ_EINVAL, "trisolve: size out of range");
  trisolve_kernel<<<1, 64, 0, s>>>(H, ldh, g, k, y);
  YQ_HIP(hipGetLastError());
}

int krylov_norm_blocks(int64_t n) { return (int)((n + KB - 1) / KB); }

void launch_update_norm(double* w, const double* V, int64_t ld, int k, const double* partial,
                        int nb, double alpha, int64_t n, double* npart, hipStream_t s) {
  YQ_REQUIRE(k >= 1, YQ_EINVAL, "update_norm: no columns");
  update_norm_kernel<<<(unsigned)krylov_norm_blocks(n), KB, (k + KB / 64) * sizeof(double), s>>>(
      w, V, ld, k, partial, nb, alpha, n, npart);
  YQ_HIP(hipGetLastError());
}

void launch_arnoldi_scale(const double* part, int nb, const double* npart, int j, int ldh,
                          double* H, double* cs, double* sn, double* g, int* stop, double bnorm,
                          double rtol, double* status, const double* w, double* vn, int64_t n,
                          const float2* rel, const double* wnx, const double* wny, double qc,
                          float4* src, hipStream_t s) {
  YQ_REQUIRE(j >= 0 && j + 1 < ldh && j < MAXR, YQ_EINVAL, "arnoldi: column out of range");
  const int nbu = krylov_norm_blocks(n);
  arnoldi_scale_kernel<<<(unsigned)nbu, KB, 0, s>>>(part, nb, npart, nbu, j, ldh, H, cs, sn, g,
                                                    stop, bnorm, rtol, status, w, vn, n, rel, wnx,
                                                    wny, qc, src);
  YQ_HIP(hipGetLastError());
}

void launch_gmres_init(double* g, int m, double beta, int* stop, hipStream_t s) {
  gmres_init_kernel<<<(unsigned)((m + 1 + 255) / 256), 256, 0, s>>>(g, m, beta, stop);
  YQ_HIP(hipGetLastError());
}

void launch_multidot(const double* V, int64_t ld, int k, const double* w, int64_t n,
                     double* partial, int nb, hipStream_t s) {
  if (k < 1) return;
  multidot_kernel<<<dim3(nb, k), KB, 0, s>>>(V, ld, k, w, n, partial);
  YQ_HIP(hipGetLastError());
}

void launch_update_partial(double* w, const double* V, int64_t ld, int k, const double* partial,
                           int nb, double alpha, int64_t n, hipStream_t s) {
  if (k < 1) return;
  update_partial_kernel<<<(unsigned)((n + KB - 1) / KB), KB, k * sizeof(double), s>>>(
      w, V, ld, k, partial, nb, alpha, n);
  YQ_HIP(hipGetLastError());
}

double sum_partials(const double* p, int nb) {
  double t = 0.0;
  for (int b = 0; b < nb; ++b) t += p[b];
  return t;
}

void launch_update(double* w, const double* V, int64_t ld, int k, const double* h, double alpha,
                   int64_t n, hipStream_t s) {
  update_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(w, V, ld, k, h, alpha, n);
  YQ_HIP(hipGetLastError());
}

void launch_axpby(double a, const double* x, double b, const double* y, double* out, int64_t n,
                  hipStream_t s) {
  axpby_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, x, b, y, out, n);
  YQ_HIP(hipGetLastError());
}


}  // namespace yq
