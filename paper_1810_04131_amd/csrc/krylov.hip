// Step a8: vector kernels for GMRES (Algorithm 1 solves eq. bie with GMRES).
// Arnoldi uses classical Gram-Schmidt applied twice, so each orthogonalisation
// is two multi-dot products and two updates.  Dot products reduce in a fixed
// order (per-block partials, then one block per column), so results do not
// depend on scheduling.  The Krylov basis V is column-major: V[k * ld + i].
#include "common.h"

namespace yq {

constexpr int KB = 256;

int krylov_blocks(int64_t n) {
  int64_t nb = (n + 2047) / 2048;
  if (nb < 1) nb = 1;
  if (nb > 1024) nb = 1024;
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
  for (int k = threadIdx.x; k < kc; k += KB) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += partial[(int64_t)k * nb + b];
    h[k] = t;
  }
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)KB + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < kc; ++k) s = fma(V[(int64_t)k * ld + i], h[k], s);
  w[i] = fma(alpha, s, w[i]);
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

// out = x * inv[0]
__global__ void scale_kernel(const double* __restrict__ x, const double* __restrict__ inv,
                             double* __restrict__ out, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = x[i] * inv[0];
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

void launch_scale(const double* x, const double* inv, double* out, int64_t n, hipStream_t s) {
  scale_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, inv, out, n);
  YQ_HIP(hipGetLastError());
}

}  // namespace yq
