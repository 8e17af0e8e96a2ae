// Vector kernels of the Krylov (GMRES) acceleration: deterministic dot
// products with per-block partial sums, and axpy / scaling with coefficients
// that stay in device memory (no host round trip per Gram-Schmidt step).
#include <hip/hip_runtime.h>

#include "rav_internal.h"

namespace rav {

constexpr int KB = 256;
constexpr int KBLOCKS = 1024;   // fixed grid: partial sums land in a 1024-entry buffer

__global__ __launch_bounds__(KB) void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                     long long n, double* __restrict__ partial) {
  __shared__ double red[KB];
  double s = 0.0;
  for (long long i = blockIdx.x * (long long)KB + threadIdx.x; i < n; i += (long long)gridDim.x * KB) s += a[i] * b[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = KB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out[0] = sum of partial[0 .. nb); if take_sqrt, out[0] = sqrt(sum).
__global__ __launch_bounds__(KB) void k_dot_final(const double* __restrict__ partial, int nb, double* __restrict__ out,
                                                   int take_sqrt) {
  __shared__ double red[KB];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += KB) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = KB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = take_sqrt ? sqrt(red[0]) : red[0];
}

// y += sign * c[0] * x
__global__ __launch_bounds__(KB) void k_axpy_dev(double* __restrict__ y, const double* __restrict__ x,
                                                  const double* __restrict__ c, double sign, long long n) {
  const double a = sign * c[0];
  for (long long i = blockIdx.x * (long long)KB + threadIdx.x; i < n; i += (long long)gridDim.x * KB) y[i] += a * x[i];
}

// y = x / c[0]  (c[0] == 0 leaves y = 0)
__global__ __launch_bounds__(KB) void k_div_dev(double* __restrict__ y, const double* __restrict__ x,
                                                 const double* __restrict__ c, long long n) {
  const double d = c[0];
  const double inv = d != 0.0 ? 1.0 / d : 0.0;
  for (long long i = blockIdx.x * (long long)KB + threadIdx.x; i < n; i += (long long)gridDim.x * KB) y[i] = x[i] * inv;
}

static inline unsigned kgrid(long long n) {
  long long b = (n + KB - 1) / KB;
  return (unsigned)(b < KBLOCKS ? (b < 1 ? 1 : b) : KBLOCKS);
}

void launch_dot(const double* a, const double* b, long long n, double* partial, double* out, int take_sqrt,
                hipStream_t s) {
  const unsigned g = kgrid(n);
  hipLaunchKernelGGL(k_dot_partial, dim3(g), dim3(KB), 0, s, a, b, n, partial);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(KB), 0, s, partial, (int)g, out, take_sqrt);
}
void launch_axpy_dev(double* y, const double* x, const double* c, double sign, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_dev, dim3(kgrid(n)), dim3(KB), 0, s, y, x, c, sign, n);
}
void launch_div_dev(double* y, const double* x, const double* c, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_div_dev, dim3(kgrid(n)), dim3(KB), 0, s, y, x, c, n);
}

}  // namespace rav
