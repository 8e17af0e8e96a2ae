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

// ---- batched vector kernels (one launch for all problems of a batch) -------
// Tasks are (problem = grid, first element = start) tiles of BV elements in
// XCD order; t.logical indexes the partial sums, which are contiguous per
// problem.  Problems with active[p] == 0 are skipped.  Pointer tables hold one
// device vector per problem.
namespace rav {

constexpr int BV = 1024;   // elements per task (256 threads x 4)

__global__ __launch_bounds__(256) void k_bdot_partial(const BlockTask* __restrict__ tasks, double* const* __restrict__ A,
                                                       double* const* __restrict__ Bv, const long long* __restrict__ n,
                                                       const int* __restrict__ active, double* __restrict__ partial) {
  __shared__ double red[256];
  const BlockTask t = tasks[blockIdx.x];
  if (t.grid < 0) return;
  double s = 0.0;
  if (active[t.grid]) {
    const double* a = A[t.grid];
    const double* b = Bv[t.grid];
    const long long end = min(t.start + (long long)BV, n[t.grid]);
    for (long long i = t.start + threadIdx.x; i < end; i += 256) s += a[i] * b[i];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[t.logical] = red[0];
}

// out[p * ostride + ooff] = sum of problem p's partials (sqrt if take_sqrt).
__global__ __launch_bounds__(256) void k_bdot_final(const double* __restrict__ partial, const int* __restrict__ first,
                                                     const int* __restrict__ count, const int* __restrict__ active,
                                                     double* __restrict__ out, long long ostride, long long ooff,
                                                     int take_sqrt) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  if (!active[p]) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < count[p]; i += 256) s += partial[first[p] + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p * ostride + ooff] = take_sqrt ? sqrt(red[0]) : red[0];
}

// mode 0: y += sign * c * x;  mode 1: y = x / c (c == 0 gives 0);  mode 2: y = sign * c * x;
// mode 3: y = 0 (x unused).  c = coef[p * cstride + coff] (coef == nullptr: c = 1).
__global__ __launch_bounds__(256) void k_bvec(const BlockTask* __restrict__ tasks, double* const* __restrict__ Y,
                                               double* const* __restrict__ X, const long long* __restrict__ n,
                                               const int* __restrict__ active, const double* __restrict__ coef,
                                               long long cstride, long long coff, double sign, int mode) {
  const BlockTask t = tasks[blockIdx.x];
  if (t.grid < 0 || !active[t.grid]) return;
  double* y = Y[t.grid];
  const double* x = X[t.grid];
  const double c = coef ? coef[t.grid * cstride + coff] : 1.0;
  const long long end = min(t.start + (long long)BV, n[t.grid]);
  if (mode == 0) {
    const double a = sign * c;
    for (long long i = t.start + threadIdx.x; i < end; i += 256) y[i] += a * x[i];
  } else if (mode == 1) {
    const double inv = c != 0.0 ? 1.0 / c : 0.0;
    for (long long i = t.start + threadIdx.x; i < end; i += 256) y[i] = x[i] * inv;
  } else if (mode == 2) {
    const double a = sign * c;
    for (long long i = t.start + threadIdx.x; i < end; i += 256) y[i] = a * x[i];
  } else {
    for (long long i = t.start + threadIdx.x; i < end; i += 256) y[i] = 0.0;
  }
}

// x_p += sum_{i < jend_p} y[p * m + i] Z_i^p  (Z[i * nprob + p] = Z_i of problem p)
__global__ __launch_bounds__(256) void k_bupdate(const BlockTask* __restrict__ tasks, double* const* __restrict__ Xk,
                                                  double* const* __restrict__ Z, int nprob, int m,
                                                  const long long* __restrict__ n, const int* __restrict__ jend,
                                                  const double* __restrict__ ycoef) {
  const BlockTask t = tasks[blockIdx.x];
  if (t.grid < 0) return;
  const int p = t.grid;
  const int je = jend[p];
  if (je <= 0) return;
  double* x = Xk[p];
  const long long end = min(t.start + (long long)BV, n[p]);
  for (long long i = t.start + threadIdx.x; i < end; i += 256) {
    double s = x[i];
    for (int j = 0; j < je; ++j) s += ycoef[p * m + j] * Z[(long long)j * nprob + p][i];
    x[i] = s;
  }
}

void launch_bdot(const BlockTask* tasks, int ntasks, double* const* A, double* const* Bv, const long long* n,
                 const int* active, double* partial, const int* first, const int* count, int nprob, double* out,
                 long long ostride, long long ooff, int take_sqrt, hipStream_t s) {
  hipLaunchKernelGGL(k_bdot_partial, dim3(ntasks), dim3(256), 0, s, tasks, A, Bv, n, active, partial);
  hipLaunchKernelGGL(k_bdot_final, dim3(nprob), dim3(256), 0, s, partial, first, count, active, out, ostride, ooff,
                     take_sqrt);
}
void launch_bvec(const BlockTask* tasks, int ntasks, double* const* Y, double* const* X, const long long* n,
                 const int* active, const double* coef, long long cstride, long long coff, double sign, int mode,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_bvec, dim3(ntasks), dim3(256), 0, s, tasks, Y, X, n, active, coef, cstride, coff, sign, mode);
}
void launch_bupdate(const BlockTask* tasks, int ntasks, double* const* Xk, double* const* Z, int nprob, int m,
                    const long long* n, const int* jend, const double* ycoef, hipStream_t s) {
  hipLaunchKernelGGL(k_bupdate, dim3(ntasks), dim3(256), 0, s, tasks, Xk, Z, nprob, m, n, jend, ycoef);
}

}  // namespace rav
