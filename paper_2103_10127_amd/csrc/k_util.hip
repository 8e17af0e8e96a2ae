// Small utility kernels of the solver: deterministic norm reductions of the
// per-tile partial sums written by the residual kernel, copies, fills, and
// the owner map of the restricted prolongation.
#include <hip/hip_runtime.h>

#include "rav_internal.h"

namespace rav {

// Deterministic sum of partials[first .. first+count) into out[0], and into
// host_out[0] (pinned host memory the host reads after a stream
// synchronisation, which spares a copy) when host_out is not null.
__global__ __launch_bounds__(256) void k_norm_finalize(const double* __restrict__ partials, int first,
                                                        int count, double* __restrict__ out,
                                                        double* __restrict__ host_out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) s += partials[first + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0];
    if (host_out) host_out[0] = red[0];
  }
}

// One block per problem: out[g] = sum of partials[first[g] .. first[g] + count[g]).
__global__ __launch_bounds__(256) void k_norm_finalize_batch(const double* __restrict__ partials,
                                                              const int* __restrict__ first,
                                                              const int* __restrict__ count,
                                                              double* __restrict__ out) {
  __shared__ double red[256];
  const int gidx = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < count[gidx]; i += 256) s += partials[first[gidx] + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[gidx] = red[0];
}

// Batched copy: task = (problem, block of 256 entries).
__global__ __launch_bounds__(256) void k_copy_batch(double* const* __restrict__ dst, const double* const* __restrict__ src,
                                                     const long long* __restrict__ n,
                                                     const BlockTask* __restrict__ tasks) {
  const BlockTask t = tasks[blockIdx.x];
  if (t.grid < 0) return;
  const long long i = t.start + threadIdx.x;
  if (i < n[t.grid]) dst[t.grid][i] = src[t.grid][i];
}

__global__ __launch_bounds__(256) void k_copy(double* __restrict__ dst, const double* __restrict__ src, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_fill(double* __restrict__ dst, double v, long long n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = v;
}

__global__ __launch_bounds__(256) void k_owner(const GridDev* __restrict__ G, int kind, long long n,
                                                int* __restrict__ owner) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Geo& g = G->g;
  if (i < g.dim * g.nV) {
    int a[3] = {0, 0, 0};
    long long nl_;
    split_vel(g, i, &nl_);
    node_of(g, nl_, a);
    if (node_dirichlet(g, a)) { owner[i] = -1; return; }
  }
  owner[i] = (int)owner_of(g, kind, i);
}

void launch_norm_finalize_batch(const double* partials, const int* first, const int* count, int ngrids,
                                double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_finalize_batch, dim3(ngrids), dim3(256), 0, s, partials, first, count, out);
}

void launch_copy_batch(double* const* dst, const double* const* src, const long long* n, const BlockTask* tasks,
                       int ntasks, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_batch, dim3(ntasks), dim3(256), 0, s, dst, src, n, tasks);
}

void launch_norm_finalize(const double* partials, int first, int count, double* out, double* host_out,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(256), 0, s, partials, first, count, out, host_out);
}

static inline unsigned grid_for(long long n) {
  long long b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

void launch_copy(double* dst, const double* src, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(256), 0, s, dst, src, n);
}
void launch_fill(double* dst, double v, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, dst, v, n);
}
void launch_owner(const GridDev* G, int kind, long long n, int* owner, hipStream_t s) {
  hipLaunchKernelGGL(k_owner, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, G, kind, n, owner);
}

}  // namespace rav
