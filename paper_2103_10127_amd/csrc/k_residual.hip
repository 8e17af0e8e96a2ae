// Residual r = b - L x on the free rows (eq. 10), with an optional partial
// sum of r^2 per block for the stopping test (Sec. 4), plus small utility
// kernels (norm reduction, copy, fill, owner map).
//
// One thread per operator row.  Every block covers rows of a single ELL
// segment, so all lanes of a wavefront share the stencil shape (compile-time
// per node parity type) and read the slot-major values coalesced.
#include <hip/hip_runtime.h>

#include "rav_internal.h"

namespace rav {

template <int DIM, int TY>
__device__ __forceinline__ double res_velocity(const GridDev& gd, int s, long long row, bool& masked) {
  const Geo& g = gd.g;
  const int c = s >> DIM;
  int a[3] = {0, 0, 0};
  vel_row_node(g, TY, row, a);
  masked = node_dirichlet(g, a);
  const long long base = node_lin(g, a);
  const long long gi = c * g.nV + base;
  if (masked) { gd.r[gi] = 0.0; return 0.0; }
  const long long rows = gd.seg_rows[s];
  const double* __restrict__ v = gd.vals + gd.seg_off[s] + row;
  const double* __restrict__ xc = gd.x + c * g.nV;
  const double* __restrict__ xp = gd.x + DIM * g.nV;
  constexpr int W0 = (TY & 1) ? 1 : 2;
  constexpr int W1 = ((TY >> 1) & 1) ? 1 : 2;
  constexpr int W2 = DIM == 3 ? (((TY >> 2) & 1) ? 1 : 2) : 0;
  const int twoN = 2 * g.N;
  const long long nn = g.nn, nn2 = g.nn * g.nn;
  double acc = 0.0;
  int slot = 0;
#pragma unroll 1
  for (int oz = -W2; oz <= W2; ++oz) {
#pragma unroll 1
    for (int oy = -W1; oy <= W1; ++oy) {
#pragma unroll
      for (int ox = -W0; ox <= W0; ++ox) {
        bool ok = a[0] + ox >= 0 && a[0] + ox <= twoN && a[1] + oy >= 0 && a[1] + oy <= twoN;
        if (DIM == 3) ok = ok && a[2] + oz >= 0 && a[2] + oz <= twoN;
        const double val = v[(long long)slot * rows];
        const double xv = ok ? xc[base + ox + nn * oy + nn2 * oz] : 0.0;
        acc += val * xv;
        ++slot;
      }
    }
  }
  constexpr int M0 = 3 - (TY & 1), M1 = 3 - ((TY >> 1) & 1), M2 = DIM == 3 ? 3 - ((TY >> 2) & 1) : 1;
  const int lo0 = (a[0] >> 1) - 1 + (TY & 1);
  const int lo1 = (a[1] >> 1) - 1 + ((TY >> 1) & 1);
  const int lo2 = DIM == 3 ? (a[2] >> 1) - 1 + ((TY >> 2) & 1) : 0;
  const long long np1 = g.np1, np12 = g.np1 * g.np1;
#pragma unroll 1
  for (int jz = 0; jz < M2; ++jz) {
#pragma unroll 1
    for (int jy = 0; jy < M1; ++jy) {
#pragma unroll
      for (int jx = 0; jx < M0; ++jx) {
        const int k0 = lo0 + jx, k1 = lo1 + jy, k2 = lo2 + jz;
        bool ok = k0 >= 0 && k0 <= g.N && k1 >= 0 && k1 <= g.N;
        if (DIM == 3) ok = ok && k2 >= 0 && k2 <= g.N;
        const double val = v[(long long)slot * rows];
        const double xv = ok ? xp[k0 + np1 * k1 + np12 * k2] : 0.0;
        acc += val * xv;
        ++slot;
      }
    }
  }
  const double r = gd.b[gi] - acc;
  gd.r[gi] = r;
  return r;
}

template <int DIM>
__device__ __forceinline__ double res_pressure(const GridDev& gd, long long row) {
  const Geo& g = gd.g;
  const int s = pressure_segment(DIM);
  int k[3] = {0, 0, 0};
  vert_of(g, row, k);
  const long long rows = gd.seg_rows[s];
  const double* __restrict__ v = gd.vals + gd.seg_off[s] + row;
  const int twoN = 2 * g.N;
  const long long nn = g.nn, nn2 = g.nn * g.nn;
  int a[3] = {2 * k[0], 2 * k[1], DIM == 3 ? 2 * k[2] : 0};
  const long long base = a[0] + nn * a[1] + nn2 * a[2];
  constexpr int WZ = DIM == 3 ? 2 : 0;
  double acc = 0.0;
#pragma unroll 1
  for (int c = 0; c < DIM; ++c) {
    const double* __restrict__ xc = gd.x + c * g.nV;
    int slot = c * ipow(5, DIM);
#pragma unroll 1
    for (int oz = -WZ; oz <= WZ; ++oz) {
#pragma unroll 1
      for (int oy = -2; oy <= 2; ++oy) {
#pragma unroll
        for (int ox = -2; ox <= 2; ++ox) {
          bool ok = a[0] + ox >= 0 && a[0] + ox <= twoN && a[1] + oy >= 0 && a[1] + oy <= twoN;
          if (DIM == 3) ok = ok && a[2] + oz >= 0 && a[2] + oz <= twoN;
          const double val = v[(long long)slot * rows];
          const double xv = ok ? xc[base + ox + nn * oy + nn2 * oz] : 0.0;
          acc += val * xv;
          ++slot;
        }
      }
    }
  }
  const long long gi = DIM * g.nV + row;
  const double r = gd.b[gi] - acc;
  gd.r[gi] = r;
  return r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int DIM>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_residual(const GridDev* __restrict__ G,
                                                     const BlockTask* __restrict__ tasks,
                                                     double* __restrict__ partials) {
  const BlockTask t = tasks[blockIdx.x];
  if (t.grid < 0) return;   // padding block of the XCD permutation (whole block)
  if (grid_idle(G[t.grid])) return;
  double sq = 0.0;
  {
    const GridDev& gd = G[t.grid];
    const int s = t.part;
    const long long row = t.start + threadIdx.x;
    if (row < gd.seg_rows[s]) {
      double r = 0.0;
      bool masked = false;
      if (s == pressure_segment(DIM)) {
        r = res_pressure<DIM>(gd, row);
      } else {
        switch (s & ((1 << DIM) - 1)) {
          case 0: r = res_velocity<DIM, 0>(gd, s, row, masked); break;
          case 1: r = res_velocity<DIM, 1>(gd, s, row, masked); break;
          case 2: r = res_velocity<DIM, 2>(gd, s, row, masked); break;
          case 3: r = res_velocity<DIM, 3>(gd, s, row, masked); break;
          case 4: r = res_velocity<DIM, 4>(gd, s, row, masked); break;
          case 5: r = res_velocity<DIM, 5>(gd, s, row, masked); break;
          case 6: r = res_velocity<DIM, 6>(gd, s, row, masked); break;
          default: r = res_velocity<DIM, 7>(gd, s, row, masked); break;
        }
      }
      sq = r * r;
    }
  }
  if (partials == nullptr) return;
  __shared__ double red[BLOCK / 64];
  sq = wave_sum(sq);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s2 = 0.0;
    for (int w = 0; w < BLOCK / 64; ++w) s2 += red[w];
    partials[t.logical] = s2;
  }
}

// Deterministic sum of partials[first .. first+count) into out[0].
__global__ __launch_bounds__(256) void k_norm_finalize(const double* __restrict__ partials, int first,
                                                        int count, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) s += partials[first + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
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

void launch_residual(int dim, const GridDev* G, const BlockTask* tasks, int ntasks, double* partials,
                     hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(k_residual<2>, dim3(ntasks), dim3(BLOCK), 0, s, G, tasks, partials);
  else
    hipLaunchKernelGGL(k_residual<3>, dim3(ntasks), dim3(BLOCK), 0, s, G, tasks, partials);
}

void launch_norm_finalize_batch(const double* partials, const int* first, const int* count, int ngrids,
                                double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_finalize_batch, dim3(ngrids), dim3(256), 0, s, partials, first, count, out);
}

void launch_copy_batch(double* const* dst, const double* const* src, const long long* n, const BlockTask* tasks,
                       int ntasks, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_batch, dim3(ntasks), dim3(256), 0, s, dst, src, n, tasks);
}

void launch_norm_finalize(const double* partials, int first, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(256), 0, s, partials, first, count, out);
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
