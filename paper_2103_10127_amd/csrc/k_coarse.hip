// Coarse-grid direct solver (Sec. 2: LU factorisation solved to machine
// accuracy on the coarsest grid).
//
// Set-up: the coarsest operator is expanded to a dense FP64 matrix (masked
// rows become identity rows; with Dirichlet velocity on the whole boundary it
// is bordered by e = (0, 1_p) to fix the pressure constant) and inverted in
// place by Gauss-Jordan elimination with partial pivoting, one pivot step per
// pair of launches spread over the whole GPU.  Each cycle the coarse solve is
// then a single dense GEMV with the stored inverse, which parallelises over all
// CUs instead of two sequential triangular solves.
#include <hip/hip_runtime.h>

#include "rav_internal.h"

namespace rav {

template <int DIM>
__global__ __launch_bounds__(256) void k_coarse_build(const GridDev* __restrict__ G, double* __restrict__ M,
                                                       long long nb, int bordered, int unit_masked) {
  const long long R = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const GridDev& gd = *G;
  const Geo& g = gd.g;
  if (R >= g.n) {
    if (bordered && R == g.n) {
      for (long long j = DIM * g.nV; j < g.n; ++j) M[R * nb + j] = 1.0;
    }
    return;
  }
  double* row = M + R * nb;
  if (bordered) row[g.n] = (R >= DIM * g.nV) ? 1.0 : 0.0;
  if (R < DIM * g.nV) {
    long long nl_;
    const int c = split_vel(g, R, &nl_);
    int a[3] = {0, 0, 0};
    node_of(g, nl_, a);
    if (node_dirichlet(g, a)) { row[R] = unit_masked ? 1.0 : 0.0; return; }
    const int t = node_type(g, a);
    const int s = c * (1 << DIM) + t;
    const long long rows = gd.seg_rows[s], rr = vel_seg_row(g, t, a);
    const double* v = gd.vals + gd.seg_off[s] + rr;
    int w[3] = {0, 0, 0}, m[3] = {1, 1, 1}, lo[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) {
      w[d] = a_halfwidth(t, d);
      m[d] = 3 - ((t >> d) & 1);
      lo[d] = (a[d] >> 1) - 1 + ((t >> d) & 1);
    }
    int slot = 0;
    for (int oz = -w[2]; oz <= w[2]; ++oz)
      for (int oy = -w[1]; oy <= w[1]; ++oy)
        for (int ox = -w[0]; ox <= w[0]; ++ox, ++slot) {
          int b[3] = {a[0] + ox, a[1] + oy, a[2] + oz};
          if (node_inside(g, b)) row[c * g.nV + node_lin(g, b)] = v[slot * rows];
        }
    for (int jz = 0; jz < m[2]; ++jz)
      for (int jy = 0; jy < m[1]; ++jy)
        for (int jx = 0; jx < m[0]; ++jx, ++slot) {
          int kk[3] = {lo[0] + jx, lo[1] + jy, lo[2] + jz};
          bool ok = true;
          for (int d = 0; d < DIM; ++d) ok = ok && kk[d] >= 0 && kk[d] <= g.N;
          if (ok) row[DIM * g.nV + vert_lin(g, kk)] = v[slot * rows];
        }
    return;
  }
  const long long rr = R - DIM * g.nV;
  int k[3] = {0, 0, 0};
  vert_of(g, rr, k);
  const int s = pressure_segment(DIM);
  const long long rows = gd.seg_rows[s];
  const double* v = gd.vals + gd.seg_off[s] + rr;
  const int wz = DIM == 3 ? 2 : 0;
  int slot = 0;
  for (int c = 0; c < DIM; ++c)
    for (int oz = -wz; oz <= wz; ++oz)
      for (int oy = -2; oy <= 2; ++oy)
        for (int ox = -2; ox <= 2; ++ox, ++slot) {
          int b[3] = {2 * k[0] + ox, 2 * k[1] + oy, DIM == 3 ? 2 * k[2] + oz : 0};
          if (node_inside(g, b)) row[c * g.nV + node_lin(g, b)] = v[slot * rows];
        }
}

// Pivot search, row interchange and scaling of pivot row kk (one block).
__global__ __launch_bounds__(1024) void k_gj_pivot(double* __restrict__ M, long long nb, long long kk,
                                                    int* __restrict__ piv, double* __restrict__ colk,
                                                    int* __restrict__ status) {
  __shared__ double bv[1024];
  __shared__ long long bi[1024];
  double best = -1.0;
  long long besti = kk;
  for (long long i = kk + threadIdx.x; i < nb; i += 1024) {
    const double v = fabs(M[i * nb + kk]);
    if (v > best) { best = v; besti = i; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = besti;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double ob = bv[threadIdx.x + w];
      const long long oi = bi[threadIdx.x + w];
      if (ob > bv[threadIdx.x] || (ob == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = ob;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const long long p = bi[0];
  if (bv[0] <= 0.0) {
    if (threadIdx.x == 0) atomicMin(status, (int)kk);
    return;
  }
  if (threadIdx.x == 0) piv[kk] = (int)p;
  if (p != kk) {
    for (long long j = threadIdx.x; j < nb; j += 1024) {
      const double tmp = M[kk * nb + j];
      M[kk * nb + j] = M[p * nb + j];
      M[p * nb + j] = tmp;
    }
  }
  __syncthreads();
  const double ipv = 1.0 / M[kk * nb + kk];
  for (long long i = threadIdx.x; i < nb; i += 1024) colk[i] = M[i * nb + kk];
  __syncthreads();
  for (long long j = threadIdx.x; j < nb; j += 1024) M[kk * nb + j] = (j == kk) ? ipv : M[kk * nb + j] * ipv;
}

// Elimination of column kk from every other row.
__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ M, long long nb, long long kk,
                                                    const double* __restrict__ colk, const int* __restrict__ status) {
  if (*status != 0x7fffffff) return;
  const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (idx >= nb * nb) return;
  const long long i = idx / nb, j = idx % nb;
  if (i == kk) return;
  const double f = colk[i];
  if (j == kk) M[idx] = -f * M[kk * nb + kk];
  else M[idx] = M[idx] - f * M[kk * nb + j];
}

__global__ __launch_bounds__(256) void k_gj_colswap(double* __restrict__ M, long long nb, const int* __restrict__ piv) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= nb) return;
  double* row = M + i * nb;
  for (long long kk = nb - 1; kk >= 0; --kk) {
    const int q = piv[kk];
    if (q != kk) {
      const double tmp = row[kk];
      row[kk] = row[q];
      row[q] = tmp;
    }
  }
}

// x[i] = sum_{j < n0} Minv[i][j] b[j] for i < n0 (the border column multiplies 0).
__global__ __launch_bounds__(256) void k_coarse_gemv(const double* __restrict__ Minv, long long nb, long long n0,
                                                      const double* __restrict__ b, double* __restrict__ x) {
  const long long row = blockIdx.x * 4LL + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n0) return;
  const double* m = Minv + row * nb;
  double s = 0.0;
  for (long long j = lane; j < n0; j += 64) s += m[j] * b[j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) x[row] = s;
}

// Batched coarse solve: task = (problem, block of 4 rows), one wavefront per row.
__global__ __launch_bounds__(256) void k_coarse_gemv_batch(const GridDev* __restrict__ G,
                                                            const BlockTask* __restrict__ tasks) {
  const BlockTask t = tasks[blockIdx.x];
  if (t.grid < 0) return;
  const GridDev& gd = G[t.grid];
  if (grid_idle(gd)) return;
  const long long n0 = gd.g.n;
  const long long row = t.start + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n0) return;
  const double* m = gd.Minv + row * gd.nbc;
  const double* b = gd.b;
  double s = 0.0;
  for (long long j = lane; j < n0; j += 64) s += m[j] * b[j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) gd.x[row] = s;
}

void launch_coarse_gemv_batch(const GridDev* G, const BlockTask* tasks, int ntasks, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_gemv_batch, dim3(ntasks), dim3(256), 0, s, G, tasks);
}

void launch_coarse_build(const GridDev* G, int dim, double* M, long long nb, int bordered, int unit_masked,
                         hipStream_t s) {
  launch_fill(M, 0.0, nb * nb, s);
  const unsigned blocks = (unsigned)((nb + 255) / 256);
  if (dim == 2) hipLaunchKernelGGL(k_coarse_build<2>, dim3(blocks), dim3(256), 0, s, G, M, nb, bordered, unit_masked);
  else hipLaunchKernelGGL(k_coarse_build<3>, dim3(blocks), dim3(256), 0, s, G, M, nb, bordered, unit_masked);
}

void launch_coarse_gj_step(double* M, long long nb, long long kk, int* piv, double* colk, int* status,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, s, M, nb, kk, piv, colk, status);
  const long long tot = nb * nb;
  hipLaunchKernelGGL(k_gj_update, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, nb, kk, colk, status);
}

void launch_coarse_colswap(double* M, long long nb, const int* piv, hipStream_t s) {
  hipLaunchKernelGGL(k_gj_colswap, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, M, nb, piv);
}

void launch_coarse_gemv(const double* Minv, long long nb, long long n0, const double* b, double* x,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_gemv, dim3((unsigned)((n0 + 3) / 4)), dim3(256), 0, s, Minv, nb, n0, b, x);
}

}  // namespace rav
