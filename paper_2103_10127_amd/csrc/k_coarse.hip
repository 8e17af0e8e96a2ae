// Coarse-grid direct solver (Sec. 2: a direct LU-type solve on the coarsest
// grid, exact up to rounding).
//
// Set-up: the coarsest operator is expanded to a dense FP64 matrix (masked
// rows become identity rows; with Dirichlet velocity on the whole boundary it
// is bordered by e = (0, 1_p) to fix the pressure constant) and inverted in
// place by blocked Gauss-Jordan elimination with partial pivoting, for all
// problems of a batch at once.  Each cycle the coarse solve is then a single
// dense GEMV with the stored inverse, which parallelises over all CUs instead
// of two sequential triangular solves.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// ---- blocked Gauss-Jordan inversion of a batch of dense matrices ----------
// The coarse matrices of all problems of a batch (same size nb) are inverted
// together, GJ_PANEL pivots at a time.  Panel step (one block per problem,
// one launch per panel): for each pivot of the panel, partial pivoting over
// the rows at and below it, the row interchange over the whole rows, then the
// Gauss-Jordan elimination restricted to the panel's columns; finally the
// panel's pivot rows are saved.  Trailing update (one launch per panel over
// all problems, 64 x 64 tiles): with C the transformed panel columns and R the
// saved pivot rows (outside the panel),
//   M[i][j] = [i not a panel pivot row] M[i][j] + sum_t C[i][t] R[t][j]
// for every column j outside the panel, which applies the panel's eliminations
// to the rest of the matrix at once (rank-GJ_PANEL update: the matrix is read
// and written once per panel instead of once per pivot).  The row
// interchanges are undone as column permutations at the end.
__global__ __launch_bounds__(1024) void k_bgj_panel(double* const* __restrict__ Ms, long long nb, long long k0,
                                                     int bw, int* __restrict__ pivs, double* __restrict__ colk,
                                                     double* __restrict__ Rsave, int* __restrict__ status) {
  __shared__ double bv[1024];
  __shared__ int bi[1024];
  const int prob = blockIdx.x;
  if (status[prob] != 0x7fffffff) return;   // an earlier panel found a zero pivot
  double* __restrict__ M = Ms[prob];
  int* __restrict__ piv = pivs + (long long)prob * nb;
  double* __restrict__ ck = colk + (long long)prob * nb;
  const int tid = threadIdx.x;
  for (long long kk = k0; kk < k0 + bw; ++kk) {
    double best = -1.0;
    int besti = (int)kk;
    for (long long i = kk + tid; i < nb; i += 1024) {
      const double v = fabs(M[i * nb + kk]);
      if (v > best) { best = v; besti = (int)i; }
    }
    bv[tid] = best;
    bi[tid] = besti;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (tid < w) {
        const double ob = bv[tid + w];
        const int oi = bi[tid + w];
        if (ob > bv[tid] || (ob == bv[tid] && oi < bi[tid])) { bv[tid] = ob; bi[tid] = oi; }
      }
      __syncthreads();
    }
    const long long pr = bi[0];
    if (!(bv[0] > 0.0)) {
      if (tid == 0) status[prob] = (int)kk;
      return;
    }
    if (tid == 0) piv[kk] = (int)pr;
    if (pr != kk) {
      for (long long j = tid; j < nb; j += 1024) {
        const double t = M[kk * nb + j];
        M[kk * nb + j] = M[pr * nb + j];
        M[pr * nb + j] = t;
      }
    }
    __syncthreads();
    const double ipv = 1.0 / M[kk * nb + kk];
    for (long long i = tid; i < nb; i += 1024) ck[i] = M[i * nb + kk];
    __syncthreads();
    for (int t = tid; t < bw; t += 1024) {
      const long long j = k0 + t;
      M[kk * nb + j] = j == kk ? ipv : M[kk * nb + j] * ipv;
    }
    __syncthreads();
    for (long long e = tid; e < nb * bw; e += 1024) {
      const long long i = e / bw, j = k0 + e % bw;
      if (i == kk) continue;
      const double f = ck[i];
      M[i * nb + j] = j == kk ? -f * ipv : M[i * nb + j] - f * M[kk * nb + j];
    }
    __syncthreads();
  }
  double* __restrict__ R = Rsave + (long long)prob * GJ_PANEL * nb;
  for (long long e = tid; e < bw * nb; e += 1024) R[e] = M[(k0 + e / nb) * nb + e % nb];
}

__global__ __launch_bounds__(256) void k_bgj_update(double* const* __restrict__ Ms, long long nb, long long k0, int bw,
                                                     const double* __restrict__ Rsave, int ntile,
                                                     const int* __restrict__ status) {
  __shared__ double Cs[64][GJ_PANEL + 1];
  __shared__ double Rs[GJ_PANEL][64 + 1];
  const int prob = blockIdx.y;
  if (status[prob] != 0x7fffffff) return;
  double* __restrict__ M = Ms[prob];
  const double* __restrict__ R = Rsave + (long long)prob * GJ_PANEL * nb;
  const long long row0 = (long long)(blockIdx.x / ntile) * 64, col0 = (long long)(blockIdx.x % ntile) * 64;
  if (col0 >= k0 && col0 + 64 <= k0 + bw) return;   // tile lies inside the panel
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * GJ_PANEL; e += 256) {
    const int r = e / GJ_PANEL, t = e % GJ_PANEL;
    const long long i = row0 + r;
    Cs[r][t] = (i < nb && t < bw) ? M[i * nb + k0 + t] : 0.0;
  }
  for (int e = tid; e < 64 * GJ_PANEL; e += 256) {
    const int t = e / 64, c = e % 64;
    const long long j = col0 + c;
    Rs[t][c] = (j < nb && t < bw) ? R[t * nb + j] : 0.0;
  }
  __syncthreads();
  const int ty = tid / 16, tx = tid % 16;
  double acc[4][4] = {};
#pragma unroll 4
  for (int t = 0; t < GJ_PANEL; ++t) {
    double a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) { a[q] = Cs[ty * 4 + q][t]; b[q] = Rs[t][tx * 4 + q]; }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[q][u] += a[q] * b[u];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const long long i = row0 + ty * 4 + q;
    if (i >= nb) continue;
    const bool pivot_row = i >= k0 && i < k0 + bw;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long j = col0 + tx * 4 + u;
      if (j >= nb || (j >= k0 && j < k0 + bw)) continue;
      const double old = pivot_row ? 0.0 : M[i * nb + j];
      M[i * nb + j] = old + acc[q][u];
    }
  }
}

// Column permutation that undoes the row interchanges: perm[j] = source column
// of column j, from the interchanges applied in reverse order (one thread per problem).
__global__ void k_bgj_perm(const int* __restrict__ pivs, long long nb, int nprob, int* __restrict__ perm,
                           const int* __restrict__ status) {
  const int prob = blockIdx.x * blockDim.x + threadIdx.x;
  if (prob >= nprob || status[prob] != 0x7fffffff) return;
  const int* piv = pivs + (long long)prob * nb;
  int* pm = perm + (long long)prob * nb;
  for (long long j = 0; j < nb; ++j) pm[j] = (int)j;
  for (long long kk = nb - 1; kk >= 0; --kk) {
    const int q = piv[kk];
    const int t = pm[kk]; pm[kk] = pm[q]; pm[q] = t;
  }
}

// One block per (row, problem): the row is staged in LDS and written back permuted.
__global__ __launch_bounds__(256) void k_bgj_colperm(double* const* __restrict__ Ms, long long nb,
                                                      const int* __restrict__ perm, const int* __restrict__ status) {
  extern __shared__ double rowbuf[];
  const int prob = blockIdx.y;
  if (status[prob] != 0x7fffffff) return;
  double* row = Ms[prob] + (long long)blockIdx.x * nb;
  const int* pm = perm + (long long)prob * nb;
  for (long long j = threadIdx.x; j < nb; j += 256) rowbuf[j] = row[j];
  __syncthreads();
  for (long long j = threadIdx.x; j < nb; j += 256) row[j] = rowbuf[pm[j]];
}

void launch_bgj_invert(double* const* Ms, long long nb, int nprob, int* pivs, double* colk, double* Rsave,
                       int* perm, int* status, hipStream_t s) {
  const int ntile = (int)((nb + 63) / 64);
  for (long long k0 = 0; k0 < nb; k0 += GJ_PANEL) {
    const int bw = (int)std::min<long long>(GJ_PANEL, nb - k0);
    hipLaunchKernelGGL(k_bgj_panel, dim3(nprob), dim3(1024), 0, s, Ms, nb, k0, bw, pivs, colk, Rsave, status);
    hipLaunchKernelGGL(k_bgj_update, dim3(ntile * ntile, nprob), dim3(256), 0, s, Ms, nb, k0, bw, Rsave, ntile,
                       status);
  }
  hipLaunchKernelGGL(k_bgj_perm, dim3((nprob + 63) / 64), dim3(64), 0, s, pivs, nb, nprob, perm, status);
  const size_t lds = sizeof(double) * nb;   // one row; above 64 KB the launch must opt in
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)k_bgj_colperm, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)lds);
  hipLaunchKernelGGL(k_bgj_colperm, dim3((unsigned)nb, nprob), dim3(256), lds, s, Ms, nb, perm, status);
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

void launch_coarse_gemv(const double* Minv, long long nb, long long n0, const double* b, double* x,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_gemv, dim3((unsigned)((n0 + 3) / 4)), dim3(256), 0, s, Minv, nb, n0, b, x);
}

}  // namespace rav
