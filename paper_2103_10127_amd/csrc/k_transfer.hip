// Grid transfer between nested uniform levels (Sec. 2, Fig. 1).
//
// P is the nested Q2/Q1 interpolation: in 1D a coarse Q2 basis function of a
// vertex node takes the values (-1/8, 3/8, 1, 3/8, -1/8) at fine offsets
// (-3, -1, 0, 1, 3) and 0 at +-2; one of a mid node (3/4, 1, 3/4) at (-1, 0, 1);
// the Q1 pressure basis (1/2, 1, 1/2).  The d-dimensional weights are tensor
// products.  Restriction is P^T.  Both are gathers (one thread per output
// DoF) so no atomics are needed; masked DoFs are skipped (their residual and
// correction are zero).
#include <hip/hip_runtime.h>

#include "rav_internal.h"

namespace rav {

// 1D restriction stencil of coarse position A: fine offsets and weights.
__device__ __forceinline__ int q2_restrict_1d(int A, int* off, double* w) {
  if ((A & 1) == 0) {
    off[0] = -3; w[0] = -0.125;
    off[1] = -1; w[1] = 0.375;
    off[2] = 0;  w[2] = 1.0;
    off[3] = 1;  w[3] = 0.375;
    off[4] = 3;  w[4] = -0.125;
    return 5;
  }
  off[0] = -1; w[0] = 0.75;
  off[1] = 0;  w[1] = 1.0;
  off[2] = 1;  w[2] = 0.75;
  return 3;
}

// 1D prolongation stencil of fine position a: coarse nodes and weights.
__device__ __forceinline__ int q2_prolong_1d(int a, int* node, double* w) {
  if ((a & 1) == 0) { node[0] = a >> 1; w[0] = 1.0; return 1; }
  const int E = a >> 2;          // coarse cell
  const int first = (a & 3) == 1;
  node[0] = 2 * E;     w[0] = first ? 0.375 : -0.125;
  node[1] = 2 * E + 1; w[1] = 0.75;
  node[2] = 2 * E + 2; w[2] = first ? -0.125 : 0.375;
  return 3;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_restrict(const GridDev* __restrict__ G, const BlockTask* __restrict__ tasks) {
  const BlockTask t = tasks[blockIdx.x];
  if (t.grid < 0) return;
  const GridDev& gd = G[t.grid];
  if (grid_idle(gd)) return;
  const long long i = t.start + threadIdx.x;
  if (i >= gd.gc.n) return;
  const Geo& gf = gd.g;
  const Geo& gc = gd.gc;
  const double* __restrict__ rf = gd.r;
  double s = 0.0;
  if (i < DIM * gc.nV) {
    long long nl_;
    const int c = split_vel(gc, i, &nl_);
    int A[3] = {0, 0, 0};
    node_of(gc, nl_, A);
    if (!node_dirichlet(gc, A)) {
      int off[3][5];
      double w[3][5];
      int n[3] = {1, 1, 1};
      for (int d = 0; d < DIM; ++d) n[d] = q2_restrict_1d(A[d], off[d], w[d]);
      if (DIM == 2) { off[2][0] = 0; w[2][0] = 1.0; }
      for (int iz = 0; iz < n[2]; ++iz)
        for (int iy = 0; iy < n[1]; ++iy)
          for (int ix = 0; ix < n[0]; ++ix) {
            int a[3] = {2 * A[0] + off[0][ix], 2 * A[1] + off[1][iy], DIM == 3 ? 2 * A[2] + off[2][iz] : 0};
            if (!node_inside(gf, a)) continue;
            const double ww = w[0][ix] * w[1][iy] * (DIM == 3 ? w[2][iz] : 1.0);
            s += ww * rf[c * gf.nV + node_lin(gf, a)];
          }
    }
  } else {
    int K[3] = {0, 0, 0};
    vert_of(gc, i - DIM * gc.nV, K);
    const double pw[3] = {0.5, 1.0, 0.5};
    for (int iz = (DIM == 3 ? -1 : 0); iz <= (DIM == 3 ? 1 : 0); ++iz)
      for (int iy = -1; iy <= 1; ++iy)
        for (int ix = -1; ix <= 1; ++ix) {
          int k[3] = {2 * K[0] + ix, 2 * K[1] + iy, DIM == 3 ? 2 * K[2] + iz : 0};
          bool ok = true;
          for (int d = 0; d < DIM; ++d) ok = ok && k[d] >= 0 && k[d] <= gf.N;
          if (!ok) continue;
          const double ww = pw[ix + 1] * pw[iy + 1] * (DIM == 3 ? pw[iz + 1] : 1.0);
          s += ww * rf[DIM * gf.nV + vert_lin(gf, k)];
        }
  }
  gd.bc[i] = s;
  gd.xc[i] = 0.0;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_prolong(const GridDev* __restrict__ G, const BlockTask* __restrict__ tasks) {
  const BlockTask t = tasks[blockIdx.x];
  if (t.grid < 0) return;
  const GridDev& gd = G[t.grid];
  if (grid_idle(gd)) return;
  const long long i = t.start + threadIdx.x;
  if (i >= gd.g.n) return;
  const Geo& gf = gd.g;
  const Geo& gc = gd.gc;
  const double* __restrict__ xc = gd.xc;
  double s = 0.0;
  if (i < DIM * gf.nV) {
    long long nl_;
    const int c = split_vel(gf, i, &nl_);
    int a[3] = {0, 0, 0};
    node_of(gf, nl_, a);
    if (node_dirichlet(gf, a)) return;
    int nodes[3][3];
    double w[3][3];
    int n[3] = {1, 1, 1};
    for (int d = 0; d < DIM; ++d) n[d] = q2_prolong_1d(a[d], nodes[d], w[d]);
    if (DIM == 2) { nodes[2][0] = 0; w[2][0] = 1.0; }
    for (int iz = 0; iz < n[2]; ++iz)
      for (int iy = 0; iy < n[1]; ++iy)
        for (int ix = 0; ix < n[0]; ++ix) {
          int A[3] = {nodes[0][ix], nodes[1][iy], DIM == 3 ? nodes[2][iz] : 0};
          const double ww = w[0][ix] * w[1][iy] * (DIM == 3 ? w[2][iz] : 1.0);
          s += ww * xc[c * gc.nV + node_lin(gc, A)];
        }
  } else {
    int k[3] = {0, 0, 0};
    vert_of(gf, i - DIM * gf.nV, k);
    int nodes[3][2];
    double w[3][2];
    int n[3] = {1, 1, 1};
    for (int d = 0; d < DIM; ++d) {
      if ((k[d] & 1) == 0) { nodes[d][0] = k[d] >> 1; w[d][0] = 1.0; n[d] = 1; }
      else { nodes[d][0] = k[d] >> 1; nodes[d][1] = (k[d] >> 1) + 1; w[d][0] = 0.5; w[d][1] = 0.5; n[d] = 2; }
    }
    if (DIM == 2) { nodes[2][0] = 0; w[2][0] = 1.0; }
    for (int iz = 0; iz < n[2]; ++iz)
      for (int iy = 0; iy < n[1]; ++iy)
        for (int ix = 0; ix < n[0]; ++ix) {
          int K[3] = {nodes[0][ix], nodes[1][iy], DIM == 3 ? nodes[2][iz] : 0};
          const double ww = w[0][ix] * w[1][iy] * (DIM == 3 ? w[2][iz] : 1.0);
          s += ww * xc[DIM * gc.nV + vert_lin(gc, K)];
        }
  }
  gd.x[i] += s;
}

void launch_restrict(int dim, const GridDev* G, const BlockTask* tasks, int ntasks, hipStream_t s) {
  if (dim == 2) hipLaunchKernelGGL(k_restrict<2>, dim3(ntasks), dim3(256), 0, s, G, tasks);
  else hipLaunchKernelGGL(k_restrict<3>, dim3(ntasks), dim3(256), 0, s, G, tasks);
}

void launch_prolong(int dim, const GridDev* G, const BlockTask* tasks, int ntasks, hipStream_t s) {
  if (dim == 2) hipLaunchKernelGGL(k_prolong<2>, dim3(ntasks), dim3(256), 0, s, G, tasks);
  else hipLaunchKernelGGL(k_prolong<3>, dim3(ntasks), dim3(256), 0, s, G, tasks);
}

}  // namespace rav
