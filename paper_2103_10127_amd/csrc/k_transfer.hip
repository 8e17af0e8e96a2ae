// Grid transfer between nested uniform levels (Sec. 2, Fig. 1).
//
// P is the nested Q2/Q1 interpolation: in 1D a coarse Q2 basis function of a
// vertex node takes the values (-1/8, 3/8, 1, 3/8, -1/8) at fine offsets
// (-3, -1, 0, 1, 3) and 0 at +-2; one of a mid node (3/4, 1, 3/4) at (-1, 0, 1);
// the Q1 pressure basis (1/2, 1, 1/2).  The d-dimensional weights are tensor
// products.  Restriction is P^T.  Both are gathers (one thread per output
// node, all components) so no atomics are needed; masked DoFs are skipped
// (their residual and correction are zero).  Restriction starts the coarse
// level from x_c = 0, so it also writes the coarse residual r_c = b_c and the
// coarse level's first smoothing sweep needs no residual launch.
#include <hip/hip_runtime.h>

#include "rav_internal.h"

namespace rav {

// Element idx of a level vector through a 32-bit byte offset from a
// wave-uniform base (level sizes stay below 2^28 elements).
__device__ __forceinline__ double ldv(const double* base, unsigned idx) {
  typedef __attribute__((address_space(1))) const char gcchar;
  typedef __attribute__((address_space(1))) const double gcdouble;
  return *(gcdouble*)((gcchar*)base + (idx << 3));
}

// 1D Q2 restriction weight of fine offset slot i (0..4) around coarse
// position A: even A uses offsets (-3,-1,0,1,3), odd A offsets (-1,0,1).
__host__ __device__ constexpr int rs_off(bool odd, int i) {
  return odd ? i - 1 : (i == 0 ? -3 : i == 4 ? 3 : i - 2);
}
__host__ __device__ constexpr double rs_w(bool odd, int i) {
  return odd ? (i == 1 ? 1.0 : 0.75) : (i == 2 ? 1.0 : (i == 1 || i == 3) ? 0.375 : -0.125);
}

// Restriction (P^T) of the velocity at coarse node A of parity type TY, all
// components: a fully unrolled stencil of 3 or 5 fine nodes per dimension,
// loads at clamped addresses, fine nodes outside the grid weighted 0.
template <int DIM, int TY>
__device__ __forceinline__ void restrict_node(const GridDev& gd, long long row) {
  const Geo& gf = gd.g;
  const Geo& gc = gd.gc;
  int A[3] = {0, 0, 0};
  vel_row_node(gc, TY, row, A);
  const long long cb = node_lin(gc, A);
  double s[DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) s[c] = 0.0;
  if (!node_dirichlet(gc, A)) {
    constexpr int P0 = (TY & 1) ? 3 : 5, P1 = ((TY >> 1) & 1) ? 3 : 5, P2 = DIM == 3 ? (((TY >> 2) & 1) ? 3 : 5) : 1;
    const int twoN = 2 * gf.N;
    const unsigned nn = (unsigned)gf.nn;
#pragma unroll(DIM == 3 ? 1 : 8)
    for (int iz = 0; iz < P2; ++iz) {
      const int fz = DIM == 3 ? 2 * A[2] + rs_off((TY >> 2) & 1, iz) : 0;
      const double wz = DIM == 3 ? rs_w((TY >> 2) & 1, iz) : 1.0;
#pragma unroll
      for (int iy = 0; iy < P1; ++iy) {
        const int fy = 2 * A[1] + rs_off((TY >> 1) & 1, iy);
#pragma unroll
        for (int ix = 0; ix < P0; ++ix) {
          const int fx = 2 * A[0] + rs_off(TY & 1, ix);
          bool in = fx >= 0 && fx <= twoN && fy >= 0 && fy <= twoN;
          if (DIM == 3) in = in && fz >= 0 && fz <= twoN;
          const unsigned lin = (unsigned)min(max(fx, 0), twoN) + nn * (unsigned)min(max(fy, 0), twoN) +
                               nn * nn * (unsigned)min(max(fz, 0), twoN);
          const double w = in ? rs_w(TY & 1, ix) * rs_w((TY >> 1) & 1, iy) * wz : 0.0;
#pragma unroll
          for (int c = 0; c < DIM; ++c) s[c] += w * ldv(gd.r + c * gf.nV, lin);
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    gd.bc[c * gc.nV + cb] = s[c];
    gd.rc[c * gc.nV + cb] = s[c];
    gd.xc[c * gc.nV + cb] = 0.0;
  }
}

// Restriction of the pressure at coarse vertex K: fine vertices 2K + o,
// o in {-1,0,1}^d, weights (1/2, 1, 1/2) per dimension.
template <int DIM>
__device__ __forceinline__ void restrict_pres(const GridDev& gd, long long row) {
  const Geo& gf = gd.g;
  const Geo& gc = gd.gc;
  int K[3] = {0, 0, 0};
  vert_of(gc, row, K);
  const int Nf = gf.N;
  const unsigned np1 = (unsigned)gf.np1;
  const double* rp = gd.r + DIM * gf.nV;
  double s = 0.0;
#pragma unroll
  for (int iz = (DIM == 3 ? -1 : 0); iz <= (DIM == 3 ? 1 : 0); ++iz) {
#pragma unroll
    for (int iy = -1; iy <= 1; ++iy) {
#pragma unroll
      for (int ix = -1; ix <= 1; ++ix) {
        const int kx = 2 * K[0] + ix, ky = 2 * K[1] + iy, kz = DIM == 3 ? 2 * K[2] + iz : 0;
        bool in = kx >= 0 && kx <= Nf && ky >= 0 && ky <= Nf;
        if (DIM == 3) in = in && kz >= 0 && kz <= Nf;
        const unsigned lin = (unsigned)min(max(kx, 0), Nf) + np1 * (unsigned)min(max(ky, 0), Nf) +
                             np1 * np1 * (unsigned)min(max(kz, 0), Nf);
        const double w = (ix == 0 ? 1.0 : 0.5) * (iy == 0 ? 1.0 : 0.5) * (iz == 0 ? 1.0 : 0.5);
        s += (in ? w : 0.0) * ldv(rp, lin);
      }
    }
  }
  const long long i = DIM * gc.nV + row;
  gd.bc[i] = s;
  gd.rc[i] = s;
  gd.xc[i] = 0.0;
}

// Prolongation (x += P xc) at fine node a of parity type TY, all components:
// per dimension one coarse node (even a, weight 1) or three (odd a: coarse
// cell E = a >> 2, weights by a & 3), always inside the coarse grid.
template <int DIM, int TY>
__device__ __forceinline__ void prolong_node(const GridDev& gd, long long row) {
  const Geo& gf = gd.g;
  const Geo& gc = gd.gc;
  int a[3] = {0, 0, 0};
  vel_row_node(gf, TY, row, a);
  if (node_dirichlet(gf, a)) return;
  constexpr int P0 = (TY & 1) ? 3 : 1, P1 = ((TY >> 1) & 1) ? 3 : 1, P2 = DIM == 3 ? (((TY >> 2) & 1) ? 3 : 1) : 1;
  int n0[3] = {0, 0, 0};
  bool first[3] = {false, false, false};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const bool odd = (TY >> d) & 1;
    n0[d] = odd ? 2 * (a[d] >> 2) : a[d] >> 1;
    first[d] = (a[d] & 3) == 1;
  }
  const unsigned nn = (unsigned)gc.nn;
  double s[DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) s[c] = 0.0;
#pragma unroll
  for (int iz = 0; iz < P2; ++iz) {
#pragma unroll
    for (int iy = 0; iy < P1; ++iy) {
#pragma unroll
      for (int ix = 0; ix < P0; ++ix) {
        const int ii[3] = {ix, iy, iz};
        double w = 1.0;
        unsigned lin = 0, st = 1;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          if ((TY >> d) & 1)
            w *= ii[d] == 1 ? 0.75 : ((ii[d] == 0) == first[d] ? 0.375 : -0.125);
          lin += st * (unsigned)(n0[d] + ii[d]);
          st *= nn;
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) s[c] += w * ldv(gd.xc + c * gc.nV, lin);
      }
    }
  }
  const long long base = node_lin(gf, a);
#pragma unroll
  for (int c = 0; c < DIM; ++c) gd.x[c * gf.nV + base] += s[c];
}

// Prolongation of the pressure at fine vertex k: even k_d takes coarse
// vertex k_d / 2, odd k_d the mean of (k_d >> 1) and (k_d >> 1) + 1.
template <int DIM>
__device__ __forceinline__ void prolong_pres(const GridDev& gd, long long row) {
  const Geo& gf = gd.g;
  const Geo& gc = gd.gc;
  int k[3] = {0, 0, 0};
  vert_of(gf, row, k);
  const unsigned np1 = (unsigned)gc.np1;
  const double* xp = gd.xc + DIM * gc.nV;
  double s = 0.0;
#pragma unroll
  for (int iz = 0; iz < (DIM == 3 ? 2 : 1); ++iz) {
#pragma unroll
    for (int iy = 0; iy < 2; ++iy) {
#pragma unroll
      for (int ix = 0; ix < 2; ++ix) {
        const int ii[3] = {ix, iy, iz};
        double w = 1.0;
        unsigned lin = 0, st = 1;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const bool odd = k[d] & 1;
          w *= odd ? 0.5 : (ii[d] == 0 ? 1.0 : 0.0);
          lin += st * (unsigned)((k[d] >> 1) + (odd ? ii[d] : 0));
          st *= np1;
        }
        s += w * ldv(xp, lin);
      }
    }
  }
  gd.x[DIM * gf.nV + row] += s;
}

// Tiles: part = parity type t (velocity nodes of that type on the output
// grid, all components) or 2^d (pressure vertices), as for the residual.
template <int DIM, bool RESTRICT>
__device__ __forceinline__ void transfer_block(const GridDev* __restrict__ G, const BlockTask* __restrict__ tasks) {
  const BlockTask t = tasks[blockIdx.x];
  if (t.grid < 0) return;
  const GridDev& gd = G[t.grid];
  if (grid_idle(gd)) return;
  const Geo& go = RESTRICT ? gd.gc : gd.g;
  const int part = t.part;
  const long long row = t.start + threadIdx.x;
  if (part == (1 << DIM)) {
    if (row >= go.nP) return;
    if (RESTRICT) restrict_pres<DIM>(gd, row);
    else prolong_pres<DIM>(gd, row);
    return;
  }
  if (row >= seg_rows(go, part)) return;
#define RAV_TRANSFER_CASE(TY)                                   \
  case TY:                                                      \
    if (RESTRICT) restrict_node<DIM, TY>(gd, row);              \
    else prolong_node<DIM, TY>(gd, row);                        \
    break;
  if constexpr (DIM == 2) {
    switch (part) { RAV_TRANSFER_CASE(0) RAV_TRANSFER_CASE(1) RAV_TRANSFER_CASE(2) default: RAV_TRANSFER_CASE(3) }
  } else {
    switch (part) {
      RAV_TRANSFER_CASE(0) RAV_TRANSFER_CASE(1) RAV_TRANSFER_CASE(2) RAV_TRANSFER_CASE(3)
      RAV_TRANSFER_CASE(4) RAV_TRANSFER_CASE(5) RAV_TRANSFER_CASE(6) default: RAV_TRANSFER_CASE(7)
    }
  }
#undef RAV_TRANSFER_CASE
}

template <int DIM>
__global__ __launch_bounds__(256) void k_restrict(const GridDev* __restrict__ G, const BlockTask* __restrict__ tasks) {
  transfer_block<DIM, true>(G, tasks);
}

template <int DIM>
__global__ __launch_bounds__(256) void k_prolong(const GridDev* __restrict__ G, const BlockTask* __restrict__ tasks) {
  transfer_block<DIM, false>(G, tasks);
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
