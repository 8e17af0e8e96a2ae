// Residual r = b - L x (eq. 10) evaluated cell by cell without reading the
// assembled operator.
//
// On a uniform grid every cell matrix of the divergence block is the same
// (B_e = -h^(d-1) x reference), and the viscous cell matrix is
// A_e = h^(d-2) eta_e x reference wherever the viscosity is constant on the
// cell; only cells cut by an inclusion keep a full stored A_e.  The reference
// matrices are the closed-form tensor products of the 1D Q2 stiffness/mass and
// Q1-Q2 coupling integrals:
//   K = 1/3 [[7,-8,1],[-8,16,-8],[1,-8,7]],  M = 1/30 [[4,2,-1],[2,16,2],[-1,2,4]],
//   G[k][a] = int psi_k phi_a' = [[-5/6, 2/3, 1/6], [-1/6, -2/3, 5/6]],
//   H[k][a] = int psi_k phi_a  = [[1/6, 1/3, 0], [0, 1/3, 1/6]].
// A thread owns one velocity node (both/all components) or one pressure
// vertex and gathers the contributions of the cells around it, so the sweep
// reads x, b, one coefficient per cell and the few cut-cell matrices instead
// of ~25 operator values per DoF.  Columns on masked (Dirichlet) nodes
// contribute nothing, exactly as the assembled operator drops them.  The
// per-cell coefficient is h^(d-2) eta_e, or -(1 + i) for the i-th cut cell
// whose full viscous matrix (h^(d-2) included) is cutA[i].
#include <hip/hip_runtime.h>

#include "rav_internal.h"

namespace rav {

__host__ __device__ constexpr double k1(int a, int b) {
  return a == b ? (a == 1 ? 16.0 / 3.0 : 7.0 / 3.0) : ((a == 1 || b == 1) ? -8.0 / 3.0 : 1.0 / 3.0);
}
__host__ __device__ constexpr double m1(int a, int b) {
  return a == b ? (a == 1 ? 16.0 / 30.0 : 4.0 / 30.0) : ((a == 1 || b == 1) ? 2.0 / 30.0 : -1.0 / 30.0);
}
__host__ __device__ constexpr double g1(int k, int a) {
  return k == 0 ? (a == 0 ? -5.0 / 6.0 : a == 1 ? 2.0 / 3.0 : 1.0 / 6.0)
                : (a == 0 ? -1.0 / 6.0 : a == 1 ? -2.0 / 3.0 : 5.0 / 6.0);
}
__host__ __device__ constexpr double h1(int k, int a) {
  return k == 0 ? (a == 0 ? 1.0 / 6.0 : a == 1 ? 1.0 / 3.0 : 0.0) : (a == 0 ? 0.0 : a == 1 ? 1.0 / 3.0 : 1.0 / 6.0);
}
// Reference viscous cell matrix (h = 1, eta = 1): sum_c K(a_c,b_c) prod_{d != c} M(a_d,b_d).
template <int DIM>
__host__ __device__ constexpr double aref(int la, int lb) {
  double s = 0.0;
  for (int c = 0; c < DIM; ++c) {
    double p = 1.0;
    int a = la, b = lb;
    for (int d = 0; d < DIM; ++d) {
      p *= (d == c) ? k1(a % 3, b % 3) : m1(a % 3, b % 3);
      a /= 3;
      b /= 3;
    }
    s += p;
  }
  return s;
}
// Reference divergence cell matrix (h = 1): -G(k_c,a_c) prod_{d != c} H(k_d,a_d).
template <int DIM>
__host__ __device__ constexpr double bref(int c, int la, int lk) {
  double p = -1.0;
  int a = la, k = lk;
  for (int d = 0; d < DIM; ++d) {
    p *= (d == c) ? g1(k & 1, a % 3) : h1(k & 1, a % 3);
    a /= 3;
    k >>= 1;
  }
  return p;
}

template <int DIM>
struct Tabs {
  double A[ipow(3, DIM) * ipow(3, DIM)];
  double B[DIM * ipow(3, DIM) * ipow(2, DIM)];
  constexpr Tabs() : A(), B() {
    for (int a = 0; a < ipow(3, DIM); ++a)
      for (int b = 0; b < ipow(3, DIM); ++b) A[a * ipow(3, DIM) + b] = aref<DIM>(a, b);
    for (int c = 0; c < DIM; ++c)
      for (int a = 0; a < ipow(3, DIM); ++a)
        for (int k = 0; k < ipow(2, DIM); ++k) B[(c * ipow(3, DIM) + a) * ipow(2, DIM) + k] = bref<DIM>(c, a, k);
  }
};
__constant__ const Tabs<2> c_tab2 = Tabs<2>();
__constant__ const Tabs<3> c_tab3 = Tabs<3>();

template <int DIM>
__device__ __forceinline__ const Tabs<DIM>& tabs();
template <>
__device__ __forceinline__ const Tabs<2>& tabs<2>() { return c_tab2; }
template <>
__device__ __forceinline__ const Tabs<3>& tabs<3>() { return c_tab3; }

// Global-memory views of the level vectors (the descriptor holds generic
// pointers; the explicit address space gives global instead of flat loads).
typedef __attribute__((address_space(1))) const double gcdouble;
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ gcdouble* gview(const double* p) { return (gcdouble*)p; }
__device__ __forceinline__ gdouble* gview(double* p) { return (gdouble*)p; }
// Element idx of a level vector (level sizes stay below 2^28 elements, so the
// byte offset is a 32-bit value added to a wave-uniform base address).
__device__ __forceinline__ double ld(gcdouble* base, unsigned idx) {
  typedef __attribute__((address_space(1))) const char gcchar;
  return *(gcdouble*)((gcchar*)base + (idx << 3));
}

// Half-grid position a_d + o_d holds a free velocity node in dimension d:
// inside the grid and not on a masked side.
__device__ __forceinline__ bool free_coord(const Geo& g, int d, int v) {
  return v >= 0 && v <= 2 * g.N && !coord_dirichlet(g, d, v);
}

// Velocity node a of parity type TY (all components).  Cells around the node:
// per dimension one cell (odd position, local index 1) or two (even position,
// local index 2 in the lower cell, 0 in the upper one).  The row is a stencil
// over the unique column nodes a + o, |o_d| <= W_d, and pressure vertices
// lo + j; the coefficient of a column is the sum over the cells that contain
// it of (cell coefficient) x (reference entry), the reference entries folding
// into immediates.  All cell coefficients and column values are loaded up
// front at clamped (in-range) addresses; missing cells get coefficient 0 and
// columns outside the grid or on a masked side are replaced by 0 with a
// select, so every path is branch-free except the correction for cut cells
// (whose full matrices replace the scaled reference).
// With OUT the row values go to out[c] (per component) instead of r.
template <int DIM, int TY, bool OUT = false>
__device__ __forceinline__ double res_node(const GridDev& gd, long long row, double* out = nullptr) {
  constexpr int NV = ipow(3, DIM), NP = ipow(2, DIM);
  constexpr int NE0 = (TY & 1) ? 1 : 2, NE1 = ((TY >> 1) & 1) ? 1 : 2;
  constexpr int NE2 = DIM == 3 ? (((TY >> 2) & 1) ? 1 : 2) : 1;
  constexpr int NE = NE0 * NE1 * NE2;
  constexpr int W0 = (TY & 1) ? 1 : 2, W1 = ((TY >> 1) & 1) ? 1 : 2;
  constexpr int W2 = DIM == 3 ? (((TY >> 2) & 1) ? 1 : 2) : 0;
  constexpr int M0 = 3 - (TY & 1), M1 = 3 - ((TY >> 1) & 1), M2 = DIM == 3 ? 3 - ((TY >> 2) & 1) : 1;
  const Geo& g = gd.g;
  const Tabs<DIM>& T = tabs<DIM>();
  gcdouble* __restrict__ X = gview(gd.x);
  gdouble* __restrict__ R = gview(gd.r);
  int a[3] = {0, 0, 0};
  vel_row_node(g, TY, row, a);
  const long long base = node_lin(g, a);
  double bv[DIM];   // right-hand sides first: their latency overlaps the row's arithmetic
#pragma unroll
  for (int c = 0; c < DIM; ++c) bv[c] = gview(gd.b)[c * g.nV + base];
  if (node_dirichlet(g, a)) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      if constexpr (OUT) out[c] = 0.0;
      else R[c * g.nV + base] = 0.0;
    }
    return 0.0;
  }
  const int N = g.N;
  const long long nn = g.nn, nn2 = g.nn * g.nn, np1 = g.np1, np12 = g.np1 * g.np1, nV = g.nV;
  // cells: coefficient (0 when missing or cut), existence, cut index
  double cef[NE];
  bool okc[NE];
  long long cut_row[NE];
  bool anycut = false;
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int eo[3] = {i % NE0, (i / NE0) % NE1, i / (NE0 * NE1)};
    int E[3] = {0, 0, 0}, la = 0;
    bool ok = true;
#pragma unroll
    for (int d = 0, st = 1; d < DIM; ++d, st *= 3) {
      const bool odd = (TY >> d) & 1;
      E[d] = odd ? (a[d] - 1) >> 1 : (a[d] >> 1) - 1 + eo[d];
      la += (odd ? 1 : 2 - 2 * eo[d]) * st;
      ok = ok && E[d] >= 0 && E[d] < N;
      E[d] = min(max(E[d], 0), N - 1);
    }
    const double ce = gd.ceta[E[0] + (long long)N * (E[1] + (long long)N * (DIM == 3 ? E[2] : 0))];
    okc[i] = ok;
    cef[i] = ok && ce >= 0.0 ? ce : 0.0;
    const bool cut = ok && ce < 0.0;
    cut_row[i] = cut ? ((long long)(-ce) - 1) * (NV * NV) + la * NV : -1;
    anycut = anycut || cut;
  }
  // columns per dimension and offset: free flag and clamped (in-range) position
  bool fv[2][5];
  unsigned cpos[2][5];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
#pragma unroll
    for (int o = -2; o <= 2; ++o) {
      fv[d][o + 2] = free_coord(g, d, a[d] + o);
      cpos[d][o + 2] = (unsigned)min(max(a[d] + o, 0), 2 * N) * (d == 0 ? 1u : (unsigned)nn);
    }
  }
  double acc[DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) acc[c] = 0.0;
#pragma unroll(DIM == 3 ? 1 : DIM)
  for (int c = 0; c < DIM; ++c) {
    gcdouble* __restrict__ xc = X + c * nV;
    double sc = 0.0;
#pragma unroll(DIM == 3 ? 1 : 8)
    for (int oz = -W2; oz <= W2; ++oz) {
#pragma unroll
      for (int oy = -W1; oy <= W1; ++oy) {
#pragma unroll
        for (int ox = -W0; ox <= W0; ++ox) {
          const int o[3] = {ox, oy, oz};
          bool fr = fv[0][ox + 2] && fv[1][oy + 2];
          unsigned lin = cpos[0][ox + 2] + cpos[1][oy + 2];
          if (DIM == 3) {
            fr = fr && free_coord(g, 2, a[2] + oz);
            lin += (unsigned)min(max(a[2] + oz, 0), 2 * N) * (unsigned)nn2;
          }
          const double xv = ld(xc, lin);
          double coef = 0.0;
#pragma unroll
          for (int i = 0; i < NE; ++i) {
            const int eo[3] = {i % NE0, (i / NE0) % NE1, i / (NE0 * NE1)};
            int la = 0, lb = 0;
            bool in = true;
#pragma unroll
            for (int d = 0, st = 1; d < DIM; ++d, st *= 3) {
              const int l = ((TY >> d) & 1) ? 1 : 2 - 2 * eo[d];
              la += l * st;
              lb += (l + o[d]) * st;
              in = in && l + o[d] >= 0 && l + o[d] <= 2;
            }
            if (in) coef += cef[i] * T.A[la * NV + lb];
          }
          sc += (fr ? coef : 0.0) * xv;
        }
      }
    }
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc) acc[cc] += cc == c ? sc : 0.0;   // register select, no indexed array
  }
  // pressure columns k = lo + j, lo_d = (a_d >> 1) - 1 + (a_d & 1), j_d < M_d
  double accB[DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) accB[c] = 0.0;
  int lo[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < DIM; ++d) lo[d] = (a[d] >> 1) - 1 + ((TY >> d) & 1);
  gcdouble* __restrict__ XP = X + DIM * nV;
  const unsigned pstr[3] = {1u, (unsigned)np1, (unsigned)np12};
#pragma unroll(DIM == 3 ? 1 : 8)
  for (int jz = 0; jz < M2; ++jz) {
#pragma unroll
    for (int jy = 0; jy < M1; ++jy) {
#pragma unroll
      for (int jx = 0; jx < M0; ++jx) {
        const int j[3] = {jx, jy, jz};
        bool in_grid = true;
        unsigned lin = 0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const int k = lo[d] + j[d];
          in_grid = in_grid && k >= 0 && k <= N;
          lin += (unsigned)min(max(k, 0), N) * pstr[d];
        }
        const double pv = ld(XP, lin);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          double coef = 0.0;
#pragma unroll
          for (int i = 0; i < NE; ++i) {
            const int eo[3] = {i % NE0, (i / NE0) % NE1, i / (NE0 * NE1)};
            int la = 0, lk = 0;
            bool in = true;
#pragma unroll
            for (int d = 0, st = 1; d < DIM; ++d, st *= 3) {
              const bool odd = (TY >> d) & 1;
              la += (odd ? 1 : 2 - 2 * eo[d]) * st;
              const int kl = j[d] - (odd ? 0 : eo[d]);   // vertex index inside the cell
              in = in && kl >= 0 && kl <= 1;
              lk |= (kl & 1) << d;
            }
            if (in) coef += okc[i] ? T.B[(c * NV + la) * NP + lk] : 0.0;
          }
          accB[c] += (in_grid ? coef : 0.0) * pv;
        }
      }
    }
  }
  // cut cells: full cell matrix rows (rare, divergent)
  if (anycut) {
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      if (cut_row[i] < 0) continue;
      const int eo[3] = {i % NE0, (i / NE0) % NE1, i / (NE0 * NE1)};
      int E2[3] = {0, 0, 0};
#pragma unroll
      for (int d = 0; d < DIM; ++d) E2[d] = ((TY >> d) & 1) ? a[d] - 1 : a[d] - 2 + 2 * eo[d];
      gcdouble* __restrict__ Ae = gview(gd.cutA) + cut_row[i];
#pragma unroll(DIM == 3 ? 9 : NV)
      for (int lb = 0; lb < NV; ++lb) {
        const int b[3] = {E2[0] + lb % 3, E2[1] + (lb / 3) % 3, DIM == 3 ? E2[2] + lb / 9 : 0};
        bool fr = true;
#pragma unroll
        for (int d = 0; d < DIM; ++d) fr = fr && !coord_dirichlet(g, d, b[d]);
        const double w = Ae[lb];
        const long long lin = b[0] + nn * b[1] + nn2 * b[2];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          const double xv = X[c * nV + lin];
          acc[c] += w * (fr ? xv : 0.0);
        }
      }
    }
  }
  const double hB = DIM == 2 ? gd.h : gd.h * gd.h;
  double sq = 0.0;
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const long long gi = c * nV + base;
    const double r = bv[c] - (acc[c] + hB * accB[c]);
    if constexpr (OUT) out[c] = r;
    else R[gi] = r;
    sq += r * r;
  }
  return sq;
}

// Pressure row of vertex k: divergence of the velocity over the (up to 2^d)
// cells around the vertex (cell k - 1 + eo, local vertex 1 - eo), as a stencil
// over the nodes 2k + o, |o_d| <= 2, with constant coefficients; missing cells
// and masked or outside columns contribute nothing (selects, no branches).
template <int DIM, bool OUT = false>
__device__ __forceinline__ double res_pres(const GridDev& gd, long long row, double* out = nullptr) {
  constexpr int NV = ipow(3, DIM), NP = ipow(2, DIM);
  const Geo& g = gd.g;
  const Tabs<DIM>& T = tabs<DIM>();
  gcdouble* __restrict__ X = gview(gd.x);
  int k[3] = {0, 0, 0};
  vert_of(g, row, k);
  const int N = g.N;
  const long long nn = g.nn, nV = g.nV;
  const double bv = gview(gd.b)[DIM * nV + row];   // issued first
  bool okc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int E = k[d] - 1 + ((i >> d) & 1);
      ok = ok && E >= 0 && E < N;
    }
    okc[i] = ok;
  }
  bool fv[2][5];
  unsigned cpos[2][5];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
#pragma unroll
    for (int o = -2; o <= 2; ++o) {
      fv[d][o + 2] = free_coord(g, d, 2 * k[d] + o);
      cpos[d][o + 2] = (unsigned)min(max(2 * k[d] + o, 0), 2 * N) * (d == 0 ? 1u : (unsigned)nn);
    }
  }
  double acc = 0.0;
#pragma unroll(DIM == 3 ? 1 : DIM)
  for (int c = 0; c < DIM; ++c) {
    gcdouble* __restrict__ xc = X + c * nV;
#pragma unroll(DIM == 3 ? 1 : 8)
    for (int oz = (DIM == 3 ? -2 : 0); oz <= (DIM == 3 ? 2 : 0); ++oz) {
#pragma unroll
      for (int oy = -2; oy <= 2; ++oy) {
#pragma unroll
        for (int ox = -2; ox <= 2; ++ox) {
          const int o[3] = {ox, oy, oz};
          bool fr = fv[0][ox + 2] && fv[1][oy + 2];
          unsigned lin = cpos[0][ox + 2] + cpos[1][oy + 2];
          if (DIM == 3) {
            fr = fr && free_coord(g, 2, 2 * k[2] + oz);
            lin += (unsigned)min(max(2 * k[2] + oz, 0), 2 * N) * (unsigned)(nn * nn);
          }
          const double xv = ld(xc, lin);
          double coef = 0.0;
#pragma unroll
          for (int i = 0; i < NP; ++i) {
            int lb = 0, lk = 0;
            bool in = true;
#pragma unroll
            for (int d = 0, st = 1; d < DIM; ++d, st *= 3) {
              const int eo = (i >> d) & 1, l = o[d] + 2 - 2 * eo;
              in = in && l >= 0 && l <= 2;
              lb += l * st;
              lk |= (1 - eo) << d;
            }
            if (in) coef += okc[i] ? T.B[(c * NV + lb) * NP + lk] : 0.0;
          }
          acc += (fr ? coef : 0.0) * xv;
        }
      }
    }
  }
  const double hB = DIM == 2 ? gd.h : gd.h * gd.h;
  const long long gi = DIM * nV + row;
  const double r = bv - hB * acc;
  if constexpr (OUT) *out = r;
  else gview(gd.r)[gi] = r;
  return r * r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block task part: velocity parity type t (0 .. 2^d - 1) or 2^d for pressure rows.
template <int DIM>
__device__ __forceinline__ void residual_block(const GridDev* __restrict__ G, const BlockTask* __restrict__ tasks,
                                               double* __restrict__ partials) {
  const BlockTask t = tasks[blockIdx.x];
  if (t.grid < 0) return;
  const GridDev& gd = G[t.grid];
  if (grid_idle(gd)) return;
  double sq = 0.0;
  const long long row = t.start + threadIdx.x;
  const int part = t.part;
  const long long rows = part == (1 << DIM) ? gd.g.nP : seg_rows(gd.g, part);
  if (row < rows) {
    if constexpr (DIM == 2) {
      switch (part) {
        case 0: sq = res_node<2, 0>(gd, row); break;
        case 1: sq = res_node<2, 1>(gd, row); break;
        case 2: sq = res_node<2, 2>(gd, row); break;
        case 3: sq = res_node<2, 3>(gd, row); break;
        default: sq = res_pres<2>(gd, row); break;
      }
    } else {
      switch (part) {
        case 0: sq = res_node<3, 0>(gd, row); break;
        case 1: sq = res_node<3, 1>(gd, row); break;
        case 2: sq = res_node<3, 2>(gd, row); break;
        case 3: sq = res_node<3, 3>(gd, row); break;
        case 4: sq = res_node<3, 4>(gd, row); break;
        case 5: sq = res_node<3, 5>(gd, row); break;
        case 6: sq = res_node<3, 6>(gd, row); break;
        case 7: sq = res_node<3, 7>(gd, row); break;
        default: sq = res_pres<3>(gd, row); break;
      }
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

__global__ __launch_bounds__(BLOCK) void k_residual2(const GridDev* __restrict__ G, const BlockTask* __restrict__ tasks,
                                                     double* __restrict__ partials) {
  residual_block<2>(G, tasks, partials);
}
__global__ __launch_bounds__(BLOCK) void k_residual3(const GridDev* __restrict__ G, const BlockTask* __restrict__ tasks,
                                                     double* __restrict__ partials) {
  residual_block<3>(G, tasks, partials);
}

// ---- 2D residual staged through LDS ------------------------------------------
// Large 2D levels: one block per tile of RT_X x RT_Y cells.  The block first
// loads the tile's velocity nodes, pressure vertices and cell coefficients with
// a two-node halo into LDS (row-contiguous, coalesced loads), then evaluates
// the rows of the nodes the tile owns, one node parity type per round so that
// a wavefront shares one compile-time stencil, reading every column value
// from LDS.  A tile owns velocity nodes a_d in [2 x0_d, 2 x0_d + 2 RT_d) and
// pressure vertices k_d in [x0_d, x0_d + RT_d), plus the last node layer
// (a_d = 2N, k_d = N) in the last tile of each direction.  The row formulas
// are those of res_node / res_pres.
// Window positions in parity-split order: per dimension the even positions l
// first, then the odd ones, so nodes of one parity sit at consecutive addresses.
__host__ __device__ constexpr int qperm(int l, int half) { return (l & 1) ? half + (l >> 1) : (l >> 1); }
// Position of l + o relative to l >> 1 in the permuted order, for l of parity t.
__host__ __device__ constexpr int qoff(int t, int o, int half) { return (((t + o) & 1) ? half : 0) + ((t + o + 4) >> 1) - 2; }

constexpr int RT_X = 32, RT_Y = 8;
constexpr int RW_X = 2 * RT_X + 5, RW_Y = 2 * RT_Y + 5;   // velocity window (node a = 2 x0 - 2 + index)
constexpr int RP_X = RT_X + 3, RP_Y = RT_Y + 3;           // pressure window (vertex k = x0 - 1 + index)
constexpr int RC_X = RT_X + 2, RC_Y = RT_Y + 2;           // cell window (cell E = x0 - 1 + index)
constexpr int RE_X = (RW_X + 1) / 2;                       // x positions in parity-split order (evens first)

struct TileLds {
  double xs[2][RW_Y][RW_X];
  double ps[RP_Y][RP_X];
  double cs[RC_Y][RC_X];
};

template <int TY>
__device__ __forceinline__ double res_node_lds(const GridDev& gd, const TileLds& S, int x0, int y0, int a0, int a1) {
  constexpr int NV = 9, NP = 4;
  constexpr int NE0 = (TY & 1) ? 1 : 2, NE1 = ((TY >> 1) & 1) ? 1 : 2, NE = NE0 * NE1;
  constexpr int W0 = (TY & 1) ? 1 : 2, W1 = ((TY >> 1) & 1) ? 1 : 2;
  constexpr int M0 = 3 - (TY & 1), M1 = 3 - ((TY >> 1) & 1);
  const Geo& g = gd.g;
  const Tabs<2>& T = tabs<2>();
  const int a[3] = {a0, a1, 0};
  const long long nn = g.nn, nV = g.nV;
  const long long base = a0 + nn * a1;
  gdouble* __restrict__ R = gview(gd.r);
  // right-hand sides first: their latency overlaps the row's arithmetic
  const double bv0 = gview(gd.b)[base], bv1 = gview(gd.b)[nV + base];
  if (node_dirichlet(g, a)) {
    R[base] = 0.0;
    R[nV + base] = 0.0;
    return 0.0;
  }
  const int N = g.N;
  double cef[NE];
  bool okc[NE];
  long long cut_row[NE];
  bool anycut = false;
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int eo[2] = {i % NE0, i / NE0};
    int E[2], la = 0;
    bool ok = true;
#pragma unroll
    for (int d = 0, st = 1; d < 2; ++d, st *= 3) {
      const bool odd = (TY >> d) & 1;
      E[d] = odd ? (a[d] - 1) >> 1 : (a[d] >> 1) - 1 + eo[d];
      la += (odd ? 1 : 2 - 2 * eo[d]) * st;
      ok = ok && E[d] >= 0 && E[d] < N;
    }
    const double ce = S.cs[E[1] - (y0 - 1)][E[0] - (x0 - 1)];
    okc[i] = ok;
    cef[i] = ok && ce >= 0.0 ? ce : 0.0;
    const bool cut = ok && ce < 0.0;
    cut_row[i] = cut ? ((long long)(-ce) - 1) * (NV * NV) + la * NV : -1;
    anycut = anycut || cut;
  }
  bool fv[2][5];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
#pragma unroll
    for (int o = -2; o <= 2; ++o) fv[d][o + 2] = free_coord(g, d, a[d] + o);
  }
  const int lx = a0 - (2 * x0 - 2), ly = a1 - (2 * y0 - 2);
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int oy = -W1; oy <= W1; ++oy) {
#pragma unroll
    for (int ox = -W0; ox <= W0; ++ox) {
      const int o[2] = {ox, oy};
      double coef = 0.0;
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const int eo[2] = {i % NE0, i / NE0};
        int la = 0, lb = 0;
        bool in = true;
#pragma unroll
        for (int d = 0, st = 1; d < 2; ++d, st *= 3) {
          const int l = ((TY >> d) & 1) ? 1 : 2 - 2 * eo[d];
          la += l * st;
          lb += (l + o[d]) * st;
          in = in && l + o[d] >= 0 && l + o[d] <= 2;
        }
        if (in) coef += cef[i] * T.A[la * NV + lb];
      }
      coef = fv[0][ox + 2] && fv[1][oy + 2] ? coef : 0.0;
      acc[0] += coef * S.xs[0][ly + oy][(lx >> 1) + qoff(TY & 1, ox, RE_X)];
      acc[1] += coef * S.xs[1][ly + oy][(lx >> 1) + qoff(TY & 1, ox, RE_X)];
    }
  }
  double accB[2] = {0.0, 0.0};
  const int lo[2] = {(a0 >> 1) - 1 + (TY & 1), (a1 >> 1) - 1 + ((TY >> 1) & 1)};
#pragma unroll
  for (int jy = 0; jy < M1; ++jy) {
#pragma unroll
    for (int jx = 0; jx < M0; ++jx) {
      const int j[2] = {jx, jy};
      const int k0 = lo[0] + jx, k1 = lo[1] + jy;
      const bool in_grid = k0 >= 0 && k0 <= N && k1 >= 0 && k1 <= N;
      const double pv = S.ps[k1 - (y0 - 1)][k0 - (x0 - 1)];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        double coef = 0.0;
#pragma unroll
        for (int i = 0; i < NE; ++i) {
          const int eo[2] = {i % NE0, i / NE0};
          int la = 0, lk = 0;
          bool in = true;
#pragma unroll
          for (int d = 0, st = 1; d < 2; ++d, st *= 3) {
            const bool odd = (TY >> d) & 1;
            la += (odd ? 1 : 2 - 2 * eo[d]) * st;
            const int kl = j[d] - (odd ? 0 : eo[d]);
            in = in && kl >= 0 && kl <= 1;
            lk |= (kl & 1) << d;
          }
          if (in) coef += okc[i] ? T.B[(c * NV + la) * NP + lk] : 0.0;
        }
        accB[c] += (in_grid ? coef : 0.0) * pv;
      }
    }
  }
  if (anycut) {
    gcdouble* __restrict__ X = gview(gd.x);
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      if (cut_row[i] < 0) continue;
      const int eo[2] = {i % NE0, i / NE0};
      int E2[2];
#pragma unroll
      for (int d = 0; d < 2; ++d) E2[d] = ((TY >> d) & 1) ? a[d] - 1 : a[d] - 2 + 2 * eo[d];
      gcdouble* __restrict__ Ae = gview(gd.cutA) + cut_row[i];
#pragma unroll
      for (int lb = 0; lb < NV; ++lb) {
        const int b0 = E2[0] + lb % 3, b1 = E2[1] + lb / 3;
        const bool fr = !coord_dirichlet(g, 0, b0) && !coord_dirichlet(g, 1, b1);
        const double w = Ae[lb];
        const long long lin = b0 + nn * b1;
        acc[0] += w * (fr ? X[lin] : 0.0);
        acc[1] += w * (fr ? X[nV + lin] : 0.0);
      }
    }
  }
  const double hB = gd.h;
  double sq = 0.0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const long long gi = c * nV + base;
    const double r = (c == 0 ? bv0 : bv1) - (acc[c] + hB * accB[c]);
    R[gi] = r;
    sq += r * r;
  }
  return sq;
}

__device__ __forceinline__ double res_pres_lds(const GridDev& gd, const TileLds& S, int x0, int y0, int k0, int k1) {
  constexpr int NV = 9, NP = 4;
  const Geo& g = gd.g;
  const long long gi = 2 * g.nV + k0 + g.np1 * k1;
  const double bv = gview(gd.b)[gi];   // issued first
  const Tabs<2>& T = tabs<2>();
  const int N = g.N;
  const int k[2] = {k0, k1};
  bool okc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int E = k[d] - 1 + ((i >> d) & 1);
      ok = ok && E >= 0 && E < N;
    }
    okc[i] = ok;
  }
  bool fv[2][5];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
#pragma unroll
    for (int o = -2; o <= 2; ++o) fv[d][o + 2] = free_coord(g, d, 2 * k[d] + o);
  }
  const int lx = 2 * k0 - (2 * x0 - 2), ly = 2 * k1 - (2 * y0 - 2);
  double acc = 0.0;
#pragma unroll
  for (int oy = -2; oy <= 2; ++oy) {
#pragma unroll
    for (int ox = -2; ox <= 2; ++ox) {
      const int o[2] = {ox, oy};
      const bool fr = fv[0][ox + 2] && fv[1][oy + 2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        double coef = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          int lb = 0, lk = 0;
          bool in = true;
#pragma unroll
          for (int d = 0, st = 1; d < 2; ++d, st *= 3) {
            const int eo = (i >> d) & 1, l = o[d] + 2 - 2 * eo;
            in = in && l >= 0 && l <= 2;
            lb += l * st;
            lk |= (1 - eo) << d;
          }
          if (in) coef += okc[i] ? T.B[(c * NV + lb) * NP + lk] : 0.0;
        }
        acc += (fr ? coef : 0.0) * S.xs[c][ly + oy][(lx >> 1) + qoff(0, ox, RE_X)];
      }
    }
  }
  const double r = bv - gd.h * acc;
  gview(gd.r)[gi] = r;
  return r * r;
}

template <int TY>
__device__ __forceinline__ double tile_round(const GridDev& gd, const TileLds& S, int x0, int y0, bool last_x,
                                             bool last_y) {
  const int cx = RT_X + ((last_x && !(TY & 1)) ? 1 : 0);
  const int cy = RT_Y + ((last_y && !((TY >> 1) & 1)) ? 1 : 0);
  double sq = 0.0;
  for (int i = threadIdx.x; i < cx * cy; i += BLOCK) {
    const int ix = i % cx, iy = i / cx;
    sq += res_node_lds<TY>(gd, S, x0, y0, 2 * (x0 + ix) + (TY & 1), 2 * (y0 + iy) + ((TY >> 1) & 1));
  }
  return sq;
}

// Hardware block b works on tile (b mod 8) T/8 + b/8 of the row-major tile
// order (T a multiple of 8), so each XCD sweeps one band of tile rows.
__global__ __launch_bounds__(BLOCK) void k_residual_tiled2(const GridDev* __restrict__ G, double* __restrict__ partials) {
  __shared__ TileLds S;
  const GridDev& gd = *G;
  const Geo& g = gd.g;
  const int N = g.N;
  const int ntx = N / RT_X, nty = N / RT_Y, T = ntx * nty;
  const int b = blockIdx.x;
  const int lt = (b % 8) * (T / 8) + b / 8;
  const int tx = lt % ntx, ty = lt / ntx;
  const int x0 = tx * RT_X, y0 = ty * RT_Y;
  const bool last_x = tx == ntx - 1, last_y = ty == nty - 1;
  {
    // every load of the tile is issued before any is stored (a loop that
    // stored each value before the next load waited out one memory latency
    // per element)
    gcdouble* __restrict__ X = gview(gd.x);
    const unsigned nn = (unsigned)g.nn, nV = (unsigned)g.nV, np1 = (unsigned)g.np1;
    const int twoN = 2 * N;
    constexpr int NXW = 2 * RW_Y * RW_X, XPER = (NXW + BLOCK - 1) / BLOCK;
    constexpr int NPW = RP_Y * RP_X, PPER = (NPW + BLOCK - 1) / BLOCK;
    constexpr int NCW = RC_Y * RC_X, CPER = (NCW + BLOCK - 1) / BLOCK;
    double xv[XPER], pv[PPER], cv[CPER];
#pragma unroll
    for (int q = 0; q < XPER; ++q) {
      const int i = min((int)threadIdx.x + q * BLOCK, NXW - 1);
      const int c = i / (RW_Y * RW_X), rem = i - c * (RW_Y * RW_X);
      const int yy = rem / RW_X, xx = rem - yy * RW_X;
      const unsigned gx = (unsigned)min(max(2 * x0 - 2 + xx, 0), twoN);
      const unsigned gy = (unsigned)min(max(2 * y0 - 2 + yy, 0), twoN);
      xv[q] = ld(X, (unsigned)c * nV + gx + nn * gy);
    }
#pragma unroll
    for (int q = 0; q < PPER; ++q) {
      const int i = min((int)threadIdx.x + q * BLOCK, NPW - 1);
      const int yy = i / RP_X, xx = i - yy * RP_X;
      const unsigned gx = (unsigned)min(max(x0 - 1 + xx, 0), N), gy = (unsigned)min(max(y0 - 1 + yy, 0), N);
      pv[q] = ld(X, 2u * nV + gx + np1 * gy);
    }
#pragma unroll
    for (int q = 0; q < CPER; ++q) {
      const int i = min((int)threadIdx.x + q * BLOCK, NCW - 1);
      const int yy = i / RC_X, xx = i - yy * RC_X;
      const unsigned gx = (unsigned)min(max(x0 - 1 + xx, 0), N - 1), gy = (unsigned)min(max(y0 - 1 + yy, 0), N - 1);
      cv[q] = ld(gview(gd.ceta), gx + (unsigned)N * gy);
    }
#pragma unroll
    for (int q = 0; q < XPER; ++q) {
      const int i = (int)threadIdx.x + q * BLOCK;
      if (i < NXW) {
        const int c = i / (RW_Y * RW_X), rem = i - c * (RW_Y * RW_X);
        const int yy = rem / RW_X, xx = rem - yy * RW_X;
        S.xs[c][yy][qperm(xx, RE_X)] = xv[q];   // one parity type's nodes contiguous: no bank conflicts
      }
    }
#pragma unroll
    for (int q = 0; q < PPER; ++q) {
      const int i = (int)threadIdx.x + q * BLOCK;
      if (i < NPW) (&S.ps[0][0])[i] = pv[q];
    }
#pragma unroll
    for (int q = 0; q < CPER; ++q) {
      const int i = (int)threadIdx.x + q * BLOCK;
      if (i < NCW) (&S.cs[0][0])[i] = cv[q];
    }
  }
  __syncthreads();
  double sq = tile_round<0>(gd, S, x0, y0, last_x, last_y);
  sq += tile_round<1>(gd, S, x0, y0, last_x, last_y);
  sq += tile_round<2>(gd, S, x0, y0, last_x, last_y);
  sq += tile_round<3>(gd, S, x0, y0, last_x, last_y);
  {
    const int cx = RT_X + (last_x ? 1 : 0), cy = RT_Y + (last_y ? 1 : 0);
    for (int i = threadIdx.x; i < cx * cy; i += BLOCK) {
      const int ix = i % cx, iy = i / cx;
      sq += res_pres_lds(gd, S, x0, y0, x0 + ix, y0 + iy);
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
    partials[lt] = s2;
  }
}

// ---- 3D residual staged through LDS ------------------------------------------
// Large 3D levels: one block per tile of Q_X x Q_Y x Q_Z cells.  Pressures and
// cell coefficients of the tile (with halo) are staged once, the velocity
// window one component at a time (the viscous block acts on each component
// separately, so a component-c velocity row needs only x_c and the
// pressures); pressure rows accumulate their divergence over the three
// component stages in registers.  Masked and outside columns are staged as
// zeros, so no row tests its columns.  Rows of nodes whose cells all exist and
// share one coefficient use the assembled reference stencil times that
// coefficient; other rows (free boundary sides, viscosity jumps, cut cells)
// sum cell by cell.
constexpr int Q_X = 8, Q_Y = 8, Q_Z = 4;
constexpr int QW_X = 2 * Q_X + 5, QW_Y = 2 * Q_Y + 5, QW_Z = 2 * Q_Z + 5;   // node a = 2 x0 - 2 + l
constexpr int QP_X = Q_X + 3, QP_Y = Q_Y + 3, QP_Z = Q_Z + 3;             // vertex k = x0 - 1 + index
constexpr int QC_X = Q_X + 2, QC_Y = Q_Y + 2, QC_Z = Q_Z + 2;             // cell E = x0 - 1 + index
// Velocity window layout: per dimension the even positions l first, then the
// odd ones, so the nodes of one parity type (one round) sit at consecutive
// addresses; rows are padded to 24 doubles (8 times an odd number), which
// spreads the 8 x 8 nodes of a wave over all banks.
constexpr int QE_X = (QW_X + 1) / 2, QE_Y = (QW_Y + 1) / 2, QE_Z = (QW_Z + 1) / 2;
constexpr int QR = 24, QPL = QW_Y * QR;

__device__ __forceinline__ int qidx(int lz, int ly, int lx) {
  return qperm(lz, QE_Z) * QPL + qperm(ly, QE_Y) * QR + qperm(lx, QE_X);
}

// With all cells around a node present and one coefficient, the assembled
// viscous row is sum_c (K in dimension c) x (M in the others), K and M the 1D
// stiffness and mass rows summed over the node's cells in each dimension
// (node of parity t, column offset o, |o| <= 2; odd nodes reach |o| <= 1).
__host__ __device__ constexpr double st1(bool stiff, int t, int o) {
  return t ? ((o >= -1 && o <= 1) ? (stiff ? k1(1, 1 + o) : m1(1, 1 + o)) : 0.0)
           : ((o <= 0 ? (stiff ? k1(2, 2 + o) : m1(2, 2 + o)) : 0.0) + (o >= 0 ? (stiff ? k1(0, o) : m1(0, o)) : 0.0));
}
// The divergence block factorizes over dimensions: summed over the cells around
// a node, an entry is -prod_d F_d, with F_d the 1D factor G (d = component) or
// H (other dimensions) summed over the node's cells in that dimension.
// Velocity node of parity t, pressure vertex lo + j (even: j < 3, odd: j < 2):
__host__ __device__ constexpr double ga1(int t, int j) {
  return t ? (j < 2 ? g1(j, 1) : 0.0) : (j == 0 ? g1(0, 2) : j == 1 ? g1(1, 2) + g1(0, 0) : g1(1, 0));
}
__host__ __device__ constexpr double ha1(int t, int j) {
  return t ? (j < 2 ? h1(j, 1) : 0.0) : (j == 0 ? h1(0, 2) : j == 1 ? h1(1, 2) + h1(0, 0) : h1(1, 0));
}
// Pressure vertex k, velocity node 2k + o (|o| <= 2):
__host__ __device__ constexpr double gv1(int o) { return (o <= 0 ? g1(1, o + 2) : 0.0) + (o >= 0 ? g1(0, o) : 0.0); }
__host__ __device__ constexpr double hv1(int o) { return (o <= 0 ? h1(1, o + 2) : 0.0) + (o >= 0 ? h1(0, o) : 0.0); }

// z factors of the column pass, per window plane p (rolled loop, scalar loads):
// K_z and M_z of node j (z = 2 z0 + j) at offset p - j - 2, and the divergence
// z factor of component c for vertex m (z0 + m) at offset p - 2 m - 2; zero
// outside a node's or vertex's reach.
struct ZCoef {
  double km[2 * Q_Z + 4][2 * Q_Z][2];
  double pz[3][2 * Q_Z + 4][Q_Z];
  constexpr ZCoef() : km(), pz() {
    for (int p = 0; p < 2 * Q_Z + 4; ++p) {
      for (int j = 0; j < 2 * Q_Z; ++j) {
        const int dz = p - j - 2;
        const bool in = dz >= -2 && dz <= 2;
        km[p][j][0] = in ? st1(true, j & 1, dz) : 0.0;
        km[p][j][1] = in ? st1(false, j & 1, dz) : 0.0;
      }
      for (int m = 0; m < Q_Z; ++m) {
        const int dz = p - 2 * m - 2;
        const bool in = dz >= -2 && dz <= 2;
        for (int c = 0; c < 3; ++c) pz[c][p][m] = in ? (c == 2 ? gv1(dz) : hv1(dz)) : 0.0;
      }
    }
  }
};
__constant__ const ZCoef c_zcoef = ZCoef();

struct Tile3Lds {
  double xs[QW_Z * QPL];
  double ps[QP_Z][QP_Y][QP_X];
  double cs[QC_Z][QC_Y][QC_X];
  double pl[Q_Z][Q_Y][Q_X];   // divergence rows of interior vertices, summed over the components
};

struct Tile3 {
  int x0[3];
  bool last[3];
};

// (z, y, x) position of element i of an NZ x NY x NX box, advanced by BLOCK
// elements per step without divisions.
template <int NZ, int NY, int NX>
struct BoxWalk {
  int z, y, x;
  __device__ explicit BoxWalk(int i) : z(i / (NY * NX)), y((i / NX) % NY), x(i % NX) {}
  __device__ void step() {
    constexpr int dz = BLOCK / (NY * NX), dy = (BLOCK / NX) % NY, dx = BLOCK % NX;
    x += dx;
    const int cx = x >= NX ? 1 : 0;
    x -= cx * NX;
    y += dy + cx;
    const int cy = y >= NY ? 1 : 0;
    y -= cy * NY;
    z += dz + cy;
  }
};
static_assert(12 * QW_X <= BLOCK && 24 >= QW_Y, "two window rows per thread");

// Staging of one velocity component's window: thread t < 12 QW_X owns window
// column xx = t mod QW_X of rows y0 = t / QW_X and y0 + 12 and loads them in
// every plane (all loads issued before any is used; positions off the grid
// read a clamped in-range address).
struct XRows {
  unsigned gxy[2];   // x + nn y of the two rows (clamped)
  int lxy[2];        // their window positions (permuted order)
  bool fxy[2];       // x and y free and inside
  bool ok[2];        // row exists
};

__device__ __forceinline__ XRows tile3_rows(const Geo& g, const Tile3& tl) {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));   // recomputed per component rather than held across the rows
  const int twoN = 2 * g.N;
  const int xx = t % QW_X, y0 = t / QW_X;
  const int ax = 2 * tl.x0[0] - 2 + xx;
  const unsigned gx = (unsigned)min(max(ax, 0), twoN);
  const bool fx = free_coord(g, 0, ax);
  XRows R;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int yy = y0 + 12 * r, ay = 2 * tl.x0[1] - 2 + yy;
    R.ok[r] = t < 12 * QW_X && yy < QW_Y;
    R.gxy[r] = gx + (unsigned)g.nn * (unsigned)min(max(ay, 0), twoN);
    R.lxy[r] = qperm(min(yy, QW_Y - 1), QE_Y) * QR + qperm(xx, QE_X);
    R.fxy[r] = fx & free_coord(g, 1, ay);
  }
  return R;
}

__device__ __forceinline__ void tile3_load_x(const GridDev& gd, const Tile3& tl, int c, const XRows& R,
                                             double (*v)[QW_Z]) {
  const Geo& g = gd.g;
  const unsigned nn2 = (unsigned)g.nn * (unsigned)g.nn;
  gcdouble* __restrict__ X = gview(gd.x) + (size_t)c * g.nV;
#pragma unroll
  for (int z = 0; z < QW_Z; ++z) {
    const unsigned zo = nn2 * (unsigned)min(max(2 * tl.x0[2] - 2 + z, 0), 2 * g.N);
#pragma unroll
    for (int r = 0; r < 2; ++r) v[r][z] = ld(X, (R.ok[r] ? R.gxy[r] : R.gxy[0]) + zo);
  }
}

// Masked and outside columns are stored as zeros: they drop out of every row.
__device__ __forceinline__ void tile3_store_x(const Geo& g, const Tile3& tl, const XRows& R, const double (*v)[QW_Z],
                                              double* xs) {
#pragma unroll
  for (int z = 0; z < QW_Z; ++z) {
    const bool fz = free_coord(g, 2, 2 * tl.x0[2] - 2 + z);
#pragma unroll
    for (int r = 0; r < 2; ++r)
      if (R.ok[r]) xs[qperm(z, QE_Z) * QPL + R.lxy[r]] = (R.fxy[r] & fz) ? v[r][z] : 0.0;
  }
}

// Velocity row (component c) of node a of parity type TY, cell by cell: the
// rows the column pass leaves (masked nodes, free sides with missing cells,
// viscosity jumps, cut cells with their stored matrices).  The staged window
// holds 0 at masked and outside columns, so no column is tested.
template <int TY>
__device__ __noinline__ double res3_vel_cells(const GridDev& gd, const Tile3Lds& S, const Tile3& tl, int c,
                                              int a0, int a1, int a2) {
  constexpr int NV = 27, NP = 8;
  constexpr int T0 = TY & 1, T1 = (TY >> 1) & 1, T2 = (TY >> 2) & 1;
  constexpr int NE0 = T0 ? 1 : 2, NE1 = T1 ? 1 : 2, NE2 = T2 ? 1 : 2;
  constexpr int NE = NE0 * NE1 * NE2;
  const int a[3] = {a0, a1, a2};
  const Geo& g = gd.g;
  const int N = g.N;
  const long long gi = c * g.nV + a[0] + g.nn * (a[1] + g.nn * (long long)a[2]);
  if (node_dirichlet(g, a)) {
    gview(gd.r)[gi] = 0.0;
    return 0.0;
  }
  const double bv = gview(gd.b)[gi];
  const Tabs<3>& T = tabs<3>();
  const int l[3] = {a[0] - (2 * tl.x0[0] - 2), a[1] - (2 * tl.x0[1] - 2), a[2] - (2 * tl.x0[2] - 2)};
  const int lo[3] = {(a[0] >> 1) - 1 + T0 - (tl.x0[0] - 1), (a[1] >> 1) - 1 + T1 - (tl.x0[1] - 1),
                     (a[2] >> 1) - 1 + T2 - (tl.x0[2] - 1)};
  double acc = 0.0, accB = 0.0;
#pragma unroll 1
  for (int i = 0; i < NE; ++i) {
    const int eo[3] = {i % NE0, (i / NE0) % NE1, i / (NE0 * NE1)};
    int E[3], la3[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      E[d] = ((TY >> d) & 1) ? (a[d] - 1) >> 1 : (a[d] >> 1) - 1 + eo[d];
      ok = ok && E[d] >= 0 && E[d] < N;
      la3[d] = ((TY >> d) & 1) ? 1 : 2 - 2 * eo[d];
    }
    if (!ok) continue;
    const double cei = S.cs[E[2] - (tl.x0[2] - 1)][E[1] - (tl.x0[1] - 1)][E[0] - (tl.x0[0] - 1)];
    int pz[3], py[3], px[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {   // permuted positions of the cell's nodes (window index l - la + q)
      pz[q] = qperm(l[2] - la3[2] + q, QE_Z) * QPL;
      py[q] = qperm(l[1] - la3[1] + q, QE_Y) * QR;
      px[q] = qperm(l[0] - la3[0] + q, QE_X);
    }
    const int la = la3[0] + 3 * la3[1] + 9 * la3[2];
    double sc = 0.0;
    if (cei > 0.0) {
#pragma unroll
      for (int lb = 0; lb < NV; ++lb) sc += T.A[la * NV + lb] * S.xs[pz[lb / 9] + py[(lb / 3) % 3] + px[lb % 3]];
      sc *= cei;
    } else {
      gcdouble* __restrict__ Ae = gview(gd.cutA) + ((long long)(-cei) - 1) * (NV * NV) + la * NV;
#pragma unroll
      for (int lb = 0; lb < NV; ++lb) sc += Ae[lb] * S.xs[pz[lb / 9] + py[(lb / 3) % 3] + px[lb % 3]];
    }
    acc += sc;
    const int p0[3] = {lo[0] + (T0 ? 0 : eo[0]), lo[1] + (T1 ? 0 : eo[1]), lo[2] + (T2 ? 0 : eo[2])};
#pragma unroll
    for (int lk = 0; lk < NP; ++lk)
      accB += T.B[(c * NV + la) * NP + lk] * S.ps[p0[2] + (lk >> 2)][p0[1] + ((lk >> 1) & 1)][p0[0] + (lk & 1)];
  }
  const double r = bv - (acc + gd.h * gd.h * accB);
  gview(gd.r)[gi] = r;
  return r * r;
}

// Component-c part of the divergence row of pressure vertex k (without h^2)
// for the vertices the column pass leaves (grid boundary, last-tile extras).
// The cells around a vertex that exist form a product set over dimensions, so
// the row keeps the factorized form, each 1D factor summed over the vertex's
// existing cells in that dimension.
__device__ __noinline__ double res3_pres_sep(const Tile3Lds& S, const Tile3& tl, int N, int c, int k0, int k1, int k2) {
  const int k[3] = {k0, k1, k2};
  double f[3][5];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const bool lo = k[d] >= 1, hi = k[d] <= N - 1;   // cells k - 1 and k
#pragma unroll
    for (int o = -2; o <= 2; ++o) {
      const double gl = o <= 0 ? g1(1, o + 2) : 0.0, gh = o >= 0 ? g1(0, o) : 0.0;
      const double hl = o <= 0 ? h1(1, o + 2) : 0.0, hh = o >= 0 ? h1(0, o) : 0.0;
      f[d][o + 2] = d == c ? (lo ? gl : 0.0) + (hi ? gh : 0.0) : (lo ? hl : 0.0) + (hi ? hh : 0.0);
    }
  }
  // window position 2 k + o: l = 2 k - (2 x0 - 2) is even, so o fixes the
  // parity half and the offsets from l / 2 are compile-time (qoff)
  const double* __restrict__ xb = S.xs + (k[2] - tl.x0[2] + 1) * QPL + (k[1] - tl.x0[1] + 1) * QR + (k[0] - tl.x0[0] + 1);
  double acc = 0.0;
#pragma unroll 1
  for (int oz = -2; oz <= 2; ++oz) {
    const double* __restrict__ xz = xb + qoff(0, oz, QE_Z) * QPL;
    double az = 0.0;
#pragma unroll
    for (int oy = -2; oy <= 2; ++oy) {
      double ay = 0.0;
#pragma unroll
      for (int ox = -2; ox <= 2; ++ox) ay += f[0][ox + 2] * xz[qoff(0, oy, QE_Y) * QR + qoff(0, ox, QE_X)];
      az += f[1][oy + 2] * ay;
    }
    acc += (oz == -2 ? f[2][0] : oz == -1 ? f[2][1] : oz == 0 ? f[2][2] : oz == 1 ? f[2][3] : f[2][4]) * az;
  }
  return -acc;
}

// Column pass of one wave: nodes of xy parity type TXY, one (x, y) column of
// the tile per lane, all 2 Q_Z nodes of the column in registers.  Window
// planes are read once and each feeds every node whose stencil reaches it
// (assembled stencil constants times the node's cell coefficient); the
// divergence entries use the factorized form plane by plane.  The wave of
// type 0 also accumulates the divergence rows of the interior pressure
// vertices of its columns (the same 5 x 5 plane values) into LDS.  Rows that
// are not uniform go to the cell-by-cell path.
template <int TXY>
__device__ __forceinline__ double tile3_columns(const GridDev& gd, Tile3Lds& S, const Tile3& tl, int c, int lane) {
  constexpr int TX = TXY & 1, TYY = TXY >> 1;
  constexpr int W0 = TX ? 1 : 2, W1 = TYY ? 1 : 2;
  constexpr int NX0 = TX ? 1 : 2, NY0 = TYY ? 1 : 2;
  constexpr int M0 = 3 - TX, M1 = 3 - TYY;
  constexpr int NZN = 2 * Q_Z;   // nodes per column (az = 2 z0 + j)
  const Geo& g = gd.g;
  const int N = g.N;
  const int ix = lane & 7, iy = lane >> 3;
  const int ax = 2 * (tl.x0[0] + ix) + TX, ay = 2 * (tl.x0[1] + iy) + TYY;
  const long long zst = g.nn * g.nn;
  const long long col = c * g.nV + ax + g.nn * ay + zst * (2 * tl.x0[2]);
  double bv[NZN];
#pragma unroll
  for (int j = 0; j < NZN; ++j) bv[j] = gview(gd.b)[col + zst * j];
  // per plane of cells: the coefficient shared by the column's cells (0 when
  // they differ, are cut or missing)
  double cz[QC_Z];
#pragma unroll
  for (int e = 0; e < QC_Z; ++e) {
    const double v0 = S.cs[e][iy + (TYY ? 1 : 0)][ix + (TX ? 1 : 0)];
    bool u = v0 > 0.0;
#pragma unroll
    for (int ey = 0; ey < NY0; ++ey)
#pragma unroll
      for (int ex = 0; ex < NX0; ++ex) u &= S.cs[e][iy + (TYY ? 1 : ey)][ix + (TX ? 1 : ex)] == v0;   // no short circuit
    cz[e] = u ? v0 : 0.0;
  }
  // divergence factors of this component
  double fx[3], fy[3], fz[2][3], px[5], py[5];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    fx[j] = c == 0 ? ga1(TX, j) : ha1(TX, j);
    fy[j] = c == 1 ? ga1(TYY, j) : ha1(TYY, j);
    fz[0][j] = c == 2 ? ga1(0, j) : ha1(0, j);
    fz[1][j] = c == 2 ? ga1(1, j) : ha1(1, j);
  }
#pragma unroll
  for (int o = 0; o < 5; ++o) {
    px[o] = c == 0 ? gv1(o - 2) : hv1(o - 2);
    py[o] = c == 1 ? gv1(o - 2) : hv1(o - 2);
  }
  // viscous part: window planes p = 0 .. 2 Q_Z + 3 (node j sits on plane j + 2).
  // Per plane, A1 = (M_y x M_x) v and A2 = (K_y x M_x + M_y x K_x) v; node j
  // then takes K_z(dz) A1 + M_z(dz) A2 (zero outside its reach).  The plane
  // loop stays rolled: one plane's values are live at a time.
  double acc[NZN], pq[Q_Z];
#pragma unroll
  for (int j = 0; j < NZN; ++j) acc[j] = 0.0;
#pragma unroll
  for (int m = 0; m < Q_Z; ++m) pq[m] = 0.0;
#pragma unroll 1
  for (int p = 0; p < NZN + 4; ++p) {
    const double* __restrict__ xp = S.xs + qperm(p, QE_Z) * QPL + (iy + 1) * QR + (ix + 1);
    double v[2 * W1 + 1][2 * W0 + 1];
#pragma unroll
    for (int oy = -W1; oy <= W1; ++oy)
#pragma unroll
      for (int ox = -W0; ox <= W0; ++ox) v[oy + W1][ox + W0] = xp[qoff(TYY, oy, QE_Y) * QR + qoff(TX, ox, QE_X)];
    double A1 = 0.0, A2 = 0.0;
#pragma unroll
    for (int oy = -W1; oy <= W1; ++oy) {
      double rm = 0.0, rk = 0.0;
#pragma unroll
      for (int ox = -W0; ox <= W0; ++ox) {
        rm += st1(false, TX, ox) * v[oy + W1][ox + W0];
        rk += st1(true, TX, ox) * v[oy + W1][ox + W0];
      }
      A1 += st1(false, TYY, oy) * rm;
      A2 += st1(true, TYY, oy) * rm + st1(false, TYY, oy) * rk;
    }
    const double(*__restrict__ km)[2] = c_zcoef.km[p];
#pragma unroll
    for (int j = 0; j < NZN; ++j) acc[j] += km[j][0] * A1 + km[j][1] * A2;
    if constexpr (TXY == 0) {
      double q = 0.0;
#pragma unroll
      for (int oy = 0; oy < 5; ++oy) {
        double rx = 0.0;
#pragma unroll
        for (int ox = 0; ox < 5; ++ox) rx += px[ox] * v[oy][ox];
        q += py[oy] * rx;
      }
      const double* __restrict__ zc = c_zcoef.pz[c][p];
#pragma unroll
      for (int m = 0; m < Q_Z; ++m) pq[m] += zc[m] * q;
    }
  }
  if constexpr (TXY == 0) {
    // the sums of vertices this pass does not own are not used (plain adds, no branches)
#pragma unroll
    for (int m = 0; m < Q_Z; ++m) S.pl[m][iy][ix] += pq[m];
  }
  // divergence part: pressure planes kp (vertex z0 - 1 + kp); node j uses lo .. lo + M2 - 1
  double accB[NZN];
#pragma unroll
  for (int j = 0; j < NZN; ++j) accB[j] = 0.0;
#pragma unroll
  for (int kp = 0; kp < Q_Z + 2; ++kp) {
    double P = 0.0;
#pragma unroll
    for (int jy = 0; jy < M1; ++jy) {
      double rr = 0.0;
#pragma unroll
      for (int jx = 0; jx < M0; ++jx) rr += fx[jx] * S.ps[kp][iy + TYY + jy][ix + TX + jx];
      P += fy[jy] * rr;
    }
#pragma unroll
    for (int j = 0; j < NZN; ++j) {
      const int jz = kp - ((j >> 1) + (j & 1)), M2 = (j & 1) ? 2 : 3;
      if (jz >= 0 && jz < M2) accB[j] += fz[j & 1][jz] * P;
    }
  }
  // rows
  const double h2 = gd.h * gd.h;
  const bool dxy = coord_dirichlet(g, 0, ax) || coord_dirichlet(g, 1, ay);
  gdouble* __restrict__ R = gview(gd.r);
  double sq = 0.0;
  unsigned slow = 0;
#pragma unroll
  for (int j = 0; j < NZN; ++j) {
    // branch-free: every row is stored here (rows of the cell-by-cell path are
    // overwritten below), so the column sums stay in registers and are not
    // sunk into per-node branches
    const bool dir = dxy || coord_dirichlet(g, 2, 2 * tl.x0[2] + j);
    const double ce = (j & 1) ? cz[(j + 1) >> 1] : cz[j >> 1];
    const bool fast = ce > 0.0 && ((j & 1) || cz[(j >> 1) + 1] == ce);
    double r = bv[j] - (ce * acc[j] - h2 * accB[j]);
    asm volatile("" : "+v"(r));   // evaluated here for every node (not moved under a branch on dir)
    r = dir ? 0.0 : r;
    R[col + zst * j] = r;
    sq += (!dir && fast) ? r * r : 0.0;
    slow |= (!dir && !fast) ? 1u << j : 0u;
  }
#pragma unroll 1
  for (int j = 0; j < NZN; ++j) {
    if (!((slow >> j) & 1u)) continue;
    if (j & 1) sq += res3_vel_cells<TXY | 4>(gd, S, tl, c, ax, ay, 2 * tl.x0[2] + j);
    else sq += res3_vel_cells<TXY>(gd, S, tl, c, ax, ay, 2 * tl.x0[2] + j);
  }
  return sq;
}

// Velocity nodes of a last tile outside its 2 Q_X x 2 Q_Y x 2 Q_Z core (on
// the upper grid sides): the slabs ix = Q_X, iy = Q_Y (ix < Q_X) and iz = Q_Z
// (ix < Q_X, iy < Q_Y) of the type's node box.
template <int TY>
__device__ __forceinline__ double tile3_extras(const GridDev& gd, const Tile3Lds& S, const Tile3& tl, int c) {
  const int ex = (tl.last[0] && !(TY & 1)) ? 1 : 0, ey = (tl.last[1] && !((TY >> 1) & 1)) ? 1 : 0,
            ez = (tl.last[2] && !((TY >> 2) & 1)) ? 1 : 0;
  const int cy = Q_Y + ey, cz = Q_Z + ez;
  const int n0 = ex * cy * cz, n1 = ey * Q_X * cz, n2 = ez * Q_X * Q_Y;
  const Geo& g = gd.g;
  double sq = 0.0;
  for (int i = threadIdx.x; i < n0 + n1 + n2; i += BLOCK) {
    int ix, iy, iz;
    if (i < n0) {
      ix = Q_X; iy = ey ? i % (Q_Y + 1) : i % Q_Y; iz = ey ? i / (Q_Y + 1) : i / Q_Y;
    } else if (i < n0 + n1) {
      const int t = i - n0;
      ix = t % Q_X; iy = Q_Y; iz = t / Q_X;
    } else {
      const int t = i - n0 - n1;
      ix = t % Q_X; iy = t / Q_X; iz = Q_Z;
    }
    const int a[3] = {2 * (tl.x0[0] + ix) + (TY & 1), 2 * (tl.x0[1] + iy) + ((TY >> 1) & 1),
                      2 * (tl.x0[2] + iz) + ((TY >> 2) & 1)};
    if (node_dirichlet(g, a)) gview(gd.r)[c * g.nV + a[0] + g.nn * (a[1] + g.nn * (long long)a[2])] = 0.0;
    else sq += res3_vel_cells<TY>(gd, S, tl, c, a[0], a[1], a[2]);
  }
  return sq;
}

// Upper-side nodes of a last tile when every upper side it touches is masked:
// all of them are Dirichlet rows, zero in every component (one pass).
__device__ __noinline__ void tile3_extras_zero(const GridDev& gd, const Tile3& tl) {
  const Geo& g = gd.g;
  const int twoN = 2 * g.N;
  const int ny = 2 * Q_Y + (tl.last[1] ? 1 : 0), nz = 2 * Q_Z + (tl.last[2] ? 1 : 0);
  const int n0 = tl.last[0] ? ny * nz : 0, n1 = tl.last[1] ? 2 * Q_X * nz : 0, n2 = tl.last[2] ? 4 * Q_X * Q_Y : 0;
  gdouble* __restrict__ R = gview(gd.r);
  for (int i = threadIdx.x; i < n0 + n1 + n2; i += BLOCK) {
    int ax, ay, az;
    if (i < n0) {
      ax = twoN; ay = 2 * tl.x0[1] + i % ny; az = 2 * tl.x0[2] + i / ny;
    } else if (i < n0 + n1) {
      const int t = i - n0;
      ax = 2 * tl.x0[0] + t % (2 * Q_X); ay = twoN; az = 2 * tl.x0[2] + t / (2 * Q_X);
    } else {
      const int t = i - n0 - n1;
      ax = 2 * tl.x0[0] + t % (2 * Q_X); ay = 2 * tl.x0[1] + t / (2 * Q_X); az = twoN;
    }
    const long long base = ax + g.nn * (ay + g.nn * (long long)az);
#pragma unroll
    for (int c = 0; c < 3; ++c) R[c * g.nV + base] = 0.0;
  }
}

// Two blocks per CU (LDS bound): at most 256 registers per lane.
__global__ __launch_bounds__(BLOCK, 2) void k_residual_tiled3(const GridDev* __restrict__ G, double* __restrict__ partials) {
  __shared__ Tile3Lds S;
  const GridDev& gd = *G;
  const Geo& g = gd.g;
  const int N = g.N;
  const int ntx = N / Q_X, nty = N / Q_Y, ntz = N / Q_Z, T = ntx * nty * ntz;
  const int b = blockIdx.x;
  const int lt = (b % 8) * (T / 8) + b / 8;
  const int tx = lt % ntx, ty = (lt / ntx) % nty, tz = lt / (ntx * nty);
  Tile3 tl;
  tl.x0[0] = tx * Q_X; tl.x0[1] = ty * Q_Y; tl.x0[2] = tz * Q_Z;
  tl.last[0] = tx == ntx - 1; tl.last[1] = ty == nty - 1; tl.last[2] = tz == ntz - 1;
  gcdouble* __restrict__ X = gview(gd.x);
  const unsigned nV = (unsigned)g.nV, np1 = (unsigned)g.np1;
  {
    constexpr int NPW = QP_Z * QP_Y * QP_X, NCW = QC_Z * QC_Y * QC_X;
    constexpr int PPER = (NPW + BLOCK - 1) / BLOCK, CPER = (NCW + BLOCK - 1) / BLOCK;
    double pv[PPER], cv[CPER];
    BoxWalk<QP_Z, QP_Y, QP_X> wp(threadIdx.x);
#pragma unroll
    for (int q = 0; q < PPER; ++q) {
      const unsigned gx = (unsigned)min(max(tl.x0[0] - 1 + wp.x, 0), N), gy = (unsigned)min(max(tl.x0[1] - 1 + wp.y, 0), N),
                     gz = (unsigned)min(max(tl.x0[2] - 1 + wp.z, 0), N);
      pv[q] = ld(X, 3u * nV + gx + np1 * (gy + np1 * gz));
      wp.step();
    }
    BoxWalk<QC_Z, QC_Y, QC_X> wc(threadIdx.x);
#pragma unroll
    for (int q = 0; q < CPER; ++q) {
      const unsigned gx = (unsigned)min(max(tl.x0[0] - 1 + wc.x, 0), N - 1),
                     gy = (unsigned)min(max(tl.x0[1] - 1 + wc.y, 0), N - 1),
                     gz = (unsigned)min(max(tl.x0[2] - 1 + wc.z, 0), N - 1);
      cv[q] = ld(gview(gd.ceta), gx + (unsigned)N * (gy + (unsigned)N * gz));
      wc.step();
    }
    static_assert(Q_X * Q_Y * Q_Z == BLOCK, "one pressure sum per thread");
    (&S.pl[0][0][0])[threadIdx.x] = 0.0;
    BoxWalk<QP_Z, QP_Y, QP_X> wp2(threadIdx.x);
#pragma unroll
    for (int q = 0; q < PPER; ++q) {
      if (q < PPER - 1 || threadIdx.x + q * BLOCK < NPW) {
        const int kx = tl.x0[0] - 1 + wp2.x, ky = tl.x0[1] - 1 + wp2.y, kz = tl.x0[2] - 1 + wp2.z;
        const bool in = kx >= 0 && kx <= N && ky >= 0 && ky <= N && kz >= 0 && kz <= N;
        S.ps[wp2.z][wp2.y][wp2.x] = in ? pv[q] : 0.0;
      }
      wp2.step();
    }
    BoxWalk<QC_Z, QC_Y, QC_X> wc2(threadIdx.x);
#pragma unroll
    for (int q = 0; q < CPER; ++q) {
      if (q < CPER - 1 || threadIdx.x + q * BLOCK < NCW) {
        const int ex = tl.x0[0] - 1 + wc2.x, ey = tl.x0[1] - 1 + wc2.y, ez = tl.x0[2] - 1 + wc2.z;
        const bool in = ex >= 0 && ex < N && ey >= 0 && ey < N && ez >= 0 && ez < N;
        S.cs[wc2.z][wc2.y][wc2.x] = in ? cv[q] : 0.0;
      }
      wc2.step();
    }
  }
  // pressure rows of this thread (at most two: 9 x 9 x 5 in a last tile); the
  // interior ones of the core come from the column passes, the others are
  // summed cell by cell here
  const int pcx = Q_X + (tl.last[0] ? 1 : 0), pcy = Q_Y + (tl.last[1] ? 1 : 0), pcz = Q_Z + (tl.last[2] ? 1 : 0);
  const int npr = pcx * pcy * pcz;
  double pacc[2] = {0.0, 0.0}, pb[2] = {0.0, 0.0};
  int pk[2][3];
  bool pcol[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int i = threadIdx.x + q * BLOCK;
    const int ix = i % pcx, iy = (i / pcx) % pcy, iz = i / (pcx * pcy);
    pk[q][0] = tl.x0[0] + ix; pk[q][1] = tl.x0[1] + iy; pk[q][2] = tl.x0[2] + iz;
    // core vertices take the column sums: interior ones, and those on a lower
    // grid side that is masked (the missing cell's terms multiply only
    // outside or masked window values, which are staged as zeros)
    pcol[q] = ix < Q_X && iy < Q_Y && iz < Q_Z && (pk[q][0] >= 1 || coord_dirichlet(g, 0, 0)) &&
              (pk[q][1] >= 1 || coord_dirichlet(g, 1, 0)) && (pk[q][2] >= 1 || coord_dirichlet(g, 2, 0));
    if (i < npr) pb[q] = gview(gd.b)[3 * g.nV + pk[q][0] + g.np1 * (pk[q][1] + g.np1 * (long long)pk[q][2])];
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double sq = 0.0;
#pragma unroll 1
  for (int c = 0; c < 3; ++c) {
    {
      const XRows R = tile3_rows(g, tl);
      double xv[2][QW_Z];
      tile3_load_x(gd, tl, c, R, xv);
      __syncthreads();   // previous component's window no longer read
      tile3_store_x(g, tl, R, xv, S.xs);
    }
    __syncthreads();
    switch ((wave + c) & 3) {   // xy parity types rotate over the waves from one component to the next
      case 0: sq += tile3_columns<0>(gd, S, tl, c, lane); break;
      case 1: sq += tile3_columns<1>(gd, S, tl, c, lane); break;
      case 2: sq += tile3_columns<2>(gd, S, tl, c, lane); break;
      default: sq += tile3_columns<3>(gd, S, tl, c, lane); break;
    }
    const bool upper_masked = (!tl.last[0] || coord_dirichlet(g, 0, 2 * N)) &&
                              (!tl.last[1] || coord_dirichlet(g, 1, 2 * N)) &&
                              (!tl.last[2] || coord_dirichlet(g, 2, 2 * N));
    if ((tl.last[0] || tl.last[1] || tl.last[2]) && upper_masked) {
      if (c == 0) tile3_extras_zero(gd, tl);
    } else if (tl.last[0] || tl.last[1] || tl.last[2]) {
      sq += tile3_extras<0>(gd, S, tl, c);
      sq += tile3_extras<1>(gd, S, tl, c);
      sq += tile3_extras<2>(gd, S, tl, c);
      sq += tile3_extras<3>(gd, S, tl, c);
      sq += tile3_extras<4>(gd, S, tl, c);
      sq += tile3_extras<5>(gd, S, tl, c);
      sq += tile3_extras<6>(gd, S, tl, c);
      sq += tile3_extras<7>(gd, S, tl, c);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
      if (threadIdx.x + q * BLOCK < npr && !pcol[q]) pacc[q] += res3_pres_sep(S, tl, N, c, pk[q][0], pk[q][1], pk[q][2]);
  }
  __syncthreads();   // column sums of the pressure rows complete
  const double h2 = gd.h * gd.h;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int i = threadIdx.x + q * BLOCK;
    if (i < npr) {
      const long long gi = 3 * g.nV + pk[q][0] + g.np1 * (pk[q][1] + g.np1 * (long long)pk[q][2]);
      const double r = pcol[q] ? pb[q] + h2 * S.pl[pk[q][2] - tl.x0[2]][pk[q][1] - tl.x0[1]][pk[q][0] - tl.x0[0]]
                               : pb[q] - h2 * pacc[q];
      gview(gd.r)[gi] = r;
      sq += r * r;
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
    partials[lt] = s2;
  }
}

// Tiles hold 1280 rows each: below 1024 tiles (N < 512) too few blocks run to
// hide the serial rounds, and the node-type kernel is faster.
// 3D: tiles of 8 x 8 x 4 cells, used from 1024 tiles (N >= 64) on.
bool residual_tiled_ok(int dim, int N) {
  if (dim == 2) return N >= 512 && N % RT_X == 0 && N % RT_Y == 0 && ((N / RT_X) * (N / RT_Y)) % 8 == 0;
  return N >= 64 && N % Q_X == 0 && N % Q_Y == 0 && N % Q_Z == 0 && ((N / Q_X) * (N / Q_Y) * (N / Q_Z)) % 8 == 0;
}
// ---- MV: one colour of patches (eq. 11 in the colour order, eq. 15) --------
// One 64-lane block per patch of the colour.  The residual on the patch rows
// is evaluated from the current x with the row formulas of the residual
// kernels (one lane per velocity node or pressure vertex of the patch, values
// kept in LDS), then y = omega L_i^{-1} r_i from the stored full inverse and x
// on the patch DoFs += y.  Patches of one colour share no residual rows and
// none of them reads x where another writes (colouring), so the colour's
// patches run concurrently and equal the sequential product in that order.
template <int DIM, int TY>
__device__ __forceinline__ void mv_node(const GridDev& gd, const int* a, double* out) {
  (void)res_node<DIM, TY, true>(gd, vel_seg_row(gd.g, TY, a), out);
}

template <int DIM>
__device__ __forceinline__ void mv_node_any(const GridDev& gd, const int* a, double* out) {
  const int t = node_type(gd.g, a);
  if constexpr (DIM == 2) {
    switch (t) {
      case 0: mv_node<2, 0>(gd, a, out); break;
      case 1: mv_node<2, 1>(gd, a, out); break;
      case 2: mv_node<2, 2>(gd, a, out); break;
      default: mv_node<2, 3>(gd, a, out); break;
    }
  } else {
    switch (t) {
      case 0: mv_node<3, 0>(gd, a, out); break;
      case 1: mv_node<3, 1>(gd, a, out); break;
      case 2: mv_node<3, 2>(gd, a, out); break;
      case 3: mv_node<3, 3>(gd, a, out); break;
      case 4: mv_node<3, 4>(gd, a, out); break;
      case 5: mv_node<3, 5>(gd, a, out); break;
      case 6: mv_node<3, 6>(gd, a, out); break;
      default: mv_node<3, 7>(gd, a, out); break;
    }
  }
}

template <int DIM, int KIND>
__global__ __launch_bounds__(64) void k_mv_colour(const GridDev* __restrict__ G, int colour, long long npc) {
  constexpr int NPAD = patch_npad(DIM, KIND);
  constexpr int NNODE = KIND == KIND_VERTEX ? ipow(5, DIM) : ipow(3, DIM);   // velocity nodes
  constexpr int NPV = KIND == KIND_VERTEX ? 1 : ipow(2, DIM);                // pressure vertices
  static_assert(NNODE + NPV <= 64, "one lane per patch node");
  __shared__ double rl[NPAD];
  const long long q = blockIdx.x;
  if (q >= npc) return;
  const GridDev& gd = *G;
  const Geo& g = gd.g;
  const int M = colour_modulus(KIND);
  const int ext = KIND == KIND_VERTEX ? g.N + 1 : g.N;
  int k[3] = {0, 0, 0};
  long long rem = q;
  int cc = colour;
  for (int d = 0; d < DIM; ++d) {
    const int cd = cc % M;
    cc /= M;
    const int cnt = (ext - cd + M - 1) / M;
    k[d] = cd + M * (int)(rem % cnt);
    rem /= cnt;
  }
  const long long p = patch_lin(g, KIND, k);
  const int lane = threadIdx.x;
  if (lane < NNODE) {
    int a[3] = {0, 0, 0}, m = lane;
    for (int d = 0; d < DIM; ++d) {
      a[d] = KIND == KIND_VERTEX ? 2 * k[d] + (m % 5) - 2 : 2 * k[d] + (m % 3);
      m /= KIND == KIND_VERTEX ? 5 : 3;
    }
    double out[DIM];
    if (node_inside(g, a)) {
      mv_node_any<DIM>(gd, a, out);   // 0 on masked nodes
    } else {
      for (int c = 0; c < DIM; ++c) out[c] = 0.0;
    }
    for (int c = 0; c < DIM; ++c) rl[c * NNODE + lane] = out[c];
  } else if (lane < NNODE + NPV) {
    const int j = lane - NNODE;
    int kk[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) kk[d] = KIND == KIND_VERTEX ? k[d] : k[d] + ((j >> d) & 1);
    double out = 0.0;
    (void)res_pres<DIM, true>(gd, vert_lin(g, kk), &out);
    rl[DIM * NNODE + j] = out;
  }
  __syncthreads();
  const double* __restrict__ Wi = gd.Winv + p * (long long)NPAD * NPAD;
  const double om = gd.omega_patch ? (double)gd.omega_patch[p] : gd.omega;
  for (int l = lane; l < NPAD; l += 64) {
    double y = 0.0;
#pragma unroll 4
    for (int c = 0; c < NPAD; ++c) y += Wi[c * NPAD + l] * rl[c];
    int comp, node[3];
    const long long gi = patch_local_dof(g, KIND, k, l, &comp, node);
    if (gi >= 0) gd.x[gi] += om * y;
  }
}

void launch_mv_colour(int dim, int kind, const GridDev* G, int colour, long long npc, hipStream_t s) {
  if (npc <= 0) return;
  if (dim == 2 && kind == KIND_VERTEX) hipLaunchKernelGGL((k_mv_colour<2, KIND_VERTEX>), dim3(npc), dim3(64), 0, s, G, colour, npc);
  else if (dim == 2) hipLaunchKernelGGL((k_mv_colour<2, KIND_ELEMENT>), dim3(npc), dim3(64), 0, s, G, colour, npc);
  else hipLaunchKernelGGL((k_mv_colour<3, KIND_ELEMENT>), dim3(npc), dim3(64), 0, s, G, colour, npc);
}

int residual_tiles(int dim, int N) {
  return dim == 2 ? (N / RT_X) * (N / RT_Y) : (N / Q_X) * (N / Q_Y) * (N / Q_Z);
}

void launch_residual_tiled(int dim, const GridDev* G, int N, double* partials, hipStream_t s) {
  if (dim == 2) hipLaunchKernelGGL(k_residual_tiled2, dim3(residual_tiles(2, N)), dim3(BLOCK), 0, s, G, partials);
  else hipLaunchKernelGGL(k_residual_tiled3, dim3(residual_tiles(3, N)), dim3(BLOCK), 0, s, G, partials);
}

void launch_residual(int dim, const GridDev* G, const BlockTask* tasks, int ntasks, double* partials,
                     hipStream_t s) {
  if (dim == 2) hipLaunchKernelGGL(k_residual2, dim3(ntasks), dim3(BLOCK), 0, s, G, tasks, partials);
  else hipLaunchKernelGGL(k_residual3, dim3(ntasks), dim3(BLOCK), 0, s, G, tasks, partials);
}

}  // namespace rav
