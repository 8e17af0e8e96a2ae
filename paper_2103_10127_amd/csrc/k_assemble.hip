// Level operator and right-hand side assembly (Sec. 2, eqs. 5-7).
//
// Every value of the ELL operator is computed by the thread that owns its
// row, as a gather over the (at most 2^d) cells that contain both the row
// node and the column node, so no two threads write the same address and no
// atomics are needed.  Cell matrices:
//   A_e[a][b] = h^(d-2) sum_q w_q eta_q grad phi_a(q) . grad phi_b(q)
//   B_e[c][a][k] = -h^(d-1) sum_q w_q psi_k(q) d_c phi_a(q)   (C = 0)
// with the viscosity taken per Gauss point (inclusions: closed disc/ball).
#include <hip/hip_runtime.h>

#include "rav_fields.h"
#include "rav_internal.h"

namespace rav {

__constant__ RefTables c_ref;

void set_ref_tables(const RefTables& t, hipStream_t s) {
  (void)hipStreamSynchronize(s);
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_ref), &t, sizeof(RefTables), 0, hipMemcpyHostToDevice);
}

// ---- viscosity at the Gauss points of every cell ---------------------------
// etaq[cell * nq + q]; uniform[cell] = 1 when all nq values are equal.

// R = 1: the cell's own 3^d Gauss points.  R > 1 (Galerkin coarse operator):
// the Gauss points of the R^d finest-grid cells inside the cell; the cell is
// uniform when they all see one viscosity, and then every entry of etaq is
// that value (non-uniform cells use their integrated cell matrix instead).
template <int DIM>
__global__ __launch_bounds__(256) void k_eta(const GridDev* G, const double* incl, int n_incl,
                                              double eta_out, double eta_in, int R, double* etaq,
                                              unsigned char* uniform) {
#pragma clang fp contract(off)
  constexpr int NQ = ipow(3, DIM);
  const Geo& g = G->g;
  long long ncell = (long long)g.N * g.N * (DIM == 3 ? g.N : 1);
  long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  int E[3] = {0, 0, 0};
  long long t = e;
  for (int d = 0; d < DIM; ++d) { E[d] = (int)(t % g.N); t /= g.N; }
  const double h = G->h;
  bool uni = true;
  double first = 0.0;
  if (R == 1) {
    for (int q = 0; q < NQ; ++q) {
      int qq = q;
      double x[3];
      for (int d = 0; d < DIM; ++d) { x[d] = ((double)E[d] + c_ref.gt[qq % 3]) * h; qq /= 3; }
      const double v = eta_at<DIM>(x, incl, n_incl, eta_out, eta_in);
      etaq[e * NQ + q] = v;
      if (q == 0) first = v;
      uni = uni && (v == first);
    }
  } else {
    const double hf = h / R;   // finest-grid cell size
    long long nsub = 1;
    for (int d = 0; d < DIM; ++d) nsub *= R;
    for (long long sidx = 0; sidx < nsub && uni; ++sidx) {
      long long ss = sidx;
      int S[3] = {0, 0, 0};
      for (int d = 0; d < DIM; ++d) { S[d] = (int)(ss % R); ss /= R; }
      for (int q = 0; q < NQ; ++q) {
        int qq = q;
        double x[3];
        for (int d = 0; d < DIM; ++d) {
          x[d] = ((double)E[d] * R + S[d] + c_ref.gt[qq % 3]) * hf;
          qq /= 3;
        }
        const double v = eta_at<DIM>(x, incl, n_incl, eta_out, eta_in);
        if (sidx == 0 && q == 0) first = v;
        uni = uni && (v == first);
      }
    }
    for (int q = 0; q < NQ; ++q) etaq[e * NQ + q] = first;
  }
  uniform[e] = uni ? 1 : 0;
}

// Viscous cell matrix entry by Gauss quadrature with the per-point viscosity (h = 1).
template <int DIM>
__device__ __forceinline__ double cell_stiffness_q(const double* etaq, long long cell, const int* la, const int* lb) {
  constexpr int NQ = ipow(3, DIM);
  double s = 0.0;
  for (int q = 0; q < NQ; ++q) {
    int qd[3], qq = q;
    for (int d = 0; d < DIM; ++d) { qd[d] = qq % 3; qq /= 3; }
    double w = 1.0, gg = 0.0;
    for (int d = 0; d < DIM; ++d) w *= c_ref.gw[qd[d]];
    for (int c = 0; c < DIM; ++c) {
      double p = 1.0;
      for (int d = 0; d < DIM; ++d)
        p *= (d == c) ? c_ref.dphi[la[d]][qd[d]] * c_ref.dphi[lb[d]][qd[d]]
                      : c_ref.phi[la[d]][qd[d]] * c_ref.phi[lb[d]][qd[d]];
      gg += p;
    }
    s += w * etaq[cell * NQ + q] * gg;
  }
  return s;
}

// h^(d-2) times the viscous cell matrix entry: the reference matrix times the
// cell's viscosity, or the stored matrix of a cut cell (h^(d-2) included).
template <int DIM>
__device__ __forceinline__ double cell_stiffness(const double* etaq, const unsigned char* uniform,
                                                 const int* cut_idx, const double* cutA, double hA,
                                                 long long cell, const int* la, const int* lb) {
  constexpr int NQ = ipow(3, DIM);
  constexpr int NV = ipow(3, DIM);
  int ia = 0, ib = 0, st = 1;
  for (int d = 0; d < DIM; ++d) { ia += la[d] * st; ib += lb[d] * st; st *= 3; }
  if (uniform[cell]) {
    double aref = DIM == 2 ? c_ref.aref2[ia][ib] : c_ref.aref3[ia][ib];
    return hA * (etaq[cell * NQ] * aref);
  }
  return cutA[((long long)cut_idx[cell] * NV + ia) * NV + ib];
}

template <int DIM>
__device__ __forceinline__ double bref(int c, const int* la, const int* lk) {
  int ia = 0, ik = 0, sa = 1, sk = 1;
  for (int d = 0; d < DIM; ++d) { ia += la[d] * sa; ik += lk[d] * sk; sa *= 3; sk *= 2; }
  return DIM == 2 ? c_ref.bref2[c][ia][ik] : c_ref.bref3[c][ia][ik];
}

__device__ __forceinline__ int ceil_half(int v) { return v >= 0 ? (v + 1) >> 1 : -((-v) >> 1); }

// Range of cells E_d containing both half-grid positions a and b (1D).
__device__ __forceinline__ void common_cells(int a, int b, int N, int& lo, int& hi) {
  lo = max(ceil_half(a - 2), ceil_half(b - 2));
  hi = min(a >> 1, b >> 1);
  lo = max(lo, 0);
  hi = min(hi, N - 1);
}

template <int DIM>
__global__ __launch_bounds__(256) void k_assemble(const GridDev* G, const BlockTask* tasks,
                                                   const double* etaq, const unsigned char* uniform,
                                                   const int* cut_idx, const double* cutA) {
  const BlockTask t = tasks[blockIdx.x];
  if (t.grid < 0) return;
  const GridDev& gd = G[t.grid];
  const Geo& g = gd.g;
  const int s = t.part;
  const long long rows = gd.seg_rows[s];
  const long long row = t.start + threadIdx.x;
  if (row >= rows) return;
  double* out = gd.vals + gd.seg_off[s] + row;
  const int nslot = seg_slots(DIM, s);
  const double h = gd.h;
  const double hA = DIM == 2 ? 1.0 : h;       // h^(d-2)
  const double hB = DIM == 2 ? h : h * h;     // h^(d-1)
  const int N = g.N;
  if (s == pressure_segment(DIM)) {
    int k[3] = {0, 0, 0};
    vert_of(g, row, k);
    for (int slot = 0; slot < nslot; ++slot) {
      int c = slot / ipow(5, DIM), r = slot % ipow(5, DIM);
      int b[3] = {0, 0, 0};
      for (int d = 0; d < DIM; ++d) { b[d] = 2 * k[d] + (r % 5) - 2; r /= 5; }
      double v = 0.0;
      if (node_inside(g, b) && !node_dirichlet(g, b)) {
        int lo[3], hi[3];
        for (int d = 0; d < DIM; ++d) {
          lo[d] = max(max(k[d] - 1, ceil_half(b[d] - 2)), 0);
          hi[d] = min(min(k[d], b[d] >> 1), N - 1);
        }
        for (int ez = (DIM == 3 ? lo[2] : 0); ez <= (DIM == 3 ? hi[2] : 0); ++ez)
          for (int ey = lo[1]; ey <= hi[1]; ++ey)
            for (int ex = lo[0]; ex <= hi[0]; ++ex) {
              int E[3] = {ex, ey, ez};
              int lb[3], lk[3];
              for (int d = 0; d < DIM; ++d) { lb[d] = b[d] - 2 * E[d]; lk[d] = k[d] - E[d]; }
              v += hB * bref<DIM>(c, lb, lk);
            }
      }
      out[(long long)slot * rows] = v;
    }
    return;
  }
  const int c = s >> DIM;
  const int ty = s & ((1 << DIM) - 1);
  int a[3] = {0, 0, 0};
  vel_row_node(g, ty, row, a);
  const bool row_masked = node_dirichlet(g, a);
  const int na = n_aslots(DIM, ty);
  for (int slot = 0; slot < nslot; ++slot) {
    double v = 0.0;
    if (!row_masked) {
      if (slot < na) {
        int b[3] = {0, 0, 0}, r = slot;
        for (int d = 0; d < DIM; ++d) {
          int w = a_halfwidth(ty, d);
          b[d] = a[d] + (r % (2 * w + 1)) - w;
          r /= 2 * w + 1;
        }
        if (node_inside(g, b) && !node_dirichlet(g, b)) {
          int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
          for (int d = 0; d < DIM; ++d) common_cells(a[d], b[d], N, lo[d], hi[d]);
          for (int ez = (DIM == 3 ? lo[2] : 0); ez <= (DIM == 3 ? hi[2] : 0); ++ez)
            for (int ey = lo[1]; ey <= hi[1]; ++ey)
              for (int ex = lo[0]; ex <= hi[0]; ++ex) {
                int E[3] = {ex, ey, ez};
                int la[3], lb[3];
                for (int d = 0; d < DIM; ++d) { la[d] = a[d] - 2 * E[d]; lb[d] = b[d] - 2 * E[d]; }
                long long cell = ex + (long long)N * (ey + (long long)N * ez);
                v += cell_stiffness<DIM>(etaq, uniform, cut_idx, cutA, hA, cell, la, lb);
              }
        }
      } else {
        int k[3] = {0, 0, 0}, r = slot - na;
        bool inside = true;
        for (int d = 0; d < DIM; ++d) {
          int px = (ty >> d) & 1, m = 3 - px, lo = (a[d] >> 1) - 1 + px;
          k[d] = lo + (r % m);
          r /= m;
          inside = inside && k[d] >= 0 && k[d] <= N;
        }
        if (inside) {
          int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
          for (int d = 0; d < DIM; ++d) {
            lo[d] = max(max(ceil_half(a[d] - 2), k[d] - 1), 0);
            hi[d] = min(min(a[d] >> 1, k[d]), N - 1);
          }
          for (int ez = (DIM == 3 ? lo[2] : 0); ez <= (DIM == 3 ? hi[2] : 0); ++ez)
            for (int ey = lo[1]; ey <= hi[1]; ++ey)
              for (int ex = lo[0]; ex <= hi[0]; ++ex) {
                int E[3] = {ex, ey, ez};
                int la[3], lk[3];
                for (int d = 0; d < DIM; ++d) { la[d] = a[d] - 2 * E[d]; lk[d] = k[d] - E[d]; }
                v += hB * bref<DIM>(c, la, lk);
              }
        }
      }
    }
    out[(long long)slot * rows] = v;
  }
}

// f at every Gauss point of every cell: fq[(cell * NQ + q) * DIM + c].
template <int DIM>
__global__ __launch_bounds__(256) void k_rhs_qp(const GridDev* G, const double* P, double* fq) {
  constexpr int NQ = ipow(3, DIM);
  const Geo& g = G->g;
  long long ncell = (long long)g.N * g.N * (DIM == 3 ? g.N : 1);
  long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  int E[3] = {0, 0, 0};
  long long t = e;
  for (int d = 0; d < DIM; ++d) { E[d] = (int)(t % g.N); t /= g.N; }
  for (int q = 0; q < NQ; ++q) {
    int qq = q;
    double x[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) { x[d] = ((double)E[d] + c_ref.gt[qq % 3]) * G->h; qq /= 3; }
    double f[3];
    forcing<DIM>(P, x, f);
    for (int c = 0; c < DIM; ++c) fq[(e * NQ + q) * DIM + c] = f[c];
  }
}

// b[row] = sum over cells containing the node of sum_q w_q h^d f_c(x_q) phi_a(q).
template <int DIM>
__global__ __launch_bounds__(256) void k_rhs_gather(const GridDev* G, const double* fq, double* b) {
  constexpr int NQ = ipow(3, DIM);
  const Geo& g = G->g;
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  if (i >= DIM * g.nV) { b[i] = 0.0; return; }
  long long nl_;
  const int c = split_vel(g, i, &nl_);
  int a[3] = {0, 0, 0};
  node_of(g, nl_, a);
  if (node_dirichlet(g, a)) { b[i] = 0.0; return; }
  double hd = 1.0;
  for (int d = 0; d < DIM; ++d) hd *= G->h;
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int d = 0; d < DIM; ++d) {
    lo[d] = max(ceil_half(a[d] - 2), 0);
    hi[d] = min(a[d] >> 1, g.N - 1);
  }
  double s = 0.0;
  for (int ez = (DIM == 3 ? lo[2] : 0); ez <= (DIM == 3 ? hi[2] : 0); ++ez)
    for (int ey = lo[1]; ey <= hi[1]; ++ey)
      for (int ex = lo[0]; ex <= hi[0]; ++ex) {
        int E[3] = {ex, ey, ez};
        long long cell = ex + (long long)g.N * (ey + (long long)g.N * ez);
        for (int q = 0; q < NQ; ++q) {
          int qq = q;
          double w = 1.0, phi = 1.0;
          for (int d = 0; d < DIM; ++d) {
            int qd = qq % 3;
            qq /= 3;
            w *= c_ref.gw[qd];
            phi *= c_ref.phi[a[d] - 2 * E[d]][qd];
          }
          s += w * hd * fq[(cell * NQ + q) * DIM + c] * phi;
        }
      }
  b[i] = s;
}

// Per-cell coefficients of the matrix-free residual: ceta[e] = h^(d-2) eta_e
// for cells with one viscosity, -(1 + i) for the i-th cut cell (cut_idx[e] = i).
template <int DIM>
__global__ __launch_bounds__(256) void k_cell_scale(const GridDev* G, long long ncell, const double* etaq,
                                                     const int* cut_idx, double* ceta) {
  constexpr int NQ = ipow(3, DIM);
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  const double hA = DIM == 2 ? 1.0 : G->h;
  const int ci = cut_idx[e];
  ceta[e] = ci < 0 ? hA * etaq[e * NQ] : -(1.0 + (double)ci);
}

// Full viscous cell matrices of the cut cells: cutA[(i * NV + a) * NV + b], one thread per entry.
template <int DIM>
__global__ __launch_bounds__(256) void k_cut_matrices(const GridDev* G, const double* etaq, const int* cut_cells,
                                                       int ncut, double* cutA) {
  constexpr int NV = ipow(3, DIM);
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)ncut * NV * NV) return;
  const int i = (int)(t / (NV * NV)), ab = (int)(t % (NV * NV));
  int la[3] = {0, 0, 0}, lb[3] = {0, 0, 0};
  for (int d = 0, a = ab / NV, b = ab % NV; d < DIM; ++d) { la[d] = a % 3; lb[d] = b % 3; a /= 3; b /= 3; }
  const double hA = DIM == 2 ? 1.0 : G->h;
  cutA[t] = hA * cell_stiffness_q<DIM>(etaq, cut_cells[i], la, lb);
}

// Galerkin form of a cut cell's viscous matrix on a coarse level: the integral
// over the cell by the Gauss rules of its R^d finest-grid sub-cells, with the
// coarse Q2 basis evaluated at those points (for nested spaces this is the
// cell's share of P^T L_fine P).  One thread per entry.
__device__ __forceinline__ void q2_at(double t, double* v, double* dv) {
  v[0] = (1 - t) * (1 - 2 * t); v[1] = 4 * t * (1 - t); v[2] = t * (2 * t - 1);
  dv[0] = 4 * t - 3; dv[1] = 4 - 8 * t; dv[2] = 4 * t - 1;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_cut_matrices_galerkin(const GridDev* G, const int* cut_cells, int ncut,
                                                                int R, const double* incl, int n_incl,
                                                                double eta_out, double eta_in, double* cutA) {
  constexpr int NV = ipow(3, DIM);
  constexpr int NQ = ipow(3, DIM);
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)ncut * NV * NV) return;
  const int i = (int)(t / (NV * NV)), ab = (int)(t % (NV * NV));
  int la[3] = {0, 0, 0}, lb[3] = {0, 0, 0};
  for (int d = 0, a = ab / NV, b = ab % NV; d < DIM; ++d) { la[d] = a % 3; lb[d] = b % 3; a /= 3; b /= 3; }
  const Geo& g = G->g;
  int E[3] = {0, 0, 0};
  long long ct = cut_cells[i];
  for (int d = 0; d < DIM; ++d) { E[d] = (int)(ct % g.N); ct /= g.N; }
  const double hf = G->h / R;
  long long nsub = 1;
  double wsub = 1.0;
  for (int d = 0; d < DIM; ++d) { nsub *= R; wsub /= R; }
  double s = 0.0;
  for (long long sidx = 0; sidx < nsub; ++sidx) {
    long long ss = sidx;
    int S[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) { S[d] = (int)(ss % R); ss /= R; }
    for (int q = 0; q < NQ; ++q) {
      int qq = q;
      double x[3], va[3], vb[3], da[3], db[3], w = wsub;
      for (int d = 0; d < DIM; ++d) {
        const int qd = qq % 3;
        qq /= 3;
        const double xi = ((double)S[d] + c_ref.gt[qd]) / R;   // position in the coarse cell
        x[d] = ((double)E[d] * R + S[d] + c_ref.gt[qd]) * hf;
        w *= c_ref.gw[qd];
        double v3[3], d3[3];
        q2_at(xi, v3, d3);
        va[d] = v3[la[d]]; da[d] = d3[la[d]];
        vb[d] = v3[lb[d]]; db[d] = d3[lb[d]];
      }
      double gg = 0.0;
      for (int c = 0; c < DIM; ++c) {
        double p = 1.0;
        for (int d = 0; d < DIM; ++d) p *= d == c ? da[d] * db[d] : va[d] * vb[d];
        gg += p;
      }
      s += w * eta_at<DIM>(x, incl, n_incl, eta_out, eta_in) * gg;
    }
  }
  const double hA = DIM == 2 ? 1.0 : G->h;
  cutA[t] = hA * s;
}

// Driven-cavity lifting (2D): the right-hand side -L[free, masked] u_D for
// the Dirichlet data u_D = (U, 0) on the top side's nodes strictly between the
// corners.  Only the top row of cells couples to the lid: threads take the
// x-velocity rows on the two node rows below the lid and the pressure rows on
// the two vertex rows at the top; the viscous entries come from the level's
// per-cell coefficients (reference matrix times h^(d-2) eta, or the stored cut
// cell matrix), the divergence entries from the reference integrals.
__global__ __launch_bounds__(256) void k_lift_lid(const GridDev* G, double U, double* b) {
  const Geo& g = G->g;
  const int N = g.N;
  const long long nvel = 2LL * (2 * N + 1), npres = 2LL * (N + 1);
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= nvel + npres) return;
  const double hB = G->h;
  double s = 0.0;
  const int E1 = N - 1;   // the top row of cells
  if (t < nvel) {
    int a[3] = {(int)(t % (2 * N + 1)), 2 * N - 2 + (int)(t / (2 * N + 1)), 0};
    if (node_dirichlet(g, a)) return;
    for (int ex = max(ceil_half(a[0] - 2), 0); ex <= min(a[0] >> 1, N - 1); ++ex) {
      const long long cell = ex + (long long)N * E1;
      const int la[2] = {a[0] - 2 * ex, a[1] - 2 * E1};
      const double ce = G->ceta[cell];
      for (int bx = 0; bx < 3; ++bx) {
        const int nbx = 2 * ex + bx;
        if (nbx <= 0 || nbx >= 2 * N) continue;   // lid nodes only (corners are walls)
        const int ia = la[0] + 3 * la[1], ib = bx + 3 * 2;
        const double v = ce >= 0.0 ? ce * c_ref.aref2[ia][ib] : G->cutA[((long long)(-ce - 1.0) * 9 + ia) * 9 + ib];
        s += v * U;
      }
    }
    b[node_lin(g, a)] = -s;   // x-velocity row (component 0)
    return;
  }
  const long long tp = t - nvel;
  int k[3] = {(int)(tp % (N + 1)), N - 1 + (int)(tp / (N + 1)), 0};
  for (int ex = max(k[0] - 1, 0); ex <= min(k[0], N - 1); ++ex) {
    const int lk[2] = {k[0] - ex, k[1] - E1};
    for (int bx = 0; bx < 3; ++bx) {
      const int nbx = 2 * ex + bx;
      if (nbx <= 0 || nbx >= 2 * N) continue;
      const int lb[2] = {bx, 2};
      s += hB * bref<2>(0, lb, lk) * U;
    }
  }
  b[2 * g.nV + vert_lin(g, k)] = -s;
}

static inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_lift_lid(const GridDev* G, const Geo& g, double U, double* b, hipStream_t s) {
  const long long nt = 2LL * (2 * g.N + 1) + 2LL * (g.N + 1);
  hipLaunchKernelGGL(k_lift_lid, dim3(nblk(nt, 256)), dim3(256), 0, s, G, U, b);
}

void launch_eta(int dim, long long ncell, const GridDev* G, const double* incl, int n_incl, double eta_out,
                double eta_in, int R, double* etaq, unsigned char* uni, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(k_eta<2>, dim3(nblk(ncell, 256)), dim3(256), 0, s, G, incl, n_incl, eta_out, eta_in, R, etaq,
                       uni);
  else
    hipLaunchKernelGGL(k_eta<3>, dim3(nblk(ncell, 256)), dim3(256), 0, s, G, incl, n_incl, eta_out, eta_in, R, etaq,
                       uni);
}

void launch_cell_coef(int dim, long long ncell, const GridDev* G, const double* etaq, const int* cut_idx,
                      const int* cut_cells, int ncut, int R, const double* incl, int n_incl, double eta_out,
                      double eta_in, double* ceta, double* cutA, hipStream_t s) {
  const long long nv2 = dim == 2 ? 81 : 729;
  if (dim == 2) {
    hipLaunchKernelGGL(k_cell_scale<2>, dim3(nblk(ncell, 256)), dim3(256), 0, s, G, ncell, etaq, cut_idx, ceta);
    if (ncut > 0 && R == 1)
      hipLaunchKernelGGL(k_cut_matrices<2>, dim3(nblk(ncut * nv2, 256)), dim3(256), 0, s, G, etaq, cut_cells, ncut,
                         cutA);
    else if (ncut > 0)
      hipLaunchKernelGGL(k_cut_matrices_galerkin<2>, dim3(nblk(ncut * nv2, 256)), dim3(256), 0, s, G, cut_cells, ncut,
                         R, incl, n_incl, eta_out, eta_in, cutA);
  } else {
    hipLaunchKernelGGL(k_cell_scale<3>, dim3(nblk(ncell, 256)), dim3(256), 0, s, G, ncell, etaq, cut_idx, ceta);
    if (ncut > 0 && R == 1)
      hipLaunchKernelGGL(k_cut_matrices<3>, dim3(nblk(ncut * nv2, 256)), dim3(256), 0, s, G, etaq, cut_cells, ncut,
                         cutA);
    else if (ncut > 0)
      hipLaunchKernelGGL(k_cut_matrices_galerkin<3>, dim3(nblk(ncut * nv2, 256)), dim3(256), 0, s, G, cut_cells, ncut,
                         R, incl, n_incl, eta_out, eta_in, cutA);
  }
}

void launch_assemble(int dim, const GridDev* G, const BlockTask* tasks, int ntasks, const double* etaq,
                     const unsigned char* uni, const int* cut_idx, const double* cutA, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(k_assemble<2>, dim3(ntasks), dim3(BLOCK), 0, s, G, tasks, etaq, uni, cut_idx, cutA);
  else
    hipLaunchKernelGGL(k_assemble<3>, dim3(ntasks), dim3(BLOCK), 0, s, G, tasks, etaq, uni, cut_idx, cutA);
}

void launch_rhs(int dim, const GridDev* Gh, const GridDev* Gd, const double* params, double* fq, double* b,
                hipStream_t s) {
  long long ncell = (long long)Gh->g.N * Gh->g.N * (dim == 3 ? Gh->g.N : 1);
  if (dim == 2) {
    hipLaunchKernelGGL(k_rhs_qp<2>, dim3(nblk(ncell, 256)), dim3(256), 0, s, Gd, params, fq);
    hipLaunchKernelGGL(k_rhs_gather<2>, dim3(nblk(Gh->g.n, 256)), dim3(256), 0, s, Gd, fq, b);
  } else {
    hipLaunchKernelGGL(k_rhs_qp<3>, dim3(nblk(ncell, 256)), dim3(256), 0, s, Gd, params, fq);
    hipLaunchKernelGGL(k_rhs_gather<3>, dim3(nblk(Gh->g.n, 256)), dim3(256), 0, s, Gd, fq, b);
  }
}

}  // namespace rav
