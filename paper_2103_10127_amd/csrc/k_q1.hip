// Kernels of the stabilized Q1-Q1 levels (Sec. 2, eqs. 5-8) and of their RAV
// smoother with the literal owned set (Sec. 3, eq. 13).  Layout, cell matrices
// and patch storage are described in rav_q1.h.
//
// Every kernel gathers: a thread owns the rows (or the patch, or the coarse
// vertex) it writes and reads what it needs from the cells around it, so no
// atomics are needed.  The unit-cell integrals are closed forms evaluated in
// fully unrolled loops, so they fold into constants.
#include <hip/hip_runtime.h>

#include "rav_fields.h"
#include "rav_q1.h"
#include "rav_q1_unit.h"

namespace rav {

namespace {

using namespace q1unit;

template <int DIM>
__device__ __forceinline__ void decode(const Q1Dev& q, long long v, int* c) {
  c[0] = (int)(v % q.np1);
  c[1] = (int)((v / q.np1) % q.np1);
  if (DIM == 3) c[2] = (int)(v / (q.np1 * q.np1));
}

template <int DIM>
__device__ __forceinline__ long long vlin(const Q1Dev& q, const int* c) {
  long long i = c[DIM - 1];
  for (int d = DIM - 2; d >= 0; --d) i = i * q.np1 + c[d];
  return i;
}

template <int DIM>
__device__ __forceinline__ long long clin(const Q1Dev& q, const int* e) {
  long long i = e[DIM - 1];
  for (int d = DIM - 2; d >= 0; --d) i = i * q.N + e[d];
  return i;
}

template <int DIM>
__device__ __forceinline__ bool inside(const Q1Dev& q, const int* c) {
  bool ok = true;
  for (int d = 0; d < DIM; ++d) ok = ok & (c[d] >= 0) & (c[d] <= q.N);
  return ok;
}

// Velocity of vertex c is on a Dirichlet side (bitwise, without short-circuit branches).
template <int DIM>
__device__ __forceinline__ bool vmasked(const Q1Dev& q, const int* c) {
  unsigned m = 0u;
  for (int d = 0; d < DIM; ++d) {
    m |= ((q.dmask >> (2 * d)) & 1u) & (unsigned)(c[d] == 0);
    m |= ((q.dmask >> (2 * d + 1)) & 1u) & (unsigned)(c[d] == q.N);
  }
  return m != 0u;
}

// A_e[a][b] of cell `cell`
template <int DIM>
__device__ __forceinline__ double acell(const Q1Dev& q, double ce, long long cut, int a, int b) {
  constexpr int NB = 1 << DIM;
  return cut >= 0 ? q.cutK[cut * NB * NB + a * NB + b] : ce * kunit<DIM>(a, b);
}

__device__ __forceinline__ long long cut_index(double ce) { return ce < 0.0 ? (long long)(-ce) - 1 : -1; }

__device__ __forceinline__ double gp(const Q1Dev& q, int i) { return i ? q.gp_hi : q.gp_lo; }

// Physical coordinate of a Gauss point of fine cell (R e + sc) on a grid of R N
// cells per side: ((R e + sc) + t) / (R N), the oracle's (cell + t) h.
__device__ __forceinline__ double gauss_x(const Q1Dev& q, int R, int e, int sc, double t) {
  const double hf = 1.0 / ((double)q.N * R);
  return ((double)(R * e + sc) + t) * hf;
}

// MV colour of vertex patch v: sum_d (v_d mod 4) 4^d; patches of colour c are
// numbered lexicographically over (v_d - c_d) / 4, and the colours follow each
// other in ascending order.  Patches whose count along a direction is
// cnt_d(c) = ceil((N + 1 - c_d) / 4).
__host__ __device__ inline long long mv_colour_count(int dim, int N, int colour) {
  long long n = 1;
  for (int d = 0; d < dim; ++d) {
    const int cd = colour % 4;
    colour /= 4;
    n *= (N + 1 - cd + 3) / 4;
  }
  return n;
}

template <int DIM>
__device__ __forceinline__ long long mv_position(const Q1Dev& q, const int* vc) {
  int colour = 0, mul = 1;
  for (int d = 0; d < DIM; ++d) { colour += (vc[d] % 4) * mul; mul *= 4; }
  long long off = 0;
  for (int c = 0; c < colour; ++c) off += mv_colour_count(DIM, q.N, c);
  long long qi = 0, st = 1;
  int cc = colour;
  for (int d = 0; d < DIM; ++d) {
    const int cd = cc % 4;
    cc /= 4;
    qi += ((vc[d] - cd) / 4) * st;
    st *= (q.N + 1 - cd + 3) / 4;
  }
  return off + qi;
}

// ---- cell viscosity ---------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(256) void k_q1_cell_eta(Q1Dev q, int R, const double* __restrict__ incl, int n_incl,
                                                      double eta_out, double eta_in, double* __restrict__ eta0,
                                                      unsigned char* __restrict__ uni) {
  long long ncell = q.N;
  for (int d = 1; d < DIM; ++d) ncell *= q.N;
  const long long cell = blockIdx.x * 256LL + threadIdx.x;
  if (cell >= ncell) return;
  int e[3] = {0, 0, 0};
  long long t = cell;
  for (int d = 0; d < DIM; ++d) { e[d] = (int)(t % q.N); t /= q.N; }
  long long nsub = R;
  for (int d = 1; d < DIM; ++d) nsub *= R;
  double first = 0.0;
  bool same = true;
  for (long long sidx = 0; sidx < nsub; ++sidx) {
    int sc[3] = {0, 0, 0};
    long long u = sidx;
    for (int d = 0; d < DIM; ++d) { sc[d] = (int)(u % R); u /= R; }
    for (int g = 0; g < (1 << DIM); ++g) {
      double x[3] = {0, 0, 0};
      for (int d = 0; d < DIM; ++d) x[d] = gauss_x(q, R, e[d], sc[d], gp(q, bit(g, d)));
      const double v = eta_at<DIM>(x, incl, n_incl, eta_out, eta_in);
      if (sidx == 0 && g == 0) first = v;
      same = same && v == first;
    }
  }
  eta0[cell] = first;
  uni[cell] = same ? 1 : 0;
}

// A_e of cut cells: sum over the R^d fine cells and their Gauss points of
// eta w grad phi_a . grad phi_b, with the coarse basis evaluated at fine points.
template <int DIM>
__global__ __launch_bounds__(256) void k_q1_cut_matrices(Q1Dev q, int R, const int* __restrict__ cells, int ncut,
                                                          const double* __restrict__ incl, int n_incl,
                                                          double eta_out, double eta_in, double* __restrict__ cutK) {
  constexpr int NB = 1 << DIM;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ncut) return;
  const long long cell = cells[i];
  int e[3] = {0, 0, 0};
  long long t = cell;
  for (int d = 0; d < DIM; ++d) { e[d] = (int)(t % q.N); t /= q.N; }
  double K[NB][NB];
  for (int a = 0; a < NB; ++a)
    for (int b = 0; b < NB; ++b) K[a][b] = 0.0;
  long long nsub = R;
  for (int d = 1; d < DIM; ++d) nsub *= R;
  double wsub = 1.0;   // Gauss weight (1/2)^d times the fine cell's share (1/R)^d of the unit cell
  for (int d = 0; d < DIM; ++d) wsub *= 0.5 / R;
  for (long long sidx = 0; sidx < nsub; ++sidx) {
    int sc[3] = {0, 0, 0};
    long long u = sidx;
    for (int d = 0; d < DIM; ++d) { sc[d] = (int)(u % R); u /= R; }
    for (int g = 0; g < NB; ++g) {
      double tl[3] = {0, 0, 0}, x[3] = {0, 0, 0};
      for (int d = 0; d < DIM; ++d) {
        tl[d] = (sc[d] + gp(q, bit(g, d))) / R;   // local coordinate in the cell
        x[d] = gauss_x(q, R, e[d], sc[d], gp(q, bit(g, d)));
      }
      const double eta = eta_at<DIM>(x, incl, n_incl, eta_out, eta_in);
      double grad[NB][3];
      for (int a = 0; a < NB; ++a)
        for (int c = 0; c < DIM; ++c) {
          double v = 1.0;
          for (int d = 0; d < DIM; ++d) {
            const double phi = bit(a, d) ? tl[d] : 1.0 - tl[d];
            const double dphi = bit(a, d) ? 1.0 : -1.0;
            v *= (d == c) ? dphi : phi;
          }
          grad[a][c] = v;
        }
      for (int a = 0; a < NB; ++a)
        for (int b = 0; b < NB; ++b) {
          double gg = 0.0;
          for (int c = 0; c < DIM; ++c) gg += grad[a][c] * grad[b][c];
          K[a][b] += wsub * eta * gg;
        }
    }
  }
  double scale = 1.0;   // h^(d-2)
  for (int d = 2; d < DIM; ++d) scale *= q.h;
  for (int a = 0; a < NB; ++a)
    for (int b = 0; b < NB; ++b) cutK[(long long)i * NB * NB + a * NB + b] = scale * K[a][b];
}

// ---- residual: one thread per vertex, all d+1 rows -------------------------
// 2D: the 3x3 neighbourhood of the vertex is loaded once (zeros outside the
// grid and for masked velocity), then the 4 cells around the vertex add their
// cell-matrix rows; a cell outside the grid carries weight 0.
// 3D: the cells are visited one after another and each reads its 2^d vertices
// (a 3^3 neighbourhood held in registers would take 108 doubles per thread).
template <int DIM>
__device__ __forceinline__ void q1_rows_cells(const Q1Dev& q, const double* __restrict__ x, const int* vc,
                                              double* au, double& ap) {
  constexpr int NB = 1 << DIM;
#pragma unroll
  for (int s = 0; s < NB; ++s) {   // cell whose local vertex s is v
    int e[3] = {0, 0, 0};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      e[d] = vc[d] - bit(s, d);
      ok = ok & (e[d] >= 0) & (e[d] < q.N);
    }
    if (!ok) continue;
    const double ce = q.ceta[clin<DIM>(q, e)];
    const long long cut = cut_index(ce);
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) {
      int w[3] = {0, 0, 0};
#pragma unroll
      for (int d = 0; d < DIM; ++d) w[d] = e[d] + bit(bb, d);
      const long long wi = vlin<DIM>(q, w);
      const bool wm = vmasked<DIM>(q, w);
      const double pw = x[DIM * q.nV + wi];
      ap += q.cC * kunit<DIM>(s, bb) * pw;
      const double kab = acell<DIM>(q, ce, cut, s, bb);
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        au[c] -= q.bscale * bunit<DIM>(c, s, bb) * pw;
        if (!wm) {
          const double uw = x[c * q.nV + wi];
          au[c] += kab * uw;
          ap -= q.bscale * bunit<DIM>(c, bb, s) * uw;
        }
      }
    }
  }
}

// A x on the d+1 rows of vertex vc (velocity rows before masking): 2D loads the
// 3x3 neighbourhood once, 3D visits the cells one after another.
template <int DIM>
__device__ __forceinline__ void q1_vertex_rows(const Q1Dev& q, const double* __restrict__ x, const int* vc,
                                               long long v, double* au, double& ap) {
  constexpr int NB = 1 << DIM;
  constexpr int NBLK = q1_nblk(DIM);
  ap = 0.0;
#pragma unroll
  for (int c = 0; c < DIM; ++c) au[c] = 0.0;
  if constexpr (DIM == 3) {
    q1_rows_cells<DIM>(q, x, vc, au, ap);
  } else {
    double u[DIM][NBLK], pv[NBLK];
#pragma unroll
    for (int m = 0; m < NBLK; ++m) {
      int w[3] = {0, 0, 0};
      int t = m;
#pragma unroll
      for (int d = 0; d < DIM; ++d) { w[d] = vc[d] + (t % 3) - 1; t /= 3; }
      const bool in = inside<DIM>(q, w);
      const bool fr = in & !vmasked<DIM>(q, w);
      const long long wi = in ? vlin<DIM>(q, w) : v;
      pv[m] = in ? x[DIM * q.nV + wi] : 0.0;
#pragma unroll
      for (int c = 0; c < DIM; ++c) u[c][m] = fr ? x[c * q.nV + wi] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < NB; ++s) {   // cell whose local vertex s is v
      int e[3] = {0, 0, 0};
      bool ok = true;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        e[d] = vc[d] - bit(s, d);
        ok = ok & (e[d] >= 0) & (e[d] < q.N);
      }
      const double ce = ok ? q.ceta[clin<DIM>(q, e)] : 0.0;
      const long long cut = cut_index(ce);
      const double wc = ok ? 1.0 : 0.0;
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) {
        int m = 0, st = 1;   // neighbourhood index of the cell's local vertex bb
#pragma unroll
        for (int d = 0; d < DIM; ++d) { m += (bit(bb, d) - bit(s, d) + 1) * st; st *= 3; }
        const double kab = acell<DIM>(q, ce, cut, s, bb);
        ap += wc * q.cC * kunit<DIM>(s, bb) * pv[m];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          au[c] += kab * u[c][m] - wc * q.bscale * bunit<DIM>(c, s, bb) * pv[m];
          ap -= wc * q.bscale * bunit<DIM>(c, bb, s) * u[c][m];
        }
      }
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_q1_residual(Q1Dev q, const double* __restrict__ x,
                                                      const double* __restrict__ b, double* __restrict__ r,
                                                      double* __restrict__ partials) {
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  double sq = 0.0;
  if (v < q.nV) {
    int vc[3] = {0, 0, 0};
    decode<DIM>(q, v, vc);
    double au[DIM], ap = 0.0;
    q1_vertex_rows<DIM>(q, x, vc, v, au, ap);
    const bool vm = vmasked<DIM>(q, vc);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const double rc = vm ? 0.0 : b[c * q.nV + v] - au[c];
      r[c * q.nV + v] = rc;
      sq += rc * rc;
    }
    const double rp = b[DIM * q.nV + v] - ap;
    r[DIM * q.nV + v] = rp;
    sq += rp * rp;
  }
  if (!partials) return;
  __shared__ double red[256];
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// ---- patch factorization: one 64-lane block per vertex patch ---------------
// K (3^d x 3^d, identity rows/columns for padding) is eliminated by
// Gauss-Jordan without pivoting (symmetric positive definite) with the d
// pressure columns b_c and the identity carried along (giving z_c = K^{-1} b_c
// and K^{-1}); then S = c_kk - sum_c b_c . z_c (negative: c_kk < 0 and K^{-1}
// is SPD).  mode: Q1_ROWS owned rows, Q1_FACTORED the factored form, Q1_FULL
// every row of L_i^{-1} (AV, MV), all value-major W[value * nV + patch].
template <int DIM>
__global__ __launch_bounds__(64) void k_q1_factor(Q1Dev q, int mode, double* __restrict__ W,
                                                   int* __restrict__ status) {
  constexpr int NB = 1 << DIM;
  constexpr int NBLK = q1_nblk(DIM);
  constexpr int CEN = (NBLK - 1) / 2;
  constexpr int NC = NBLK + DIM + NBLK;   // K | b_1..b_d | I
  constexpr int KI = NBLK + DIM;          // first column of K^{-1}
  constexpr int NPAD = q1_npad(DIM);
  __shared__ double M[NBLK][NC];
  __shared__ double bsave[DIM][NBLK];
  __shared__ double fac[NBLK];
  __shared__ double ckk;
  const long long k = blockIdx.x;
  const int lane = threadIdx.x;
  int vc[3] = {0, 0, 0};
  decode<DIM>(q, k, vc);
  auto blk = [&](int m, int* w) {
    int t = m;
    for (int d = 0; d < DIM; ++d) { w[d] = vc[d] + (t % 3) - 1; t /= 3; }
  };
  auto valid = [&](const int* w) { return inside<DIM>(q, w) & !vmasked<DIM>(q, w); };
  // K entries and the pressure columns
  for (int idx = lane; idx < NBLK * NC; idx += 64) {
    const int m1i = idx / NC, col = idx % NC;
    int w1[3] = {0, 0, 0};
    blk(m1i, w1);
    double val = 0.0;
    if (col >= KI) {
      val = (m1i == col - KI) ? 1.0 : 0.0;
    } else if (!valid(w1)) {
      val = (col == m1i) ? 1.0 : 0.0;
      if (col >= NBLK) bsave[col - NBLK][m1i] = 0.0;
    } else if (col < NBLK) {
      int w2[3] = {0, 0, 0};
      blk(col, w2);
      if (valid(w2)) {
        // cells e with w1, w2 in e + {0,1}^d
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int d = 0; d < DIM; ++d) {
          lo[d] = max(max(w1[d], w2[d]) - 1, 0);
          hi[d] = min(min(w1[d], w2[d]), q.N - 1);
        }
        for (int s = 0; s < NB; ++s) {
          int e[3] = {0, 0, 0};
          bool ok = true;
          for (int d = 0; d < DIM; ++d) { e[d] = lo[d] + bit(s, d); ok = ok && e[d] <= hi[d]; }
          if (!ok) continue;
          int a1 = 0, a2 = 0;
          for (int d = 0; d < DIM; ++d) { a1 |= (w1[d] - e[d]) << d; a2 |= (w2[d] - e[d]) << d; }
          const double ce = q.ceta[clin<DIM>(q, e)];
          val += acell<DIM>(q, ce, cut_index(ce), a1, a2);
        }
      }
    } else {
      const int c = col - NBLK;   // L[(c, w1), p_k]: cells containing w1 and the vertex k
      int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
      for (int d = 0; d < DIM; ++d) {
        lo[d] = max(max(w1[d], vc[d]) - 1, 0);
        hi[d] = min(min(w1[d], vc[d]), q.N - 1);
      }
      for (int s = 0; s < NB; ++s) {
        int e[3] = {0, 0, 0};
        bool ok = true;
        for (int d = 0; d < DIM; ++d) { e[d] = lo[d] + bit(s, d); ok = ok && e[d] <= hi[d]; }
        if (!ok) continue;
        int a1 = 0, ak = 0;
        for (int d = 0; d < DIM; ++d) { a1 |= (w1[d] - e[d]) << d; ak |= (vc[d] - e[d]) << d; }
        val -= q.bscale * bunit<DIM>(c, a1, ak);
      }
      bsave[c][m1i] = val;
    }
    M[m1i][col] = val;
  }
  if (lane == 0) {
    double c = 0.0;
    for (int s = 0; s < NB; ++s) {
      int e[3] = {0, 0, 0};
      bool ok = true;
      for (int d = 0; d < DIM; ++d) { e[d] = vc[d] - bit(s, d); ok = ok && e[d] >= 0 && e[d] < q.N; }
      if (ok) c += q.cC * kunit<DIM>(s, s);
    }
    ckk = c;
  }
  __syncthreads();
  bool bad = false;
  for (int p = 0; p < NBLK; ++p) {
    const double piv = M[p][p];
    if (!(piv > 0.0)) bad = true;
    const double inv = 1.0 / piv;
    __syncthreads();
    for (int j = lane; j < NC; j += 64) M[p][j] *= inv;
    for (int i = lane; i < NBLK; i += 64) fac[i] = M[i][p];
    __syncthreads();
    for (int idx = lane; idx < NBLK * NC; idx += 64) {
      const int i = idx / NC, j = idx % NC;
      if (i != p) M[i][j] -= fac[i] * M[p][j];
    }
    __syncthreads();
  }
  // S = c_kk - sum_c b_c . z_c, reduced over the wavefront
  double part = 0.0;
  for (int idx = lane; idx < DIM * NBLK; idx += 64) {
    const int c = idx / NBLK, m = idx % NBLK;
    part += bsave[c][m] * M[m][NBLK + c];
  }
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  const double S = ckk - part;
  const double sinv = 1.0 / S;
  if (!(S < 0.0) || !isfinite(sinv)) bad = true;
  if (bad && lane == 0) atomicMin(status, (int)k);
  const long long stride = q.nV;
  const long long kpos = mode == Q1_FULL_MV ? mv_position<DIM>(q, vc) : k;   // patch slot in W
  if (mode == Q1_FACTORED) {
    for (int idx = lane; idx < q1_nvals(DIM, Q1_FACTORED); idx += 64) {
      double v;
      if (idx < NBLK) v = M[idx][KI + CEN];
      else if (idx < NBLK + DIM * NBLK) { const int c = (idx - NBLK) / NBLK, m = (idx - NBLK) % NBLK; v = M[m][NBLK + c]; }
      else v = sinv;
      W[idx * stride + k] = v;
    }
  } else if (mode == Q1_ROWS) {
    // owned rows: velocity component c at the centre (rows 0..d-1), pressure (row d)
    for (int idx = lane; idx < q1_nvals(DIM, Q1_ROWS); idx += 64) {
      const int row = idx / NPAD, col = idx % NPAD;
      double v;
      if (row < DIM) {
        const double zc0 = M[CEN][NBLK + row];
        if (col < DIM * NBLK) {
          const int c2 = col / NBLK, m = col % NBLK;
          v = (c2 == row ? M[m][KI + CEN] : 0.0) + zc0 * sinv * M[m][NBLK + c2];
        } else {
          v = -zc0 * sinv;
        }
      } else {
        if (col < DIM * NBLK) {
          const int c2 = col / NBLK, m = col % NBLK;
          v = -sinv * M[m][NBLK + c2];
        } else {
          v = sinv;
        }
      }
      W[idx * stride + k] = v;
    }
  } else {
    // every row: (c, m) velocity rows then the pressure row, same columns
    for (int idx = lane; idx < q1_nvals(DIM, Q1_FULL); idx += 64) {
      const int row = idx / NPAD, col = idx % NPAD;
      const bool rv = row < DIM * NBLK, cv = col < DIM * NBLK;
      double v;
      if (rv && cv) {
        const int c1 = row / NBLK, m1 = row % NBLK, c2 = col / NBLK, m2 = col % NBLK;
        v = (c1 == c2 ? M[m1][KI + m2] : 0.0) + M[m1][NBLK + c1] * sinv * M[m2][NBLK + c2];
      } else if (rv) {
        v = -M[row % NBLK][NBLK + row / NBLK] * sinv;
      } else if (cv) {
        v = -sinv * M[col % NBLK][NBLK + col / NBLK];
      } else {
        v = sinv;
      }
      if (mode == Q1_FULL_MV) W[kpos * (long long)(NPAD * NPAD) + idx] = v;   // patch-major
      else W[idx * stride + k] = v;
    }
  }
}

// ---- RAV apply: one thread per vertex patch --------------------------------
// y = L_i^{-1} r_i on the owned rows, x_owned += omega y (eq. 13).
template <int DIM, bool FACT>
__global__ __launch_bounds__(256) void k_q1_apply(Q1Dev q, const double* __restrict__ W,
                                                   const double* __restrict__ r, double* __restrict__ x,
                                                   double omega) {
  constexpr int NBLK = q1_nblk(DIM);
  constexpr int CEN = (NBLK - 1) / 2;
  constexpr int NPAD = q1_npad(DIM);
  const long long k = blockIdx.x * 256LL + threadIdx.x;
  if (k >= q.nV) return;
  const long long st = q.nV;
  int vc[3] = {0, 0, 0};
  decode<DIM>(q, k, vc);
  const double rp = r[DIM * q.nV + k];
  double yu[DIM], yp = 0.0, t = 0.0;
#pragma unroll
  for (int c = 0; c < DIM; ++c) yu[c] = 0.0;
#pragma unroll
  for (int m = 0; m < NBLK; ++m) {
    int w[3] = {0, 0, 0};
    int tm = m;
#pragma unroll
    for (int d = 0; d < DIM; ++d) { w[d] = vc[d] + (tm % 3) - 1; tm /= 3; }
    const bool ok = inside<DIM>(q, w) & !vmasked<DIM>(q, w);
    const long long wi = ok ? vlin<DIM>(q, w) : 0;
    double rc[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) rc[c] = ok ? r[c * q.nV + wi] : 0.0;
    if (FACT) {
      const double kin = W[m * st + k];
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        yu[c] += kin * rc[c];
        t += W[(NBLK + c * NBLK + m) * st + k] * rc[c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
#pragma unroll
        for (int row = 0; row < DIM; ++row) yu[row] += W[(row * NPAD + c * NBLK + m) * st + k] * rc[c];
        yp += W[(DIM * NPAD + c * NBLK + m) * st + k] * rc[c];
      }
    }
  }
  if (FACT) {
    const double s = W[(NBLK + DIM * NBLK) * st + k];
    const double u = s * (t - rp);
    yp = -u;
#pragma unroll
    for (int c = 0; c < DIM; ++c) yu[c] += W[(NBLK + c * NBLK + CEN) * st + k] * u;
  } else {
#pragma unroll
    for (int row = 0; row < DIM; ++row) yu[row] += W[(row * NPAD + DIM * NBLK) * st + k] * rp;
    yp += W[(DIM * NPAD + DIM * NBLK) * st + k] * rp;
  }
  x[DIM * q.nV + k] += omega * yp;
  if (!vmasked<DIM>(q, vc)) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) x[c * q.nV + k] += omega * yu[c];
  }
}

// ---- AV (eq. 12): every row of the local inverse, corrections summed -------
// k_q1_av_apply: one thread per patch, Y[row * nV + k] = omega (L_i^{-1} r_i)[row];
// k_q1_av_gather: one thread per vertex w, adding the rows of the patches that
// hold its DoFs (velocity: the patches of the vertices within one of w, at
// block position w - k; pressure: its own patch), so no two threads write
// the same entry.
template <int DIM>
__global__ __launch_bounds__(256) void k_q1_av_apply(Q1Dev q, const double* __restrict__ W,
                                                      const double* __restrict__ r, double* __restrict__ Y,
                                                      double omega) {
  constexpr int NBLK = q1_nblk(DIM);
  constexpr int NPAD = q1_npad(DIM);
  const long long k = blockIdx.x * 256LL + threadIdx.x;
  if (k >= q.nV) return;
  const long long st = q.nV;
  int vc[3] = {0, 0, 0};
  decode<DIM>(q, k, vc);
  double rl[NPAD];
#pragma unroll
  for (int m = 0; m < NBLK; ++m) {
    int w[3] = {0, 0, 0};
    int t = m;
#pragma unroll
    for (int d = 0; d < DIM; ++d) { w[d] = vc[d] + (t % 3) - 1; t /= 3; }
    const bool ok = inside<DIM>(q, w) & !vmasked<DIM>(q, w);
    const long long wi = ok ? vlin<DIM>(q, w) : 0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) rl[c * NBLK + m] = ok ? r[c * q.nV + wi] : 0.0;
  }
  rl[DIM * NBLK] = r[DIM * q.nV + k];
#pragma unroll 1
  for (int row = 0; row < NPAD; ++row) {
    double y = 0.0;
#pragma unroll
    for (int col = 0; col < NPAD; ++col) y += W[(long long)(row * NPAD + col) * st + k] * rl[col];
    Y[(long long)row * st + k] = omega * y;
  }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_q1_av_gather(Q1Dev q, const double* __restrict__ Y, double* __restrict__ x) {
  constexpr int NBLK = q1_nblk(DIM);
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v >= q.nV) return;
  const long long st = q.nV;
  int vc[3] = {0, 0, 0};
  decode<DIM>(q, v, vc);
  x[DIM * q.nV + v] += Y[(long long)(DIM * NBLK) * st + v];
  if (vmasked<DIM>(q, vc)) return;
  double acc[DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) acc[c] = 0.0;
#pragma unroll
  for (int o = 0; o < NBLK; ++o) {   // patch k = v - (offset o), v at block position o of that patch
    int kk[3] = {0, 0, 0};
    int t = o;
#pragma unroll
    for (int d = 0; d < DIM; ++d) { kk[d] = vc[d] - ((t % 3) - 1); t /= 3; }
    if (!inside<DIM>(q, kk)) continue;
    const long long ki = vlin<DIM>(q, kk);
#pragma unroll
    for (int c = 0; c < DIM; ++c) acc[c] += Y[(long long)(c * NBLK + o) * st + ki];
  }
#pragma unroll
  for (int c = 0; c < DIM; ++c) x[c * q.nV + v] += acc[c];
}

// ---- MV (eqs. 11, 15): one colour of patches ----------------------------------
// Patch k of colour sum_d (k_d mod 4) 4^d: its residual rows are recomputed from
// the current x, then x on its DoFs += omega L_i^{-1} r_i.  A patch writes x
// within one vertex of k and reads x within two vertices, so same-colour
// patches (4 or more vertices apart in some direction) are independent.
constexpr int MV_LANES = 32;   // lanes per patch of the MV kernel
constexpr int MV_BLOCK = 64;   // two patches per block

// One 32-lane group per patch: lane m < 3^d evaluates the rows of block vertex
// m (the centre lane also the pressure row) into LDS, then lane r computes row
// r of L_i^{-1} r_i from the patch-major stored inverse and updates that DoF.
template <int DIM>
__global__ __launch_bounds__(MV_BLOCK) void k_q1_mv_colour(Q1Dev q, const double* __restrict__ W,
                                                            const double* __restrict__ b, double* __restrict__ x,
                                                            double omega, int colour, long long npc) {
  constexpr int NBLK = q1_nblk(DIM);
  constexpr int NPAD = q1_npad(DIM);
  constexpr int CEN = (NBLK - 1) / 2;
  static_assert(NBLK <= MV_LANES, "one lane per block vertex");
  __shared__ double rls[MV_BLOCK / MV_LANES][NPAD];
  const int grp = threadIdx.x / MV_LANES, lane = threadIdx.x % MV_LANES;
  const long long qi = blockIdx.x * (long long)(MV_BLOCK / MV_LANES) + grp;
  const bool active = qi < npc;
  double* rl = rls[grp];
  int vc[3] = {0, 0, 0};
  long long k = 0, pos = 0;
  if (active) {
    long long rem = qi;
    int cc = colour;
    for (int d = 0; d < DIM; ++d) {
      const int cd = cc % 4;
      cc /= 4;
      const int cnt = (q.N + 1 - cd + 3) / 4;
      vc[d] = cd + 4 * (int)(rem % cnt);
      rem /= cnt;
    }
    k = vlin<DIM>(q, vc);
    pos = qi;   // colour-major slot of this patch's inverse
    for (int c = 0; c < colour; ++c) pos += mv_colour_count(DIM, q.N, c);
  }
  auto block_vertex = [&](int m, int* w) {
    int t = m;
    for (int d = 0; d < DIM; ++d) { w[d] = vc[d] + (t % 3) - 1; t /= 3; }
    return inside<DIM>(q, w) & !vmasked<DIM>(q, w);
  };
  // residual rows of the patch from the current x (eq. 15)
  if (active && lane < NBLK) {
    int w[3] = {0, 0, 0};
    const bool ok = block_vertex(lane, w);
    if (ok || lane == CEN) {
      const long long wi = vlin<DIM>(q, w);
      double au[DIM], ap = 0.0;
      q1_vertex_rows<DIM>(q, x, w, wi, au, ap);
      for (int c = 0; c < DIM; ++c) rl[c * NBLK + lane] = ok ? b[c * q.nV + wi] - au[c] : 0.0;
      if (lane == CEN) rl[DIM * NBLK] = b[DIM * q.nV + k] - ap;
    } else {
      for (int c = 0; c < DIM; ++c) rl[c * NBLK + lane] = 0.0;
    }
  }
  __syncthreads();
  if (!active) return;
  // x on the patch DoFs += omega L_i^{-1} r_i, one row per lane
  const double* __restrict__ Wp = W + pos * (long long)(NPAD * NPAD);
  for (int row = lane; row < NPAD; row += MV_LANES) {
    double y = 0.0;
#pragma unroll
    for (int col = 0; col < NPAD; ++col) y += Wp[row * NPAD + col] * rl[col];
    if (row == DIM * NBLK) {
      x[DIM * q.nV + k] += omega * y;
    } else {
      int w[3] = {0, 0, 0};
      if (block_vertex(row % NBLK, w)) x[(row / NBLK) * q.nV + vlin<DIM>(q, w)] += omega * y;
    }
  }
}

// ---- transfers -------------------------------------------------------------
// b_c = P^T r_f on the coarse vertices (masked rows 0), x_c = 0 and, when rc
// is given, r_c = b_c (the residual of the zero iterate).
template <int DIM>
__global__ __launch_bounds__(256) void k_q1_restrict(Q1Dev f, Q1Dev c, const double* __restrict__ rf,
                                                      double* __restrict__ bc, double* __restrict__ xc,
                                                      double* __restrict__ rc) {
  const long long W = blockIdx.x * 256LL + threadIdx.x;
  if (W >= c.nV) return;
  int wc[3] = {0, 0, 0};
  decode<DIM>(c, W, wc);
  const bool cm = vmasked<DIM>(c, wc);
  double acc[DIM + 1];
#pragma unroll
  for (int fl = 0; fl <= DIM; ++fl) acc[fl] = 0.0;
  constexpr int NO = DIM == 2 ? 9 : 27;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    int V[3] = {0, 0, 0};
    int t = o;
    double wgt = 1.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int od = (t % 3) - 1;
      t /= 3;
      V[d] = 2 * wc[d] + od;
      if (od != 0) wgt *= 0.5;
    }
    if (!inside<DIM>(f, V)) continue;
    const long long vi = vlin<DIM>(f, V);
    const bool fm = vmasked<DIM>(f, V);
#pragma unroll
    for (int fl = 0; fl < DIM; ++fl)
      if (!fm) acc[fl] += wgt * rf[fl * f.nV + vi];
    acc[DIM] += wgt * rf[DIM * f.nV + vi];
  }
#pragma unroll
  for (int fl = 0; fl <= DIM; ++fl) {
    const double val = (fl < DIM && cm) ? 0.0 : acc[fl];
    bc[fl * c.nV + W] = val;
    xc[fl * c.nV + W] = 0.0;
    if (rc) rc[fl * c.nV + W] = val;
  }
}

// x_f += P x_c (masked fine rows and masked coarse columns skipped).
template <int DIM>
__global__ __launch_bounds__(256) void k_q1_prolong(Q1Dev f, Q1Dev c, const double* __restrict__ xc,
                                                     double* __restrict__ xf) {
  const long long V = blockIdx.x * 256LL + threadIdx.x;
  if (V >= f.nV) return;
  int vf[3] = {0, 0, 0};
  decode<DIM>(f, V, vf);
  const bool fm = vmasked<DIM>(f, vf);
  double acc[DIM + 1];
#pragma unroll
  for (int fl = 0; fl <= DIM; ++fl) acc[fl] = 0.0;
#pragma unroll
  for (int s = 0; s < (1 << DIM); ++s) {
    int W[3] = {0, 0, 0};
    bool ok = true;
    double wgt = 1.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      if (vf[d] & 1) {
        W[d] = (vf[d] >> 1) + bit(s, d);
        wgt *= 0.5;
      } else {
        W[d] = vf[d] >> 1;
        ok = ok && bit(s, d) == 0;
      }
    }
    if (!ok) continue;
    const long long wi = vlin<DIM>(c, W);
    const bool cm = vmasked<DIM>(c, W);
#pragma unroll
    for (int fl = 0; fl < DIM; ++fl)
      if (!cm) acc[fl] += wgt * xc[fl * c.nV + wi];
    acc[DIM] += wgt * xc[DIM * c.nV + wi];
  }
  if (!fm) {
#pragma unroll
    for (int fl = 0; fl < DIM; ++fl) xf[fl * f.nV + V] += acc[fl];
  }
  xf[DIM * f.nV + V] += acc[DIM];
}

// ---- dense coarse matrix ----------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(256) void k_q1_dense(Q1Dev q, double* __restrict__ M, long long nb, int bordered) {
  constexpr int NB = 1 << DIM;
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= nb * nb) return;
  const long long i = idx / nb, j = idx % nb;
  double val = 0.0;
  if (bordered && (i == q.n || j == q.n)) {
    const long long o = i == q.n ? j : i;
    val = (o < q.n && o >= DIM * q.nV) ? 1.0 : 0.0;
    M[idx] = val;
    return;
  }
  const int fi = (int)(i / q.nV), fj = (int)(j / q.nV);
  int vi[3] = {0, 0, 0}, vj[3] = {0, 0, 0};
  decode<DIM>(q, i % q.nV, vi);
  decode<DIM>(q, j % q.nV, vj);
  const bool mi = (fi < DIM) & vmasked<DIM>(q, vi);
  const bool mj = (fj < DIM) & vmasked<DIM>(q, vj);
  if (mi || mj) {
    M[idx] = (i == j) ? 1.0 : 0.0;
    return;
  }
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int d = 0; d < DIM; ++d) {
    lo[d] = max(max(vi[d], vj[d]) - 1, 0);
    hi[d] = min(min(vi[d], vj[d]), q.N - 1);
  }
  for (int s = 0; s < NB; ++s) {
    int e[3] = {0, 0, 0};
    bool ok = true;
    for (int d = 0; d < DIM; ++d) { e[d] = lo[d] + bit(s, d); ok = ok && e[d] <= hi[d]; }
    if (!ok) continue;
    int a = 0, b = 0;
    for (int d = 0; d < DIM; ++d) { a |= (vi[d] - e[d]) << d; b |= (vj[d] - e[d]) << d; }
    if (fi < DIM && fj < DIM) {
      if (fi == fj) {
        const double ce = q.ceta[clin<DIM>(q, e)];
        val += acell<DIM>(q, ce, cut_index(ce), a, b);
      }
    } else if (fi < DIM) {
      val -= q.bscale * bunit<DIM>(fi, a, b);
    } else if (fj < DIM) {
      val -= q.bscale * bunit<DIM>(fj, b, a);
    } else {
      val += q.cC * kunit<DIM>(a, b);
    }
  }
  M[idx] = val;
}

// ---- right-hand sides -------------------------------------------------------
// b = [(f, phi); 0], 2^d Gauss points per cell.
template <int DIM>
__global__ __launch_bounds__(256) void k_q1_rhs(Q1Dev q, const double* __restrict__ P, double* __restrict__ b) {
  constexpr int NB = 1 << DIM;
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v >= q.nV) return;
  int vc[3] = {0, 0, 0};
  decode<DIM>(q, v, vc);
  double acc[DIM];
  for (int c = 0; c < DIM; ++c) acc[c] = 0.0;
  double hd = 1.0, w = 1.0;
  for (int d = 0; d < DIM; ++d) { hd *= q.h; w *= 0.5; }
  for (int s = 0; s < NB; ++s) {
    int e[3] = {0, 0, 0};
    bool ok = true;
    for (int d = 0; d < DIM; ++d) { e[d] = vc[d] - bit(s, d); ok = ok && e[d] >= 0 && e[d] < q.N; }
    if (!ok) continue;
    for (int g = 0; g < NB; ++g) {
      double x[3] = {0, 0, 0}, phi = 1.0;
      for (int d = 0; d < DIM; ++d) {
        const double t = gp(q, bit(g, d));
        x[d] = (e[d] + t) * q.h;
        phi *= bit(s, d) ? t : 1.0 - t;
      }
      double f[3] = {0, 0, 0};
      forcing<DIM>(P, x, f);
      for (int c = 0; c < DIM; ++c) acc[c] += w * hd * phi * f[c];
    }
  }
  const bool vm = vmasked<DIM>(q, vc);
  for (int c = 0; c < DIM; ++c) b[c * q.nV + v] = vm ? 0.0 : acc[c];
  b[DIM * q.nV + v] = 0.0;
}

// b = -L_all[free, masked] u_D with u_D = (U, 0) on the top side's inner vertices (2D).
__global__ __launch_bounds__(256) void k_q1_lid(Q1Dev q, double U, double* __restrict__ b) {
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v >= q.nV) return;
  int vc[3] = {0, 0, 0};
  decode<2>(q, v, vc);
  double bu = 0.0, bp = 0.0;
  for (int s = 0; s < 4; ++s) {
    int e[3] = {vc[0] - bit(s, 0), vc[1] - bit(s, 1), 0};
    if (e[0] < 0 || e[0] >= q.N || e[1] != q.N - 1) continue;
    const double ce = q.ceta[clin<2>(q, e)];
    const long long cut = cut_index(ce);
    for (int bb = 2; bb < 4; ++bb) {   // local vertices on the cell's top side
      const int wx = e[0] + bit(bb, 0);
      if (wx <= 0 || wx >= q.N) continue;   // corners are walls
      bu -= U * acell<2>(q, ce, cut, s, bb);
      bp += U * q.bscale * bunit<2>(0, bb, s);
    }
  }
  const bool vm = vmasked<2>(q, vc);
  b[v] = vm ? 0.0 : bu;
  b[q.nV + v] = 0.0;
  b[2 * q.nV + v] = bp;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_q1_owner(Q1Dev q, int* __restrict__ owner) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= q.n) return;
  const long long v = i % q.nV;
  const int fl = (int)(i / q.nV);
  int vc[3] = {0, 0, 0};
  decode<DIM>(q, v, vc);
  const int mk = (int)(fl < DIM) & (int)vmasked<DIM>(q, vc);
  owner[i] = (int)v - mk * ((int)v + 1);   // -1 for masked velocity, else the vertex
}

inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

#define Q1_DISPATCH(dim, K, grid, blk, ...)                                           \
  do {                                                                                \
    if ((dim) == 2) hipLaunchKernelGGL(K<2>, dim3(grid), dim3(blk), 0, s, __VA_ARGS__); \
    else hipLaunchKernelGGL(K<3>, dim3(grid), dim3(blk), 0, s, __VA_ARGS__);            \
  } while (0)

void q1_launch_cell_eta(int dim, const Q1Dev& q, int R, const double* incl, int n_incl, double eta_out,
                        double eta_in, double* eta0, unsigned char* uni, hipStream_t s) {
  long long ncell = q.N;
  for (int d = 1; d < dim; ++d) ncell *= q.N;
  Q1_DISPATCH(dim, k_q1_cell_eta, nblk(ncell), 256, q, R, incl, n_incl, eta_out, eta_in, eta0, uni);
}

void q1_launch_cut_matrices(int dim, const Q1Dev& q, int R, const int* cells, int ncut, const double* incl,
                            int n_incl, double eta_out, double eta_in, double* cutK, hipStream_t s) {
  if (ncut <= 0) return;
  Q1_DISPATCH(dim, k_q1_cut_matrices, nblk(ncut), 256, q, R, cells, ncut, incl, n_incl, eta_out, eta_in, cutK);
}

int q1_residual_blocks(const Q1Dev& q) { return (int)nblk(q.nV); }

void q1_launch_residual(int dim, const Q1Dev& q, const double* x, const double* b, double* r, double* partials,
                        hipStream_t s) {
  Q1_DISPATCH(dim, k_q1_residual, nblk(q.nV), 256, q, x, b, r, partials);
}

void q1_launch_factor(int dim, const Q1Dev& q, int mode, double* W, int* status, hipStream_t s) {
  Q1_DISPATCH(dim, k_q1_factor, (unsigned)q.nV, 64, q, mode, W, status);
}

void q1_launch_av(int dim, const Q1Dev& q, const double* W, const double* r, double* Y, double* x, double omega,
                  hipStream_t s) {
  Q1_DISPATCH(dim, k_q1_av_apply, nblk(q.nV), 256, q, W, r, Y, omega);
  Q1_DISPATCH(dim, k_q1_av_gather, nblk(q.nV), 256, q, Y, x);
}

void q1_launch_mv_colour(int dim, const Q1Dev& q, const double* W, const double* b, double* x, double omega,
                         int colour, hipStream_t s) {
  const long long npc = mv_colour_count(dim, q.N, colour);
  if (npc <= 0) return;
  const long long per_block = MV_BLOCK / MV_LANES;
  const unsigned g = (unsigned)((npc + per_block - 1) / per_block);
  Q1_DISPATCH(dim, k_q1_mv_colour, g, MV_BLOCK, q, W, b, x, omega, colour, npc);
}

void q1_launch_apply(int dim, const Q1Dev& q, int mode, const double* W, const double* r, double* x,
                     double omega, hipStream_t s) {
  const bool factored = mode == Q1_FACTORED;
  const unsigned g = nblk(q.nV);
  if (dim == 2) {
    if (factored) hipLaunchKernelGGL((k_q1_apply<2, true>), dim3(g), dim3(256), 0, s, q, W, r, x, omega);
    else hipLaunchKernelGGL((k_q1_apply<2, false>), dim3(g), dim3(256), 0, s, q, W, r, x, omega);
  } else {
    if (factored) hipLaunchKernelGGL((k_q1_apply<3, true>), dim3(g), dim3(256), 0, s, q, W, r, x, omega);
    else hipLaunchKernelGGL((k_q1_apply<3, false>), dim3(g), dim3(256), 0, s, q, W, r, x, omega);
  }
}

void q1_launch_restrict(int dim, const Q1Dev& f, const Q1Dev& c, const double* rf, double* bc, double* xc,
                        double* rc, hipStream_t s) {
  Q1_DISPATCH(dim, k_q1_restrict, nblk(c.nV), 256, f, c, rf, bc, xc, rc);
}

void q1_launch_prolong(int dim, const Q1Dev& f, const Q1Dev& c, const double* xc, double* xf, hipStream_t s) {
  Q1_DISPATCH(dim, k_q1_prolong, nblk(f.nV), 256, f, c, xc, xf);
}

void q1_launch_dense(int dim, const Q1Dev& q, double* M, long long nb, int bordered, hipStream_t s) {
  Q1_DISPATCH(dim, k_q1_dense, nblk(nb * nb), 256, q, M, nb, bordered);
}

void q1_launch_rhs(int dim, const Q1Dev& q, const double* params, double* b, hipStream_t s) {
  Q1_DISPATCH(dim, k_q1_rhs, nblk(q.nV), 256, q, params, b);
}

void q1_launch_lid(const Q1Dev& q, double U, double* b, hipStream_t s) {
  hipLaunchKernelGGL(k_q1_lid, dim3(nblk(q.nV)), dim3(256), 0, s, q, U, b);
}

void q1_launch_owner(int dim, const Q1Dev& q, int* owner, hipStream_t s) {
  Q1_DISPATCH(dim, k_q1_owner, nblk(q.n), 256, q, owner);
}

}  // namespace rav
