// Stabilized equal-order Q1-Q1 levels (Sec. 2, eqs. 5-8) with vertex patches
// and the literal RAV owned set of Sec. 3 (eq. 13): the patch of vertex k owns
// the pressure at k and the velocity at k.
//
// Numbering: vertex v in [0, N]^d, lin(v) = sum_d v_d (N+1)^d (x fastest);
// the level vector is [u_1; ...; u_d; p], field f of vertex v at f*nV + lin(v).
// Velocity on a Dirichlet side is masked (x = 0, residual 0).
//
// Cell matrices on a cell of side h (local vertex a = sum_d a_d 2^d):
//   A_e[a][b] = h^(d-2) sum_g w_g eta_g grad phi_a . grad phi_b   (2-point Gauss)
//   B_e[c][a][k] = -h^(d-1) int d_c phi_a psi_k
//   C_e[a][b] = -beta diam_s^2 h^(d-2) int grad psi_a . grad psi_b, diam_s^2 = d hs^2
// where hs is the level's own h (rediscretised) or the finest h (Galerkin).
// The unit-cell integrals are products of the 1D Q1 mass [1/3 1/6; 1/6 1/3],
// stiffness [1 -1; -1 1] and derivative-mass (-1/2 for the left function,
// +1/2 for the right one) entries.
//
// Vertex patch of k: the 3^d vertex block k + o, o in [-1,1]^d (lexicographic,
// x fastest), all velocity components, then p_k: npad = d 3^d + 1 local DoFs
// (19 in 2D, 82 in 3D); block vertices outside the grid or masked are padding.
// Stored per patch, value-major W[q * npad_patches + k]:
//   factored: row m0 (block centre) of K^{-1} (3^d values), z_c = K^{-1} b_c
//             (d 3^d values), s = 1/S (1 value), where K is the scalar viscous
//             block of the patch, b_c its pressure column and S = c_kk - sum_c b_c.z_c;
//   rows:     the d+1 owned rows of L_i^{-1} over the npad local columns;
//   full:     all npad rows (AV, MV), row-major over the local DoFs.
#pragma once
#include <hip/hip_runtime.h>

namespace rav {

struct Q1Dev {
  int dim, N;
  long long np1, nV, n;
  unsigned dmask;
  double h;
  double bscale;        // h^(d-1)
  double cC;            // -beta d hs^2 h^(d-2)
  double gp_lo, gp_hi;  // 2-point Gauss abscissae on [0,1]: 1/2 -+ 1/(2 sqrt 3)
  const double* ceta;   // per cell: >= 0: A_e = ceta * unit stiffness; < 0: cut cell -(1 + i)
  const double* cutK;   // cut cell i: A_e as [i][a][b], 2^d x 2^d
};

constexpr int q1_nblk(int dim) { return dim == 2 ? 9 : 27; }
constexpr int q1_npad(int dim) { return dim * q1_nblk(dim) + 1; }
// Stored values per patch: owned rows (RAV), factored owned rows (RAV), or
// the full inverse (AV, MV).
// Q1_FULL_MV: the full inverse patch-major (NPAD^2 contiguous values per
// patch), patches in MV colour-major order.
enum { Q1_ROWS = 0, Q1_FACTORED = 1, Q1_FULL = 2, Q1_FULL_MV = 3 };
constexpr int q1_nvals(int dim, int mode) {
  return mode == Q1_FACTORED ? (dim + 1) * q1_nblk(dim) + 1
       : mode == Q1_ROWS ? (dim + 1) * q1_npad(dim) : q1_npad(dim) * q1_npad(dim);
}

// Cell viscosity pass: eta at every (R^d fine cells x 2^d) Gauss point of
// each cell; uni[cell] = 1 when all are equal, eta0[cell] = the first value.
void q1_launch_cell_eta(int dim, const Q1Dev& q, int R, const double* incl, int n_incl, double eta_out,
                        double eta_in, double* eta0, unsigned char* uni, hipStream_t s);
// A_e of the listed cut cells, integrated with the Gauss points of their R^d fine cells.
void q1_launch_cut_matrices(int dim, const Q1Dev& q, int R, const int* cells, int ncut, const double* incl,
                            int n_incl, double eta_out, double eta_in, double* cutK, hipStream_t s);
int q1_residual_blocks(const Q1Dev& q);
void q1_launch_residual(int dim, const Q1Dev& q, const double* x, const double* b, double* r, double* partials,
                        hipStream_t s);
// status receives (atomicMin) the first patch with a non-positive pivot of K
// or a non-finite Schur complement.  mode: Q1_ROWS, Q1_FACTORED, Q1_FULL or
// Q1_FULL_MV (patch slots in colour order, contiguous per colour launch).
void q1_launch_factor(int dim, const Q1Dev& q, int mode, double* W, int* status, hipStream_t s);
// RAV (eq. 13): x_owned += omega (owned rows of L_i^{-1}) r_i (mode Q1_ROWS or Q1_FACTORED).
void q1_launch_apply(int dim, const Q1Dev& q, int mode, const double* W, const double* r, double* x,
                     double omega, hipStream_t s);
// AV (eq. 12): Y_i = omega L_i^{-1} r_i per patch, then x += sum_i R_i^T Y_i (gather, no atomics).
void q1_launch_av(int dim, const Q1Dev& q, const double* W, const double* r, double* Y, double* x, double omega,
                  hipStream_t s);
// MV (eq. 11): the patches of one colour sum_d (k_d mod 4) 4^d, each recomputing
// its residual rows from the current x (eq. 15) and adding omega L_i^{-1} r_i.
void q1_launch_mv_colour(int dim, const Q1Dev& q, const double* W, const double* b, double* x, double omega,
                         int colour, hipStream_t s);
void q1_launch_restrict(int dim, const Q1Dev& f, const Q1Dev& c, const double* rf, double* bc, double* xc,
                        double* rc, hipStream_t s);   // rc may be null
void q1_launch_prolong(int dim, const Q1Dev& f, const Q1Dev& c, const double* xc, double* xf, hipStream_t s);
// Dense coarse matrix, row-major nb x nb; masked rows/columns identity;
// bordered: row/column n holds the pressure ones (zero-mean constraint).
void q1_launch_dense(int dim, const Q1Dev& q, double* M, long long nb, int bordered, hipStream_t s);
void q1_launch_rhs(int dim, const Q1Dev& q, const double* params, double* b, hipStream_t s);
void q1_launch_lid(const Q1Dev& q, double U, double* b, hipStream_t s);
void q1_launch_owner(int dim, const Q1Dev& q, int* owner, hipStream_t s);

}  // namespace rav
