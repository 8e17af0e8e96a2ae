// Stabilized Q1-Q1 on adaptively refined quadtree grids with hanging nodes
// (Sec. 2, eqs. 5-8 and Fig. 2; Sec. 4.1, Table 1): device layout shared by
// the host driver (rav_adapt.hip) and the kernels (k_adapt.hip).
//
// A level has nV regular vertices (leaf corners that are not hanging nodes),
// numbered lexicographically (y slowest, x fastest), and 3 nV unknowns
// [u_x; u_y; p], field f of vertex v at f nV + v.  Velocity on the boundary
// of the unit square is Dirichlet (masked).
//
// Operator: the conforming space is reached through the hanging-node
// constraints, L = T^T L_corners T, assembled once on the host.  It is stored
// by vertex pairs (i, j) in SELL-64 form: vertices in slices of 64, slice s
// has width w_s = its longest row and entry k of the vertex at lane t sits at
// soff[s] + 64 k + t, so a wavefront reads every plane with unit stride.  An
// entry holds the column vertex and six planes (stride nnz): A_ij (viscous
// block, the same for both components), BT_x,ij and BT_y,ij (row u_c,i,
// column p_j), B_x,ij and B_y,ij (row p_i, column u_c,j) and C_ij
// (stabilization).  Masked rows and columns are zero; padding entries point
// at the row's own vertex with zero values.
//
// Patches (smoothed levels): patch i is vertex i.  Its free velocity vertices
// (the vertices of the leaves around i, a hanging corner standing for the
// vertices that constrain it) are stored sorted in the same SELL-64 form over
// patches (poff, pv; padding -1); pown[i] is the position of i in its own list
// (-1: velocity of i masked).  The patch matrix is [[K,0,b_x],[0,K,b_y],
// [b_x^T, b_y^T, c]] with K SPD, so its inverse is kept factored:
// z_c = K^{-1} b_c, 1/S with S = c - b_x.z_x - b_y.z_y, and
//   RAV: row pown[i] of K^{-1} (plane kr, SELL layout) -- the owned rows;
//   AV/MV: all of K^{-1}, slice s holding w_s^2 x 64 values from koff[s],
//          entry (a, b) of lane t at koff[s] + 64 (a w_s + b) + t.
#pragma once

#include <hip/hip_runtime.h>

namespace rav {

constexpr int AD_SLICE = 64;
constexpr int AD_NFMAX = 16;   // free velocity vertices per patch

struct AdDev {
  int nV;
  int nslice;
  long long nnz;                    // padded operator entries (plane stride)
  long long pnnz;                   // padded patch entries
  const unsigned char* vmask;       // velocity Dirichlet per vertex
  const int* soff;                  // nslice + 1
  const int* col;
  const double* val;                // 6 planes of nnz
  const int* poff;                  // nslice + 1 (patch slices)
  const int* pv;
  const int* pown;
  const long long* koff;            // nslice + 1 (full K^{-1} slices)
};

enum { AD_A = 0, AD_BTX = 1, AD_BTY = 2, AD_BX = 3, AD_BY = 4, AD_C = 5 };
enum { AD_RAV = 0, AD_FULL = 1 };

// Factored patch inverses: zx, zy (pnnz each), invS (nV), and kr (pnnz, RAV)
// or kfull (koff[nslice], AV/MV).
struct AdFactors {
  double* zx;
  double* zy;
  double* invS;
  double* kr;
  double* kfull;
};

int ad_residual_blocks(int nV);
void ad_launch_residual(const AdDev& a, const double* x, const double* b, double* r, double* partials,
                        hipStream_t s);
void ad_launch_factor(const AdDev& a, int mode, AdFactors f, int* status, hipStream_t s);
void ad_launch_rav(const AdDev& a, AdFactors f, const double* r, double* x, double omega, hipStream_t s);
// AV: corrections of every patch into (yx, yy: pnnz, yp: nV), then each DoF
// gathers the corrections of the patches that hold it (tsoff/tpos: SELL-64
// over vertices, entry = slot of the vertex in a patch list, padding -1).
void ad_launch_av(const AdDev& a, AdFactors f, const int* tsoff, const int* tpos, const double* r, double* yx,
                  double* yy, double* yp, double* x, double omega, hipStream_t s);
// MV: the patches order[first .. first+count) (one colour) recompute their
// residual rows from b and x and update x in place.
void ad_launch_mv(const AdDev& a, AdFactors f, const int* order, int first, int count, const double* b, double* x,
                  double omega, hipStream_t s);
// Transfers: P (fine rows, CSR over vertices, the same weights for the three
// fields; masked velocity rows and columns dropped) and its transpose.
void ad_launch_prolong(const AdDev& f, const AdDev& c, const int* ptr, const int* idx, const double* w,
                       const double* xc, double* xf, hipStream_t s);
void ad_launch_restrict(const AdDev& f, const AdDev& c, const int* ptr, const int* idx, const double* w,
                        const double* rf, double* bc, double* xc, double* rc, hipStream_t s);
void ad_launch_scale(const double* src, double alpha, double* dst, long long n, hipStream_t s);
void ad_launch_owner(const AdDev& a, int* owner, hipStream_t s);

}  // namespace rav
