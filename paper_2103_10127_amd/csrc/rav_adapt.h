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
// constraints, L = T^T L_corners T, assembled once on the host.  An entry is
// a vertex pair (i, j) with six values: A_ij (viscous block, the same for both
// components), BT_x,ij and BT_y,ij (row u_c,i, column p_j), B_x,ij and B_y,ij
// (row p_i, column u_c,j) and C_ij (stabilization); masked rows and columns
// are zero.  A grid built from a few leaf sizes has only a few hundred
// distinct value tuples, so each tuple is stored once in vtab (8 doubles per
// tuple: the six values and two zeros) and an entry holds only the column and
// the tuple id -- packed into one 32-bit word (the signed column offset j - i
// in the high 32 - id_bits bits, the id in the low id_bits bits) when every
// offset fits, else as two int32 arrays (the wide format).  Entries are in
// SELL-64 form: vertices in slices of 64, slice s has width w_s = its longest row and entry
// k of the vertex at lane t sits at soff[s] + 64 k + t.  Padding entries point
// at the row's own vertex with the all-zero tuple.
//
// Patches (smoothed levels): patch i is vertex i.  Its free velocity vertices
// (the vertices of the leaves around i, a hanging corner standing for the
// vertices that constrain it) are stored sorted, in the same SELL-64 form
// over patches (pv; padding -1).  The patch matrix
// [[K,0,b_x],[0,K,b_y],[b_x^T, b_y^T, c]] (K SPD) is fixed by the tuple ids of
// its entries, so patches with equal ids
// share one configuration; each configuration is factored once:
// z_c = K^{-1} b_c, 1/S with S = c - b_x.z_x - b_y.z_y, and
//   RAV: the row of K^{-1} of the owned vertex (kr) -- the owned rows;
//   AV/MV: all of K^{-1} (kfull).
// Configuration tables are config-major with AD_NFMAX slots per vector.
#pragma once

#include <hip/hip_runtime.h>

namespace rav {

constexpr int AD_SLICE = 64;
constexpr int AD_NFMAX = 16;   // free velocity vertices per patch
constexpr int AD_LDS_TUPLES = 1024;   // value tables up to this size are staged in LDS (residual, MV)
// The residual stages the table only on grids of at least this many vertices:
// on smaller ones the 256-thread kernel's extra blocks are worth more.
constexpr int AD_RES_LDS_MIN_VERTICES = 150000;

struct AdDev {
  int nV;
  int nslice;
  int wide;                         // 0: packed entries; 1: column and id arrays
  int id_bits;                      // packed: bits of the tuple id
  int ntuple;                       // distinct value tuples (rows of vtab)
  int table_lds;                    // MV stages vtab in LDS (ntuple <= AD_LDS_TUPLES)
  int res_lds;                      // the residual stages vtab in LDS (table_lds and a large grid)
  long long nnz;                    // padded operator entries
  long long pnnz;                   // padded patch entries
  const unsigned char* vmask;       // velocity Dirichlet per vertex
  const int* soff;                  // nslice + 1
  const unsigned* ent;              // packed entry, or (wide) the tuple id
  const int* col;                   // wide: column vertex
  const double* vtab;               // 8 doubles per tuple
  const int* poff;                  // nslice + 1 (patch slices)
  const int* pv;                    // patch vertices
  const int* pcfg;                  // configuration of every patch
  const int* cnf;                   // free velocity vertices per configuration
  const int* cown;                  // position of the patch's own vertex (-1: masked) per configuration
};

enum { AD_A = 0, AD_BTX = 1, AD_BTY = 2, AD_BX = 3, AD_BY = 4, AD_C = 5 };
enum { AD_RAV = 0, AD_FULL = 1 };

// Factors per configuration: zx, zy, kr (AD_NFMAX each), invS (1), kfull
// (AD_NFMAX^2, AV/MV only).
struct AdFactors {
  double* zx;
  double* zy;
  double* invS;
  double* kr;
  double* kfull;
};

// Partial sums the residual writes when asked for its norm (one per block).
int ad_residual_blocks(const AdDev& a);
void ad_launch_residual(const AdDev& a, const double* x, const double* b, double* r, double* partials,
                        hipStream_t s);
// One block per configuration c, built from its representative patch rep[c].
void ad_launch_factor(const AdDev& a, int mode, const int* rep, int ncfg, AdFactors f, int* status, hipStream_t s);
void ad_launch_rav(const AdDev& a, AdFactors f, const double* r, double* x, double omega, hipStream_t s);
// AV: corrections of every patch into (yx, yy: pnnz slots, yp: nV), then each
// DoF gathers the corrections of the patches that hold it (tsoff/tpos: SELL-64
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
