// Internal device-side descriptors of the RAV library.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "rav_index.h"

namespace rav {

constexpr int MAX_SEG = 25;      // 3 components x 8 parity types + pressure
constexpr int MAX_BUCKETS = 8;
constexpr int MAX_INCL = 64;
constexpr int BLOCK = 256;       // threads per block of the streaming kernels
constexpr int APPLY_SPLIT = 8;   // lanes per patch of the mid-size-level RAV apply
constexpr int APPLY_SPLIT_SMALL = 32;   // lanes per patch on the smallest levels
// Threads per block of the RAV apply: one-wavefront blocks keep the tail of a
// streaming launch short (a straggling block holds one wavefront of work); the
// 8-lane split variant runs best with 256-thread blocks.
constexpr int APPLY_BLOCK_MAX = 256;
// Buckets of at most 64 patches (3D element patches on top edges and the top
// corner: up to 89 owned rows each) use the row-parallel apply: one wavefront
// per patch, one lane per owned row.
constexpr int APPLY_ROWS = 64;
__host__ __device__ constexpr int apply_block(int split) {
  return split == APPLY_SPLIT || split == APPLY_ROWS ? 256 : 64;
}

enum Prec { P_FP64 = 0, P_FP32 = 1, P_BF16 = 2 };

// Owned inverse rows of one bucket of patches (same owned pattern).
// Entry e = c * nown + j (column c of the padded patch, owned row j) of patch p
// lives in 16-byte vector m = e / V (V = 16 bytes / element size), slot e % V.
// Vectors are chunk-major: vector m of patch p is vector m * count_pad + p, so
// a wavefront reads 1 KiB contiguously per load and the wavefronts of a launch,
// which advance through the chunks at similar rates, sweep W plane by plane
// (close to one sequential stream, the access order HBM serves fastest).
struct Bucket {
  int cls;
  int nown;
  long long count;       // patches in the bucket
  long long count_pad;   // rounded up to a multiple of 64
  long long nchunk;      // ceil(values per patch / V): npad * nown, or fact_nvals(dim) when factored
  void* W;
  int factored;          // W holds the factored form (vertex patches; see fact_nvals)
};

// Index (in 16-byte vectors) of vector m of patch p.
__host__ __device__ __forceinline__ long long w_vec(const Bucket& bk, long long p, long long m) {
  return m * bk.count_pad + p;
}

// One level of one problem, resident in device memory.
struct GridDev {
  Geo g;
  int kind;
  double h;
  double* x;             // level iterate
  double* b;             // level right-hand side
  double* r;             // level residual
  double* vals;          // ELL operator values
  // per-cell coefficients of the matrix-free residual: h^(d-2) eta for cells
  // with one viscosity at all Gauss points, -(1 + i) for the i-th cut cell,
  // whose full viscous cell matrix (h^(d-2) included) is cutA[i][a][b]
  const double* ceta;
  const double* cutA;
  long long seg_off[MAX_SEG];
  long long seg_rows[MAX_SEG];
  // coarser level (transfer target), valid when has_coarse
  int has_coarse;
  Geo gc;
  double* xc;
  double* bc;
  double* rc;            // coarser level's residual: restriction also writes it (x_c = 0, so r_c = b_c)
  // smoother data
  int nbk;
  Bucket bk[MAX_BUCKETS];
  double* Winv;          // AV/MV: full local inverses, [patch][npad][npad], column-major per patch
  double* Y;             // AV: per-patch corrections [patch][npad]
  const float* omega_patch;
  double omega;
  // coarsest level only: dense inverse of the (bordered) coarse matrix
  const double* Minv;
  long long nbc;
  // batched solves: problem stops being updated once *active == 0 (null = always)
  const int* active;
};

__host__ __device__ __forceinline__ bool grid_idle(const GridDev& gd) { return gd.active && *gd.active == 0; }

// One block of a streaming launch.  `part` selects the ELL segment or patch
// bucket, `start` the first row/patch of the tile, `logical` the tile's
// position in grid order (blocks are permuted so that each XCD walks a
// contiguous range of tiles), grid = -1 marks padding blocks.
struct BlockTask {
  int grid;
  int part;
  long long start;
  int logical;
  int pad;
};

// Reference-element tables (filled on the host from the Lagrange bases).
struct RefTables {
  double gt[3], gw[3];            // 3-point Gauss on [0,1]
  double phi[3][3], dphi[3][3];   // Q2 1D basis / derivative [node][qp]
  double psi[2][3];               // Q1 1D basis [node][qp]
  double aref2[9][9];             // sum_q w_q grad.grad, 2D reference cell (h = 1)
  double aref3[27][27];
  double bref2[2][9][4];          // -sum_q w_q psi_k d_c phi_a (h = 1)
  double bref3[3][27][8];
};

// ---- kernel launchers (defined in the .hip files) --------------------------
void set_ref_tables(const RefTables& t, hipStream_t s);

// Viscosity per Gauss point and per-cell uniformity; R > 1 samples the Gauss
// points of the R^d finest-grid cells inside each cell (Galerkin coarse operator).
void launch_eta(int dim, long long ncell, const GridDev* G, const double* incl, int n_incl, double eta_out,
                double eta_in, int R, double* etaq, unsigned char* uni, hipStream_t s);
// ELL operator values; non-uniform cells take their stored cell matrix cutA[cut_idx[cell]].
void launch_assemble(int dim, const GridDev* G, const BlockTask* tasks, int ntasks, const double* etaq,
                     const unsigned char* uni, const int* cut_idx, const double* cutA, hipStream_t s);
void launch_rhs(int dim, const GridDev* Gh, const GridDev* Gd, const double* params, double* fq,
                double* b, hipStream_t s);
// Residual tiles: part = velocity node parity type t (rows of seg_rows(g, t))
// or 2^d for the pressure rows.
void launch_residual(int dim, const GridDev* G, const BlockTask* tasks, int ntasks, double* partials,
                     hipStream_t s);
// Large levels (2D N >= 512, 3D N >= 64): the residual staged through LDS, one block per tile of cells.
bool residual_tiled_ok(int dim, int N);
int residual_tiles(int dim, int N);
void launch_residual_tiled(int dim, const GridDev* G, int N, double* partials, hipStream_t s);
// Driven-cavity lifting -L[free, masked] u_D (2D, u_D = (U, 0) on the lid) added into b.
void launch_lift_lid(const GridDev* G, const Geo& g, double U, double* b, hipStream_t s);
void launch_cell_coef(int dim, long long ncell, const GridDev* G, const double* etaq, const int* cut_idx,
                      const int* cut_cells, int ncut, int R, const double* incl, int n_incl, double eta_out,
                      double eta_in, double* ceta, double* cutA, hipStream_t s);
void launch_norm_finalize(const double* partials, int first, int count, double* out, double* host_out,
                          hipStream_t s);
void launch_rav_apply(int dim, int kind, int cls, int prec, int split, const GridDev* G, const BlockTask* tasks,
                      int ntasks, hipStream_t s, int factored = 0);
// Several buckets of one level in one launch (tasks carry the variant in pad:
// 4, APPLY_SPLIT or APPLY_ROWS).  edges: some task runs a 3D edge or corner
// class (3, 5, 6, 7) on a column-group variant.
void launch_rav_apply_multi(int dim, int kind, int prec, bool edges, const GridDev* G, const BlockTask* tasks,
                            int ntasks, hipStream_t s);
void launch_factor(int dim, int kind, int cls, int prec, int full, const GridDev* G, long long count,
                   int bucket, int* status, hipStream_t s);
void launch_av_apply(int dim, int kind, const GridDev* G, long long npatch, hipStream_t s);
void launch_av_gather(int dim, int kind, const GridDev* G, long long n, hipStream_t s);
void launch_mv_colour(int dim, int kind, const GridDev* G, int colour, long long npatch_colour,
                      hipStream_t s);
void launch_restrict(int dim, const GridDev* G, const BlockTask* tasks, int ntasks, hipStream_t s);
void launch_prolong(int dim, const GridDev* G, const BlockTask* tasks, int ntasks, hipStream_t s);
void launch_coarse_gemv_batch(const GridDev* G, const BlockTask* tasks, int ntasks, hipStream_t s);
void launch_norm_finalize_batch(const double* partials, const int* first, const int* count, int ngrids,
                                double* out, hipStream_t s);
void launch_copy_batch(double* const* dst, const double* const* src, const long long* n, const BlockTask* tasks,
                       int ntasks, hipStream_t s);
void launch_coarse_build(const GridDev* G, int dim, double* M, long long nb, int bordered, int unit_masked,
                         hipStream_t s);
// Blocked Gauss-Jordan inversion with partial pivoting of nprob dense nb x nb
// matrices (device pointer array Ms), in place.  Scratch: pivs, perm (nprob*nb
// int), colk (nprob*nb double), Rsave (nprob*GJ_PANEL*nb double); status
// (nprob int) must hold INT_MAX on entry and receives the first zero-pivot
// column of each singular matrix.
constexpr int GJ_PANEL = 32;
void launch_bgj_invert(double* const* Ms, long long nb, int nprob, int* pivs, double* colk, double* Rsave,
                       int* perm, int* status, hipStream_t s);
void launch_coarse_gemv(const double* Minv, long long nb, long long n0, const double* b, double* x,
                        hipStream_t s);
void launch_features(const GridDev* G, long long npatch, const double* incl, int n_incl, double eta_out,
                     double eta_in, float* F, hipStream_t s);
void launch_mlp_forward(const float* theta, const float* F, long long n, float* omega, hipStream_t s);
int mlp_backward_blocks(long long n);
void launch_mlp_backward(const float* theta, const float* F, const double* gom, long long n, double* partial,
                         double* grad, hipStream_t s);
void launch_adam(float* theta, double* m, double* v, const double* grad, double lr, int t, hipStream_t s);
void launch_rav_grad(const GridDev* G, long long npatch, const double* r, const double* lam, double* gom,
                     hipStream_t s);
void launch_rav_transpose(const GridDev* G, long long npatch, const double* lam, const float* omega, double* Y,
                          hipStream_t s);
void launch_patch_gather(const GridDev* G, long long n, const double* Y, double* z, hipStream_t s);
void launch_axpby(double a, const double* x, double b, double* y, long long n, hipStream_t s);
void launch_owner(const GridDev* G, int kind, long long n, int* owner, hipStream_t s);
void launch_copy(double* dst, const double* src, long long n, hipStream_t s);
void launch_fill(double* dst, double v, long long n, hipStream_t s);

}  // namespace rav
