// Host driver of the stabilized Q1-Q1 discretization (Sec. 2, eqs. 5-8) with
// the literal RAV owned set (Sec. 3, eq. 13): hierarchy set-up, patch
// factorization, smoothing, transfers, the coarse direct solve, V-cycles
// (Sec. 2, Fig. 1) and the solve to a relative residual (Sec. 4).  The public
// entry points of rav.h route here when the descriptor selects
// RAV_Q1Q1_STAB; the kernels are in k_q1.hip.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "rav_ctx.h"
#include "rav_q1.h"

using namespace rav;

struct rav_q1_state {
  struct Level {
    Q1Dev q{};
    double *x = nullptr, *b = nullptr, *r = nullptr;
    double *ceta = nullptr, *cutK = nullptr;
    long long ncut = 0;
    double* W = nullptr;          // patch inverses (smoothed levels)
    double* Y = nullptr;          // AV: per-patch corrections (row-major over the patch DoFs)
    double* partials = nullptr;   // residual norm partial sums
    int nres = 0;
  };
  std::vector<Level> lv;
  double* Minv = nullptr;
  long long nb = 0;
  int bordered = 0;
  int mode = Q1_FACTORED;   // storage of the patch inverses (Q1_ROWS / Q1_FACTORED for RAV, full for AV/MV)
  bool have_factors = false;
};

#define QCK(expr)                                                                    \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                  \
      return e_ == hipErrorOutOfMemory ? RAV_ENOMEM : RAV_EDEVICE;                   \
    }                                                                                \
  } while (0)

namespace {

using Level = rav_q1_state::Level;

long long ipowll(long long b, int e) {
  long long r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

bool all_dirichlet(const rav_problem_desc& d) {
  for (int b = 0; b < 2 * d.dim; ++b)
    if (!((d.bc_dirichlet_mask >> b) & 1u)) return false;
  return true;
}

bool vert_masked(const Q1Dev& q, const int* v) {
  for (int d = 0; d < q.dim; ++d) {
    if (((q.dmask >> (2 * d)) & 1u) && v[d] == 0) return true;
    if (((q.dmask >> (2 * d + 1)) & 1u) && v[d] == q.N) return true;
  }
  return false;
}

void vert_of(const Q1Dev& q, long long v, int* c) {
  c[0] = (int)(v % q.np1);
  c[1] = (int)((v / q.np1) % q.np1);
  c[2] = q.dim == 3 ? (int)(v / (q.np1 * q.np1)) : 0;
}

Q1Dev make_q1(const rav_problem_desc& d, int level) {
  Q1Dev q{};
  q.dim = d.dim;
  q.N = d.n_cells >> (d.n_levels - 1 - level);
  q.np1 = q.N + 1;
  q.nV = ipowll(q.np1, d.dim);
  q.n = (d.dim + 1) * q.nV;
  q.dmask = d.bc_dirichlet_mask;
  q.h = 1.0 / q.N;
  q.bscale = std::pow(q.h, d.dim - 1);
  const double hs = d.coarse_galerkin ? 1.0 / d.n_cells : q.h;
  q.cC = -d.beta * d.dim * hs * hs * std::pow(q.h, d.dim - 2);
  q.gp_lo = 0.5 - 0.5 / std::sqrt(3.0);
  q.gp_hi = 0.5 + 0.5 / std::sqrt(3.0);
  return q;
}

rav_q1_state* st(const rav_ctx* ctx) { return ctx->q1; }

rav_status check_lv(const rav_ctx* ctx, int level, bool smoothed) {
  if (level < 0 || level >= (int)st(ctx)->lv.size()) return RAV_EINVAL;
  if (smoothed && level == 0) return RAV_EINVAL;
  return RAV_OK;
}

// Per-cell coefficients of one level: eta folded with h^(d-2) where the
// viscosity is one value at every Gauss point (of the R^d finest-grid cells
// inside the cell when R > 1), the full cell matrix otherwise.
rav_status build_cells(rav_ctx* ctx, Level& L, int R) {
  const rav_problem_desc& D = ctx->desc;
  const long long ncell = ipowll(L.q.N, D.dim);
  double* eta0 = nullptr;
  unsigned char* uni = nullptr;
  QCK(rav_dmalloc((void**)&eta0, sizeof(double) * ncell));
  QCK(rav_dmalloc((void**)&uni, ncell));
  QCK(rav_dmalloc((void**)&L.ceta, sizeof(double) * ncell));
  q1_launch_cell_eta(D.dim, L.q, R, ctx->d_incl, D.n_incl, D.eta_out, D.eta_in, eta0, uni, ctx->stream);
  QCK(hipGetLastError());
  std::vector<double> he(ncell);
  std::vector<unsigned char> hu(ncell);
  QCK(hipMemcpyAsync(he.data(), eta0, sizeof(double) * ncell, hipMemcpyDeviceToHost, ctx->stream));
  QCK(hipMemcpyAsync(hu.data(), uni, ncell, hipMemcpyDeviceToHost, ctx->stream));
  QCK(hipStreamSynchronize(ctx->stream));
  (void)rav_dfree(eta0);
  (void)rav_dfree(uni);
  const double ascale = std::pow(L.q.h, D.dim - 2);
  std::vector<int> cut;
  for (long long c = 0; c < ncell; ++c) {
    if (hu[c]) {
      he[c] = ascale * he[c];
    } else {
      he[c] = -(double)(1 + cut.size());
      cut.push_back((int)c);
    }
  }
  QCK(hipMemcpy(L.ceta, he.data(), sizeof(double) * ncell, hipMemcpyHostToDevice));
  L.q.ceta = L.ceta;
  L.ncut = (long long)cut.size();
  if (!cut.empty()) {
    const int nb = 1 << D.dim;
    int* dcells = nullptr;
    QCK(rav_dmalloc((void**)&dcells, sizeof(int) * cut.size()));
    QCK(hipMemcpy(dcells, cut.data(), sizeof(int) * cut.size(), hipMemcpyHostToDevice));
    QCK(rav_dmalloc((void**)&L.cutK, sizeof(double) * cut.size() * nb * nb));
    q1_launch_cut_matrices(D.dim, L.q, R, dcells, (int)cut.size(), ctx->d_incl, D.n_incl, D.eta_out, D.eta_in,
                           L.cutK, ctx->stream);
    QCK(hipGetLastError());
    QCK(hipStreamSynchronize(ctx->stream));
    (void)rav_dfree(dcells);
  }
  L.q.cutK = L.cutK;
  return RAV_OK;
}

rav_status build_coarse(rav_ctx* ctx) {
  rav_q1_state* S = st(ctx);
  const Level& L0 = S->lv[0];
  S->bordered = all_dirichlet(ctx->desc) ? 1 : 0;
  S->nb = L0.q.n + S->bordered;
  const long long nb = S->nb;
  QCK(rav_dmalloc((void**)&S->Minv, sizeof(double) * nb * nb));
  q1_launch_dense(ctx->desc.dim, L0.q, S->Minv, nb, S->bordered, ctx->stream);
  QCK(hipGetLastError());
  double** dM = nullptr;
  int *piv = nullptr, *perm = nullptr, *pst = nullptr;
  double *colk = nullptr, *Rs = nullptr;
  const int big = INT_MAX;
  QCK(rav_dmalloc((void**)&dM, sizeof(double*)));
  QCK(rav_dmalloc((void**)&piv, sizeof(int) * nb));
  QCK(rav_dmalloc((void**)&perm, sizeof(int) * nb));
  QCK(rav_dmalloc((void**)&pst, sizeof(int)));
  QCK(rav_dmalloc((void**)&colk, sizeof(double) * nb));
  QCK(rav_dmalloc((void**)&Rs, sizeof(double) * GJ_PANEL * nb));
  QCK(hipMemcpy(dM, &S->Minv, sizeof(double*), hipMemcpyHostToDevice));
  QCK(hipMemcpy(pst, &big, sizeof(int), hipMemcpyHostToDevice));
  launch_bgj_invert(dM, nb, 1, piv, colk, Rs, perm, pst, ctx->stream);
  QCK(hipGetLastError());
  int status = 0;
  QCK(hipMemcpyAsync(&status, pst, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  QCK(hipStreamSynchronize(ctx->stream));
  (void)rav_dfree(dM); (void)rav_dfree(piv); (void)rav_dfree(perm); (void)rav_dfree(pst); (void)rav_dfree(colk);
  (void)rav_dfree(Rs);
  if (status != INT_MAX)
    return rav_set_error(ctx, RAV_ESINGULAR, "zero pivot in the coarse matrix at column " + std::to_string(status));
  return RAV_OK;
}

void residual(rav_ctx* ctx, int l, bool with_norm) {
  Level& L = st(ctx)->lv[l];
  q1_launch_residual(ctx->desc.dim, L.q, L.x, L.b, L.r, with_norm ? L.partials : nullptr, ctx->stream);
  if (with_norm) launch_norm_finalize(L.partials, 0, L.nres, ctx->d_norm, ctx->h_norm_dev, ctx->stream);
}

// `sweeps` smoothing sweeps: RAV (eq. 13) and AV (eq. 12) from one residual
// (r_valid: L.r already holds b - L x), MV (eq. 11) colour by colour, each
// patch recomputing its residual rows (eq. 15).
void smooth(rav_ctx* ctx, int l, int sweeps, bool r_valid) {
  Level& L = st(ctx)->lv[l];
  const rav_problem_desc& D = ctx->desc;
  for (int k = 0; k < sweeps; ++k) {
    if (D.smoother == RAV_SMOOTHER_MV) {
      const int ncol = D.dim == 2 ? 16 : 64;
      for (int c = 0; c < ncol; ++c) q1_launch_mv_colour(D.dim, L.q, L.W, L.b, L.x, D.omega, c, ctx->stream);
      continue;
    }
    if (!(k == 0 && r_valid)) residual(ctx, l, false);
    if (D.smoother == RAV_SMOOTHER_AV) q1_launch_av(D.dim, L.q, L.W, L.r, L.Y, L.x, D.omega, ctx->stream);
    else q1_launch_apply(D.dim, L.q, st(ctx)->mode, L.W, L.r, L.x, D.omega, ctx->stream);
  }
}

void coarse_solve(rav_ctx* ctx) {
  rav_q1_state* S = st(ctx);
  Level& L0 = S->lv[0];
  launch_coarse_gemv(S->Minv, S->nb, L0.q.n, L0.b, L0.x, ctx->stream);
}

// V-cycle on level l (Sec. 2, Fig. 1); r_valid: L.r holds the residual of
// the current x (coarse levels: restriction writes r_c = b_c for x_c = 0).
void vcycle(rav_ctx* ctx, int l, bool r_valid) {
  if (l == 0) {
    coarse_solve(ctx);
    return;
  }
  rav_q1_state* S = st(ctx);
  Level& L = S->lv[l];
  Level& C = S->lv[l - 1];
  smooth(ctx, l, ctx->desc.nu_pre, r_valid);
  if (ctx->desc.nu_pre > 0 || !r_valid) residual(ctx, l, false);
  q1_launch_restrict(ctx->desc.dim, L.q, C.q, L.r, C.b, C.x, l - 1 > 0 ? C.r : nullptr, ctx->stream);
  vcycle(ctx, l - 1, true);
  q1_launch_prolong(ctx->desc.dim, L.q, C.q, C.x, L.x, ctx->stream);
  smooth(ctx, l, ctx->desc.nu_post, false);
}

// One solve cycle from a current finest residual: V-cycle, then the new
// finest residual and its norm (replayed from a graph, rav_graph_cycle).
void issue_cycle(rav_ctx* ctx) {
  const int lf = (int)st(ctx)->lv.size() - 1;
  vcycle(ctx, lf, true);
  residual(ctx, lf, true);
}

void solve_cycle(rav_ctx* ctx) { rav_graph_cycle(ctx, issue_cycle); }

rav_status need_factors(rav_ctx* ctx) {
  if (!st(ctx)->have_factors) return rav_set_error(ctx, RAV_EINVAL, "rav_factor_patches has not been called");
  return RAV_OK;
}

}  // namespace

// ============================================================================
rav_status rav_q1_create(const rav_problem_desc* d, void* hip_stream, rav_ctx** out) {
  if (d->dim != 2 && d->dim != 3) return rav_set_error(nullptr, RAV_EINVAL, "dim must be 2 or 3");
  if (d->n_levels < 2) return rav_set_error(nullptr, RAV_EINVAL, "n_levels must be >= 2");
  if (d->n_levels > 20 || d->n_cells <= 0 || d->n_cells % (1 << (d->n_levels - 1)))
    return rav_set_error(nullptr, RAV_EINVAL, "n_cells must be divisible by 2^(n_levels-1)");
  const long long n0 = (d->dim + 1) * ipowll((d->n_cells >> (d->n_levels - 1)) + 1, d->dim);
  if (n0 + 1 > MAX_COARSE)
    return rav_set_error(nullptr, RAV_EINVAL, "coarsest grid too large for the dense direct solve (" +
                         std::to_string(n0) + " DoFs, limit " + std::to_string(MAX_COARSE) + "): use more levels");
  if ((d->dim + 1) * ipowll(d->n_cells + 1LL, d->dim) >= (1LL << 31))
    return rav_set_error(nullptr, RAV_EUNSUPPORTED, "finest level beyond 2^31 DoFs");
  if (!(d->beta > 0.0)) return rav_set_error(nullptr, RAV_EINVAL, "the stabilization constant beta must be > 0");
  if (!(d->omega > 0.0) || d->nu_pre < 0 || d->nu_post < 0)
    return rav_set_error(nullptr, RAV_EINVAL, "omega must be > 0 and smoothing steps >= 0");
  if (!(d->eta_out > 0.0) || !(d->eta_in > 0.0)) return rav_set_error(nullptr, RAV_EINVAL, "viscosities must be > 0");
  if (d->n_incl < 0 || d->n_incl > MAX_INCL || (d->n_incl > 0 && !d->incl))
    return rav_set_error(nullptr, RAV_EINVAL, "n_incl must be in [0, 64] with a valid array");
  if (d->bc_dirichlet_mask >> (2 * d->dim))
    return rav_set_error(nullptr, RAV_EINVAL, "bc mask has bits beyond 2*dim");
  if (d->coarse_galerkin != 0 && d->coarse_galerkin != 1)
    return rav_set_error(nullptr, RAV_EINVAL, "coarse_galerkin must be 0 or 1");
  if (d->smoother < RAV_SMOOTHER_RAV || d->smoother > RAV_SMOOTHER_MV)
    return rav_set_error(nullptr, RAV_EINVAL, "bad smoother");
  if (d->patch != RAV_PATCH_VERTEX || d->inv_precision != RAV_FP64)
    return rav_set_error(nullptr, RAV_EUNSUPPORTED, "the stabilized Q1-Q1 discretization is provided with "
                         "vertex patches and FP64 inverses");
  if (d->inv_format != RAV_ROWS && d->inv_format != RAV_FACTORED)
    return rav_set_error(nullptr, RAV_EINVAL, "bad inverse format");

  rav_ctx* ctx = new rav_ctx();
  ctx->desc = *d;
  if (d->n_incl > 0) ctx->incl.assign(d->incl, d->incl + d->n_incl);
  ctx->desc.incl = ctx->incl.empty() ? nullptr : ctx->incl.data();
  ctx->stream = (hipStream_t)hip_stream;
  ctx->prec = P_FP64;
  ctx->q1 = new rav_q1_state();
  auto fail = [&](rav_status s) {
    rav_set_error(nullptr, s, ctx->err);
    rav_destroy(ctx);
    return s;
  };
  rav_status s = rav_init_common(ctx, d);
  if (s != RAV_OK) return fail(s);
  rav_q1_state* S = ctx->q1;
  S->mode = d->smoother == RAV_SMOOTHER_AV ? Q1_FULL
          : d->smoother == RAV_SMOOTHER_MV ? Q1_FULL_MV
          : d->inv_format == RAV_FACTORED ? Q1_FACTORED : Q1_ROWS;
  S->lv.resize(d->n_levels);
  for (int l = 0; l < d->n_levels; ++l) {
    Level& L = S->lv[l];
    L.q = make_q1(*d, l);
    const long long n = L.q.n;
    hipError_t e = rav_dmalloc((void**)&L.x, sizeof(double) * n);
    if (e == hipSuccess) e = rav_dmalloc((void**)&L.b, sizeof(double) * n);
    if (e == hipSuccess) e = rav_dmalloc((void**)&L.r, sizeof(double) * n);
    L.nres = q1_residual_blocks(L.q);
    if (e == hipSuccess) e = rav_dmalloc((void**)&L.partials, sizeof(double) * L.nres);
    if (e == hipSuccess) e = hipMemsetAsync(L.x, 0, sizeof(double) * n, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(L.b, 0, sizeof(double) * n, ctx->stream);
    if (e != hipSuccess) { ctx->err = hipGetErrorString(e); return fail(RAV_EDEVICE); }
    const int R = d->coarse_galerkin ? d->n_cells / L.q.N : 1;
    if ((s = build_cells(ctx, L, R)) != RAV_OK) return fail(s);
  }
  if ((s = build_coarse(ctx)) != RAV_OK) return fail(s);
  *out = ctx;
  return RAV_OK;
}

void rav_q1_free(rav_ctx* ctx) {
  rav_q1_state* S = ctx->q1;
  if (!S) return;
  for (Level& L : S->lv) {
    (void)rav_dfree(L.x); (void)rav_dfree(L.b); (void)rav_dfree(L.r); (void)rav_dfree(L.ceta); (void)rav_dfree(L.cutK);
    (void)rav_dfree(L.W); (void)rav_dfree(L.Y); (void)rav_dfree(L.partials);
  }
  (void)rav_dfree(S->Minv);
  delete S;
  ctx->q1 = nullptr;
}

rav_status rav_q1_factor(rav_ctx* ctx) {
  rav_q1_state* S = st(ctx);
  const int dim = ctx->desc.dim;
  const int nvals = q1_nvals(dim, S->mode);
  const int big = INT_MAX;
  for (size_t l = 1; l < S->lv.size(); ++l) {
    Level& L = S->lv[l];
    if (!L.W) QCK(rav_dmalloc((void**)&L.W, sizeof(double) * nvals * L.q.nV));
    if (S->mode == Q1_FULL && !L.Y) QCK(rav_dmalloc((void**)&L.Y, sizeof(double) * q1_npad(dim) * L.q.nV));
    QCK(hipMemcpy(ctx->d_status, &big, sizeof(int), hipMemcpyHostToDevice));
    q1_launch_factor(dim, L.q, S->mode, L.W, ctx->d_status, ctx->stream);
    QCK(hipGetLastError());
    int stv = 0;
    QCK(hipMemcpyAsync(&stv, ctx->d_status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    QCK(hipStreamSynchronize(ctx->stream));
    if (stv != INT_MAX)
      return rav_set_error(ctx, RAV_ESINGULAR,
                           "singular local system in patch " + std::to_string(stv) + " on level " + std::to_string(l));
  }
  S->have_factors = true;
  ctx->factored = 1;
  return RAV_OK;
}

rav_status rav_q1_dofs(const rav_ctx* ctx, int level, long* n_total, long* n_free) {
  if (check_lv(ctx, level, false) != RAV_OK) return RAV_EINVAL;
  const Q1Dev& q = st(ctx)->lv[level].q;
  if (n_total) *n_total = (long)q.n;
  if (n_free) {
    long long masked = 0;
    for (long long v = 0; v < q.nV; ++v) {
      int c[3];
      vert_of(q, v, c);
      if (vert_masked(q, c)) ++masked;
    }
    *n_free = (long)(q.n - q.dim * masked);
  }
  return RAV_OK;
}

int rav_q1_n_levels(const rav_ctx* ctx) { return (int)st(ctx)->lv.size(); }

rav_status rav_q1_n_patches(const rav_ctx* ctx, int level, long* n) {
  if (check_lv(ctx, level, false) != RAV_OK || !n) return RAV_EINVAL;
  *n = (long)st(ctx)->lv[level].q.nV;
  return RAV_OK;
}

rav_status rav_q1_assemble_rhs(rav_ctx* ctx, const double* params, int n_params, double* b_dev) {
  const int need = ctx->desc.dim == 2 ? 25 : 65;
  if (n_params != need)
    return rav_set_error(ctx, RAV_EINVAL, "mms parameter array must have " + std::to_string(need) + " entries");
  Level& L = st(ctx)->lv.back();
  double* dp = nullptr;
  QCK(rav_dmalloc((void**)&dp, sizeof(double) * n_params));
  QCK(hipMemcpy(dp, params, sizeof(double) * n_params, hipMemcpyHostToDevice));
  q1_launch_rhs(ctx->desc.dim, L.q, dp, b_dev, ctx->stream);
  QCK(hipGetLastError());
  QCK(hipStreamSynchronize(ctx->stream));
  QCK(rav_dfree(dp));
  return RAV_OK;
}

rav_status rav_q1_assemble_rhs_lid(rav_ctx* ctx, double lid_u, double* b_dev) {
  Level& L = st(ctx)->lv.back();
  q1_launch_lid(L.q, lid_u, b_dev, ctx->stream);
  QCK(hipGetLastError());
  QCK(hipStreamSynchronize(ctx->stream));
  return RAV_OK;
}

rav_status rav_q1_residual(rav_ctx* ctx, int level, const double* x, const double* b, double* r, double* norm) {
  if (check_lv(ctx, level, false) != RAV_OK) return RAV_EINVAL;
  Level& L = st(ctx)->lv[level];
  launch_copy(L.x, x, L.q.n, ctx->stream);
  launch_copy(L.b, b, L.q.n, ctx->stream);
  residual(ctx, level, norm != nullptr);
  launch_copy(r, L.r, L.q.n, ctx->stream);
  QCK(hipGetLastError());
  if (norm) return rav_read_norm(ctx, norm);
  return RAV_OK;
}

rav_status rav_q1_smooth(rav_ctx* ctx, int level, int sweeps, double* x, const double* b) {
  if (check_lv(ctx, level, true) != RAV_OK) return RAV_EINVAL;
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  Level& L = st(ctx)->lv[level];
  launch_copy(L.x, x, L.q.n, ctx->stream);
  launch_copy(L.b, b, L.q.n, ctx->stream);
  smooth(ctx, level, sweeps, false);
  launch_copy(x, L.x, L.q.n, ctx->stream);
  QCK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_q1_restrict(rav_ctx* ctx, int level, const double* rf, double* bc) {
  if (check_lv(ctx, level, true) != RAV_OK) return RAV_EINVAL;
  Level& L = st(ctx)->lv[level];
  Level& C = st(ctx)->lv[level - 1];
  launch_copy(L.r, rf, L.q.n, ctx->stream);
  q1_launch_restrict(ctx->desc.dim, L.q, C.q, L.r, C.b, C.x, nullptr, ctx->stream);
  launch_copy(bc, C.b, C.q.n, ctx->stream);
  QCK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_q1_prolong_add(rav_ctx* ctx, int level, const double* xc, double* xf) {
  if (check_lv(ctx, level, true) != RAV_OK) return RAV_EINVAL;
  Level& L = st(ctx)->lv[level];
  Level& C = st(ctx)->lv[level - 1];
  launch_copy(C.x, xc, C.q.n, ctx->stream);
  launch_copy(L.x, xf, L.q.n, ctx->stream);
  q1_launch_prolong(ctx->desc.dim, L.q, C.q, C.x, L.x, ctx->stream);
  launch_copy(xf, L.x, L.q.n, ctx->stream);
  QCK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_q1_coarse_solve(rav_ctx* ctx, const double* b0, double* x0) {
  rav_q1_state* S = st(ctx);
  launch_coarse_gemv(S->Minv, S->nb, S->lv[0].q.n, b0, x0, ctx->stream);
  QCK(hipGetLastError());
  return RAV_OK;
}

// FGMRES hooks (rav_krylov.hip): the finest level's vectors, its residual
// (norm into the context's norm slot) and one V-cycle in place on them.
RavFinest rav_q1_finest(rav_ctx* ctx) {
  const int lf = (int)st(ctx)->lv.size() - 1;
  Level& L = st(ctx)->lv[lf];
  return RavFinest{L.q.n, L.x, L.b, L.r, st(ctx)->have_factors};
}
void rav_q1_residual_finest(rav_ctx* ctx, bool with_norm) { residual(ctx, (int)st(ctx)->lv.size() - 1, with_norm); }
void rav_q1_vcycle_finest(rav_ctx* ctx) { vcycle(ctx, (int)st(ctx)->lv.size() - 1, false); }

rav_status rav_q1_vcycle(rav_ctx* ctx, double* x, const double* b) {
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  const int lf = (int)st(ctx)->lv.size() - 1;
  Level& L = st(ctx)->lv[lf];
  launch_copy(L.x, x, L.q.n, ctx->stream);
  launch_copy(L.b, b, L.q.n, ctx->stream);
  vcycle(ctx, lf, false);
  launch_copy(x, L.x, L.q.n, ctx->stream);
  QCK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_q1_solve(rav_ctx* ctx, double* x, const double* b, double rtol, int maxit, int* iters,
                        double* rel_res) {
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  const int lf = (int)st(ctx)->lv.size() - 1;
  Level& L = st(ctx)->lv[lf];
  launch_copy(L.x, x, L.q.n, ctx->stream);
  launch_copy(L.b, b, L.q.n, ctx->stream);
  residual(ctx, lf, true);
  double r0 = 0.0;
  rav_status s = rav_read_norm(ctx, &r0);
  if (s != RAV_OK) return s;
  if (iters) *iters = 0;
  if (rel_res) *rel_res = r0 > 0.0 ? 1.0 : 0.0;
  if (!std::isfinite(r0)) return rav_set_error(ctx, RAV_EDIVERGED, "initial residual is not finite");
  rav_status result = r0 == 0.0 ? RAV_OK : RAV_NOT_CONVERGED;
  int k = 0;
  double rk = r0;
  while (result == RAV_NOT_CONVERGED && k < maxit) {
    solve_cycle(ctx);   // the finest residual is current from the norm evaluation
    if ((s = rav_read_norm(ctx, &rk)) != RAV_OK) return s;
    ++k;
    if (!std::isfinite(rk) || rk > 1e3 * r0) {
      result = RAV_EDIVERGED;
      ctx->err = "residual diverged at cycle " + std::to_string(k);
    } else if (rk <= rtol * r0) {
      result = RAV_OK;
    }
  }
  if (iters) *iters = k;
  if (rel_res) *rel_res = r0 > 0.0 ? rk / r0 : 0.0;
  launch_copy(x, L.x, L.q.n, ctx->stream);
  QCK(hipGetLastError());
  QCK(hipStreamSynchronize(ctx->stream));
  return result;
}

// Local DoFs of the patch of vertex k, in local order: velocity components
// over the valid vertices of the 3^d block, then p_k.  Fills the padded local
// index of each (pad) and its global index (dofs); owned marks p_k and the
// velocity at k.
static int q1_patch_list(const Q1Dev& q, long long k, int* dofs, int* owned, int* pad) {
  const int dim = q.dim;
  const int nblk = dim == 2 ? 9 : 27;
  int vc[3];
  vert_of(q, k, vc);
  int cnt = 0;
  for (int c = 0; c < dim; ++c)
    for (int m = 0; m < nblk; ++m) {
      int w[3] = {0, 0, 0}, t = m;
      bool ok = true;
      for (int d = 0; d < dim; ++d) {
        w[d] = vc[d] + (t % 3) - 1;
        t /= 3;
        ok = ok && w[d] >= 0 && w[d] <= q.N;
      }
      if (!ok || vert_masked(q, w)) continue;
      long long wi = w[dim - 1];
      for (int d = dim - 2; d >= 0; --d) wi = wi * q.np1 + w[d];
      if (dofs) dofs[cnt] = (int)(c * q.nV + wi);
      if (owned) owned[cnt] = wi == k ? 1 : 0;
      if (pad) pad[cnt] = c * nblk + m;
      ++cnt;
    }
  if (dofs) dofs[cnt] = (int)(dim * q.nV + k);
  if (owned) owned[cnt] = 1;
  if (pad) pad[cnt] = dim * nblk;
  return cnt + 1;
}

rav_status rav_q1_map_patch(const rav_problem_desc* d, int level, long patch, int* dofs, int* n, int* owned) {
  if (!d || (d->dim != 2 && d->dim != 3) || d->n_levels < 1 || d->n_levels > 20 || level < 0 ||
      level >= d->n_levels || d->n_cells <= 0 || d->n_cells % (1 << (d->n_levels - 1)) || !dofs || !n)
    return RAV_EINVAL;
  const Q1Dev q = make_q1(*d, level);
  if (patch < 0 || patch >= q.nV) return RAV_EINVAL;
  *n = q1_patch_list(q, patch, dofs, owned, nullptr);
  return RAV_OK;
}

rav_status rav_q1_map_owner(const rav_problem_desc* d, int level, int* owner) {
  if (!d || (d->dim != 2 && d->dim != 3) || d->n_levels < 1 || d->n_levels > 20 || level < 0 ||
      level >= d->n_levels || d->n_cells <= 0 || d->n_cells % (1 << (d->n_levels - 1)) || !owner)
    return RAV_EINVAL;
  const Q1Dev q = make_q1(*d, level);
  for (long long i = 0; i < q.n; ++i) {
    const long long v = i % q.nV;
    int c[3];
    vert_of(q, v, c);
    owner[i] = (i < q.dim * q.nV && vert_masked(q, c)) ? -1 : (int)v;
  }
  return RAV_OK;
}

rav_status rav_q1_get_owner(rav_ctx* ctx, int level, int* owner_dev) {
  if (check_lv(ctx, level, false) != RAV_OK) return RAV_EINVAL;
  q1_launch_owner(ctx->desc.dim, st(ctx)->lv[level].q, owner_dev, ctx->stream);
  QCK(hipGetLastError());
  QCK(hipStreamSynchronize(ctx->stream));
  return RAV_OK;
}

rav_status rav_q1_get_patch_map(const rav_ctx* ctx, int level, long patch, int* dofs, int* n, int* owned) {
  if (check_lv(ctx, level, false) != RAV_OK || !dofs || !n) return RAV_EINVAL;
  const Q1Dev& q = st(ctx)->lv[level].q;
  if (patch < 0 || patch >= q.nV) return RAV_EINVAL;
  *n = q1_patch_list(q, patch, dofs, owned, nullptr);
  return RAV_OK;
}

// Owned rows of L_i^{-1} (owned DoFs in local order x patch DoFs), rebuilt
// from the stored values in either format.
rav_status rav_q1_get_patch_inverse(rav_ctx* ctx, int level, long patch, double* out, int* rows, int* cols) {
  if (check_lv(ctx, level, true) != RAV_OK) return RAV_EINVAL;
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  rav_q1_state* S = st(ctx);
  const Level& L = S->lv[level];
  const Q1Dev& q = L.q;
  if (patch < 0 || patch >= q.nV) return RAV_EINVAL;
  const int dim = q.dim, nblk = dim == 2 ? 9 : 27, npad = dim * nblk + 1, cen = (nblk - 1) / 2;
  const int nvals = q1_nvals(dim, S->mode);
  std::vector<double> W(nvals);
  QCK(hipStreamSynchronize(ctx->stream));
  long long slot = patch;   // MV stores the inverses in colour-major order
  if (S->mode == Q1_FULL_MV) {
    int c[3];
    vert_of(q, patch, c);
    int colour = 0, mul = 1;
    for (int d = 0; d < dim; ++d) { colour += (c[d] % 4) * mul; mul *= 4; }
    slot = 0;
    for (int cc = 0; cc < colour; ++cc) {
      long long cnt = 1;
      int t = cc;
      for (int d = 0; d < dim; ++d) { const int cd = t % 4; t /= 4; cnt *= (q.N + 1 - cd + 3) / 4; }
      slot += cnt;
    }
    long long qi = 0, stv = 1;
    int t = colour;
    for (int d = 0; d < dim; ++d) {
      const int cd = t % 4;
      t /= 4;
      qi += ((c[d] - cd) / 4) * stv;
      stv *= (q.N + 1 - cd + 3) / 4;
    }
    slot += qi;
  }
  if (S->mode == Q1_FULL_MV)   // patch-major
    QCK(hipMemcpy(W.data(), L.W + slot * nvals, sizeof(double) * nvals, hipMemcpyDeviceToHost));
  else
    QCK(hipMemcpy2D(W.data(), sizeof(double), L.W + slot, sizeof(double) * q.nV, sizeof(double), nvals,
                    hipMemcpyDeviceToHost));
  std::vector<int> dofs(npad), own(npad), pad(npad);
  const int n = q1_patch_list(q, patch, dofs.data(), own.data(), pad.data());
  const bool full = S->mode == Q1_FULL || S->mode == Q1_FULL_MV;
  // entry of owned row `row` (0..d-1 velocity at the centre, d pressure) at padded column col
  auto entry = [&](int row, int col) -> double {
    if (S->mode == Q1_ROWS) return W[(size_t)row * npad + col];
    const double sinv = W[nblk + dim * nblk];
    auto z = [&](int c, int m) { return W[nblk + c * nblk + m]; };
    const bool cv = col < dim * nblk;
    if (row < dim) {
      if (cv) {
        const int c2 = col / nblk, m = col % nblk;
        return (c2 == row ? W[m] : 0.0) + z(row, cen) * sinv * z(c2, m);
      }
      return -z(row, cen) * sinv;
    }
    if (cv) return -sinv * z(col / nblk, col % nblk);
    return sinv;
  };
  int nr = 0;
  if (full) {   // every row: the full local inverse over the patch DoFs
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < n; ++j) out[(size_t)i * n + j] = W[(size_t)pad[i] * npad + pad[j]];
      ++nr;
    }
  } else {
    for (int i = 0; i < n; ++i) {
      if (!own[i]) continue;
      const int row = pad[i] == dim * nblk ? dim : pad[i] / nblk;
      for (int j = 0; j < n; ++j) out[(size_t)nr * n + j] = entry(row, pad[j]);
      ++nr;
    }
  }
  *rows = nr;
  *cols = n;
  return RAV_OK;
}

rav_status rav_q1_time_sweep(rav_ctx* ctx, int level, int reps, double* x, const double* b, float* ms_res,
                             float* ms_apply) {
  if (check_lv(ctx, level, true) != RAV_OK) return RAV_EINVAL;
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  Level& L = st(ctx)->lv[level];
  launch_copy(L.x, x, L.q.n, ctx->stream);
  launch_copy(L.b, b, L.q.n, ctx->stream);
  std::vector<hipEvent_t> ev(3 * reps);
  for (auto& e : ev) QCK(hipEventCreate(&e));
  for (int i = 0; i < reps; ++i) {
    QCK(hipEventRecord(ev[3 * i], ctx->stream));
    residual(ctx, level, false);
    QCK(hipEventRecord(ev[3 * i + 1], ctx->stream));
    if (ctx->desc.smoother == RAV_SMOOTHER_AV)
      q1_launch_av(ctx->desc.dim, L.q, L.W, L.r, L.Y, L.x, ctx->desc.omega, ctx->stream);
    else
      q1_launch_apply(ctx->desc.dim, L.q, st(ctx)->mode, L.W, L.r, L.x, ctx->desc.omega, ctx->stream);
    QCK(hipEventRecord(ev[3 * i + 2], ctx->stream));
  }
  QCK(hipEventSynchronize(ev.back()));
  double tr = 0.0, ta = 0.0;
  for (int i = 0; i < reps; ++i) {
    float a = 0.f, c = 0.f;
    QCK(hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]));
    QCK(hipEventElapsedTime(&c, ev[3 * i + 1], ev[3 * i + 2]));
    tr += a;
    ta += c;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (ms_res) *ms_res = (float)(tr / reps);
  if (ms_apply) *ms_apply = (float)(ta / reps);
  launch_copy(x, L.x, L.q.n, ctx->stream);
  QCK(hipStreamSynchronize(ctx->stream));
  return RAV_OK;
}
