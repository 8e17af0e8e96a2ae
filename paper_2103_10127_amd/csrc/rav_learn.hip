// Learned per-patch damping: network object, per-level weights, and the
// gradient of an exact two-grid cycle with respect to the network parameters.
//
// The per-patch weight omega_i is the diagonal weighting of eq. (11) reduced to
// one scalar per subdomain and applied in the RAV sweep of eq. (13).  Training
// differentiates the residual reduction ||L x_out||^2 / ||L x0||^2 of the cycle
//   nu RAV sweeps (omega_i) -> exact coarse correction -> nu RAV sweeps
// (b = 0) by running the cycle's linear steps backwards:
//   sweep x' = x + S_w(-L x):  dJ/dw_i += lam_owned(i) . W_i r_i,
//                              lam <- lam - L S_w^T lam
//   coarse x' = x + P C P^T(-L x):  lam <- lam - L P C P^T lam   (C symmetric)
// then back-propagates sum_i dJ/dw_i dw_i/dtheta through the network.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "rav_ctx.h"

using namespace rav;

namespace {

constexpr int NPARAM = 5313;

struct LearnState {
  int nu = 0;
  long long n = 0, npatch = 0;
  std::vector<double*> states;     // x before/after every step of the cycle
  double *z = nullptr, *rbuf = nullptr, *lam = nullptr, *zero = nullptr, *Y = nullptr, *gom = nullptr;
  float* F = nullptr;              // features of the fine level
  float* omega = nullptr;          // per-patch weights of the fine level
  std::vector<GridDev*> vx;        // descriptor variants: x = states[s], b = 0, r = rbuf
  GridDev* vz = nullptr;           // x = z, b = 0, r = rbuf
  GridDev* vlam = nullptr;         // x = z, b = 0, r = lam (restriction of lam, prolongation into z)
  double* partial = nullptr;
  std::vector<float*> level_omega; // per-level weights for solves (rav_learn_set_omega)
  std::vector<float*> level_feat;
};

void learn_free(rav_ctx* ctx) {
  LearnState* S = static_cast<LearnState*>(ctx->learn);
  if (!S) return;
  for (double* p : S->states) (void)rav_dfree(p);
  (void)rav_dfree(S->z); (void)rav_dfree(S->rbuf); (void)rav_dfree(S->lam); (void)rav_dfree(S->zero);
  (void)rav_dfree(S->Y); (void)rav_dfree(S->gom); (void)rav_dfree(S->F); (void)rav_dfree(S->omega);
  for (GridDev* p : S->vx) (void)rav_dfree(p);
  (void)rav_dfree(S->vz); (void)rav_dfree(S->vlam); (void)rav_dfree(S->partial);
  for (float* p : S->level_omega) (void)rav_dfree(p);
  for (float* p : S->level_feat) (void)rav_dfree(p);
  delete S;
  ctx->learn = nullptr;
}

LearnState* state(rav_ctx* ctx) {
  if (!ctx->learn) {
    ctx->learn = new LearnState();
    ctx->learn_free = learn_free;
  }
  return static_cast<LearnState*>(ctx->learn);
}

}  // namespace

struct rav_mlp {
  LiveCount live_;
  float* theta = nullptr;
  double *m = nullptr, *v = nullptr, *grad = nullptr;
  int t = 0;
};

#define LCK(expr)                                                                  \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      if (ctx) ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);       \
      return e_ == hipErrorOutOfMemory ? RAV_ENOMEM : RAV_EDEVICE;                 \
    }                                                                              \
  } while (0)

static rav_status check_learn_ctx(rav_ctx* ctx) {
  if (!ctx) return RAV_EINVAL;
  const rav_problem_desc& D = ctx->desc;
  if (ctx->q1 || ctx->ad || D.dim != 2 || D.patch != RAV_PATCH_VERTEX || D.smoother != RAV_SMOOTHER_RAV) {
    ctx->err = "learned damping is provided for 2D vertex-patch RAV";
    return RAV_EUNSUPPORTED;
  }
  if (!ctx->factored) { ctx->err = "rav_factor_patches has not been called"; return RAV_EINVAL; }
  return RAV_OK;
}

static rav_status level_features(rav_ctx* ctx, int l, float** F) {
  LearnState* S = state(ctx);
  if ((int)S->level_feat.size() < (int)ctx->lv.size()) S->level_feat.resize(ctx->lv.size(), nullptr);
  LevelHost& L = ctx->lv[l];
  if (!S->level_feat[l]) {
    LCK(rav_dmalloc((void**)&S->level_feat[l], sizeof(float) * 16 * L.npatch));
    launch_features(L.dd, L.npatch, ctx->d_incl, ctx->desc.n_incl, ctx->desc.eta_out, ctx->desc.eta_in,
                    S->level_feat[l], ctx->stream);
    LCK(hipGetLastError());
  }
  *F = S->level_feat[l];
  return RAV_OK;
}

extern "C" {

rav_status rav_mlp_create(const float* theta_host, rav_mlp** out) {
  rav_ctx* ctx = nullptr;
  if (!theta_host || !out) return RAV_EINVAL;
  rav_mlp* M = new rav_mlp();
  if (rav_dmalloc((void**)&M->theta, sizeof(float) * NPARAM) != hipSuccess ||
      rav_dmalloc((void**)&M->m, sizeof(double) * NPARAM) != hipSuccess ||
      rav_dmalloc((void**)&M->v, sizeof(double) * NPARAM) != hipSuccess ||
      rav_dmalloc((void**)&M->grad, sizeof(double) * NPARAM) != hipSuccess) {
    rav_mlp_destroy(M);
    return RAV_ENOMEM;
  }
  LCK(hipMemcpy(M->theta, theta_host, sizeof(float) * NPARAM, hipMemcpyHostToDevice));
  LCK(hipMemset(M->m, 0, sizeof(double) * NPARAM));
  LCK(hipMemset(M->v, 0, sizeof(double) * NPARAM));
  LCK(hipMemset(M->grad, 0, sizeof(double) * NPARAM));
  *out = M;
  return RAV_OK;
}

rav_status rav_mlp_get(const rav_mlp* M, float* theta_host, double* grad_host) {
  rav_ctx* ctx = nullptr;
  if (!M) return RAV_EINVAL;
  LCK(hipDeviceSynchronize());
  if (theta_host) LCK(hipMemcpy(theta_host, M->theta, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
  if (grad_host) LCK(hipMemcpy(grad_host, M->grad, sizeof(double) * NPARAM, hipMemcpyDeviceToHost));
  return RAV_OK;
}

rav_status rav_mlp_destroy(rav_mlp* M) {
  if (!M) return RAV_OK;
  (void)rav_dfree(M->theta); (void)rav_dfree(M->m); (void)rav_dfree(M->v); (void)rav_dfree(M->grad);
  delete M;
  return RAV_OK;
}

rav_status rav_learn_patch_omega(rav_ctx* ctx, const rav_mlp* M, int level, float* omega_dev) {
  rav_status st = check_learn_ctx(ctx);
  if (st != RAV_OK) return st;
  if (!M || !omega_dev || level < 1 || level >= (int)ctx->lv.size()) return RAV_EINVAL;
  float* F = nullptr;
  if ((st = level_features(ctx, level, &F)) != RAV_OK) return st;
  launch_mlp_forward(M->theta, F, ctx->lv[level].npatch, omega_dev, ctx->stream);
  LCK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_learn_set_omega(rav_ctx* ctx, const rav_mlp* M) {
  rav_status st = check_learn_ctx(ctx);
  if (st != RAV_OK) return st;
  LearnState* S = state(ctx);
  if ((int)S->level_omega.size() < (int)ctx->lv.size()) S->level_omega.resize(ctx->lv.size(), nullptr);
  for (int l = 1; l < (int)ctx->lv.size(); ++l) {
    LevelHost& L = ctx->lv[l];
    if (!M) {
      L.hd.omega_patch = nullptr;
    } else {
      if (!S->level_omega[l]) LCK(rav_dmalloc((void**)&S->level_omega[l], sizeof(float) * L.npatch));
      if ((st = rav_learn_patch_omega(ctx, M, l, S->level_omega[l])) != RAV_OK) return st;
      L.hd.omega_patch = S->level_omega[l];
    }
    if ((st = rav_upload_desc(ctx, L)) != RAV_OK) return st;
  }
  return RAV_OK;
}

static rav_status ensure_twogrid(rav_ctx* ctx, int nu) {
  LearnState* S = state(ctx);
  LevelHost& Lf = ctx->lv[1];
  if (S->nu == nu && !S->states.empty()) return RAV_OK;
  for (double* p : S->states) (void)rav_dfree(p);
  for (GridDev* p : S->vx) (void)rav_dfree(p);
  S->states.assign(2 * nu + 2, nullptr);
  S->vx.assign(2 * nu + 2, nullptr);
  S->nu = nu;
  S->n = Lf.hd.g.n;
  S->npatch = Lf.npatch;
  const long long n = S->n;
  for (double*& p : S->states) LCK(rav_dmalloc((void**)&p, sizeof(double) * n));
  if (!S->z) {
    LCK(rav_dmalloc((void**)&S->z, sizeof(double) * n));
    LCK(rav_dmalloc((void**)&S->rbuf, sizeof(double) * n));
    LCK(rav_dmalloc((void**)&S->lam, sizeof(double) * n));
    LCK(rav_dmalloc((void**)&S->zero, sizeof(double) * n));
    LCK(hipMemset(S->zero, 0, sizeof(double) * n));
    LCK(rav_dmalloc((void**)&S->Y, sizeof(double) * S->npatch * 51));
    LCK(rav_dmalloc((void**)&S->gom, sizeof(double) * S->npatch));
    LCK(rav_dmalloc((void**)&S->omega, sizeof(float) * S->npatch));
    LCK(rav_dmalloc((void**)&S->partial, sizeof(double) * NPARAM * mlp_backward_blocks(S->npatch)));
    LCK(rav_dmalloc((void**)&S->vz, sizeof(GridDev)));
    LCK(rav_dmalloc((void**)&S->vlam, sizeof(GridDev)));
  }
  GridDev v = Lf.hd;
  v.b = S->zero;
  v.r = S->rbuf;
  v.omega_patch = S->omega;
  for (int s = 0; s < 2 * nu + 2; ++s) {
    v.x = S->states[s];
    LCK(rav_dmalloc((void**)&S->vx[s], sizeof(GridDev)));
    LCK(hipMemcpy(S->vx[s], &v, sizeof(GridDev), hipMemcpyHostToDevice));
  }
  v.x = S->z;
  LCK(hipMemcpy(S->vz, &v, sizeof(GridDev), hipMemcpyHostToDevice));
  v.r = S->lam;
  LCK(hipMemcpy(S->vlam, &v, sizeof(GridDev), hipMemcpyHostToDevice));
  return RAV_OK;
}

static double residual_sq(rav_ctx* ctx, GridDev* D, rav_status* st) {
  LevelHost& L = ctx->lv[1];
  launch_residual(2, D, L.res_tasks, L.n_res_tasks, L.partials, ctx->stream);
  launch_norm_finalize(L.partials, 0, L.n_res_tiles, ctx->d_norm, ctx->h_norm_dev, ctx->stream);
  double v = 0.0;
  *st = rav_read_norm(ctx, &v);
  return v * v;
}

// Gradient of the two-grid residual reduction from x0 with respect to theta
// (and, optionally, to every per-patch omega).  Requires a 2-level context.
rav_status rav_learn_twogrid(rav_ctx* ctx, const rav_mlp* M, const double* x0, int nu, double* loss,
                             double* grad_omega_dev, double* grad_theta_host) {
  rav_status st = check_learn_ctx(ctx);
  if (st != RAV_OK) return st;
  if (!M || !x0 || nu < 1 || nu > 8) return RAV_EINVAL;
  if (ctx->lv.size() != 2) { ctx->err = "the two-grid loss needs a 2-level context (exact coarse solve)"; return RAV_EINVAL; }
  if (ctx->prec != P_FP64 || ctx->desc.inv_format != RAV_ROWS) {
    ctx->err = "training uses FP64 inverse rows (RAV_ROWS)";
    return RAV_EUNSUPPORTED;
  }
  if ((st = ensure_twogrid(ctx, nu)) != RAV_OK) return st;
  LearnState* S = state(ctx);
  LevelHost& Lf = ctx->lv[1];
  hipStream_t s = ctx->stream;
  const long long n = S->n, np = S->npatch;
  const int R = Lf.n_res_tasks;
  float* F = nullptr;
  if ((st = level_features(ctx, 1, &F)) != RAV_OK) return st;
  launch_mlp_forward(M->theta, F, np, S->omega, s);
  // ---- forward: states[0] = x0, sweeps, coarse correction, sweeps ----
  launch_copy(S->states[0], x0, n, s);
  auto sweep = [&](int to) {
    launch_copy(S->states[to], S->states[to - 1], n, s);
    launch_residual(2, S->vx[to], Lf.res_tasks, R, nullptr, s);
    for (const ApplyLaunch& al : Lf.apply)
      launch_rav_apply(2, KIND_VERTEX, al.cls, P_FP64, al.split, S->vx[to], al.tasks, al.ntasks, s);
  };
  for (int k = 1; k <= nu; ++k) sweep(k);
  {
    const int to = nu + 1;
    launch_copy(S->states[to], S->states[to - 1], n, s);
    launch_residual(2, S->vx[to], Lf.res_tasks, R, nullptr, s);
    launch_restrict(2, S->vx[to], Lf.rtasks, Lf.n_rtasks, s);
    launch_coarse_gemv_batch(ctx->lv[0].dd, ctx->coarse_tasks, ctx->n_coarse_tasks, s);
    launch_prolong(2, S->vx[to], Lf.ptasks, Lf.n_ptasks, s);
  }
  for (int k = nu + 2; k <= 2 * nu + 1; ++k) sweep(k);
  const int last = 2 * nu + 1;
  const double den = residual_sq(ctx, S->vx[0], &st);
  if (st != RAV_OK) return st;
  const double num = residual_sq(ctx, S->vx[last], &st);   // leaves rbuf = -L x_out
  if (st != RAV_OK) return st;
  if (loss) *loss = num / den;
  // ---- reverse: lam = 2 L L x_out / den ----
  launch_copy(S->z, S->rbuf, n, s);                       // z = -L x_out
  launch_residual(2, S->vz, Lf.res_tasks, R, nullptr, s);  // rbuf = -L z = L L x_out
  launch_axpby(2.0 / den, S->rbuf, 0.0, S->lam, n, s);
  LCK(hipMemsetAsync(S->gom, 0, sizeof(double) * np, s));
  auto sweep_back = [&](int pre) {
    launch_residual(2, S->vx[pre], Lf.res_tasks, R, nullptr, s);   // rbuf = -L x_pre
    launch_rav_grad(S->vx[pre], np, S->rbuf, S->lam, S->gom, s);
    launch_rav_transpose(S->vx[pre], np, S->lam, S->omega, S->Y, s);
    launch_patch_gather(S->vx[pre], n, S->Y, S->z, s);             // z = S_w^T lam
    launch_residual(2, S->vz, Lf.res_tasks, R, nullptr, s);        // rbuf = -L z
    launch_axpby(1.0, S->rbuf, 1.0, S->lam, n, s);                 // lam -= L z
  };
  for (int k = last; k >= nu + 2; --k) sweep_back(k - 1);
  {
    launch_fill(S->z, 0.0, n, s);
    launch_restrict(2, S->vlam, Lf.rtasks, Lf.n_rtasks, s);        // coarse b = P^T lam
    launch_coarse_gemv_batch(ctx->lv[0].dd, ctx->coarse_tasks, ctx->n_coarse_tasks, s);
    launch_prolong(2, S->vlam, Lf.ptasks, Lf.n_ptasks, s);         // z = P C P^T lam
    launch_residual(2, S->vz, Lf.res_tasks, R, nullptr, s);        // rbuf = -L z
    launch_axpby(1.0, S->rbuf, 1.0, S->lam, n, s);
  }
  for (int k = nu; k >= 1; --k) sweep_back(k - 1);
  if (grad_omega_dev) launch_copy(grad_omega_dev, S->gom, np, s);
  launch_mlp_backward(M->theta, F, S->gom, np, S->partial, M->grad, s);
  LCK(hipGetLastError());
  LCK(hipStreamSynchronize(s));
  if (grad_theta_host) LCK(hipMemcpy(grad_theta_host, M->grad, sizeof(double) * NPARAM, hipMemcpyDeviceToHost));
  return RAV_OK;
}

rav_status rav_learn_step(rav_ctx* ctx, rav_mlp* M, const double* x0, int nu, double lr, double* loss) {
  rav_status st = rav_learn_twogrid(ctx, M, x0, nu, loss, nullptr, nullptr);
  if (st != RAV_OK) return st;
  M->t += 1;
  launch_adam(M->theta, M->m, M->v, M->grad, lr, M->t, ctx->stream);
  LCK(hipGetLastError());
  return RAV_OK;
}

}  // extern "C"
