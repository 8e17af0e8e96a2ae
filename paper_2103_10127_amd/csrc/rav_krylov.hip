// Krylov acceleration of the multigrid solver: restarted, right-preconditioned
// flexible GMRES whose preconditioner is one V-cycle (with zero initial guess)
// of the context's smoother (Sec. 4 remarks that the multigrid cycle may
// equally serve as the preconditioner of a Krylov method).  The Arnoldi
// coefficients stay in device memory; one small read-back per iteration feeds
// the Givens update of the least-squares residual on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "rav_ctx.h"

using namespace rav;

namespace rav {
void launch_dot(const double* a, const double* b, long long n, double* partial, double* out, int take_sqrt,
                hipStream_t s);
void launch_axpy_dev(double* y, const double* x, const double* c, double sign, long long n, hipStream_t s);
void launch_div_dev(double* y, const double* x, const double* c, long long n, hipStream_t s);
}  // namespace rav

// Internal: one V-cycle of the context on its finest level (defined in rav_capi.hip).
void rav_vcycle_finest(rav_ctx* ctx);

#define KCK(expr)                                                              \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);            \
      return e_ == hipErrorOutOfMemory ? RAV_ENOMEM : RAV_EDEVICE;             \
    }                                                                          \
  } while (0)

namespace {

// The finest level of any discretization: its vectors, its residual (norm in
// the context's norm slot when asked) and one V-cycle in place on them.
struct Finest {
  RavFinest v;
  void (*residual)(rav_ctx*, bool);
  void (*vcycle)(rav_ctx*);
};

void th_residual_finest(rav_ctx* ctx, bool with_norm) {
  rav_residual_level(ctx, (int)ctx->lv.size() - 1, with_norm);
}

Finest finest_of(rav_ctx* ctx) {
  if (ctx->q1) return Finest{rav_q1_finest(ctx), rav_q1_residual_finest, rav_q1_vcycle_finest};
  if (ctx->ad) return Finest{rav_ad_finest(ctx), rav_ad_residual_finest, rav_ad_vcycle_finest};
  LevelHost& L = ctx->lv.back();
  return Finest{RavFinest{L.hd.g.n, L.hd.x, L.hd.b, L.hd.r, ctx->factored != 0}, th_residual_finest, rav_vcycle_finest};
}

// Device and host buffers of one FGMRES(m) solve.  Device: the Krylov basis
// V_0..V_m and the preconditioned directions Z_0..Z_{m-1} (n doubles each),
// the iterate xk and right-hand side bk, 1024 dot-product partial sums and
// the Arnoldi columns hdev ((m + 2) per column).  Host: the Hessenberg matrix
// H ((m + 1) x m), the Givens rotations, the least-squares right-hand side g,
// the update coefficients y and hhost (m + 2), which receives one Arnoldi
// column per iteration.  Every buffer is written before it is read, so none
// needs clearing.
struct GmresWork {
  double** V;
  double** Z;
  double *xk, *bk, *partial, *hdev;
  double *hhost, *H, *cs, *sn, *g, *y;
};

rav_status gmres_run(rav_ctx* ctx, double* x_dev, const double* b_dev, double rtol, int maxit, int m,
                     const GmresWork& w, int* iters, double* rel_res) {
  const Finest F = finest_of(ctx);
  const long long n = F.v.n;
  double *Lx = F.v.x, *Lb = F.v.b, *Lr = F.v.r;
  hipStream_t s = ctx->stream;
  double** V = w.V;
  double** Z = w.Z;
  double *xk = w.xk, *bk = w.bk, *partial = w.partial, *hdev = w.hdev, *hhost = w.hhost;
  double *H = w.H, *cs = w.cs, *sn = w.sn, *g = w.g, *y = w.y;
  launch_copy(xk, x_dev, n, s);
  launch_copy(bk, b_dev, n, s);
  // residual of the current iterate into the level's r (norm in ctx->d_norm)
  auto true_residual = [&](double* nrm) -> rav_status {
    launch_copy(Lx, xk, n, s);
    launch_copy(Lb, bk, n, s);
    F.residual(ctx, true);
    return rav_read_norm(ctx, nrm);
  };
  double beta0 = 0.0;
  rav_status result = true_residual(&beta0);
  if (result != RAV_OK) return result;
  if (!std::isfinite(beta0)) { ctx->err = "initial residual is not finite"; return RAV_EDIVERGED; }
  int total = 0;
  double res = beta0;
  result = RAV_NOT_CONVERGED;
  if (beta0 == 0.0) result = RAV_OK;
  while (result == RAV_NOT_CONVERGED && total < maxit) {
    double beta = 0.0;
    if (total > 0) {
      rav_status st = true_residual(&beta);
      if (st != RAV_OK) return st;
      res = beta;
      if (!std::isfinite(beta) || beta > 1e3 * beta0) { result = RAV_EDIVERGED; break; }
      if (beta <= rtol * beta0) { result = RAV_OK; break; }
    } else {
      beta = beta0;
    }
    // V_0 = r / beta
    launch_axpby(1.0 / beta, Lr, 0.0, V[0], n, s);
    for (int i = 0; i <= m; ++i) g[i] = 0.0;
    g[0] = beta;
    int jend = 0;
    for (int j = 0; j < m && total < maxit; ++j) {
      // Z_j = M V_j (one V-cycle from zero)
      launch_copy(Lb, V[j], n, s);
      launch_fill(Lx, 0.0, n, s);
      if (ctx->prof_level < 0) rav_graph_issue(ctx, F.vcycle, &ctx->pc_exec);   // captured once, replayed
      else F.vcycle(ctx);
      launch_copy(Z[j], Lx, n, s);
      // w = L Z_j  (residual with b = 0 gives -L Z_j)
      launch_fill(Lb, 0.0, n, s);
      F.residual(ctx, false);
      double* wv = V[j + 1];
      launch_axpby(-1.0, Lr, 0.0, wv, n, s);
      // modified Gram-Schmidt, coefficients h[i][j] in device memory
      for (int i = 0; i <= j; ++i) {
        double* hij = hdev + (size_t)j * (m + 2) + i;
        launch_dot(wv, V[i], n, partial, hij, 0, s);
        launch_axpy_dev(wv, V[i], hij, -1.0, n, s);
      }
      double* hn = hdev + (size_t)j * (m + 2) + j + 1;
      launch_dot(wv, wv, n, partial, hn, 1, s);
      launch_div_dev(wv, wv, hn, n, s);
      KCK(hipGetLastError());
      KCK(hipMemcpyAsync(hhost, hdev + (size_t)j * (m + 2), sizeof(double) * (j + 2), hipMemcpyDeviceToHost, s));
      KCK(hipStreamSynchronize(s));
      ++total;
      for (int i = 0; i <= j + 1; ++i) H[(size_t)i * m + j] = hhost[i];
      // apply previous rotations to column j, then a new one
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
      }
      const double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
      const double rr = std::hypot(a, c);
      cs[j] = rr > 0.0 ? a / rr : 1.0;
      sn[j] = rr > 0.0 ? c / rr : 0.0;
      H[(size_t)j * m + j] = rr;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      res = std::fabs(g[j + 1]);
      jend = j + 1;
      if (!std::isfinite(res)) { result = RAV_EDIVERGED; break; }
      if (res <= rtol * beta0 || hhost[j + 1] == 0.0) break;
    }
    if (result == RAV_EDIVERGED) break;
    // y = R^{-1} g, x += Z y
    for (int i = jend - 1; i >= 0; --i) {
      double t = g[i];
      for (int k = i + 1; k < jend; ++k) t -= H[(size_t)i * m + k] * y[k];
      y[i] = H[(size_t)i * m + i] != 0.0 ? t / H[(size_t)i * m + i] : 0.0;
    }
    for (int i = 0; i < jend; ++i) launch_axpby(y[i], Z[i], 1.0, xk, n, s);
    if (res <= rtol * beta0) {
      double beta_true = 0.0;
      rav_status st = true_residual(&beta_true);
      if (st != RAV_OK) return st;
      res = beta_true;
      if (beta_true <= rtol * beta0) result = RAV_OK;
    }
  }
  launch_copy(x_dev, xk, n, s);
  KCK(hipGetLastError());
  KCK(hipStreamSynchronize(s));
  if (iters) *iters = total;
  if (rel_res) *rel_res = beta0 > 0.0 ? res / beta0 : 0.0;
  if (result == RAV_EDIVERGED) ctx->err = "GMRES residual diverged";
  return result;
}

rav_status gmres_check(rav_ctx* ctx, double* x_dev, const double* b_dev, double rtol, int maxit, int restart,
                       int max_restart) {
  if (!ctx || !x_dev || !b_dev || !(rtol > 0.0) || maxit < 0 || restart < 1 || restart > max_restart)
    return RAV_EINVAL;
  if (!finest_of(ctx).v.factored) { ctx->err = "rav_factor_patches has not been called"; return RAV_EINVAL; }
  return RAV_OK;
}

// ---- allocation-free variant ------------------------------------------------
// Workspace of rav_solve_gmres_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code must not pass `scratch`
// itself to a kernel (in host code the name is a host-side stand-in); it uses
// the device address obtained once per device with hipGetSymbolAddress.
constexpr long long SCRATCH_DOUBLES = RAV_NOALLOC_SCRATCH_BYTES / 8;
constexpr long long SCRATCH_HEAD = 8192;   // partial sums (1024) and Arnoldi columns (<= 66 x 65)
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

rav_status scratch_address(rav_ctx* ctx, double** out) {
  int dev = 0;
  KCK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) { ctx->err = "device index out of range"; return RAV_EDEVICE; }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    KCK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return RAV_OK;
}

}  // namespace

namespace {

// Work vectors of rav_solve_gmres, kept by the context between calls: the
// first call (and one with another restart) allocates them, rav_destroy
// releases them, so a solve loop allocates nothing after its first solve.
struct GmCache {
  int m = 0;
  long long n = 0;
  std::vector<double*> V, Z;
  double *xk = nullptr, *bk = nullptr, *partial = nullptr, *hdev = nullptr, *hhost = nullptr;
};

void gm_release(rav_ctx* ctx) {
  GmCache* c = static_cast<GmCache*>(ctx->gm_cache);
  if (!c) return;
  for (double* p : c->V) (void)rav_dfree(p);
  for (double* p : c->Z) (void)rav_dfree(p);
  (void)rav_dfree(c->xk); (void)rav_dfree(c->bk); (void)rav_dfree(c->partial); (void)rav_dfree(c->hdev);
  if (c->hhost) (void)hipHostFree(c->hhost);
  delete c;
  ctx->gm_cache = nullptr;
}

rav_status gm_workspace(rav_ctx* ctx, int m, long long n, GmCache** out) {
  GmCache* c = static_cast<GmCache*>(ctx->gm_cache);
  if (c && c->m == m && c->n == n) { *out = c; return RAV_OK; }
  gm_release(ctx);
  c = new GmCache();
  ctx->gm_cache = c;
  ctx->gm_free = gm_release;
  c->m = m;
  c->n = n;
  c->V.assign(m + 1, nullptr);
  c->Z.assign(m, nullptr);
  auto alloc = [&]() -> rav_status {
    for (double*& p : c->V) KCK(rav_dmalloc((void**)&p, sizeof(double) * n));
    for (double*& p : c->Z) KCK(rav_dmalloc((void**)&p, sizeof(double) * n));
    KCK(rav_dmalloc((void**)&c->xk, sizeof(double) * n));
    KCK(rav_dmalloc((void**)&c->bk, sizeof(double) * n));
    KCK(rav_dmalloc((void**)&c->partial, sizeof(double) * 1024));
    KCK(rav_dmalloc((void**)&c->hdev, sizeof(double) * (m + 2) * (m + 1)));
    KCK(hipHostMalloc((void**)&c->hhost, sizeof(double) * (m + 2), hipHostMallocDefault));
    return RAV_OK;
  };
  const rav_status st = alloc();
  if (st != RAV_OK) { gm_release(ctx); return st; }
  *out = c;
  return RAV_OK;
}

}  // namespace

extern "C" rav_status rav_solve_gmres(rav_ctx* ctx, double* x_dev, const double* b_dev, double rtol, int maxit,
                                      int restart, int* iters, double* rel_res) {
  rav_status result = gmres_check(ctx, x_dev, b_dev, rtol, maxit, restart, 200);
  if (result != RAV_OK) return result;
  const int m = restart;
  GmCache* c = nullptr;
  if ((result = gm_workspace(ctx, m, finest_of(ctx).v.n, &c)) != RAV_OK) return result;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  const GmresWork w{c->V.data(), c->Z.data(), c->xk, c->bk, c->partial, c->hdev, c->hhost, H.data(), cs.data(),
                    sn.data(), g.data(), y.data()};
  return gmres_run(ctx, x_dev, b_dev, rtol, maxit, m, w, iters, rel_res);
}

extern "C" rav_status rav_solve_gmres_noalloc(rav_ctx* ctx, double* x_dev, const double* b_dev, double rtol,
                                              int maxit, int restart, int* iters, double* rel_res) {
  rav_status result = gmres_check(ctx, x_dev, b_dev, rtol, maxit, restart, RAV_NOALLOC_MAX_RESTART);
  if (result != RAV_OK) return result;
  const long long n = finest_of(ctx).v.n;
  const long long stride = (n + 31) / 32 * 32;   // 256-byte aligned vectors
  const int m = restart;
  const long long need = SCRATCH_HEAD + (2LL * m + 3) * stride;
  if (need > SCRATCH_DOUBLES) {
    ctx->err = "rav_solve_gmres_noalloc: restart " + std::to_string(m) + " on " + std::to_string(n) +
               " DoFs needs " + std::to_string(need * 8) + " bytes of workspace, more than its " +
               std::to_string(SCRATCH_DOUBLES * 8) + "-byte maximum";
    return RAV_EINVAL;
  }
  double* base = nullptr;
  if ((result = scratch_address(ctx, &base)) != RAV_OK) return result;
  double* V[RAV_NOALLOC_MAX_RESTART + 1];
  double* Z[RAV_NOALLOC_MAX_RESTART];
  double* vec = base + SCRATCH_HEAD;
  for (int i = 0; i <= m; ++i) V[i] = vec + (long long)i * stride;
  for (int i = 0; i < m; ++i) Z[i] = vec + (long long)(m + 1 + i) * stride;
  double* xk = vec + (2LL * m + 1) * stride;
  double* bk = vec + (2LL * m + 2) * stride;
  double hhost[RAV_NOALLOC_MAX_RESTART + 2];
  double H[(RAV_NOALLOC_MAX_RESTART + 1) * RAV_NOALLOC_MAX_RESTART];
  double cs[RAV_NOALLOC_MAX_RESTART], sn[RAV_NOALLOC_MAX_RESTART], g[RAV_NOALLOC_MAX_RESTART + 1];
  double y[RAV_NOALLOC_MAX_RESTART];
  const GmresWork w{V, Z, xk, bk, base, base + 1024, hhost, H, cs, sn, g, y};
  return gmres_run(ctx, x_dev, b_dev, rtol, maxit, m, w, iters, rel_res);
}
