// Batched RAV multigrid: many independent problems of different sizes solved
// together (the additive, colouring-free RAV sweep of Sec. 3, eq. 13 needs no
// ordering between patches, so patches of all problems can share one launch).
//
// Every problem keeps its own hierarchy (an ordinary context).  Levels are
// aligned at the coarsest grid: depth d = 0 is the common coarsest size and
// all problems that own depth d have the same grid size there.  For each depth
// the batch keeps a device array of the level descriptors of all problems
// owning it and block-task tables spanning all of them, so each stage of the
// V-cycle (residual, RAV apply, restriction, prolongation, coarse solve) is a
// single launch over the whole batch.  A problem that has converged is marked
// inactive in device memory and its blocks exit at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>
#include <vector>

#include "rav_ctx.h"

using namespace rav;

namespace {

struct DepthPlan {
  std::vector<int> probs;                 // problems owning this depth
  GridDev* dG = nullptr;                  // descriptors, one per entry of probs
  BlockTask* res = nullptr; int n_res = 0;
  std::vector<ApplyLaunch> apply;
  BlockTask* rtask = nullptr; int n_rtask = 0;   // restriction into depth-1
  BlockTask* ptask = nullptr; int n_ptask = 0;   // prolongation from depth-1
  // problems whose finest level is this depth: residual + norm for the stop test
  std::vector<int> top;                   // indices into probs
  BlockTask* top_res = nullptr; int n_top_res = 0;
  double* partials = nullptr;
  int* first = nullptr; int* count = nullptr; int* pid = nullptr;
  BlockTask* coarse = nullptr; int n_coarse = 0;   // depth 0 only
};

__global__ __launch_bounds__(256) void k_norm_scatter(const double* __restrict__ partials,
                                                       const int* __restrict__ first,
                                                       const int* __restrict__ count,
                                                       const int* __restrict__ pid, double* __restrict__ out) {
  __shared__ double red[256];
  const int g = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < count[g]; i += 256) s += partials[first[g] + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[pid[g]] = red[0];
}

}  // namespace

struct rav_batch {
  std::vector<rav_ctx*> sub;
  hipStream_t stream = nullptr;
  int dim = 2, prec = P_FP64, nu_pre = 2, nu_post = 2, kind = 0;
  std::vector<DepthPlan> depth;
  int* d_active = nullptr;
  double* d_norm2 = nullptr;
  double* h_norm2 = nullptr;
  // user vector tables (device) and finest-level copy tasks
  double** d_dst = nullptr;
  const double** d_src = nullptr;
  long long* d_n = nullptr;
  BlockTask* copy_tasks = nullptr; int n_copy = 0;
  std::vector<long long> n_fine;
  std::string err;
  bool factored = false;
};

#define BCK(expr)                                                         \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) {                                               \
      B->err = std::string(#expr) + ": " + hipGetErrorString(e_);         \
      return e_ == hipErrorOutOfMemory ? RAV_ENOMEM : RAV_EDEVICE;        \
    }                                                                     \
  } while (0)

static std::string g_batch_error;

static rav_status upload(rav_batch* B, const std::vector<BlockTask>& logical, BlockTask** out, int* n) {
  std::vector<BlockTask> t = xcd_order(logical);
  *n = (int)t.size();
  BCK(hipMalloc((void**)out, sizeof(BlockTask) * std::max<size_t>(t.size(), 1)));
  BCK(hipMemcpy(*out, t.data(), sizeof(BlockTask) * t.size(), hipMemcpyHostToDevice));
  return RAV_OK;
}

template <typename T>
static rav_status upload_vec(rav_batch* B, const std::vector<T>& v, T** out) {
  BCK(hipMalloc((void**)out, sizeof(T) * std::max<size_t>(v.size(), 1)));
  if (!v.empty()) BCK(hipMemcpy(*out, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return RAV_OK;
}

// Level of problem p at depth d.
static LevelHost& level_at(rav_batch* B, int p, int d) { return B->sub[p]->lv[d]; }

static rav_status build_plans(rav_batch* B) {
  int dmax = 0;
  for (rav_ctx* c : B->sub) dmax = std::max(dmax, (int)c->lv.size() - 1);
  B->depth.assign(dmax + 1, DepthPlan());
  for (int d = 0; d <= dmax; ++d) {
    DepthPlan& P = B->depth[d];
    for (int p = 0; p < (int)B->sub.size(); ++p)
      if ((int)B->sub[p]->lv.size() > d) P.probs.push_back(p);
    std::vector<GridDev> gds;
    for (int p : P.probs) {
      GridDev g = level_at(B, p, d).hd;
      g.active = B->d_active + p;
      gds.push_back(g);
    }
    rav_status st = upload_vec(B, gds, &P.dG);
    if (st != RAV_OK) return st;
    const int ng = (int)P.probs.size();
    const Geo& g0 = gds[0].g;
    std::vector<BlockTask> rt, pt, res;
    for (int i = 0; i < ng; ++i)
      append_residual_tiles(res, i, gds[i].g);
    if ((st = upload(B, res, &P.res, &P.n_res)) != RAV_OK) return st;
    if (d > 0) {
      for (int i = 0; i < ng; ++i) append_residual_tiles(rt, i, gds[i].gc);
      for (int i = 0; i < ng; ++i) append_residual_tiles(pt, i, gds[i].g);
      if ((st = upload(B, rt, &P.rtask, &P.n_rtask)) != RAV_OK) return st;
      if ((st = upload(B, pt, &P.ptask, &P.n_ptask)) != RAV_OK) return st;
      // one apply launch per bucket class; every problem at this depth has the same buckets
      const long long total = (long long)ng * n_patches(g0, B->kind);
      for (int bi = 0; bi < gds[0].nbk; ++bi) {
        ApplyLaunch al;
        al.bucket = bi;
        al.cls = gds[0].bk[bi].cls;
        al.split = apply_split(total, SPLIT_BELOW);
        std::vector<BlockTask> at;
        for (int i = 0; i < ng; ++i) append_tiles(at, i, bi, gds[i].bk[bi].count, apply_block(al.split) / al.split);
        if ((st = upload(B, at, &al.tasks, &al.ntasks)) != RAV_OK) return st;
        P.apply.push_back(al);
      }
    } else {
      std::vector<BlockTask> ct;
      for (int i = 0; i < ng; ++i) append_tiles(ct, i, 0, gds[i].g.n, 4);
      if ((st = upload(B, ct, &P.coarse, &P.n_coarse)) != RAV_OK) return st;
    }
    // stop-test residual on the problems whose finest level is this depth
    std::vector<BlockTask> tr;
    std::vector<int> first, count, pid;
    for (int i = 0; i < ng; ++i) {
      const int p = P.probs[i];
      if ((int)B->sub[p]->lv.size() - 1 != d) continue;
      P.top.push_back(i);
      const int f = (int)tr.size();
      append_residual_tiles(tr, i, gds[i].g);
      first.push_back(f);
      count.push_back((int)tr.size() - f);
      pid.push_back(p);
    }
    if (!P.top.empty()) {
      if ((st = upload(B, tr, &P.top_res, &P.n_top_res)) != RAV_OK) return st;
      BCK(hipMalloc((void**)&P.partials, sizeof(double) * tr.size()));
      if ((st = upload_vec(B, first, &P.first)) != RAV_OK) return st;
      if ((st = upload_vec(B, count, &P.count)) != RAV_OK) return st;
      if ((st = upload_vec(B, pid, &P.pid)) != RAV_OK) return st;
    }
  }
  return RAV_OK;
}

// r_valid: every level at this depth holds its current residual (levels
// entered through restriction always do; top levels after a norm evaluation).
static bool smooth_depth(rav_batch* B, int d, int sweeps, bool r_valid) {
  DepthPlan& P = B->depth[d];
  for (int s = 0; s < sweeps; ++s) {
    if (!r_valid) launch_residual(B->dim, P.dG, P.res, P.n_res, nullptr, B->stream);
    for (const ApplyLaunch& al : P.apply)
      launch_rav_apply(B->dim, B->kind, al.cls, B->prec, al.split, P.dG, al.tasks, al.ntasks, B->stream);
    r_valid = false;
  }
  return r_valid;
}

// One batched V-cycle; top_valid: the top levels' residuals are current.
static void batch_vcycle(rav_batch* B, bool top_valid) {
  const int dmax = (int)B->depth.size() - 1;
  for (int d = dmax; d >= 1; --d) {
    DepthPlan& P = B->depth[d];
    if (!smooth_depth(B, d, B->nu_pre, top_valid || P.top.empty()))
      launch_residual(B->dim, P.dG, P.res, P.n_res, nullptr, B->stream);
    launch_restrict(B->dim, P.dG, P.rtask, P.n_rtask, B->stream);
  }
  launch_coarse_gemv_batch(B->depth[0].dG, B->depth[0].coarse, B->depth[0].n_coarse, B->stream);
  for (int d = 1; d <= dmax; ++d) {
    DepthPlan& P = B->depth[d];
    launch_prolong(B->dim, P.dG, P.ptask, P.n_ptask, B->stream);
    smooth_depth(B, d, B->nu_post, false);
  }
}

static rav_status batch_norms(rav_batch* B, std::vector<double>& out) {
  for (DepthPlan& P : B->depth) {
    if (P.top.empty()) continue;
    launch_residual(B->dim, P.dG, P.top_res, P.n_top_res, P.partials, B->stream);
    hipLaunchKernelGGL(k_norm_scatter, dim3((unsigned)P.top.size()), dim3(256), 0, B->stream, P.partials, P.first,
                       P.count, P.pid, B->d_norm2);
  }
  BCK(hipGetLastError());
  BCK(hipMemcpyAsync(B->h_norm2, B->d_norm2, sizeof(double) * B->sub.size(), hipMemcpyDeviceToHost, B->stream));
  BCK(hipStreamSynchronize(B->stream));
  out.resize(B->sub.size());
  for (size_t p = 0; p < B->sub.size(); ++p) out[p] = std::sqrt(B->h_norm2[p]);
  return RAV_OK;
}

static rav_status copy_user(rav_batch* B, double* const* dst, const double* const* src) {
  const size_t n = B->sub.size();
  BCK(hipStreamSynchronize(B->stream));   // the pointer tables may still be read by a previous copy
  BCK(hipMemcpy(B->d_dst, dst, sizeof(double*) * n, hipMemcpyHostToDevice));
  BCK(hipMemcpy((void*)B->d_src, src, sizeof(double*) * n, hipMemcpyHostToDevice));
  launch_copy_batch(B->d_dst, B->d_src, B->d_n, B->copy_tasks, B->n_copy, B->stream);
  BCK(hipGetLastError());
  return RAV_OK;
}

static rav_status set_active(rav_batch* B, const std::vector<int>& act) {
  BCK(hipStreamSynchronize(B->stream));
  BCK(hipMemcpy(B->d_active, act.data(), sizeof(int) * act.size(), hipMemcpyHostToDevice));
  return RAV_OK;
}

extern "C" {

rav_status rav_batch_create(const rav_problem_desc* descs, int n, void* hip_stream, rav_batch** out) {
  if (!descs || n <= 0 || !out) { g_batch_error = "null descriptors or n <= 0"; return RAV_EINVAL; }
  *out = nullptr;
  const rav_problem_desc& d0 = descs[0];
  const int coarsest = d0.n_cells >> (d0.n_levels - 1);
  for (int i = 0; i < n; ++i) {
    const rav_problem_desc& d = descs[i];
    if (d.dim != d0.dim || d.patch != d0.patch || d.inv_precision != d0.inv_precision || d.nu_pre != d0.nu_pre ||
        d.nu_post != d0.nu_post) {
      g_batch_error = "all problems of a batch must share dim, patch kind, precision and smoothing steps";
      return RAV_EINVAL;
    }
    if (d.smoother != RAV_SMOOTHER_RAV) { g_batch_error = "batched solves use the RAV smoother"; return RAV_EUNSUPPORTED; }
    if (d.n_levels < 2 || d.n_levels > 20 || d.n_cells % (1 << (d.n_levels - 1)) ||
        (d.n_cells >> (d.n_levels - 1)) != coarsest) {
      g_batch_error = "all problems of a batch must share the coarsest grid size";
      return RAV_EINVAL;
    }
  }
  rav_batch* B = new rav_batch();
  B->stream = (hipStream_t)hip_stream;
  B->dim = d0.dim; B->prec = d0.inv_precision; B->nu_pre = d0.nu_pre; B->nu_post = d0.nu_post; B->kind = d0.patch;
  auto fail = [&](rav_status st, const std::string& m) {
    g_batch_error = m;
    rav_batch_destroy(B);
    return st;
  };
  for (int i = 0; i < n; ++i) {
    rav_ctx* c = nullptr;
    rav_status st = rav_create(&descs[i], hip_stream, &c);
    if (st != RAV_OK) return fail(st, "problem " + std::to_string(i) + ": " + rav_last_error(nullptr));
    B->sub.push_back(c);
    B->n_fine.push_back(c->lv.back().hd.g.n);
  }
  if (hipMalloc((void**)&B->d_active, sizeof(int) * n) != hipSuccess ||
      hipMalloc((void**)&B->d_norm2, sizeof(double) * n) != hipSuccess ||
      hipHostMalloc((void**)&B->h_norm2, sizeof(double) * n, hipHostMallocDefault) != hipSuccess ||
      hipMalloc((void**)&B->d_dst, sizeof(double*) * n) != hipSuccess ||
      hipMalloc((void**)&B->d_src, sizeof(double*) * n) != hipSuccess)
    return fail(RAV_ENOMEM, "batch table allocation failed");
  std::vector<int> ones(n, 1);
  if (hipMemcpy(B->d_active, ones.data(), sizeof(int) * n, hipMemcpyHostToDevice) != hipSuccess)
    return fail(RAV_EDEVICE, "hipMemcpy failed");
  rav_status st = upload_vec(B, B->n_fine, &B->d_n);
  if (st != RAV_OK) return fail(st, B->err);
  std::vector<BlockTask> ct;
  for (int i = 0; i < n; ++i) append_tiles(ct, i, 0, B->n_fine[i], BLOCK);
  if ((st = upload(B, ct, &B->copy_tasks, &B->n_copy)) != RAV_OK) return fail(st, B->err);
  *out = B;
  return RAV_OK;
}

rav_status rav_batch_factor(rav_batch* B) {
  if (!B) return RAV_EINVAL;
  for (size_t i = 0; i < B->sub.size(); ++i) {
    rav_status st = rav_factor_patches(B->sub[i]);
    if (st != RAV_OK) {
      B->err = "problem " + std::to_string(i) + ": " + rav_last_error(B->sub[i]);
      return st;
    }
  }
  // descriptors now hold the inverse-row buffers: build the batched plans
  rav_status st = build_plans(B);
  if (st != RAV_OK) return st;
  B->factored = true;
  return RAV_OK;
}

rav_status rav_batch_size(const rav_batch* B, int* n_problems) {
  if (!B || !n_problems) return RAV_EINVAL;
  *n_problems = (int)B->sub.size();
  return RAV_OK;
}

rav_status rav_batch_dofs(const rav_batch* B, int problem, long* n_total, long* n_free) {
  if (!B || problem < 0 || problem >= (int)B->sub.size()) return RAV_EINVAL;
  rav_ctx* c = B->sub[problem];
  return rav_dofs(c, (int)c->lv.size() - 1, n_total, n_free);
}

rav_status rav_batch_assemble_rhs(rav_batch* B, int problem, const double* params, int n_params, double* b_dev) {
  if (!B || problem < 0 || problem >= (int)B->sub.size()) return RAV_EINVAL;
  rav_status st = rav_assemble_rhs(B->sub[problem], params, n_params, b_dev);
  if (st != RAV_OK) B->err = rav_last_error(B->sub[problem]);
  return st;
}

rav_status rav_batch_vcycle(rav_batch* B, double* const* x, const double* const* b) {
  if (!B || !x || !b) return RAV_EINVAL;
  if (!B->factored) { B->err = "rav_batch_factor has not been called"; return RAV_EINVAL; }
  const size_t n = B->sub.size();
  std::vector<double*> xi(n), bi(n);
  for (size_t p = 0; p < n; ++p) {
    if (!x[p] || !b[p]) return RAV_EINVAL;
    xi[p] = B->sub[p]->lv.back().hd.x;
    bi[p] = B->sub[p]->lv.back().hd.b;
  }
  rav_status st = set_active(B, std::vector<int>(n, 1));
  if (st != RAV_OK) return st;
  if ((st = copy_user(B, xi.data(), x)) != RAV_OK) return st;
  if ((st = copy_user(B, bi.data(), b)) != RAV_OK) return st;
  batch_vcycle(B, false);
  std::vector<const double*> xs(xi.begin(), xi.end());
  if ((st = copy_user(B, const_cast<double* const*>(x), xs.data())) != RAV_OK) return st;
  BCK(hipStreamSynchronize(B->stream));
  return RAV_OK;
}

rav_status rav_batch_solve(rav_batch* B, double* const* x, const double* const* b, double rtol, int maxit,
                           int* iters, double* rel_res) {
  if (!B || !x || !b || !(rtol > 0.0) || maxit < 0) return RAV_EINVAL;
  if (!B->factored) { B->err = "rav_batch_factor has not been called"; return RAV_EINVAL; }
  const size_t n = B->sub.size();
  std::vector<double*> xi(n), bi(n);
  for (size_t p = 0; p < n; ++p) {
    if (!x[p] || !b[p]) return RAV_EINVAL;
    xi[p] = B->sub[p]->lv.back().hd.x;
    bi[p] = B->sub[p]->lv.back().hd.b;
  }
  std::vector<int> act(n, 1);
  rav_status st = set_active(B, act);
  if (st != RAV_OK) return st;
  if ((st = copy_user(B, xi.data(), x)) != RAV_OK) return st;
  if ((st = copy_user(B, bi.data(), b)) != RAV_OK) return st;
  std::vector<double> r0, rk;
  if ((st = batch_norms(B, r0)) != RAV_OK) return st;
  std::vector<int> it(n, 0), status(n, 1);
  rk = r0;
  for (size_t p = 0; p < n; ++p) {
    if (!std::isfinite(r0[p])) { status[p] = -4; act[p] = 0; }
    else if (r0[p] == 0.0) { status[p] = 0; act[p] = 0; }
  }
  int k = 0;
  while (k < maxit && std::count(act.begin(), act.end(), 1) > 0) {
    if ((st = set_active(B, act)) != RAV_OK) return st;
    batch_vcycle(B, true);   // top residuals are current from the norm evaluation
    std::vector<double> nk;
    if ((st = batch_norms(B, nk)) != RAV_OK) return st;
    ++k;
    for (size_t p = 0; p < n; ++p) {
      if (!act[p]) continue;
      rk[p] = nk[p];
      it[p] = k;
      if (!std::isfinite(nk[p]) || nk[p] > 1e3 * r0[p]) { status[p] = -4; act[p] = 0; }
      else if (nk[p] <= rtol * r0[p]) { status[p] = 0; act[p] = 0; }
    }
  }
  if ((st = set_active(B, std::vector<int>(n, 1))) != RAV_OK) return st;
  std::vector<const double*> xs(xi.begin(), xi.end());
  if ((st = copy_user(B, const_cast<double* const*>(x), xs.data())) != RAV_OK) return st;
  BCK(hipStreamSynchronize(B->stream));
  rav_status result = RAV_OK;
  for (size_t p = 0; p < n; ++p) {
    if (iters) iters[p] = it[p];
    if (rel_res) rel_res[p] = r0[p] > 0.0 ? rk[p] / r0[p] : 0.0;
    if (status[p] == -4) result = RAV_EDIVERGED;
    else if (status[p] == 1 && result == RAV_OK) result = RAV_NOT_CONVERGED;
  }
  if (result == RAV_EDIVERGED) B->err = "at least one problem diverged";
  return result;
}

rav_status rav_batch_destroy(rav_batch* B) {
  if (!B) return RAV_OK;
  (void)hipStreamSynchronize(B->stream);
  for (DepthPlan& P : B->depth) {
    (void)hipFree(P.dG); (void)hipFree(P.res); (void)hipFree(P.rtask); (void)hipFree(P.ptask);
    (void)hipFree(P.top_res); (void)hipFree(P.partials); (void)hipFree(P.first); (void)hipFree(P.count);
    (void)hipFree(P.pid); (void)hipFree(P.coarse);
    for (ApplyLaunch& a : P.apply) (void)hipFree(a.tasks);
  }
  for (rav_ctx* c : B->sub) rav_destroy(c);
  (void)hipFree(B->d_active); (void)hipFree(B->d_norm2); (void)hipFree(B->d_dst); (void)hipFree((void*)B->d_src);
  (void)hipFree(B->d_n); (void)hipFree(B->copy_tasks);
  if (B->h_norm2) (void)hipHostFree(B->h_norm2);
  delete B;
  return RAV_OK;
}

const char* rav_batch_last_error(const rav_batch* B) { return B ? B->err.c_str() : g_batch_error.c_str(); }

}  // extern "C"
