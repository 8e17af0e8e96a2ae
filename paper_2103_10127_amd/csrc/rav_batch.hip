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

constexpr int BV_TILE = 1024;   // elements per task of the batched Krylov vector kernels

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
  LiveCount live_;
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
  double* h_norm2_dev = nullptr;          // device alias of the pinned h_norm2
  // one batched V-cycle plus the top-level residual norms, captured once and
  // replayed by rav_batch_solve (RAV_GRAPH=0 launches directly)
  hipGraphExec_t cycle_exec = nullptr;
  bool graph_failed = false;
  // per-problem vector tiles for the batched Krylov kernels
  BlockTask* vtasks = nullptr; int n_vtasks = 0;
  int* v_first = nullptr; int* v_count = nullptr;
  double* v_partial = nullptr;
  std::vector<int> apply_split_log;        // chosen lanes per patch, (depth, bucket) order
};

namespace rav {
void launch_bdot(const BlockTask* tasks, int ntasks, double* const* A, double* const* Bv, const long long* n,
                 const int* active, double* partial, const int* first, const int* count, int nprob, double* out,
                 long long ostride, long long ooff, int take_sqrt, hipStream_t s);
void launch_bvec(const BlockTask* tasks, int ntasks, double* const* Y, double* const* X, const long long* n,
                 const int* active, const double* coef, long long cstride, long long coff, double sign, int mode,
                 hipStream_t s);
void launch_bupdate(const BlockTask* tasks, int ntasks, double* const* Xk, double* const* Z, int nprob, int m,
                    const long long* n, const int* jend, const double* ycoef, hipStream_t s);
}  // namespace rav

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
  BCK(rav_dmalloc((void**)out, sizeof(BlockTask) * std::max<size_t>(t.size(), 1)));
  BCK(hipMemcpy(*out, t.data(), sizeof(BlockTask) * t.size(), hipMemcpyHostToDevice));
  return RAV_OK;
}

template <typename T>
static rav_status upload_vec(rav_batch* B, const std::vector<T>& v, T** out) {
  BCK(rav_dmalloc((void**)out, sizeof(T) * std::max<size_t>(v.size(), 1)));
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
        if (gds[0].bk[bi].factored && al.split == APPLY_ROWS) al.split = APPLY_SPLIT_SMALL;
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
      BCK(rav_dmalloc((void**)&P.partials, sizeof(double) * tr.size()));
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
      launch_rav_apply(B->dim, B->kind, al.cls, B->prec, al.split, P.dG, al.tasks, al.ntasks, B->stream,
                       level_at(B, P.probs[0], d).hd.bk[al.bucket].factored);
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

// Residual of every problem's finest level; with norms, the squared norms are
// written straight into pinned host memory (h_norm2).
static void batch_top_residual(rav_batch* B, bool norms) {
  for (DepthPlan& P : B->depth) {
    if (P.top.empty()) continue;
    launch_residual(B->dim, P.dG, P.top_res, P.n_top_res, norms ? P.partials : nullptr, B->stream);
    if (norms)
      hipLaunchKernelGGL(k_norm_scatter, dim3((unsigned)P.top.size()), dim3(256), 0, B->stream, P.partials, P.first,
                         P.count, P.pid, B->h_norm2_dev);
  }
}

static rav_status read_norms(rav_batch* B, std::vector<double>& out) {
  BCK(hipGetLastError());
  BCK(hipStreamSynchronize(B->stream));
  out.resize(B->sub.size());
  for (size_t p = 0; p < B->sub.size(); ++p) out[p] = std::sqrt(B->h_norm2[p]);
  return RAV_OK;
}

static rav_status batch_norms(rav_batch* B, std::vector<double>& out) {
  batch_top_residual(B, true);
  return read_norms(B, out);
}

// One solve cycle (V-cycle from current top residuals, then the new top
// residuals and their norms), replayed from a captured graph when possible.
static void batch_solve_cycle(rav_batch* B) {
  static const bool graphs = [] {
    const char* e = std::getenv("RAV_GRAPH");
    return !(e && std::string(e) == "0");
  }();
  if (graphs && !B->graph_failed) {
    if (!B->cycle_exec) {
      hipGraph_t g = nullptr;
      bool ok = hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        batch_vcycle(B, true);
        batch_top_residual(B, true);
        ok = hipStreamEndCapture(B->stream, &g) == hipSuccess && g != nullptr;
      }
      if (ok) ok = hipGraphInstantiate(&B->cycle_exec, g, nullptr, nullptr, 0) == hipSuccess;
      if (g) (void)hipGraphDestroy(g);
      if (!ok) {
        (void)hipGetLastError();
        B->cycle_exec = nullptr;
        B->graph_failed = true;
      }
    }
    if (B->cycle_exec && hipGraphLaunch(B->cycle_exec, B->stream) == hipSuccess) return;
    (void)hipGetLastError();
    B->graph_failed = true;
  }
  batch_vcycle(B, true);
  batch_top_residual(B, true);
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
    if (d.dim != d0.dim || d.patch != d0.patch || d.inv_precision != d0.inv_precision ||
        d.inv_format != d0.inv_format || d.nu_pre != d0.nu_pre ||
        d.nu_post != d0.nu_post) {
      g_batch_error = "all problems of a batch must share dim, patch kind, precision, inverse format and smoothing "
                      "steps";
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
    rav_status st = rav_create_ex(&descs[i], hip_stream, &c, false);
    if (st != RAV_OK) return fail(st, "problem " + std::to_string(i) + ": " + rav_last_error(nullptr));
    c->autotune = false;
    B->sub.push_back(c);
    B->n_fine.push_back(c->lv.back().hd.g.n);
  }
  // the coarse matrices of all problems (grouped by size) inverted together
  for (size_t i = 0; i < B->sub.size(); ++i) {
    if (B->sub[i]->coarse_tasks) continue;   // already inverted with an earlier group
    std::vector<rav_ctx*> grp;
    for (size_t j = i; j < B->sub.size(); ++j)
      if (!B->sub[j]->coarse_tasks && B->sub[j]->nb == B->sub[i]->nb) grp.push_back(B->sub[j]);
    std::vector<int> piv_status;
    std::string err;
    rav_status st = rav_invert_coarse(grp.data(), (int)grp.size(), B->stream, &piv_status, &err);
    if (st != RAV_OK) return fail(st, err);
    for (size_t g = 0; g < grp.size(); ++g) {
      st = rav_finish_coarse(grp[g], piv_status[g]);
      if (st != RAV_OK) return fail(st, "coarse matrix: " + grp[g]->err);
    }
  }
  if (rav_dmalloc((void**)&B->d_active, sizeof(int) * n) != hipSuccess ||
      rav_dmalloc((void**)&B->d_norm2, sizeof(double) * n) != hipSuccess ||
      hipHostMalloc((void**)&B->h_norm2, sizeof(double) * n, hipHostMallocDefault) != hipSuccess ||
      hipHostGetDevicePointer((void**)&B->h_norm2_dev, B->h_norm2, 0) != hipSuccess ||
      rav_dmalloc((void**)&B->d_dst, sizeof(double*) * n) != hipSuccess ||
      rav_dmalloc((void**)&B->d_src, sizeof(double*) * n) != hipSuccess)
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

// Autotuner of the batched apply: for every depth and bucket, the 1-, 4-,
// APPLY_SPLIT- and APPLY_SPLIT_SMALL-lanes-per-patch launches over all
// problems are timed (HIP events, mean of three after one warm-up, on the
// levels' own vectors, which every solve overwrites) and the fastest kept.
// RAV_AUTOTUNE=0 keeps the size rule.
static rav_status autotune_batch(rav_batch* B) {
  if (const char* e = std::getenv("RAV_AUTOTUNE"))
    if (std::string(e) == "0") return RAV_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BCK(hipEventCreate(&e0));
  BCK(hipEventCreate(&e1));
  rav_status result = RAV_OK;
  const int cands[4] = {1, 4, APPLY_SPLIT, APPLY_SPLIT_SMALL};
  for (size_t d = 1; d < B->depth.size() && result == RAV_OK; ++d) {
    DepthPlan& P = B->depth[d];
    const int ng = (int)P.probs.size();
    for (ApplyLaunch& al : P.apply) {
      float best = 1e30f;
      int best_split = al.split;
      BlockTask* best_tasks = nullptr;
      int best_n = 0;
      for (int split : cands) {
        std::vector<BlockTask> at;
        for (int i = 0; i < ng; ++i)
          append_tiles(at, i, al.bucket, level_at(B, P.probs[i], (int)d).hd.bk[al.bucket].count,
                       apply_block(split) / split);
        BlockTask* tasks = nullptr;
        int nt = 0;
        if ((result = upload(B, at, &tasks, &nt)) != RAV_OK) break;
        const int fac = level_at(B, P.probs[0], (int)d).hd.bk[al.bucket].factored;
        launch_rav_apply(B->dim, B->kind, al.cls, B->prec, split, P.dG, tasks, nt, B->stream, fac);
        (void)hipEventRecord(e0, B->stream);
        for (int r = 0; r < 3; ++r)
          launch_rav_apply(B->dim, B->kind, al.cls, B->prec, split, P.dG, tasks, nt, B->stream, fac);
        (void)hipEventRecord(e1, B->stream);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = 1e30f;
        if (ms < best) {
          if (best_tasks) (void)rav_dfree(best_tasks);
          best = ms; best_split = split; best_tasks = tasks; best_n = nt;
        } else {
          (void)rav_dfree(tasks);
        }
      }
      if (best_tasks) {
        (void)rav_dfree(al.tasks);
        al.tasks = best_tasks; al.ntasks = best_n; al.split = best_split;
      }
      B->apply_split_log.push_back(al.split);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  BCK(hipGetLastError());
  return result;
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
  if ((st = autotune_batch(B)) != RAV_OK) return st;
  if (B->cycle_exec) { (void)hipGraphExecDestroy(B->cycle_exec); B->cycle_exec = nullptr; }
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
    batch_solve_cycle(B);   // top residuals are current from the norm evaluation
    std::vector<double> nk;
    if ((st = read_norms(B, nk)) != RAV_OK) return st;
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

// Per-problem vector tiles of the batched Krylov kernels (built on first use).
static rav_status build_vector_tasks(rav_batch* B) {
  if (B->vtasks) return RAV_OK;
  std::vector<BlockTask> vt;
  std::vector<int> first, count;
  for (size_t p = 0; p < B->sub.size(); ++p) {
    first.push_back((int)vt.size());
    append_tiles(vt, (int)p, 0, B->n_fine[p], BV_TILE);
    count.push_back((int)vt.size() - first.back());
  }
  rav_status st = upload(B, vt, &B->vtasks, &B->n_vtasks);
  if (st != RAV_OK) return st;
  if ((st = upload_vec(B, first, &B->v_first)) != RAV_OK) return st;
  if ((st = upload_vec(B, count, &B->v_count)) != RAV_OK) return st;
  BCK(rav_dmalloc((void**)&B->v_partial, sizeof(double) * std::max<size_t>(vt.size(), 1)));
  return RAV_OK;
}

rav_status rav_batch_solve_gmres(rav_batch* B, double* const* x, const double* const* b, double rtol, int maxit,
                                 int restart, int* iters, double* rel_res) {
  if (!B || !x || !b || !(rtol > 0.0) || maxit < 0 || restart < 1 || restart > 200) return RAV_EINVAL;
  if (!B->factored) { B->err = "rav_batch_factor has not been called"; return RAV_EINVAL; }
  const int P = (int)B->sub.size();
  const int m = restart;
  for (int p = 0; p < P; ++p)
    if (!x[p] || !b[p]) return RAV_EINVAL;
  rav_status st = build_vector_tasks(B);
  if (st != RAV_OK) return st;
  hipStream_t s = B->stream;
  // work vectors of every problem in one allocation
  long long total = 0;
  std::vector<long long> off(P);
  for (int p = 0; p < P; ++p) { off[p] = total; total += (2LL * m + 3) * ((B->n_fine[p] + 31) / 32 * 32); }
  double* work = nullptr;
  double** tabs = nullptr;     // device pointer tables: V[i][p], Z[i][p], xk[p], bk[p], X[p], Bf[p], R[p]
  double *hdev = nullptr, *ydev = nullptr;
  int* jdev = nullptr;
  const long long ntab = (long long)P * (2LL * m + 6);
  auto cleanup = [&]() {
    (void)rav_dfree(work); (void)rav_dfree(tabs); (void)rav_dfree(hdev); (void)rav_dfree(ydev); (void)rav_dfree(jdev);
  };
  auto fail = [&](hipError_t e, const char* what) {
    B->err = std::string(what) + ": " + hipGetErrorString(e);
    cleanup();
    return e == hipErrorOutOfMemory ? RAV_ENOMEM : RAV_EDEVICE;
  };
  hipError_t e;
  if ((e = rav_dmalloc((void**)&work, sizeof(double) * std::max(total, 1LL))) != hipSuccess) return fail(e, "work");
  if ((e = rav_dmalloc((void**)&tabs, sizeof(double*) * ntab)) != hipSuccess) return fail(e, "tables");
  if ((e = rav_dmalloc((void**)&hdev, sizeof(double) * P * (m + 2) * (m + 1))) != hipSuccess) return fail(e, "h");
  if ((e = rav_dmalloc((void**)&ydev, sizeof(double) * P * m)) != hipSuccess) return fail(e, "y");
  if ((e = rav_dmalloc((void**)&jdev, sizeof(int) * P)) != hipSuccess) return fail(e, "jend");
  std::vector<double*> ht(ntab);
  double** const dV = tabs;                       // V_i of problem p at dV[i * P + p]
  double** const dZ = tabs + (long long)P * (m + 1);
  double** const dXk = dZ + (long long)P * m;
  double** const dBk = dXk + P;
  double** const dX = dBk + P;                     // finest-level x, b, r of each problem
  double** const dBf = dX + P;
  double** const dR = dBf + P;
  for (int p = 0; p < P; ++p) {
    const long long str = (B->n_fine[p] + 31) / 32 * 32;
    double* base = work + off[p];
    for (int i = 0; i <= m; ++i) ht[(long long)i * P + p] = base + i * str;
    for (int i = 0; i < m; ++i) ht[(long long)P * (m + 1) + (long long)i * P + p] = base + (m + 1 + i) * str;
    ht[(long long)P * (2 * m + 1) + p] = base + (2LL * m + 1) * str;
    ht[(long long)P * (2 * m + 2) + p] = base + (2LL * m + 2) * str;
    const GridDev& top = B->sub[p]->lv.back().hd;
    ht[(long long)P * (2 * m + 3) + p] = top.x;
    ht[(long long)P * (2 * m + 4) + p] = top.b;
    ht[(long long)P * (2 * m + 5) + p] = top.r;
  }
  if ((e = hipMemcpy(tabs, ht.data(), sizeof(double*) * ntab, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e, "tables");
  const BlockTask* vt = B->vtasks;
  const int nv = B->n_vtasks;
  const int* act = B->d_active;
  auto vec = [&](double** Y, double** X, const double* c, long long cstr, long long coff, double sign, int mode) {
    launch_bvec(vt, nv, Y, X, B->d_n, act, c, cstr, coff, sign, mode, s);
  };
  auto dot = [&](double** A, double** Bv, double* out, long long ostr, long long ooff, int sq) {
    launch_bdot(vt, nv, A, Bv, B->d_n, act, B->v_partial, B->v_first, B->v_count, P, out, ostr, ooff, sq, s);
  };
  // initial iterate and residual of every problem
  std::vector<int> on(P, 1);
  if ((st = set_active(B, on)) != RAV_OK) { cleanup(); return st; }
  if ((st = copy_user(B, ht.data() + (long long)P * (2 * m + 1), (const double* const*)x)) != RAV_OK) {
    cleanup(); return st;
  }
  if ((st = copy_user(B, ht.data() + (long long)P * (2 * m + 2), b)) != RAV_OK) { cleanup(); return st; }
  auto true_residuals = [&](std::vector<double>& out) -> rav_status {
    vec(dX, dXk, nullptr, 0, 0, 1.0, 2);
    vec(dBf, dBk, nullptr, 0, 0, 1.0, 2);
    return batch_norms(B, out);
  };
  std::vector<double> beta0, res;
  if ((st = true_residuals(beta0)) != RAV_OK) { cleanup(); return st; }
  res = beta0;
  std::vector<int> status(P, 1), it(P, 0);   // 1 = running, 0 = converged, -4 = diverged
  for (int p = 0; p < P; ++p) {
    if (!std::isfinite(beta0[p])) status[p] = -4;
    else if (beta0[p] == 0.0) status[p] = 0;
  }
  const long long hs = (long long)(m + 2) * (m + 1);   // Arnoldi coefficients per problem
  std::vector<double> H((size_t)P * (m + 1) * m), cs((size_t)P * m), sn((size_t)P * m), g((size_t)P * (m + 1)),
      y((size_t)P * m), hcol((size_t)P * (m + 2)), beta(P), binv(P);
  std::vector<int> jend(P, 0);
  bool first_cycle = true;
  while (true) {
    std::vector<int> cyc(P, 0);   // problems taking part in this restart cycle
    for (int p = 0; p < P; ++p) cyc[p] = status[p] == 1 && it[p] < maxit;
    if (std::count(cyc.begin(), cyc.end(), 1) == 0) break;
    if ((st = set_active(B, cyc)) != RAV_OK) { cleanup(); return st; }
    if (!first_cycle) {   // residuals of the updated iterates
      std::vector<double> rn;
      if ((st = true_residuals(rn)) != RAV_OK) { cleanup(); return st; }
      for (int p = 0; p < P; ++p) {
        if (!cyc[p]) continue;
        res[p] = rn[p];
        if (!std::isfinite(rn[p]) || rn[p] > 1e3 * beta0[p]) { status[p] = -4; cyc[p] = 0; }
        else if (rn[p] <= rtol * beta0[p]) { status[p] = 0; cyc[p] = 0; }
      }
      if (std::count(cyc.begin(), cyc.end(), 1) == 0) break;
      if ((st = set_active(B, cyc)) != RAV_OK) { cleanup(); return st; }
    }
    first_cycle = false;
    // V_0 = r / beta (beta = ||r||, per problem in ydev[p * m])
    for (int p = 0; p < P; ++p) {
      beta[p] = res[p];
      binv[p] = res[p] > 0.0 ? 1.0 / res[p] : 0.0;
      for (int i = 0; i <= m; ++i) g[(size_t)p * (m + 1) + i] = 0.0;
      g[(size_t)p * (m + 1)] = res[p];
      jend[p] = 0;
    }
    if ((e = hipMemcpy(ydev, binv.data(), sizeof(double) * P, hipMemcpyHostToDevice)) != hipSuccess)
      return fail(e, "scale");
    vec(dV, dR, ydev, 1, 0, 1.0, 2);
    std::vector<int> arn = cyc;   // still extending their Krylov basis
    for (int j = 0; j < m; ++j) {
      // Z_j = M V_j: one batched V-cycle from zero with b = V_j
      vec(dBf, dV + (long long)j * P, nullptr, 0, 0, 1.0, 2);
      vec(dX, dX, nullptr, 0, 0, 0.0, 3);
      batch_vcycle(B, false);
      vec(dZ + (long long)j * P, dX, nullptr, 0, 0, 1.0, 2);
      // w = L Z_j = -(0 - L Z_j)
      vec(dBf, dBf, nullptr, 0, 0, 0.0, 3);
      batch_top_residual(B, false);
      double** W = dV + (long long)(j + 1) * P;
      vec(W, dR, nullptr, 0, 0, -1.0, 2);
      for (int i = 0; i <= j; ++i) {
        dot(W, dV + (long long)i * P, hdev, hs, (long long)j * (m + 2) + i, 0);
        vec(W, dV + (long long)i * P, hdev, hs, (long long)j * (m + 2) + i, -1.0, 0);
      }
      dot(W, W, hdev, hs, (long long)j * (m + 2) + j + 1, 1);
      vec(W, W, hdev, hs, (long long)j * (m + 2) + j + 1, 1.0, 1);
      if ((e = hipGetLastError()) != hipSuccess) return fail(e, "arnoldi");
      if ((e = hipMemcpy2DAsync(hcol.data(), sizeof(double) * (m + 2), hdev + (long long)j * (m + 2),
                                sizeof(double) * hs, sizeof(double) * (j + 2), P, hipMemcpyDeviceToHost, s)) !=
          hipSuccess)
        return fail(e, "readback");
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "sync");
      bool changed = false;
      for (int p = 0; p < P; ++p) {
        if (!arn[p]) continue;
        double* Hp = H.data() + (size_t)p * (m + 1) * m;
        double* c = cs.data() + (size_t)p * m;
        double* sv = sn.data() + (size_t)p * m;
        double* gp = g.data() + (size_t)p * (m + 1);
        const double* hc = hcol.data() + (size_t)p * (m + 2);
        ++it[p];
        for (int i = 0; i <= j + 1; ++i) Hp[(size_t)i * m + j] = hc[i];
        for (int i = 0; i < j; ++i) {
          const double a = Hp[(size_t)i * m + j], cc = Hp[(size_t)(i + 1) * m + j];
          Hp[(size_t)i * m + j] = c[i] * a + sv[i] * cc;
          Hp[(size_t)(i + 1) * m + j] = -sv[i] * a + c[i] * cc;
        }
        const double a = Hp[(size_t)j * m + j], cc = Hp[(size_t)(j + 1) * m + j];
        const double rr = std::hypot(a, cc);
        c[j] = rr > 0.0 ? a / rr : 1.0;
        sv[j] = rr > 0.0 ? cc / rr : 0.0;
        Hp[(size_t)j * m + j] = rr;
        Hp[(size_t)(j + 1) * m + j] = 0.0;
        gp[j + 1] = -sv[j] * gp[j];
        gp[j] = c[j] * gp[j];
        res[p] = std::fabs(gp[j + 1]);
        jend[p] = j + 1;
        if (!std::isfinite(res[p])) { status[p] = -4; arn[p] = 0; changed = true; continue; }
        if (res[p] <= rtol * beta0[p] || hc[j + 1] == 0.0 || it[p] >= maxit) { arn[p] = 0; changed = true; }
      }
      if (std::count(arn.begin(), arn.end(), 1) == 0) break;
      if (changed && (st = set_active(B, arn)) != RAV_OK) { cleanup(); return st; }
    }
    // x += Z y with y = R^{-1} g, per problem
    for (int p = 0; p < P; ++p) {
      if (!cyc[p] || status[p] == -4) { jend[p] = 0; continue; }
      const double* Hp = H.data() + (size_t)p * (m + 1) * m;
      const double* gp = g.data() + (size_t)p * (m + 1);
      double* yp = y.data() + (size_t)p * m;
      for (int i = jend[p] - 1; i >= 0; --i) {
        double t = gp[i];
        for (int k = i + 1; k < jend[p]; ++k) t -= Hp[(size_t)i * m + k] * yp[k];
        yp[i] = Hp[(size_t)i * m + i] != 0.0 ? t / Hp[(size_t)i * m + i] : 0.0;
      }
    }
    if ((e = hipMemcpy(ydev, y.data(), sizeof(double) * P * m, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(jdev, jend.data(), sizeof(int) * P, hipMemcpyHostToDevice)) != hipSuccess)
      return fail(e, "update");
    launch_bupdate(vt, nv, dXk, dZ, P, m, B->d_n, jdev, ydev, s);
  }
  // results: x = xk for every problem
  if ((st = set_active(B, on)) != RAV_OK) { cleanup(); return st; }
  if ((st = copy_user(B, const_cast<double* const*>(x), (const double* const*)(ht.data() + (long long)P * (2 * m + 1)))) !=
      RAV_OK) {
    cleanup(); return st;
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e, "sync");
  rav_status result = RAV_OK;
  for (int p = 0; p < P; ++p) {
    if (iters) iters[p] = it[p];
    if (rel_res) rel_res[p] = beta0[p] > 0.0 ? res[p] / beta0[p] : 0.0;
    if (status[p] == -4) result = RAV_EDIVERGED;
    else if (status[p] == 1 && result == RAV_OK) result = RAV_NOT_CONVERGED;
  }
  if (result == RAV_EDIVERGED) B->err = "at least one problem diverged";
  cleanup();
  return result;
}

rav_status rav_batch_destroy(rav_batch* B) {
  if (!B) return RAV_OK;
  (void)hipStreamSynchronize(B->stream);
  for (DepthPlan& P : B->depth) {
    (void)rav_dfree(P.dG); (void)rav_dfree(P.res); (void)rav_dfree(P.rtask); (void)rav_dfree(P.ptask);
    (void)rav_dfree(P.top_res); (void)rav_dfree(P.partials); (void)rav_dfree(P.first); (void)rav_dfree(P.count);
    (void)rav_dfree(P.pid); (void)rav_dfree(P.coarse);
    for (ApplyLaunch& a : P.apply) (void)rav_dfree(a.tasks);
  }
  if (B->cycle_exec) (void)hipGraphExecDestroy(B->cycle_exec);
  (void)rav_dfree(B->vtasks); (void)rav_dfree(B->v_first); (void)rav_dfree(B->v_count); (void)rav_dfree(B->v_partial);
  for (rav_ctx* c : B->sub) rav_destroy(c);
  (void)rav_dfree(B->d_active); (void)rav_dfree(B->d_norm2); (void)rav_dfree(B->d_dst); (void)rav_dfree((void*)B->d_src);
  (void)rav_dfree(B->d_n); (void)rav_dfree(B->copy_tasks);
  if (B->h_norm2) (void)hipHostFree(B->h_norm2);
  delete B;
  return RAV_OK;
}

const char* rav_batch_last_error(const rav_batch* B) { return B ? B->err.c_str() : g_batch_error.c_str(); }

rav_status rav_create_batch(const rav_problem_desc* descs, int n, void* hip_stream, rav_batch** out) {
  return rav_batch_create(descs, n, hip_stream, out);
}

rav_status rav_solve_batch(rav_batch* B, double* const* x, const double* const* b, double rtol, int maxit,
                           int* iters, double* rel_res) {
  return rav_batch_solve(B, x, b, rtol, maxit, iters, rel_res);
}

}  // extern "C"
