// Host driver and C-ABI of the RAV multigrid library.
//
// Builds the uniform level hierarchy (Sec. 2), uploads one GridDev
// descriptor per level, and orders every step of a V-cycle (Fig. 1) on the
// caller's stream: smoothing (Sec. 3, eqs. 10-13), residual, restriction,
// recursion, coarse direct solve, prolongation.  The solve loop reads back one
// FP64 norm per cycle for the stopping test (Sec. 4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rav_ctx.h"

using namespace rav;

namespace {
std::string g_create_error;
}  // namespace

#define CK(expr)                                                                     \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                  \
      return e_ == hipErrorOutOfMemory ? RAV_ENOMEM : RAV_EDEVICE;                   \
    }                                                                                \
  } while (0)

namespace {

// ---- reference-element tables from the Lagrange bases ----------------------
void q2(double t, double* v) { v[0] = (1 - t) * (1 - 2 * t); v[1] = 4 * t * (1 - t); v[2] = t * (2 * t - 1); }
void dq2(double t, double* v) { v[0] = 4 * t - 3; v[1] = 4 - 8 * t; v[2] = 4 * t - 1; }

RefTables make_tables() {
  RefTables T{};
  T.gt[0] = 0.5 - 0.5 * std::sqrt(0.6); T.gt[1] = 0.5; T.gt[2] = 0.5 + 0.5 * std::sqrt(0.6);
  T.gw[0] = 5.0 / 18.0; T.gw[1] = 8.0 / 18.0; T.gw[2] = 5.0 / 18.0;
  for (int q = 0; q < 3; ++q) {
    double v[3], dv[3];
    q2(T.gt[q], v);
    dq2(T.gt[q], dv);
    for (int a = 0; a < 3; ++a) { T.phi[a][q] = v[a]; T.dphi[a][q] = dv[a]; }
    T.psi[0][q] = 1 - T.gt[q];
    T.psi[1][q] = T.gt[q];
  }
  // 2D and 3D reference stiffness (h = 1) and divergence tables.
  for (int dim = 2; dim <= 3; ++dim) {
    const int nv = dim == 2 ? 9 : 27, np = dim == 2 ? 4 : 8, nq = nv;
    for (int a = 0; a < nv; ++a)
      for (int b = 0; b < nv; ++b) {
        double s = 0.0;
        for (int q = 0; q < nq; ++q) {
          int ia[3] = {a % 3, (a / 3) % 3, a / 9}, ib[3] = {b % 3, (b / 3) % 3, b / 9}, iq[3] = {q % 3, (q / 3) % 3, q / 9};
          double w = 1.0, gg = 0.0;
          for (int d = 0; d < dim; ++d) w *= T.gw[iq[d]];
          for (int c = 0; c < dim; ++c) {
            double p = 1.0;
            for (int d = 0; d < dim; ++d)
              p *= (d == c) ? T.dphi[ia[d]][iq[d]] * T.dphi[ib[d]][iq[d]] : T.phi[ia[d]][iq[d]] * T.phi[ib[d]][iq[d]];
            gg += p;
          }
          s += w * gg;
        }
        if (dim == 2) T.aref2[a][b] = s; else T.aref3[a][b] = s;
      }
    for (int c = 0; c < dim; ++c)
      for (int a = 0; a < nv; ++a)
        for (int k = 0; k < np; ++k) {
          double s = 0.0;
          for (int q = 0; q < nq; ++q) {
            int ia[3] = {a % 3, (a / 3) % 3, a / 9}, ik[3] = {k & 1, (k >> 1) & 1, k >> 2},
                iq[3] = {q % 3, (q / 3) % 3, q / 9};
            double w = 1.0, ps = 1.0, dphi = 1.0;
            for (int d = 0; d < dim; ++d) {
              w *= T.gw[iq[d]];
              ps *= T.psi[ik[d]][iq[d]];
              dphi *= (d == c) ? T.dphi[ia[d]][iq[d]] : T.phi[ia[d]][iq[d]];
            }
            s += w * ps * dphi;
          }
          if (dim == 2) T.bref2[c][a][k] = -s; else T.bref3[c][a][k] = -s;
        }
  }
  return T;
}

}  // namespace

namespace rav {
std::vector<BlockTask> xcd_order(const std::vector<BlockTask>& logical) {
  const size_t T = (logical.size() + 7) / 8 * 8;
  std::vector<BlockTask> out(T);
  for (size_t b = 0; b < T; ++b) {
    const size_t l = (b % 8) * (T / 8) + b / 8;
    if (l < logical.size()) out[b] = logical[l];
    else { out[b].grid = -1; out[b].part = 0; out[b].start = 0; out[b].logical = 0; out[b].pad = 0; }
  }
  return out;
}

void append_tiles(std::vector<BlockTask>& out, int grid, int part, long long n, int per_block) {
  for (long long s0 = 0; s0 < n; s0 += per_block) {
    BlockTask t{};
    t.grid = grid; t.part = part; t.start = s0; t.logical = (int)out.size();
    out.push_back(t);
  }
}

void append_residual_tiles(std::vector<BlockTask>& out, int grid, const Geo& g) {
  // Tiles of all node types are ordered by the half-grid row (then plane) of
  // their first row, so the contiguous tile range an XCD receives covers one
  // band of the grid for every type and the band of x stays in that XCD's L2.
  struct Keyed { long long key; BlockTask t; };
  std::vector<Keyed> kt;
  const int np = (1 << g.dim) + 1;
  for (int part = 0; part < np; ++part) {
    const bool pres = part == (1 << g.dim);
    const long long rows = pres ? g.nP : seg_rows(g, part);
    for (long long r0 = 0; r0 < rows; r0 += BLOCK) {
      int a[3] = {0, 0, 0};
      if (pres) {
        vert_of(g, r0, a);
        for (int d = 0; d < g.dim; ++d) a[d] *= 2;
      } else {
        vel_row_node(g, part, r0, a);
      }
      const long long key = ((long long)a[2] * (2 * g.N + 1) + a[1]) * 16 + part;
      BlockTask t{};
      t.grid = grid; t.part = part; t.start = r0;
      kt.push_back({key, t});
    }
  }
  std::stable_sort(kt.begin(), kt.end(), [](const Keyed& x, const Keyed& y) { return x.key < y.key; });
  for (Keyed& k : kt) {
    k.t.logical = (int)out.size();
    out.push_back(k.t);
  }
}
}  // namespace rav

rav_status rav_set_error(rav_ctx* ctx, rav_status st, const std::string& msg) {
  if (ctx) ctx->err = msg; else g_create_error = msg;
  return st;
}

static rav_status set_err(rav_ctx* ctx, rav_status st, const std::string& msg) { return rav_set_error(ctx, st, msg); }

// Status word, norm buffers (device and pinned host) and the inclusion table.
// ---- device memory ------------------------------------------------------------
std::atomic<long> rav_live_objects{0};

namespace {
struct DeviceAllocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*release)(void*, void*) = nullptr;
  void* user = nullptr;
};
DeviceAllocator g_alloc;
std::mutex g_alloc_mutex;
}  // namespace

hipError_t rav_dmalloc(void** p, size_t bytes) {
  if (!g_alloc.alloc) return hipMalloc(p, bytes);
  *p = nullptr;
  if (bytes == 0) return hipSuccess;   // as hipMalloc
  *p = g_alloc.alloc(bytes, g_alloc.user);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

hipError_t rav_dfree(void* p) {
  if (!p) return hipSuccess;
  if (!g_alloc.release) return hipFree(p);
  g_alloc.release(p, g_alloc.user);
  return hipSuccess;
}

rav_status rav_init_common(rav_ctx* ctx, const rav_problem_desc* d) {
  CK(rav_dmalloc((void**)&ctx->d_status, sizeof(int)));
  CK(rav_dmalloc((void**)&ctx->d_norm, sizeof(double)));
  CK(hipHostMalloc((void**)&ctx->h_norm, sizeof(double), hipHostMallocDefault));
  CK(hipHostGetDevicePointer((void**)&ctx->h_norm_dev, ctx->h_norm, 0));
  std::vector<double> inc(4 * std::max(d->n_incl, 1), 0.0);
  for (int i = 0; i < d->n_incl; ++i) {
    const rav_inclusion& c = d->incl[i];
    inc[4 * i + 0] = c.cx; inc[4 * i + 1] = c.cy; inc[4 * i + 2] = c.cz; inc[4 * i + 3] = c.r;
  }
  CK(rav_dmalloc((void**)&ctx->d_incl, sizeof(double) * inc.size()));
  CK(hipMemcpy(ctx->d_incl, inc.data(), sizeof(double) * inc.size(), hipMemcpyHostToDevice));
  return RAV_OK;
}

rav_status rav_upload_tasks(rav_ctx* ctx, const std::vector<BlockTask>& logical, BlockTask** out, int* n) {
  std::vector<BlockTask> t = xcd_order(logical);
  *n = (int)t.size();
  CK(rav_dmalloc((void**)out, sizeof(BlockTask) * std::max<size_t>(t.size(), 1)));
  CK(hipMemcpy(*out, t.data(), sizeof(BlockTask) * t.size(), hipMemcpyHostToDevice));
  return RAV_OK;
}

rav_status rav_upload_desc(rav_ctx* ctx, LevelHost& L) {
  CK(hipStreamSynchronize(ctx->stream));
  CK(hipMemcpy(L.dd, &L.hd, sizeof(GridDev), hipMemcpyHostToDevice));
  return RAV_OK;
}

// Apply tiles of one bucket for the given lanes-per-patch variant.
static rav_status make_apply_tasks(rav_ctx* ctx, ApplyLaunch& al, long long count, int split) {
  const int per_block = apply_block(split) / split;
  std::vector<BlockTask> at;
  for (long long p0 = 0; p0 < count; p0 += per_block) {
    BlockTask t{};
    t.grid = 0; t.part = al.bucket; t.start = p0; t.logical = (int)at.size();
    at.push_back(t);
  }
  al.split = split;
  return rav_upload_tasks(ctx, at, &al.tasks, &al.ntasks);
}

static rav_status build_level(rav_ctx* ctx, int l) {
  const rav_problem_desc& D = ctx->desc;
  LevelHost& L = ctx->lv[l];
  const int N = D.n_cells >> (D.n_levels - 1 - l);
  GridDev& h = L.hd;
  std::memset(&h, 0, sizeof(GridDev));
  h.g = make_geo(D.dim, N, D.bc_dirichlet_mask);
  h.kind = D.patch;
  h.h = 1.0 / N;
  h.omega = D.omega;
  const Geo& g = h.g;
  const int nseg = n_segments(D.dim);
  long long off = 0;
  for (int s = 0; s < nseg; ++s) {
    h.seg_off[s] = off;
    h.seg_rows[s] = seg_rows(g, s);
    off += h.seg_rows[s] * seg_slots(D.dim, s);
  }
  L.nvals = off;
  CK(rav_dmalloc((void**)&h.x, sizeof(double) * g.n));
  CK(rav_dmalloc((void**)&h.b, sizeof(double) * g.n));
  CK(rav_dmalloc((void**)&h.r, sizeof(double) * g.n));
  CK(rav_dmalloc((void**)&h.vals, sizeof(double) * off));
  CK(hipMemsetAsync(h.x, 0, sizeof(double) * g.n, ctx->stream));
  CK(hipMemsetAsync(h.b, 0, sizeof(double) * g.n, ctx->stream));
  CK(hipMemsetAsync(h.r, 0, sizeof(double) * g.n, ctx->stream));
  CK(rav_dmalloc((void**)&L.dd, sizeof(GridDev)));
  L.npatch = n_patches(g, D.patch);
  std::vector<BlockTask> tiles;
  append_residual_tiles(tiles, 0, g);
  L.n_res_tiles = (int)tiles.size();
  rav_status st = rav_upload_tasks(ctx, tiles, &L.res_tasks, &L.n_res_tasks);
  if (st != RAV_OK) return st;
  if (l > 0) {
    const Geo gc = make_geo(D.dim, N / 2, D.bc_dirichlet_mask);
    std::vector<BlockTask> rt, pt;
    append_residual_tiles(rt, 0, gc);
    append_residual_tiles(pt, 0, g);
    st = rav_upload_tasks(ctx, rt, &L.rtasks, &L.n_rtasks);
    if (st != RAV_OK) return st;
    st = rav_upload_tasks(ctx, pt, &L.ptasks, &L.n_ptasks);
    if (st != RAV_OK) return st;
  }
  const int n_part = std::max(L.n_res_tiles, residual_tiled_ok(D.dim, N) ? residual_tiles(D.dim, N) : 1);
  CK(rav_dmalloc((void**)&L.partials, sizeof(double) * n_part));
  // patch buckets (smoothed levels only)
  if (l > 0) {
    const int nbk = n_buckets(D.dim, D.patch);
    for (int m = 0; m < nbk; ++m) {
      const long long cnt = bucket_count(g, D.patch, m);
      if (cnt <= 0) continue;
      Bucket& B = h.bk[h.nbk];
      B.cls = D.patch == KIND_VERTEX ? 0 : m;
      B.nown = bucket_nown(D.dim, D.patch, B.cls);
      B.count = cnt;
      B.count_pad = (cnt + 63) / 64 * 64;
      B.factored = D.inv_format == RAV_FACTORED ? 1 : 0;
      ApplyLaunch al;
      al.bucket = h.nbk;
      al.cls = B.cls;
      int split = apply_split(cnt, ctx->split_below);
      if (B.factored && split == APPLY_ROWS) split = APPLY_SPLIT_SMALL;   // no row-parallel factored kernel
      st = make_apply_tasks(ctx, al, cnt, split);
      if (st != RAV_OK) return st;
      L.apply.push_back(al);
      ++h.nbk;
    }
  }
  // operator assembly on the device
  st = rav_upload_desc(ctx, L);
  if (st != RAV_OK) return st;
  const long long ncell = (long long)N * N * (D.dim == 3 ? N : 1);
  double* etaq = nullptr;
  unsigned char* uni = nullptr;
  CK(rav_dmalloc((void**)&etaq, sizeof(double) * ncell * (D.dim == 2 ? 9 : 27)));
  CK(rav_dmalloc((void**)&uni, ncell));
  std::vector<BlockTask> at;
  for (int s = 0; s < nseg; ++s)
    for (long long r0 = 0; r0 < h.seg_rows[s]; r0 += BLOCK) {
      BlockTask t{};
      t.grid = 0; t.part = s; t.start = r0; t.logical = (int)at.size();
      at.push_back(t);
    }
  BlockTask* atd = nullptr;
  int natd = 0;
  st = rav_upload_tasks(ctx, at, &atd, &natd);
  if (st != RAV_OK) return st;
  // Galerkin coarse operators: cell integrals by the finest grid's Gauss points
  const int R = D.coarse_galerkin ? (1 << (D.n_levels - 1 - l)) : 1;
  launch_eta(D.dim, ncell, L.dd, ctx->d_incl, D.n_incl, D.eta_out, D.eta_in, R, etaq, uni, ctx->stream);
  CK(hipGetLastError());
  CK(hipStreamSynchronize(ctx->stream));
  // cells cut by an inclusion keep their full viscous cell matrix (matrix-free
  // residual and operator assembly); the others one coefficient
  std::vector<unsigned char> hu(ncell);
  CK(hipMemcpy(hu.data(), uni, ncell, hipMemcpyDeviceToHost));
  std::vector<int> cut_idx(ncell, -1), cut_cells;
  for (long long e = 0; e < ncell; ++e)
    if (!hu[e]) { cut_idx[e] = (int)cut_cells.size(); cut_cells.push_back((int)e); }
  L.ncut = (long long)cut_cells.size();
  const long long nv2 = D.dim == 2 ? 81 : 729;
  int *d_cut_idx = nullptr, *d_cut_cells = nullptr;
  CK(rav_dmalloc((void**)&L.ceta, sizeof(double) * ncell));
  CK(rav_dmalloc((void**)&L.cutA, sizeof(double) * std::max<long long>(L.ncut * nv2, 1)));
  CK(rav_dmalloc((void**)&d_cut_idx, sizeof(int) * ncell));
  CK(rav_dmalloc((void**)&d_cut_cells, sizeof(int) * std::max<long long>(L.ncut, 1)));
  CK(hipMemcpy(d_cut_idx, cut_idx.data(), sizeof(int) * ncell, hipMemcpyHostToDevice));
  if (L.ncut) CK(hipMemcpy(d_cut_cells, cut_cells.data(), sizeof(int) * L.ncut, hipMemcpyHostToDevice));
  launch_cell_coef(D.dim, ncell, L.dd, etaq, d_cut_idx, d_cut_cells, (int)L.ncut, R, ctx->d_incl, D.n_incl,
                   D.eta_out, D.eta_in, L.ceta, L.cutA, ctx->stream);
  launch_assemble(D.dim, L.dd, atd, natd, etaq, uni, d_cut_idx, L.cutA, ctx->stream);
  CK(hipGetLastError());
  CK(hipStreamSynchronize(ctx->stream));
  CK(rav_dfree(d_cut_idx));
  CK(rav_dfree(d_cut_cells));
  CK(rav_dfree(etaq));
  CK(rav_dfree(uni));
  CK(rav_dfree(atd));
  h.ceta = L.ceta;
  h.cutA = L.cutA;
  return rav_upload_desc(ctx, L);
}

// Coarsest level, part 1: the dense (bordered) matrix in ctx->Minv, not yet inverted.
static rav_status build_coarse_matrix(rav_ctx* ctx) {
  LevelHost& L = ctx->lv[0];
  const Geo& g = L.hd.g;
  bool all_dir = true;
  for (int b = 0; b < 2 * g.dim; ++b) all_dir = all_dir && ((g.dmask >> b) & 1u);
  ctx->bordered = all_dir ? 1 : 0;
  ctx->nb = g.n + ctx->bordered;
  const long long nb = ctx->nb;
  if (nb > MAX_COARSE)
    return set_err(ctx, RAV_EINVAL, "the coarsest grid has " + std::to_string(nb) + " unknowns; its dense direct "
                   "solve is limited to " + std::to_string(MAX_COARSE) + " (use more levels)");
  CK(rav_dmalloc((void**)&ctx->Minv, sizeof(double) * nb * nb));
  launch_coarse_build(L.dd, g.dim, ctx->Minv, nb, ctx->bordered, 1, ctx->stream);
  CK(hipGetLastError());
  return RAV_OK;
}

// Part 2, after the inversion: zero-pivot check, the coarse solve's tasks and descriptor.
rav_status rav_finish_coarse(rav_ctx* ctx, int pivot_status) {
  if (pivot_status != INT_MAX)
    return set_err(ctx, RAV_ESINGULAR, "zero pivot in the coarse matrix at column " + std::to_string(pivot_status));
  LevelHost& L = ctx->lv[0];
  L.hd.Minv = ctx->Minv;
  L.hd.nbc = ctx->nb;
  std::vector<BlockTask> ct;
  append_tiles(ct, 0, 0, L.hd.g.n, 4);
  rav_status rs = rav_upload_tasks(ctx, ct, &ctx->coarse_tasks, &ctx->n_coarse_tasks);
  if (rs != RAV_OK) return rs;
  return rav_upload_desc(ctx, L);
}

// Blocked Gauss-Jordan inversion of the coarse matrices of n contexts (same nb).
rav_status rav_invert_coarse(rav_ctx* const* ctxs, int n, hipStream_t s, std::vector<int>* status_out,
                             std::string* err) {
  const long long nb = ctxs[0]->nb;
  double** dM = nullptr;
  int *piv = nullptr, *perm = nullptr, *st = nullptr;
  double *colk = nullptr, *Rs = nullptr;
  rav_status result = RAV_OK;
  auto chk = [&](hipError_t e) {
    if (e != hipSuccess && result == RAV_OK) {
      *err = std::string("coarse inversion: ") + hipGetErrorString(e);
      result = e == hipErrorOutOfMemory ? RAV_ENOMEM : RAV_EDEVICE;
    }
    return e == hipSuccess;
  };
  std::vector<double*> hM(n);
  for (int i = 0; i < n; ++i) hM[i] = ctxs[i]->Minv;
  std::vector<int> big(n, INT_MAX);
  if (chk(rav_dmalloc((void**)&dM, sizeof(double*) * n)) && chk(rav_dmalloc((void**)&piv, sizeof(int) * n * nb)) &&
      chk(rav_dmalloc((void**)&perm, sizeof(int) * n * nb)) && chk(rav_dmalloc((void**)&st, sizeof(int) * n)) &&
      chk(rav_dmalloc((void**)&colk, sizeof(double) * n * nb)) &&
      chk(rav_dmalloc((void**)&Rs, sizeof(double) * n * GJ_PANEL * nb)) &&
      chk(hipMemcpy(dM, hM.data(), sizeof(double*) * n, hipMemcpyHostToDevice)) &&
      chk(hipMemcpy(st, big.data(), sizeof(int) * n, hipMemcpyHostToDevice))) {
    launch_bgj_invert(dM, nb, n, piv, colk, Rs, perm, st, s);
    if (chk(hipGetLastError()) && chk(hipStreamSynchronize(s))) {
      status_out->assign(n, INT_MAX);
      chk(hipMemcpy(status_out->data(), st, sizeof(int) * n, hipMemcpyDeviceToHost));
    }
  }
  (void)rav_dfree(dM); (void)rav_dfree(piv); (void)rav_dfree(perm); (void)rav_dfree(st); (void)rav_dfree(colk);
  (void)rav_dfree(Rs);
  return result;
}

static rav_status build_coarse(rav_ctx* ctx, bool invert) {
  rav_status st = build_coarse_matrix(ctx);
  if (st != RAV_OK || !invert) return st;
  std::vector<int> piv_status;
  st = rav_invert_coarse(&ctx, 1, ctx->stream, &piv_status, &ctx->err);
  if (st != RAV_OK) return st;
  return rav_finish_coarse(ctx, piv_status[0]);
}

// ---- device sequences -------------------------------------------------------
void rav_residual_level(rav_ctx* ctx, int l, bool with_norm) {
  LevelHost& L = ctx->lv[l];
  const int N = L.hd.g.N;
  if (residual_tiled_ok(ctx->desc.dim, N)) {
    launch_residual_tiled(ctx->desc.dim, L.dd, N, with_norm ? L.partials : nullptr, ctx->stream);
    if (with_norm) launch_norm_finalize(L.partials, 0, residual_tiles(ctx->desc.dim, N), ctx->d_norm, ctx->h_norm_dev,
                                         ctx->stream);
    return;
  }
  launch_residual(ctx->desc.dim, L.dd, L.res_tasks, L.n_res_tasks, with_norm ? L.partials : nullptr, ctx->stream);
  if (with_norm) launch_norm_finalize(L.partials, 0, L.n_res_tiles, ctx->d_norm, ctx->h_norm_dev, ctx->stream);
}

static bool prof_mark(rav_ctx* ctx, int l, std::vector<hipEvent_t>& ev, int& n, bool start) {
  if (ctx->prof_level != l) return false;
  if (ctx->prof_capture) {   // markers inside the profiled cycle graph
    const bool res = &ev == &ctx->prof_res;
    std::vector<hipEvent_t>& gev = res ? ctx->gprof_res : ctx->gprof_app;
    int& gn = res ? ctx->gprof_nres : ctx->gprof_napp;
    if (start) {
      while ((int)gev.size() < 2 * (gn + 1)) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return false;
        gev.push_back(e);
      }
      (void)hipEventRecord(gev[2 * gn], ctx->stream);
    } else {
      (void)hipEventRecord(gev[2 * gn + 1], ctx->stream);
      ++gn;
    }
    return true;
  }
  if (start) {
    if (n >= ctx->prof_max) return false;
    (void)hipEventRecord(ev[2 * n], ctx->stream);
  } else {
    (void)hipEventRecord(ev[2 * n + 1], ctx->stream);
    ++n;
  }
  return true;
}

void rav_apply_level(rav_ctx* ctx, int l) {
  LevelHost& L = ctx->lv[l];
  const rav_problem_desc& D = ctx->desc;
  const bool timed = prof_mark(ctx, l, ctx->prof_app, ctx->prof_napp, true);
  if (D.smoother == RAV_SMOOTHER_RAV) {
    for (const ApplyLaunch& al : L.apply)
      if (!al.merged)
        launch_rav_apply(D.dim, D.patch, al.cls, ctx->prec, al.split, L.dd, al.tasks, al.ntasks, ctx->stream,
                         L.hd.bk[al.bucket].factored);
    if (L.n_multi > 0)
      launch_rav_apply_multi(D.dim, D.patch, ctx->prec, L.multi_edges, L.dd, L.multi_tasks, L.n_multi, ctx->stream);
  } else if (D.smoother == RAV_SMOOTHER_AV) {
    launch_av_apply(D.dim, D.patch, L.dd, L.npatch, ctx->stream);
    launch_av_gather(D.dim, D.patch, L.dd, L.hd.g.n, ctx->stream);
  }
  if (timed) prof_mark(ctx, l, ctx->prof_app, ctx->prof_napp, false);
}

static void mv_sweep(rav_ctx* ctx, int l) {
  LevelHost& L = ctx->lv[l];
  const rav_problem_desc& D = ctx->desc;
  const Geo& g = L.hd.g;
  const int M = colour_modulus(D.patch);
  const int ext = D.patch == KIND_VERTEX ? g.N + 1 : g.N;
  int ncol = 1;
  for (int d = 0; d < D.dim; ++d) ncol *= M;
  for (int col = 0; col < ncol; ++col) {
    long long cnt = 1;
    int cc = col;
    for (int d = 0; d < D.dim; ++d) {
      const int cd = cc % M;
      cc /= M;
      cnt *= std::max(0, (ext - cd + M - 1) / M);
    }
    launch_mv_colour(D.dim, D.patch, L.dd, col, cnt, ctx->stream);
  }
}

// `r_valid`: the level's r already holds b - L x for the current x (after a
// norm evaluation, or after restriction onto the level); the first sweep then
// skips its residual launch.  Returns whether r is still current afterwards.
static bool smooth_level(rav_ctx* ctx, int l, int sweeps, bool r_valid) {
  for (int s = 0; s < sweeps; ++s) {
    if (ctx->desc.smoother == RAV_SMOOTHER_MV) {
      mv_sweep(ctx, l);
    } else {
      if (!r_valid) {
        const bool timed = prof_mark(ctx, l, ctx->prof_res, ctx->prof_nres, true);
        rav_residual_level(ctx, l, false);
        if (timed) prof_mark(ctx, l, ctx->prof_res, ctx->prof_nres, false);
      }
      rav_apply_level(ctx, l);
    }
    r_valid = false;
  }
  return r_valid;
}

static void coarse_solve_level(rav_ctx* ctx) {
  launch_coarse_gemv_batch(ctx->lv[0].dd, ctx->coarse_tasks, ctx->n_coarse_tasks, ctx->stream);
}

// One V-cycle on level l; r_valid as for smooth_level (levels below the top
// are entered through restriction, which leaves their residual current).
static void vcycle_level(rav_ctx* ctx, int l, bool r_valid) {
  if (l == 0) { coarse_solve_level(ctx); return; }
  LevelHost& L = ctx->lv[l];
  if (!smooth_level(ctx, l, ctx->desc.nu_pre, r_valid)) rav_residual_level(ctx, l, false);
  launch_restrict(ctx->desc.dim, L.dd, L.rtasks, L.n_rtasks, ctx->stream);
  vcycle_level(ctx, l - 1, true);
  launch_prolong(ctx->desc.dim, L.dd, L.ptasks, L.n_ptasks, ctx->stream);
  smooth_level(ctx, l, ctx->desc.nu_post, false);
}

void rav_vcycle_finest(rav_ctx* ctx) { vcycle_level(ctx, (int)ctx->lv.size() - 1, false); }

void rav_drop_graph(rav_ctx* ctx) {
  if (ctx->cycle_exec) (void)hipGraphExecDestroy(ctx->cycle_exec);
  if (ctx->prof_exec) (void)hipGraphExecDestroy(ctx->prof_exec);
  if (ctx->pc_exec) (void)hipGraphExecDestroy(ctx->pc_exec);
  ctx->cycle_exec = ctx->prof_exec = ctx->pc_exec = nullptr;
  ctx->prof_exec_level = -1;
}

// Issues `issue(ctx)` on the context stream: captured into a graph on first
// use and replayed afterwards (RAV_GRAPH=0 in the environment, or a failed
// capture, issues the launches directly).
void rav_graph_cycle(rav_ctx* ctx, void (*issue)(rav_ctx*)) { rav_graph_issue(ctx, issue, &ctx->cycle_exec); }

void rav_graph_issue(rav_ctx* ctx, void (*issue)(rav_ctx*), hipGraphExec_t* slot) {
  static const bool graphs = [] {
    const char* e = std::getenv("RAV_GRAPH");
    return !(e && std::string(e) == "0");
  }();
  if (graphs && !ctx->graph_failed) {
    if (!*slot) {
      hipGraph_t g = nullptr;
      bool ok = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        issue(ctx);
        ok = hipStreamEndCapture(ctx->stream, &g) == hipSuccess && g != nullptr;
      }
      if (ok) ok = hipGraphInstantiate(slot, g, nullptr, nullptr, 0) == hipSuccess;
      if (g) (void)hipGraphDestroy(g);
      if (!ok) {
        (void)hipGetLastError();
        *slot = nullptr;
        ctx->graph_failed = true;
      }
    }
    if (*slot && hipGraphLaunch(*slot, ctx->stream) == hipSuccess) return;
    (void)hipGetLastError();
    rav_drop_graph(ctx);
    ctx->graph_failed = true;
  }
  issue(ctx);
}

// One solve cycle: V-cycle from a current finest residual, then the new
// finest residual and its squared norm in d_norm.  Replayed from a graph when
// possible; with profiling markers active (their events count launches on the
// host) the launches are issued directly.
static bool capture_cycle(rav_ctx* ctx, hipGraphExec_t* out) {
  const int lf = (int)ctx->lv.size() - 1;
  hipGraph_t g = nullptr;
  bool ok = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    vcycle_level(ctx, lf, true);
    rav_residual_level(ctx, lf, true);
    ok = hipStreamEndCapture(ctx->stream, &g) == hipSuccess && g != nullptr;
  }
  if (ok) ok = hipGraphInstantiate(out, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (!ok) {
    (void)hipGetLastError();
    *out = nullptr;
  }
  return ok;
}

static void solve_cycle(rav_ctx* ctx) {
  const int lf = (int)ctx->lv.size() - 1;
  static const bool graphs = [] {
    const char* e = std::getenv("RAV_GRAPH");
    return !(e && std::string(e) == "0");
  }();
  if (graphs && !ctx->graph_failed) {
    const bool prof = ctx->prof_level >= 0;
    if (prof && ctx->prof_exec && ctx->prof_exec_level != ctx->prof_level) rav_drop_graph(ctx);
    hipGraphExec_t* ex = prof ? &ctx->prof_exec : &ctx->cycle_exec;
    if (!*ex) {
      if (prof) {
        ctx->gprof_nres = ctx->gprof_napp = 0;
        ctx->prof_capture = true;
      }
      const bool ok = capture_cycle(ctx, ex);
      ctx->prof_capture = false;
      if (prof) ctx->prof_exec_level = ctx->prof_level;
      if (!ok) ctx->graph_failed = true;   // issue the launches directly from now on
    }
    if (*ex && hipGraphLaunch(*ex, ctx->stream) == hipSuccess) return;
    (void)hipGetLastError();
    rav_drop_graph(ctx);
    ctx->graph_failed = true;
  }
  vcycle_level(ctx, lf, true);
  rav_residual_level(ctx, lf, true);
}

// After a replay of the profiled cycle (stream synchronized): add its marker
// intervals to the profile sums.
static void collect_graph_profile(rav_ctx* ctx) {
  if (ctx->prof_level < 0 || !ctx->prof_exec) return;
  for (int i = 0; i < ctx->gprof_nres; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->gprof_res[2 * i], ctx->gprof_res[2 * i + 1]) == hipSuccess) {
      ctx->prof_sum_res += ms;
      ++ctx->prof_cnt_res;
    }
  }
  for (int i = 0; i < ctx->gprof_napp; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->gprof_app[2 * i], ctx->gprof_app[2 * i + 1]) == hipSuccess) {
      ctx->prof_sum_app += ms;
      ++ctx->prof_cnt_app;
    }
  }
}

rav_status rav_read_norm(rav_ctx* ctx, double* out) {
  // the norm kernel also wrote the value into pinned host memory
  CK(hipStreamSynchronize(ctx->stream));
  *out = std::sqrt(*ctx->h_norm);
  return RAV_OK;
}

static rav_status check_level(const rav_ctx* ctx, int level, bool smoothed) {
  if (!ctx) return RAV_EINVAL;
  if (level < 0 || level >= (int)ctx->lv.size()) return RAV_EINVAL;
  if (smoothed && level == 0) return RAV_EINVAL;
  return RAV_OK;
}

static rav_status need_factors(rav_ctx* ctx) {
  if (!ctx->factored) return set_err(ctx, RAV_EINVAL, "rav_factor_patches has not been called");
  return RAV_OK;
}

// ============================================================================
// rav_create; invert_coarse = false leaves the coarse matrix uninverted, for a
// batch that inverts the coarse matrices of all its problems together
// (rav_invert_coarse, then rav_finish_coarse).
rav_status rav_create_ex(const rav_problem_desc* d, void* hip_stream, rav_ctx** out, bool invert_coarse) {
  if (!d || !out) return set_err(nullptr, RAV_EINVAL, "null descriptor or output pointer");
  *out = nullptr;
  if (d->discretization == RAV_Q1Q1_ADAPTIVE)
    return set_err(nullptr, RAV_EINVAL, "adaptive grids are created with rav_create_adaptive");
  if (d->discretization == RAV_Q1Q1_STAB) {
    if (!invert_coarse)
      return set_err(nullptr, RAV_EUNSUPPORTED, "batches are provided for the Taylor-Hood discretization");
    return rav_q1_create(d, hip_stream, out);
  }
  if (d->discretization != RAV_TAYLOR_HOOD) return set_err(nullptr, RAV_EINVAL, "bad discretization");
  if (d->dim != 2 && d->dim != 3) return set_err(nullptr, RAV_EINVAL, "dim must be 2 or 3");
  if (d->n_levels < 2) return set_err(nullptr, RAV_EINVAL, "n_levels must be >= 2");
  if (d->n_levels > 20 || d->n_cells <= 0 || d->n_cells % (1 << (d->n_levels - 1)))
    return set_err(nullptr, RAV_EINVAL, "n_cells must be divisible by 2^(n_levels-1)");
  {
    const long long n0 = d->n_cells >> (d->n_levels - 1);
    long long nv = 1, np = 1;
    for (int k = 0; k < d->dim; ++k) { nv *= 2 * n0 + 1; np *= n0 + 1; }
    if (d->dim * nv + np + 1 > MAX_COARSE)
      return set_err(nullptr, RAV_EINVAL, "coarsest grid too large for the dense direct solve (" +
                     std::to_string(d->dim * nv + np) + " DoFs, limit " + std::to_string(MAX_COARSE) +
                     "): use more levels");
  }
  {
    // the kernels keep level vector indices in 32-bit integers and decode
    // them with 32-bit division; they assume fewer than 2^28 entries
    const long long nf = d->n_cells;
    long long nv = 1, np = 1;
    for (int k = 0; k < d->dim; ++k) { nv *= 2 * nf + 1; np *= nf + 1; }
    if (d->dim * nv + np >= (1LL << 28))
      return set_err(nullptr, RAV_EUNSUPPORTED, "finest level has " + std::to_string(d->dim * nv + np) +
                     " DoFs; the kernels' 32-bit index math supports fewer than 2^28");
  }
  if (!(d->omega > 0.0) || d->nu_pre < 0 || d->nu_post < 0)
    return set_err(nullptr, RAV_EINVAL, "omega must be > 0 and smoothing steps >= 0");
  if (!(d->eta_out > 0.0) || !(d->eta_in > 0.0)) return set_err(nullptr, RAV_EINVAL, "viscosities must be > 0");
  if (d->n_incl < 0 || d->n_incl > MAX_INCL || (d->n_incl > 0 && !d->incl))
    return set_err(nullptr, RAV_EINVAL, "n_incl must be in [0, 64] with a valid array");
  if (d->bc_dirichlet_mask >> (2 * d->dim)) return set_err(nullptr, RAV_EINVAL, "bc mask has bits beyond 2*dim");
  if (d->coarse_galerkin != 0 && d->coarse_galerkin != 1)
    return set_err(nullptr, RAV_EINVAL, "coarse_galerkin must be 0 or 1");
  if (d->patch != RAV_PATCH_VERTEX && d->patch != RAV_PATCH_ELEMENT) return set_err(nullptr, RAV_EINVAL, "bad patch kind");
  if (d->smoother < RAV_SMOOTHER_RAV || d->smoother > RAV_SMOOTHER_MV) return set_err(nullptr, RAV_EINVAL, "bad smoother");
  if (d->inv_precision < RAV_FP64 || d->inv_precision > RAV_BF16) return set_err(nullptr, RAV_EINVAL, "bad precision");
  if (d->dim == 3 && d->patch == RAV_PATCH_VERTEX && d->smoother != RAV_SMOOTHER_RAV)
    return set_err(nullptr, RAV_EUNSUPPORTED, "3D vertex patches (376 DoFs) are provided for RAV only: AV/MV "
                   "would store full 376x376 inverses");
  if (d->smoother != RAV_SMOOTHER_RAV && d->inv_precision != RAV_FP64)
    return set_err(nullptr, RAV_EUNSUPPORTED, "low-precision inverses are provided for RAV only");
  if (d->inv_format != RAV_ROWS && d->inv_format != RAV_FACTORED)
    return set_err(nullptr, RAV_EINVAL, "bad inverse format");
  if (d->inv_format == RAV_FACTORED && (d->smoother != RAV_SMOOTHER_RAV || d->patch != RAV_PATCH_VERTEX))
    return set_err(nullptr, RAV_EUNSUPPORTED, "the factored inverse format is provided for RAV with vertex patches");

  rav_ctx* ctx = new rav_ctx();
  ctx->desc = *d;
  if (d->n_incl > 0) ctx->incl.assign(d->incl, d->incl + d->n_incl);
  ctx->desc.incl = ctx->incl.empty() ? nullptr : ctx->incl.data();
  ctx->stream = (hipStream_t)hip_stream;
  ctx->prec = d->inv_precision;
  if (const char* e = std::getenv("RAV_SPLIT_BELOW")) ctx->split_below = std::atoll(e);
  auto fail = [&](rav_status st) {
    g_create_error = ctx->err;
    rav_destroy(ctx);
    return st;
  };
  {
    const rav_status s0 = rav_init_common(ctx, d);
    if (s0 != RAV_OK) return fail(s0);
  }
  set_ref_tables(make_tables(), ctx->stream);
  ctx->lv.resize(d->n_levels);
  for (int l = 0; l < d->n_levels; ++l) {
    rav_status st = build_level(ctx, l);
    if (st != RAV_OK) return fail(st);
  }
  for (int l = 1; l < d->n_levels; ++l) {
    LevelHost& L = ctx->lv[l];
    L.hd.has_coarse = 1;
    L.hd.gc = ctx->lv[l - 1].hd.g;
    L.hd.xc = ctx->lv[l - 1].hd.x;
    L.hd.bc = ctx->lv[l - 1].hd.b;
    L.hd.rc = ctx->lv[l - 1].hd.r;
    rav_status st = rav_upload_desc(ctx, L);
    if (st != RAV_OK) return fail(st);
  }
  rav_status st = build_coarse(ctx, invert_coarse);
  if (st != RAV_OK) return fail(st);
  *out = ctx;
  return RAV_OK;
}

extern "C" {

rav_status rav_create(const rav_problem_desc* d, void* hip_stream, rav_ctx** out) {
  return rav_create_ex(d, hip_stream, out, true);
}

}  // extern "C"

// Set-up autotuner of the RAV apply: for every bucket of more than 64 patches
// the 1-, 4-, 8- and 32-lanes-per-patch variants are timed (HIP events, mean of
// three launches after one warm-up, on the level's own vectors, which every
// solve overwrites) and the fastest is kept.  RAV_AUTOTUNE=0 keeps the
// size-based choice.
// Buckets of a level on the 4- or APPLY_SPLIT-lanes-per-patch or the
// row-parallel variant go into one merged launch of 256-thread blocks when
// there are at least two of them: the 3D boundary buckets (faces, edges, corner) are small
// and latency-bound, and separate launches serialize their tails.
static rav_status merge_apply(rav_ctx* ctx) {
  for (size_t l = 1; l < ctx->lv.size(); ++l) {
    LevelHost& L = ctx->lv[l];
    std::vector<BlockTask> mt;
    int nb = 0;
    L.multi_edges = false;
    for (ApplyLaunch& al : L.apply) al.merged = false;
    auto mergeable = [](int split) { return split == 4 || split == APPLY_SPLIT || split == APPLY_ROWS; };
    for (const ApplyLaunch& al : L.apply) nb += mergeable(al.split) ? 1 : 0;
    if (nb < 2) continue;
    for (ApplyLaunch& al : L.apply) {
      if (!mergeable(al.split)) continue;
      const long long cnt = L.hd.bk[al.bucket].count;
      const int per_block = APPLY_BLOCK_MAX / (al.split == APPLY_ROWS ? 64 : al.split);
      for (long long p0 = 0; p0 < cnt; p0 += per_block) {
        BlockTask t{};
        t.grid = 0; t.part = al.bucket; t.start = p0; t.logical = (int)mt.size(); t.pad = al.split;
        mt.push_back(t);
      }
      al.merged = true;
      const int cls = L.hd.bk[al.bucket].cls;
      if (ctx->desc.dim == 3 && al.split != APPLY_ROWS && (cls == 3 || cls >= 5)) L.multi_edges = true;
    }
    (void)rav_dfree(L.multi_tasks);
    L.multi_tasks = nullptr;
    L.n_multi = 0;
    const rav_status st = rav_upload_tasks(ctx, mt, &L.multi_tasks, &L.n_multi);
    if (st != RAV_OK) return st;
  }
  return RAV_OK;
}

static rav_status autotune_apply(rav_ctx* ctx) {
  if (ctx->desc.smoother != RAV_SMOOTHER_RAV || !ctx->autotune) return RAV_OK;
  if (const char* e = std::getenv("RAV_AUTOTUNE"))
    if (std::string(e) == "0") return RAV_OK;
  const rav_problem_desc& D = ctx->desc;
  const char* lg = std::getenv("RAV_AUTOTUNE_LOG");   // "1": print every candidate's time to stderr
  const bool log = lg && std::string(lg) == "1";
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  rav_status result = RAV_OK;
  for (size_t l = 1; l < ctx->lv.size() && result == RAV_OK; ++l) {
    LevelHost& L = ctx->lv[l];
    for (ApplyLaunch& al : L.apply) {
      const long long cnt = L.hd.bk[al.bucket].count;
      if (cnt <= 64) continue;
      float best_ms = 0.0f;
      ApplyLaunch best = al;
      bool have = false;
      for (int split : {1, 4, APPLY_SPLIT, APPLY_SPLIT_SMALL}) {
        ApplyLaunch cand = al;
        if (split == al.split) {
          cand = al;
        } else if ((result = make_apply_tasks(ctx, cand, cnt, split)) != RAV_OK) {
          break;
        }
        auto run = [&]() {
          launch_rav_apply(D.dim, D.patch, cand.cls, ctx->prec, cand.split, L.dd, cand.tasks, cand.ntasks,
                           ctx->stream, L.hd.bk[cand.bucket].factored);
        };
        run();
        (void)hipEventRecord(e0, ctx->stream);
        for (int r = 0; r < 3; ++r) run();
        (void)hipEventRecord(e1, ctx->stream);
        if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess) {
          ctx->err = "apply autotuning launch failed";
          result = RAV_EDEVICE;
          break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (log) std::fprintf(stderr, "rav autotune: level %zu bucket %d (%lld patches) split %d: %.1f us\n", l,
                              al.bucket, cnt, split, 1e3f * ms / 3.0f);
        if (!have || ms < best_ms) {
          if (have && best.tasks != al.tasks) (void)rav_dfree(best.tasks);
          best = cand;
          best_ms = ms;
          have = true;
        } else if (cand.tasks != al.tasks) {
          (void)rav_dfree(cand.tasks);
        }
      }
      if (result != RAV_OK) {
        if (have && best.tasks != al.tasks) (void)rav_dfree(best.tasks);
        break;
      }
      if (best.tasks != al.tasks) {
        (void)rav_dfree(al.tasks);
        al = best;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return result;
}

extern "C" {

rav_status rav_factor_patches(rav_ctx* ctx) {
  if (ctx && ctx->q1) return rav_q1_factor(ctx);
  if (ctx && ctx->ad) return rav_ad_factor(ctx);
  if (!ctx) return RAV_EINVAL;
  rav_drop_graph(ctx);
  const rav_problem_desc& D = ctx->desc;
  const bool full = D.smoother != RAV_SMOOTHER_RAV;
  const int npad = patch_npad(D.dim, D.patch);
  const int big = INT_MAX;
  for (size_t l = 1; l < ctx->lv.size(); ++l) {
    LevelHost& L = ctx->lv[l];
    GridDev& h = L.hd;
    if (full) {
      if (!h.Winv) {
        CK(rav_dmalloc((void**)&h.Winv, sizeof(double) * L.npatch * npad * npad));
        if (D.smoother == RAV_SMOOTHER_AV) CK(rav_dmalloc((void**)&h.Y, sizeof(double) * L.npatch * npad));
      }
    } else {
      const int V = ctx->prec == P_FP64 ? 2 : ctx->prec == P_FP32 ? 4 : 8;
      const size_t esz = ctx->prec == P_FP64 ? 8 : ctx->prec == P_FP32 ? 4 : 2;
      for (int bi = 0; bi < h.nbk; ++bi) {
        Bucket& B = h.bk[bi];
        B.nchunk = ((B.factored ? (long long)fact_nvals(D.dim) : (long long)npad * B.nown) + V - 1) / V;
        if (!B.W) {
          const size_t bytes = esz * (size_t)V * (size_t)B.nchunk * (size_t)B.count_pad;
          CK(rav_dmalloc(&B.W, bytes));
          CK(hipMemsetAsync(B.W, 0, bytes, ctx->stream));
        }
      }
    }
    rav_status st = rav_upload_desc(ctx, L);
    if (st != RAV_OK) return st;
    CK(hipMemcpy(ctx->d_status, &big, sizeof(int), hipMemcpyHostToDevice));
    if (full) {
      launch_factor(D.dim, D.patch, 0, P_FP64, 1, L.dd, L.npatch, 0, ctx->d_status, ctx->stream);
    } else {
      for (int bi = 0; bi < h.nbk; ++bi)
        launch_factor(D.dim, D.patch, h.bk[bi].cls, ctx->prec, 0, L.dd, h.bk[bi].count, bi, ctx->d_status,
                      ctx->stream);
    }
    CK(hipGetLastError());
    int stv = 0;
    CK(hipMemcpyAsync(&stv, ctx->d_status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    if (stv != INT_MAX)
      return set_err(ctx, RAV_ESINGULAR,
                     "zero pivot in patch " + std::to_string(stv) + " on level " + std::to_string(l));
  }
  ctx->factored = 1;
  const rav_status st = autotune_apply(ctx);
  return st != RAV_OK ? st : merge_apply(ctx);
}

rav_status rav_dofs(const rav_ctx* ctx, int level, long* n_total, long* n_free) {
  if (ctx && ctx->q1) return rav_q1_dofs(ctx, level, n_total, n_free);
  if (ctx && ctx->ad) return rav_ad_dofs(ctx, level, n_total, n_free);
  if (check_level(ctx, level, false) != RAV_OK) return RAV_EINVAL;
  const Geo& g = ctx->lv[level].hd.g;
  if (n_total) *n_total = (long)g.n;
  if (n_free) {
    long long masked1 = 0;   // masked nodes per component
    for (long long i = 0; i < g.nV; ++i) {
      int a[3] = {0, 0, 0};
      node_of(g, i, a);
      if (node_dirichlet(g, a)) ++masked1;
    }
    *n_free = (long)(g.n - g.dim * masked1);
  }
  return RAV_OK;
}

rav_status rav_n_levels(const rav_ctx* ctx, int* n) {
  if (ctx && ctx->q1 && n) {
    *n = rav_q1_n_levels(ctx);
    return RAV_OK;
  }
  if (ctx && ctx->ad && n) {
    *n = rav_ad_n_levels(ctx);
    return RAV_OK;
  }
  if (!ctx || !n) return RAV_EINVAL;
  *n = (int)ctx->lv.size();
  return RAV_OK;
}

rav_status rav_n_patches(const rav_ctx* ctx, int level, long* n) {
  if (ctx && ctx->q1) return rav_q1_n_patches(ctx, level, n);
  if (ctx && ctx->ad) return rav_ad_n_patches(ctx, level, n);
  if (check_level(ctx, level, false) != RAV_OK || !n) return RAV_EINVAL;
  *n = (long)ctx->lv[level].npatch;
  return RAV_OK;
}

rav_status rav_assemble_rhs(rav_ctx* ctx, const double* params, int n_params, double* b_dev) {
  if (ctx && ctx->q1 && params && b_dev) return rav_q1_assemble_rhs(ctx, params, n_params, b_dev);
  if (ctx && ctx->ad)
    return set_err(ctx, RAV_EUNSUPPORTED,
                   "adaptive grids take their data through the lifting (rav_assemble_rhs_lid, rav_assemble_rhs_dirichlet)");
  if (!ctx || !params || !b_dev) return RAV_EINVAL;
  const int need = ctx->desc.dim == 2 ? 25 : 65;
  if (n_params != need) return set_err(ctx, RAV_EINVAL, "mms parameter array must have " + std::to_string(need) + " entries");
  LevelHost& L = ctx->lv.back();
  const Geo& g = L.hd.g;
  const long long ncell = (long long)g.N * g.N * (g.dim == 3 ? g.N : 1);
  const int nq = g.dim == 2 ? 9 : 27;
  double *dp = nullptr, *fq = nullptr;
  CK(rav_dmalloc((void**)&dp, sizeof(double) * n_params));
  CK(rav_dmalloc((void**)&fq, sizeof(double) * ncell * nq * g.dim));
  CK(hipMemcpy(dp, params, sizeof(double) * n_params, hipMemcpyHostToDevice));
  launch_rhs(g.dim, &L.hd, L.dd, dp, fq, b_dev, ctx->stream);
  CK(hipGetLastError());
  CK(hipStreamSynchronize(ctx->stream));
  CK(rav_dfree(dp));
  CK(rav_dfree(fq));
  return RAV_OK;
}

rav_status rav_assemble_rhs_lid(rav_ctx* ctx, double lid_u, double* b_dev) {
  if (!ctx || !b_dev || !std::isfinite(lid_u)) return RAV_EINVAL;
  const rav_problem_desc& D = ctx->desc;
  if (D.dim != 2 || !((D.bc_dirichlet_mask >> 3) & 1u))
    return set_err(ctx, RAV_EINVAL, "the driven cavity needs a 2D grid with a Dirichlet top side (bit 3)");
  if (ctx->q1) return rav_q1_assemble_rhs_lid(ctx, lid_u, b_dev);
  if (ctx->ad) return rav_ad_assemble_rhs_lid(ctx, lid_u, b_dev);
  LevelHost& L = ctx->lv.back();
  launch_fill(b_dev, 0.0, L.hd.g.n, ctx->stream);
  launch_lift_lid(L.dd, L.hd.g, lid_u, b_dev, ctx->stream);
  CK(hipGetLastError());
  CK(hipStreamSynchronize(ctx->stream));
  return RAV_OK;
}

rav_status rav_residual(rav_ctx* ctx, int level, const double* x, const double* b, double* r, double* norm) {
  if (ctx && ctx->q1 && x && b && r) return rav_q1_residual(ctx, level, x, b, r, norm);
  if (ctx && ctx->ad && x && b && r) return rav_ad_residual(ctx, level, x, b, r, norm);
  if (check_level(ctx, level, false) != RAV_OK || !x || !b || !r) return RAV_EINVAL;
  LevelHost& L = ctx->lv[level];
  const long long n = L.hd.g.n;
  launch_copy(L.hd.x, x, n, ctx->stream);
  launch_copy(L.hd.b, b, n, ctx->stream);
  rav_residual_level(ctx, level, norm != nullptr);
  launch_copy(r, L.hd.r, n, ctx->stream);
  CK(hipGetLastError());
  if (norm) return rav_read_norm(ctx, norm);
  return RAV_OK;
}

rav_status rav_smooth(rav_ctx* ctx, int level, int sweeps, double* x, const double* b) {
  if (ctx && ctx->q1 && x && b && sweeps >= 0) return rav_q1_smooth(ctx, level, sweeps, x, b);
  if (ctx && ctx->ad && x && b && sweeps >= 0) return rav_ad_smooth(ctx, level, sweeps, x, b);
  if (check_level(ctx, level, true) != RAV_OK || !x || !b || sweeps < 0) return RAV_EINVAL;
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  LevelHost& L = ctx->lv[level];
  const long long n = L.hd.g.n;
  launch_copy(L.hd.x, x, n, ctx->stream);
  launch_copy(L.hd.b, b, n, ctx->stream);
  smooth_level(ctx, level, sweeps, false);
  launch_copy(x, L.hd.x, n, ctx->stream);
  CK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_restrict(rav_ctx* ctx, int level, const double* rf, double* bc) {
  if (ctx && ctx->q1 && rf && bc) return rav_q1_restrict(ctx, level, rf, bc);
  if (ctx && ctx->ad && rf && bc) return rav_ad_restrict(ctx, level, rf, bc);
  if (check_level(ctx, level, true) != RAV_OK || !rf || !bc) return RAV_EINVAL;
  LevelHost& L = ctx->lv[level];
  launch_copy(L.hd.r, rf, L.hd.g.n, ctx->stream);
  launch_restrict(ctx->desc.dim, L.dd, L.rtasks, L.n_rtasks, ctx->stream);
  launch_copy(bc, ctx->lv[level - 1].hd.b, L.hd.gc.n, ctx->stream);
  CK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_prolong_add(rav_ctx* ctx, int level, const double* xc, double* xf) {
  if (ctx && ctx->q1 && xc && xf) return rav_q1_prolong_add(ctx, level, xc, xf);
  if (ctx && ctx->ad && xc && xf) return rav_ad_prolong_add(ctx, level, xc, xf);
  if (check_level(ctx, level, true) != RAV_OK || !xc || !xf) return RAV_EINVAL;
  LevelHost& L = ctx->lv[level];
  launch_copy(ctx->lv[level - 1].hd.x, xc, L.hd.gc.n, ctx->stream);
  launch_copy(L.hd.x, xf, L.hd.g.n, ctx->stream);
  launch_prolong(ctx->desc.dim, L.dd, L.ptasks, L.n_ptasks, ctx->stream);
  launch_copy(xf, L.hd.x, L.hd.g.n, ctx->stream);
  CK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_coarse_solve(rav_ctx* ctx, const double* b0, double* x0) {
  if (ctx && ctx->q1 && b0 && x0) return rav_q1_coarse_solve(ctx, b0, x0);
  if (ctx && ctx->ad && b0 && x0) return rav_ad_coarse_solve(ctx, b0, x0);
  if (!ctx || !b0 || !x0) return RAV_EINVAL;
  launch_coarse_gemv(ctx->Minv, ctx->nb, ctx->lv[0].hd.g.n, b0, x0, ctx->stream);
  CK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_vcycle(rav_ctx* ctx, double* x, const double* b) {
  if (ctx && ctx->q1 && x && b) return rav_q1_vcycle(ctx, x, b);
  if (ctx && ctx->ad && x && b) return rav_ad_vcycle(ctx, x, b);
  if (!ctx || !x || !b) return RAV_EINVAL;
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  const int lf = (int)ctx->lv.size() - 1;
  LevelHost& L = ctx->lv[lf];
  const long long n = L.hd.g.n;
  launch_copy(L.hd.x, x, n, ctx->stream);
  launch_copy(L.hd.b, b, n, ctx->stream);
  vcycle_level(ctx, lf, false);
  launch_copy(x, L.hd.x, n, ctx->stream);
  CK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_solve(rav_ctx* ctx, double* x, const double* b, double rtol, int maxit, int* iters,
                     double* rel_res) {
  if (!ctx || !x || !b || !(rtol > 0.0) || maxit < 0) return RAV_EINVAL;
  if (ctx->q1) return rav_q1_solve(ctx, x, b, rtol, maxit, iters, rel_res);
  if (ctx->ad) return rav_ad_solve(ctx, x, b, rtol, maxit, iters, rel_res);
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  const int lf = (int)ctx->lv.size() - 1;
  LevelHost& L = ctx->lv[lf];
  const long long n = L.hd.g.n;
  launch_copy(L.hd.x, x, n, ctx->stream);
  launch_copy(L.hd.b, b, n, ctx->stream);
  rav_residual_level(ctx, lf, true);
  double r0 = 0.0;
  rav_status st = rav_read_norm(ctx, &r0);
  if (st != RAV_OK) return st;
  if (iters) *iters = 0;
  if (rel_res) *rel_res = r0 > 0.0 ? 1.0 : 0.0;
  if (!std::isfinite(r0)) return set_err(ctx, RAV_EDIVERGED, "initial residual is not finite");
  rav_status result = RAV_NOT_CONVERGED;
  if (r0 == 0.0) result = RAV_OK;
  int k = 0;
  double rk = r0;
  ctx->fell_back = 0;
  // the fallback drops the per-patch weights for the rest of this solve only:
  // they are put back before returning, so the next solve starts with them
  std::vector<const float*> saved_omega;
  for (const LevelHost& Lv : ctx->lv) saved_omega.push_back(Lv.hd.omega_patch);
  auto restore_omega = [&]() -> rav_status {
    if (!ctx->fell_back) return RAV_OK;
    for (size_t l = 0; l < ctx->lv.size(); ++l) {
      if (ctx->lv[l].hd.omega_patch == saved_omega[l]) continue;
      ctx->lv[l].hd.omega_patch = saved_omega[l];
      const rav_status s2 = rav_upload_desc(ctx, ctx->lv[l]);
      if (s2 != RAV_OK) return s2;
    }
    return RAV_OK;
  };
  while (result == RAV_NOT_CONVERGED && k < maxit) {
    const double rprev = rk;
    solve_cycle(ctx);   // r of the finest level is current from the norm evaluation
    st = rav_read_norm(ctx, &rk);
    if (st != RAV_OK) { (void)restore_omega(); return st; }
    collect_graph_profile(ctx);
    ++k;
    if (ctx->fallback_rho > 0.0 && !ctx->fell_back && rk > ctx->fallback_rho * rprev) {
      // the per-patch weights reduce the residual less than the fixed-omega
      // reference rate: continue with the scalar omega
      bool any = false;
      for (LevelHost& Lv : ctx->lv) {
        if (!Lv.hd.omega_patch) continue;
        Lv.hd.omega_patch = nullptr;
        any = true;
        ctx->fell_back = 1;
        if ((st = rav_upload_desc(ctx, Lv)) != RAV_OK) { (void)restore_omega(); return st; }
      }
      ctx->fell_back = any ? 1 : 0;
    }
    if (!std::isfinite(rk) || rk > 1e3 * r0) {
      result = RAV_EDIVERGED;
      ctx->err = "residual diverged at cycle " + std::to_string(k);
    } else if (rk <= rtol * r0) {
      result = RAV_OK;
    }
  }
  if (iters) *iters = k;
  if (rel_res) *rel_res = r0 > 0.0 ? rk / r0 : 0.0;
  launch_copy(x, L.hd.x, n, ctx->stream);
  CK(hipGetLastError());
  CK(hipStreamSynchronize(ctx->stream));
  if ((st = restore_omega()) != RAV_OK) return st;
  return result;
}

rav_status rav_set_params(rav_ctx* ctx, double omega, int nu_pre, int nu_post) {
  if (!ctx || !(omega > 0.0) || nu_pre < 0 || nu_post < 0) return RAV_EINVAL;
  rav_drop_graph(ctx);
  ctx->desc.omega = omega;
  ctx->desc.nu_pre = nu_pre;
  ctx->desc.nu_post = nu_post;
  if (ctx->q1 || ctx->ad) return RAV_OK;
  for (LevelHost& L : ctx->lv) {
    L.hd.omega = omega;
    rav_status st = rav_upload_desc(ctx, L);
    if (st != RAV_OK) return st;
  }
  return RAV_OK;
}

rav_status rav_set_fallback(rav_ctx* ctx, double rho_max, int* fell_back) {
  if (!ctx || rho_max < 0.0) return RAV_EINVAL;
  ctx->fallback_rho = rho_max;
  if (fell_back) *fell_back = ctx->fell_back;
  return RAV_OK;
}

rav_status rav_set_patch_omega(rav_ctx* ctx, int level, const float* omega_dev) {
  if (ctx && (ctx->q1 || ctx->ad)) return set_err(ctx, RAV_EUNSUPPORTED, "per-patch weights are provided for Taylor-Hood");
  if (check_level(ctx, level, true) != RAV_OK) return RAV_EINVAL;
  ctx->lv[level].hd.omega_patch = omega_dev;
  return rav_upload_desc(ctx, ctx->lv[level]);
}

static rav_status map_patch_geo(const Geo& g, int kind, long long npatch, long patch, int* dofs, int* n,
                                int* owned) {
  if (patch < 0 || patch >= npatch || !dofs || !n) return RAV_EINVAL;
  int k[3] = {0, 0, 0};
  patch_anchor(g, kind, patch, k);
  const int npad = patch_npad(g.dim, kind);
  int cnt = 0;
  for (int l = 0; l < npad; ++l) {
    int comp, node[3];
    const long long gi = patch_local_dof(g, kind, k, l, &comp, node);
    if (gi < 0) continue;
    dofs[cnt] = (int)gi;
    if (owned) owned[cnt] = owner_of(g, kind, gi) == patch ? 1 : 0;
    ++cnt;
  }
  *n = cnt;
  return RAV_OK;
}

static rav_status desc_geo(const rav_problem_desc* d, int level, Geo* g) {
  if (!d || (d->dim != 2 && d->dim != 3) || d->n_levels < 1 || d->n_levels > 20 || level < 0 ||
      level >= d->n_levels || d->n_cells <= 0 || d->n_cells % (1 << (d->n_levels - 1)) ||
      (d->patch != RAV_PATCH_VERTEX && d->patch != RAV_PATCH_ELEMENT))
    return RAV_EINVAL;
  *g = make_geo(d->dim, d->n_cells >> (d->n_levels - 1 - level), d->bc_dirichlet_mask);
  return RAV_OK;
}

rav_status rav_map_patch(const rav_problem_desc* d, int level, long patch, int* dofs, int* n, int* owned) {
  if (d && d->discretization == RAV_Q1Q1_STAB) return rav_q1_map_patch(d, level, patch, dofs, n, owned);
  if (d && d->discretization == RAV_Q1Q1_ADAPTIVE)
    return set_err(nullptr, RAV_EUNSUPPORTED, "adaptive patch maps need the grids: use rav_get_patch_map");
  Geo g;
  if (desc_geo(d, level, &g) != RAV_OK) return RAV_EINVAL;
  return map_patch_geo(g, d->patch, n_patches(g, d->patch), patch, dofs, n, owned);
}

rav_status rav_map_owner(const rav_problem_desc* d, int level, int* owner) {
  if (d && d->discretization == RAV_Q1Q1_STAB) return rav_q1_map_owner(d, level, owner);
  if (d && d->discretization == RAV_Q1Q1_ADAPTIVE)
    return set_err(nullptr, RAV_EUNSUPPORTED, "adaptive owner maps need the grids: use rav_get_owner");
  Geo g;
  if (desc_geo(d, level, &g) != RAV_OK || !owner) return RAV_EINVAL;
  for (long long i = 0; i < g.n; ++i) {
    if (i < g.dim * g.nV) {
      int a[3] = {0, 0, 0};
      node_of(g, i % g.nV, a);
      if (node_dirichlet(g, a)) { owner[i] = -1; continue; }
    }
    owner[i] = (int)owner_of(g, d->patch, i);
  }
  return RAV_OK;
}

rav_status rav_get_patch_map(const rav_ctx* ctx, int level, long patch, int* dofs, int* n, int* owned) {
  if (ctx && ctx->q1) return rav_q1_get_patch_map(ctx, level, patch, dofs, n, owned);
  if (ctx && ctx->ad) return rav_ad_get_patch_map(ctx, level, patch, dofs, n, owned);
  if (check_level(ctx, level, false) != RAV_OK) return RAV_EINVAL;
  const LevelHost& L = ctx->lv[level];
  return map_patch_geo(L.hd.g, ctx->desc.patch, L.npatch, patch, dofs, n, owned);
}

rav_status rav_get_owner(rav_ctx* ctx, int level, int* owner_dev) {
  if (ctx && ctx->q1 && owner_dev) return rav_q1_get_owner(ctx, level, owner_dev);
  if (ctx && ctx->ad && owner_dev) return rav_ad_get_owner(ctx, level, owner_dev);
  if (check_level(ctx, level, false) != RAV_OK || !owner_dev) return RAV_EINVAL;
  LevelHost& L = ctx->lv[level];
  launch_owner(L.dd, ctx->desc.patch, L.hd.g.n, owner_dev, ctx->stream);
  CK(hipGetLastError());
  CK(hipStreamSynchronize(ctx->stream));
  return RAV_OK;
}

rav_status rav_get_patch_inverse(rav_ctx* ctx, int level, long patch, double* out, int* rows, int* cols) {
  if (ctx && ctx->q1 && out && rows && cols) return rav_q1_get_patch_inverse(ctx, level, patch, out, rows, cols);
  if (ctx && ctx->ad && out && rows && cols) return rav_ad_get_patch_inverse(ctx, level, patch, out, rows, cols);
  if (check_level(ctx, level, true) != RAV_OK || !out || !rows || !cols) return RAV_EINVAL;
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  LevelHost& L = ctx->lv[level];
  if (patch < 0 || patch >= L.npatch) return RAV_EINVAL;
  const Geo& g = L.hd.g;
  const int kind = ctx->desc.patch;
  const int npad = patch_npad(g.dim, kind);
  int k[3] = {0, 0, 0};
  patch_anchor(g, kind, patch, k);
  std::vector<int> vcol;
  for (int c = 0; c < npad; ++c) {
    int comp, node[3];
    if (patch_local_dof(g, kind, k, c, &comp, node) >= 0) vcol.push_back(c);
  }
  CK(hipStreamSynchronize(ctx->stream));
  if (ctx->desc.smoother != RAV_SMOOTHER_RAV) {
    std::vector<double> A((size_t)npad * npad);
    CK(hipMemcpy(A.data(), L.hd.Winv + (long long)patch * npad * npad, sizeof(double) * A.size(),
                 hipMemcpyDeviceToHost));
    for (size_t i = 0; i < vcol.size(); ++i)
      for (size_t j = 0; j < vcol.size(); ++j) out[i * vcol.size() + j] = A[(size_t)vcol[j] * npad + vcol[i]];
    *rows = *cols = (int)vcol.size();
    return RAV_OK;
  }
  const int cls = kind == KIND_VERTEX ? 0 : element_class(g, k);
  int bi = -1;
  for (int i = 0; i < L.hd.nbk; ++i)
    if (L.hd.bk[i].cls == cls) bi = i;
  if (bi < 0) return set_err(ctx, RAV_EINVAL, "patch bucket not found");
  const Bucket& B = L.hd.bk[bi];
  const long long pos = kind == KIND_VERTEX ? patch : bucket_pos(g, cls, k);
  const int V = ctx->prec == P_FP64 ? 2 : ctx->prec == P_FP32 ? 4 : 8;
  const size_t esz = ctx->prec == P_FP64 ? 8 : ctx->prec == P_FP32 ? 4 : 2;
  std::vector<double> W((size_t)B.nchunk * V);
  std::vector<unsigned char> chunk(16);
  for (long long m = 0; m < B.nchunk; ++m) {
    CK(hipMemcpy(chunk.data(), (const char*)B.W + 16 * (size_t)w_vec(B, pos, m), 16, hipMemcpyDeviceToHost));
    for (int v = 0; v < V; ++v) {
      double val;
      if (esz == 8) { double t; std::memcpy(&t, chunk.data() + 8 * v, 8); val = t; }
      else if (esz == 4) { float t; std::memcpy(&t, chunk.data() + 4 * v, 4); val = t; }
      else { unsigned short u; std::memcpy(&u, chunk.data() + 2 * v, 2); unsigned bits = (unsigned)u << 16; float t; std::memcpy(&t, &bits, 4); val = t; }
      W[(size_t)m * V + v] = val;
    }
  }
  // entry (owned row j, padded column c) of the owned rows of L_i^{-1}
  auto entry = [&](int j, int c) -> double {
    if (!B.factored) return W[(size_t)c * B.nown + j];
    // factored vertex patch: rows from K^{-1}[owned, :], z = K^{-1} B and S^{-1}
    const int NN = fact_nn(g.dim), NO = fact_nown_nodes(g.dim), GV = fact_per_node(g.dim);
    const double sinv = W[(size_t)NN * GV];
    auto z = [&](int comp, int node) { return W[(size_t)node * GV + NO + comp]; };
    const int l = bucket_own_local(g.dim, kind, cls, j);
    const bool rv = l < g.dim * NN, cv = c < g.dim * NN;
    if (rv) {
      const int rc = l / NN, a = j % NO;
      const int an = l % NN;
      if (cv) {
        const int cc = c / NN, b = c % NN;
        return (rc == cc ? W[(size_t)b * GV + a] : 0.0) + z(rc, an) * sinv * z(cc, b);
      }
      return -z(rc, an) * sinv;
    }
    if (cv) return -sinv * z(c / NN, c % NN);
    return sinv;
  };
  int nr = 0;
  for (int j = 0; j < B.nown; ++j) {
    const int l = bucket_own_local(g.dim, kind, cls, j);
    int comp, node[3];
    if (patch_local_dof(g, kind, k, l, &comp, node) < 0) continue;
    for (size_t c = 0; c < vcol.size(); ++c) out[(size_t)nr * vcol.size() + c] = entry(j, vcol[c]);
    ++nr;
  }
  *rows = nr;
  *cols = (int)vcol.size();
  return RAV_OK;
}

rav_status rav_export_matrix(rav_ctx* ctx, int level, double* out) {
  if (ctx && (ctx->q1 || ctx->ad)) return set_err(ctx, RAV_EUNSUPPORTED, "dense export is provided for Taylor-Hood");
  if (check_level(ctx, level, false) != RAV_OK || !out) return RAV_EINVAL;
  LevelHost& L = ctx->lv[level];
  const long long n = L.hd.g.n;
  if (n > 20000) return set_err(ctx, RAV_EINVAL, "level too large for a dense export");
  double* M = nullptr;
  CK(rav_dmalloc((void**)&M, sizeof(double) * n * n));
  launch_coarse_build(L.dd, ctx->desc.dim, M, n, 0, 0, ctx->stream);
  CK(hipGetLastError());
  CK(hipStreamSynchronize(ctx->stream));
  CK(hipMemcpy(out, M, sizeof(double) * n * n, hipMemcpyDeviceToHost));
  CK(rav_dfree(M));
  return RAV_OK;
}

rav_status rav_time_sweep(rav_ctx* ctx, int level, int reps, double* x, const double* b, float* ms_res,
                          float* ms_apply) {
  if (ctx && ctx->q1 && x && b && reps > 0) return rav_q1_time_sweep(ctx, level, reps, x, b, ms_res, ms_apply);
  if (ctx && ctx->ad && x && b && reps > 0) return rav_ad_time_sweep(ctx, level, reps, x, b, ms_res, ms_apply);
  if (check_level(ctx, level, true) != RAV_OK || !x || !b || reps <= 0) return RAV_EINVAL;
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  if (ctx->desc.smoother == RAV_SMOOTHER_MV) return set_err(ctx, RAV_EUNSUPPORTED, "MV has no separate residual kernel");
  LevelHost& L = ctx->lv[level];
  const long long n = L.hd.g.n;
  launch_copy(L.hd.x, x, n, ctx->stream);
  launch_copy(L.hd.b, b, n, ctx->stream);
  std::vector<hipEvent_t> ev(3 * reps);
  for (auto& e : ev) CK(hipEventCreate(&e));
  for (int i = 0; i < reps; ++i) {
    CK(hipEventRecord(ev[3 * i], ctx->stream));
    rav_residual_level(ctx, level, false);
    CK(hipEventRecord(ev[3 * i + 1], ctx->stream));
    rav_apply_level(ctx, level);
    CK(hipEventRecord(ev[3 * i + 2], ctx->stream));
  }
  CK(hipEventSynchronize(ev.back()));
  double tr = 0.0, ta = 0.0;
  for (int i = 0; i < reps; ++i) {
    float a = 0.f, c = 0.f;
    CK(hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]));
    CK(hipEventElapsedTime(&c, ev[3 * i + 1], ev[3 * i + 2]));
    tr += a;
    ta += c;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (ms_res) *ms_res = (float)(tr / reps);
  if (ms_apply) *ms_apply = (float)(ta / reps);
  launch_copy(x, L.hd.x, n, ctx->stream);
  CK(hipStreamSynchronize(ctx->stream));
  return RAV_OK;
}

rav_status rav_profile_begin(rav_ctx* ctx, int level, int max_launches) {
  if (ctx && (ctx->q1 || ctx->ad)) return set_err(ctx, RAV_EUNSUPPORTED, "profiling markers are provided for Taylor-Hood");
  if (check_level(ctx, level, true) != RAV_OK || max_launches <= 0) return RAV_EINVAL;
  for (auto& e : ctx->prof_res) (void)hipEventDestroy(e);
  for (auto& e : ctx->prof_app) (void)hipEventDestroy(e);
  ctx->prof_res.assign(2 * (size_t)max_launches, nullptr);
  ctx->prof_app.assign(2 * (size_t)max_launches, nullptr);
  // timing markers only: no system-scope fence (the host reads them after a
  // stream synchronisation, which orders everything before it)
  for (auto& e : ctx->prof_res) CK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  for (auto& e : ctx->prof_app) CK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  ctx->prof_max = max_launches;
  ctx->prof_nres = ctx->prof_napp = 0;
  ctx->prof_sum_res = ctx->prof_sum_app = 0.0;
  ctx->prof_cnt_res = ctx->prof_cnt_app = 0;
  ctx->prof_level = level;
  return RAV_OK;
}

rav_status rav_profile_end(rav_ctx* ctx, float* avg_res, float* avg_app, int* n_app) {
  if (!ctx) return RAV_EINVAL;
  ctx->prof_level = -1;
  CK(hipStreamSynchronize(ctx->stream));
  double tr = 0.0, ta = 0.0;
  for (int i = 0; i < ctx->prof_nres; ++i) {
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, ctx->prof_res[2 * i], ctx->prof_res[2 * i + 1]));
    tr += ms;
  }
  for (int i = 0; i < ctx->prof_napp; ++i) {
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, ctx->prof_app[2 * i], ctx->prof_app[2 * i + 1]));
    ta += ms;
  }
  tr += ctx->prof_sum_res;
  ta += ctx->prof_sum_app;
  const long long nr = ctx->prof_nres + ctx->prof_cnt_res, na = ctx->prof_napp + ctx->prof_cnt_app;
  if (avg_res) *avg_res = nr ? (float)(tr / nr) : 0.f;
  if (avg_app) *avg_app = na ? (float)(ta / na) : 0.f;
  if (n_app) *n_app = (int)na;
  return RAV_OK;
}

rav_status rav_stream_copy(void* stream, double* dst, const double* src, long n) {
  if (!dst || !src || n < 0) return RAV_EINVAL;
  launch_copy(dst, src, n, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? RAV_OK : RAV_EDEVICE;
}

rav_status rav_create_adaptive(const rav_problem_desc* desc, const int* leaves_host, const long* n_leaves_host,
                               long lattice_x, long lattice_y, void* hip_stream, rav_ctx** out) {
  if (out) *out = nullptr;
  return rav_ad_create(desc, leaves_host, n_leaves_host, lattice_x, lattice_y, hip_stream, out);
}

rav_status rav_adaptive_host_export(const rav_problem_desc* desc, const int* leaves_host, const long* n_leaves_host,
                                    long lattice_x, long lattice_y, int level, int what, double* out_host, long* rows,
                                    long* cols) {
  return rav_ad_host_export(desc, leaves_host, n_leaves_host, lattice_x, lattice_y, level, what, out_host, rows, cols);
}

rav_status rav_assemble_rhs_dirichlet(rav_ctx* ctx, const double* ud_host, double* b_dev) {
  if (!ctx || !ud_host || !b_dev) return RAV_EINVAL;
  if (!ctx->ad) return set_err(ctx, RAV_EUNSUPPORTED, "rav_assemble_rhs_dirichlet serves adaptive-grid contexts");
  return rav_ad_assemble_rhs_dirichlet(ctx, ud_host, b_dev);
}

rav_status rav_adaptive_level_info(const rav_ctx* ctx, int level, long* info_host) {
  if (!ctx || !ctx->ad) return RAV_EINVAL;
  return rav_ad_level_info(ctx, level, info_host);
}

rav_status rav_set_device_allocator(void* (*alloc)(size_t bytes, void* user), void (*release)(void* ptr, void* user),
                                    void* user) {
  std::lock_guard<std::mutex> lock(g_alloc_mutex);
  if ((alloc == nullptr) != (release == nullptr))
    return set_err(nullptr, RAV_EINVAL, "the allocator needs both functions, or neither");
  if (rav_live_objects.load() != 0)
    return set_err(nullptr, RAV_EINVAL, "the device allocator can only change while no context, batch or network exists");
  g_alloc.alloc = alloc;
  g_alloc.release = release;
  g_alloc.user = user;
  return RAV_OK;
}

rav_status rav_destroy(rav_ctx* ctx) {
  if (!ctx) return RAV_OK;
  (void)hipStreamSynchronize(ctx->stream);
  rav_drop_graph(ctx);
  if (ctx->learn_free) ctx->learn_free(ctx);
  if (ctx->gm_free) ctx->gm_free(ctx);
  rav_q1_free(ctx);
  rav_ad_free(ctx);
  for (LevelHost& L : ctx->lv) {
    GridDev& h = L.hd;
    (void)rav_dfree(h.x); (void)rav_dfree(h.b); (void)rav_dfree(h.r); (void)rav_dfree(h.vals);
    (void)rav_dfree(h.Winv); (void)rav_dfree(h.Y);
    for (int i = 0; i < h.nbk; ++i) (void)rav_dfree(h.bk[i].W);
    (void)rav_dfree(L.dd); (void)rav_dfree(L.res_tasks); (void)rav_dfree(L.partials);
    (void)rav_dfree(L.rtasks); (void)rav_dfree(L.ptasks);
    (void)rav_dfree(L.ceta); (void)rav_dfree(L.cutA);
    for (ApplyLaunch& a : L.apply) (void)rav_dfree(a.tasks);
    (void)rav_dfree(L.multi_tasks);
  }
  (void)rav_dfree(ctx->d_incl); (void)rav_dfree(ctx->Minv); (void)rav_dfree(ctx->d_status);
  (void)rav_dfree(ctx->d_norm);
  (void)rav_dfree(ctx->coarse_tasks);
  if (ctx->h_norm) (void)hipHostFree(ctx->h_norm);
  for (auto& e : ctx->gprof_res) if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->gprof_app) if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->prof_res) if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->prof_app) if (e) (void)hipEventDestroy(e);
  delete ctx;
  return RAV_OK;
}

const char* rav_last_error(const rav_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
