// Host-side context of the RAV library (shared by the single-problem and
// batched drivers).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <string>
#include <vector>

#include "rav.h"
#include "rav_internal.h"

namespace rav {

struct ApplyLaunch {
  int bucket = 0;
  int cls = 0;
  int split = 1;
  BlockTask* tasks = nullptr;
  int ntasks = 0;
  bool merged = false;   // launched within the level's merged launch
};

// Buckets with fewer patches than SPLIT_BELOW run the split apply variant
// (APPLY_SPLIT lanes per patch), below SPLIT_BELOW / 60 the one with
// APPLY_SPLIT_SMALL lanes per patch: with few wavefronts in flight, splitting a
// patch over more lanes shortens the dependent load chain of each lane.
constexpr long long SPLIT_BELOW = 120000;

// Largest coarsest-level system (unknowns incl. the pressure border) solved by
// the dense direct solver: 2 GB of FP64 inverse (2D 32x32 and 3D 8x8x8 fit).
constexpr long long MAX_COARSE = 16384;
inline int apply_split(long long count, long long split_below) {
  if (count <= 64) return APPLY_ROWS;
  return count < split_below / 60 ? APPLY_SPLIT_SMALL : count < split_below ? APPLY_SPLIT : 1;
}

struct LevelHost {
  GridDev hd{};
  GridDev* dd = nullptr;
  long long nvals = 0;
  double* ceta = nullptr;        // per-cell coefficients of the matrix-free residual
  double* cutA = nullptr;        // cell matrices of the cut cells
  long long ncut = 0;
  BlockTask* res_tasks = nullptr;
  int n_res_tasks = 0;
  int n_res_tiles = 0;
  double* partials = nullptr;
  std::vector<ApplyLaunch> apply;
  BlockTask* multi_tasks = nullptr;   // merged launch of the buckets marked merged
  int n_multi = 0;
  bool multi_edges = false;           // it holds column-group tasks of 3D edge or corner classes
  long long npatch = 0;
  BlockTask* rtasks = nullptr;   // restriction: node-type tiles over the coarser level
  int n_rtasks = 0;
  BlockTask* ptasks = nullptr;   // prolongation: node-type tiles over this level
  int n_ptasks = 0;
};

// Permute logical tiles so that hardware block b (dispatched to XCD b % 8)
// processes logical tile (b % 8) * (T / 8) + b / 8: each XCD sweeps one
// contiguous range of the grid and its L2 sees the overlapping reads.
std::vector<BlockTask> xcd_order(const std::vector<BlockTask>& logical);

// Logical tiles of `per_block` items over [0, n) for one grid.
void append_tiles(std::vector<BlockTask>& out, int grid, int part, long long n, int per_block);

// Node-type tiles of one grid (residual, restriction onto it, prolongation
// onto it): BLOCK rows of one velocity node parity type (part = t, all
// components) or of the pressure rows (part = 2^d).
void append_residual_tiles(std::vector<BlockTask>& out, int grid, const Geo& g);

}  // namespace rav

struct rav_q1_state;   // stabilized Q1-Q1 hierarchy (rav_q1.hip)
struct rav_ad_state;   // stabilized Q1-Q1 on adaptive quadtree grids (rav_adapt.hip)

// Device memory of the library's buffers: hipMalloc/hipFree, or the caller's
// allocator set by rav_set_device_allocator.  Every context, batch and network
// counts itself in rav_live_objects, so the allocator cannot change while a
// buffer it made is alive.
hipError_t rav_dmalloc(void** p, size_t bytes);
hipError_t rav_dfree(void* p);
extern std::atomic<long> rav_live_objects;
struct LiveCount {
  LiveCount() { ++rav_live_objects; }
  ~LiveCount() { --rav_live_objects; }
  LiveCount(const LiveCount&) = delete;
  LiveCount& operator=(const LiveCount&) = delete;
};

struct rav_ctx {
  LiveCount live_;
  rav_problem_desc desc{};
  rav_q1_state* q1 = nullptr;   // set for RAV_Q1Q1_STAB: the entry points route to rav_q1_*
  rav_ad_state* ad = nullptr;   // set by rav_create_adaptive: the entry points route to rav_ad_*
  std::vector<rav_inclusion> incl;
  hipStream_t stream = nullptr;
  std::vector<rav::LevelHost> lv;
  double* d_incl = nullptr;
  double* Minv = nullptr;
  long long nb = 0;
  int bordered = 0;
  int* d_status = nullptr;
  double* d_norm = nullptr;
  double* h_norm = nullptr;       // pinned; the norm kernel writes it through h_norm_dev
  double* h_norm_dev = nullptr;
  int factored = 0;
  bool autotune = true;   // rav_factor_patches times the apply variants (a batch plans its own launches)
  int prec = rav::P_FP64;
  long long split_below = rav::SPLIT_BELOW;
  std::string err;
  // kernel timing (rav_profile_begin / rav_profile_end)
  int prof_level = -1;
  int prof_max = 0;
  int prof_nres = 0, prof_napp = 0;
  std::vector<hipEvent_t> prof_res, prof_app;
  rav::BlockTask* coarse_tasks = nullptr;
  int n_coarse_tasks = 0;
  // learned damping: state owned by rav_learn.hip, released through learn_free
  void* learn = nullptr;
  void (*learn_free)(rav_ctx*) = nullptr;
  // FGMRES work vectors kept between rav_solve_gmres calls (rav_krylov.hip),
  // released through gm_free
  void* gm_cache = nullptr;
  void (*gm_free)(rav_ctx*) = nullptr;
  // fall back to the scalar omega when a cycle reduces the residual by less than this factor (0 = off)
  double fallback_rho = 0.0;
  int fell_back = 0;
  // one V-cycle plus the finest residual and its norm, captured from the
  // stream on the first solve cycle and replayed for the others (RAV_GRAPH=0
  // disables); dropped whenever parameters, factors or tasks change
  hipGraphExec_t cycle_exec = nullptr;
  hipGraphExec_t pc_exec = nullptr;      // FGMRES: the preconditioner's V-cycle on the finest vectors
  bool graph_failed = false;
  // the same cycle captured with the profiling markers of prof_level: its
  // event pairs are re-recorded by every replay and read after each cycle
  hipGraphExec_t prof_exec = nullptr;
  int prof_exec_level = -1;
  bool prof_capture = false;
  std::vector<hipEvent_t> gprof_res, gprof_app;   // marker events inside prof_exec
  int gprof_nres = 0, gprof_napp = 0;
  double prof_sum_res = 0.0, prof_sum_app = 0.0;  // accumulated from prof_exec replays
  long long prof_cnt_res = 0, prof_cnt_app = 0;
};

// Shared helpers (rav_capi.hip).
rav_status rav_set_error(rav_ctx* ctx, rav_status st, const std::string& msg);   // ctx may be null
rav_status rav_init_common(rav_ctx* ctx, const rav_problem_desc* d);   // status, norm, inclusion buffers
rav_status rav_create_ex(const rav_problem_desc* d, void* hip_stream, rav_ctx** out, bool invert_coarse);
rav_status rav_invert_coarse(rav_ctx* const* ctxs, int n, hipStream_t s, std::vector<int>* status_out,
                             std::string* err);
rav_status rav_finish_coarse(rav_ctx* ctx, int pivot_status);
rav_status rav_upload_desc(rav_ctx* ctx, rav::LevelHost& L);
void rav_residual_level(rav_ctx* ctx, int l, bool with_norm);
void rav_apply_level(rav_ctx* ctx, int l);
rav_status rav_read_norm(rav_ctx* ctx, double* out);
void rav_drop_graph(rav_ctx* ctx);   // forget the captured solve cycle
void rav_graph_cycle(rav_ctx* ctx, void (*issue)(rav_ctx*));   // issue, captured and replayed
void rav_graph_issue(rav_ctx* ctx, void (*issue)(rav_ctx*), hipGraphExec_t* slot);   // the same, own graph
rav_status rav_upload_tasks(rav_ctx* ctx, const std::vector<rav::BlockTask>& logical, rav::BlockTask** out, int* n);

// The finest level of a hierarchy as FGMRES sees it: n unknowns, the level's
// own iterate, right-hand side and residual vectors (device), and whether the
// patches are factored.
struct RavFinest {
  long long n;
  double *x, *b, *r;
  bool factored;
};

// Stabilized Q1-Q1 (rav_q1.hip), reached through the public entry points.
rav_status rav_q1_create(const rav_problem_desc* d, void* hip_stream, rav_ctx** out);
void rav_q1_free(rav_ctx* ctx);
rav_status rav_q1_factor(rav_ctx* ctx);
rav_status rav_q1_dofs(const rav_ctx* ctx, int level, long* n_total, long* n_free);
int rav_q1_n_levels(const rav_ctx* ctx);
rav_status rav_q1_n_patches(const rav_ctx* ctx, int level, long* n);
rav_status rav_q1_assemble_rhs(rav_ctx* ctx, const double* params, int n_params, double* b_dev);
rav_status rav_q1_assemble_rhs_lid(rav_ctx* ctx, double lid_u, double* b_dev);
rav_status rav_q1_residual(rav_ctx* ctx, int level, const double* x, const double* b, double* r, double* norm);
rav_status rav_q1_smooth(rav_ctx* ctx, int level, int sweeps, double* x, const double* b);
rav_status rav_q1_restrict(rav_ctx* ctx, int level, const double* rf, double* bc);
rav_status rav_q1_prolong_add(rav_ctx* ctx, int level, const double* xc, double* xf);
rav_status rav_q1_coarse_solve(rav_ctx* ctx, const double* b0, double* x0);
rav_status rav_q1_vcycle(rav_ctx* ctx, double* x, const double* b);
RavFinest rav_q1_finest(rav_ctx* ctx);
void rav_q1_residual_finest(rav_ctx* ctx, bool with_norm);
void rav_q1_vcycle_finest(rav_ctx* ctx);
rav_status rav_q1_solve(rav_ctx* ctx, double* x, const double* b, double rtol, int maxit, int* iters,
                        double* rel_res);
rav_status rav_q1_map_patch(const rav_problem_desc* d, int level, long patch, int* dofs, int* n, int* owned);
rav_status rav_q1_map_owner(const rav_problem_desc* d, int level, int* owner);
rav_status rav_q1_get_owner(rav_ctx* ctx, int level, int* owner_dev);
rav_status rav_q1_get_patch_map(const rav_ctx* ctx, int level, long patch, int* dofs, int* n, int* owned);
rav_status rav_q1_get_patch_inverse(rav_ctx* ctx, int level, long patch, double* out, int* rows, int* cols);
rav_status rav_q1_time_sweep(rav_ctx* ctx, int level, int reps, double* x, const double* b, float* ms_res,
                             float* ms_apply);

// Stabilized Q1-Q1 on adaptive quadtree grids (rav_adapt.hip).
rav_status rav_ad_create(const rav_problem_desc* d, const int* leaves, const long* n_leaves, long lattice_x,
                         long lattice_y, void* hip_stream, rav_ctx** out);
void rav_ad_free(rav_ctx* ctx);
rav_status rav_ad_factor(rav_ctx* ctx);
rav_status rav_ad_dofs(const rav_ctx* ctx, int level, long* n_total, long* n_free);
int rav_ad_n_levels(const rav_ctx* ctx);
rav_status rav_ad_n_patches(const rav_ctx* ctx, int level, long* n);
rav_status rav_ad_assemble_rhs_lid(rav_ctx* ctx, double lid_u, double* b_dev);
rav_status rav_ad_assemble_rhs_dirichlet(rav_ctx* ctx, const double* ud_host, double* b_dev);
rav_status rav_ad_residual(rav_ctx* ctx, int level, const double* x, const double* b, double* r, double* norm);
rav_status rav_ad_smooth(rav_ctx* ctx, int level, int sweeps, double* x, const double* b);
rav_status rav_ad_restrict(rav_ctx* ctx, int level, const double* rf, double* bc);
rav_status rav_ad_prolong_add(rav_ctx* ctx, int level, const double* xc, double* xf);
rav_status rav_ad_coarse_solve(rav_ctx* ctx, const double* b0, double* x0);
rav_status rav_ad_vcycle(rav_ctx* ctx, double* x, const double* b);
RavFinest rav_ad_finest(rav_ctx* ctx);
void rav_ad_residual_finest(rav_ctx* ctx, bool with_norm);
void rav_ad_vcycle_finest(rav_ctx* ctx);
rav_status rav_ad_solve(rav_ctx* ctx, double* x, const double* b, double rtol, int maxit, int* iters,
                        double* rel_res);
rav_status rav_ad_get_owner(rav_ctx* ctx, int level, int* owner_dev);
rav_status rav_ad_get_patch_map(const rav_ctx* ctx, int level, long patch, int* dofs, int* n, int* owned);
rav_status rav_ad_get_patch_inverse(rav_ctx* ctx, int level, long patch, double* out, int* rows, int* cols);
rav_status rav_ad_time_sweep(rav_ctx* ctx, int level, int reps, double* x, const double* b, float* ms_res,
                             float* ms_apply);
rav_status rav_ad_level_info(const rav_ctx* ctx, int level, long* info);
rav_status rav_ad_host_export(const rav_problem_desc* d, const int* leaves, const long* n_leaves, long lattice_x,
                              long lattice_y, int level, int what, double* out, long* rows, long* cols);
