// Patch corrections of the three Vanka smoothers (Sec. 3).
//
// RAV (eq. 13, Sec. 4.3): x[owned(i)] += omega_i W_i r[I_i] where W_i holds the
//   owned rows of L_i^{-1}.  One lane per patch: the lane gathers r at the
//   patch's columns (the overlapping reads of neighbouring lanes hit the
//   caches) and streams its W_i with 16-byte loads from the chunk-major
//   layout, so a wavefront reads 1 KiB contiguously per load.  Owned sets
//   partition the DoFs, so the scatter needs no atomics and no colouring.
//   Low-precision W (FP32/BF16) is expanded to FP32 and accumulated in FP32;
//   the correction is added to the FP64 iterate.
// AV (eq. 12): the full L_i^{-1} r_i of every patch is written to a per-patch
//   buffer, then every DoF gathers the corrections of the patches that
//   contain it (deterministic, no atomics).
// MV (eqs. 11, 15): one launch per colour; patches of one colour touch
//   disjoint residual rows, so each wavefront recomputes its patch residual
//   b_i - L[I_i,:] x, applies L_i^{-1} and updates x[I_i] in place, which is
//   the sequential product of eq. (11) in colour-major order.
#include <hip/hip_runtime.h>

#include "rav_internal.h"

namespace rav {

struct bf16_t { unsigned short u; };

template <typename WT> struct WTraits;
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef unsigned int uvec4 __attribute__((ext_vector_type(4)));
template <> struct WTraits<double> { static constexpr int V = 2; typedef double acc_t; typedef dvec2 vec_t; };
template <> struct WTraits<float> { static constexpr int V = 4; typedef float acc_t; typedef fvec4 vec_t; };
template <> struct WTraits<bf16_t> { static constexpr int V = 8; typedef float acc_t; typedef uvec4 vec_t; };

template <typename WT>
__device__ __forceinline__ typename WTraits<WT>::acc_t vec_elem(const typename WTraits<WT>::vec_t& v, int i);
template <>
__device__ __forceinline__ double vec_elem<double>(const dvec2& v, int i) { return v[i]; }
template <>
__device__ __forceinline__ float vec_elem<float>(const fvec4& v, int i) { return v[i]; }
template <>
__device__ __forceinline__ float vec_elem<bf16_t>(const uvec4& v, int i) {
  const unsigned w = v[i >> 1];
  const unsigned bits = (i & 1) ? (w & 0xffff0000u) : (w << 16);
  return __uint_as_float(bits);
}

// Global index of local column `l` of the patch anchored at k, -1 if the
// column is outside the grid (masked columns carry r = 0 and zero weights).
template <int DIM, int KIND>
__device__ __forceinline__ long long patch_col(const Geo& g, const int* k, int l) {
  if (KIND == KIND_VERTEX) {
    constexpr int NV = ipow(5, DIM);
    if (l < DIM * NV) {
      const int c = l / NV;
      int r = l % NV;
      int a[3] = {0, 0, 0};
      bool ok = true;
      for (int d = 0; d < DIM; ++d) {
        a[d] = 2 * k[d] + (r % 5) - 2;
        r /= 5;
        ok = ok && a[d] >= 0 && a[d] <= 2 * g.N;
      }
      return ok ? c * g.nV + node_lin(g, a) : -1;
    }
    return DIM * g.nV + vert_lin(g, k);
  }
  constexpr int NV = ipow(3, DIM);
  if (l < DIM * NV) {
    const int c = l / NV;
    int r = l % NV;
    int a[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) { a[d] = 2 * k[d] + (r % 3); r /= 3; }
    return c * g.nV + node_lin(g, a);
  }
  int r = l - DIM * NV;
  int v[3] = {0, 0, 0};
  for (int d = 0; d < DIM; ++d) { v[d] = k[d] + (r & 1); r >>= 1; }
  return DIM * g.nV + vert_lin(g, v);
}

// ---- RAV apply: column and owned-DoF maps with compile-time dimension ------
typedef __attribute__((address_space(1))) const double gcdouble;
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) const char gcchar;

// Level sizes held in registers by the apply kernel.
struct ColMap {
  unsigned nn, nV, np1, twoN;
  unsigned dmask;
};

// Global index of local column l of the patch anchored at k.  Vertex-patch
// columns outside the grid are clamped to an in-range node: the owned inverse
// rows are exactly zero there (padding columns of the local matrix are unit
// rows and columns), and r at the clamped node is a finite residual, so the
// product contributes nothing.  Element-patch columns are always inside.
// With a wave-uniform l the decoding stays on the scalar unit.
template <int DIM, int KIND>
__device__ __forceinline__ unsigned col_index(const ColMap& cm, const int* k, int l) {
  constexpr int NN = KIND == KIND_VERTEX ? ipow(5, DIM) : ipow(3, DIM);
  if (l < DIM * NN) {
    const int c = l / NN;
    int r = l - c * NN;
    unsigned lin = 0, st = 1;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      int a;
      if (KIND == KIND_VERTEX) {
        a = 2 * k[d] + r % 5 - 2;
        a = min(max(a, 0), (int)cm.twoN);
        r /= 5;
      } else {
        a = 2 * k[d] + r % 3;
        r /= 3;
      }
      lin += st * (unsigned)a;
      st *= cm.nn;
    }
    return (unsigned)c * cm.nV + lin;
  }
  int r = l - DIM * NN;
  unsigned lin = 0, st = 1;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    lin += st * (unsigned)(k[d] + (KIND == KIND_VERTEX ? 0 : (r & 1)));
    r >>= 1;
    st *= cm.np1;
  }
  return (unsigned)DIM * cm.nV + lin;
}

// Global index of local DoF l of the patch (compile-time l), -1 for padding
// (outside the grid or on a masked side).
template <int DIM, int KIND>
__device__ __forceinline__ long long own_index(const ColMap& cm, const int* k, int l) {
  constexpr int NN = KIND == KIND_VERTEX ? ipow(5, DIM) : ipow(3, DIM);
  if (l < DIM * NN) {
    const int c = l / NN;
    int r = l - c * NN;
    unsigned lin = 0, st = 1;
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const int a = KIND == KIND_VERTEX ? 2 * k[d] + r % 5 - 2 : 2 * k[d] + r % 3;
      r /= KIND == KIND_VERTEX ? 5 : 3;
      ok = ok && a >= 0 && a <= (int)cm.twoN;
      ok = ok && !(((cm.dmask >> (2 * d)) & 1u) && a == 0) && !(((cm.dmask >> (2 * d + 1)) & 1u) && a == (int)cm.twoN);
      lin += st * (unsigned)a;
      st *= cm.nn;
    }
    return ok ? (long long)((unsigned)c * cm.nV + lin) : -1;
  }
  int r = l - DIM * NN;
  unsigned lin = 0, st = 1;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    lin += st * (unsigned)(k[d] + (KIND == KIND_VERTEX ? 0 : (r & 1)));
    r >>= 1;
    st *= cm.np1;
  }
  return (long long)((unsigned)DIM * cm.nV + lin);
}

__device__ __forceinline__ double ldr(gcdouble* base, unsigned idx) {
  return *(gcdouble*)((gcchar*)base + ((size_t)idx << 3));
}

__host__ __device__ constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

// Columns are processed in groups of G = V / gcd(nown, V) so that every group
// starts on a 16-byte chunk boundary: the group loop runs at run time (small
// code, bounded registers), the chunks inside a group and the ragged tail are
// unrolled at compile time.  SPLIT lanes share one patch (column groups dealt
// round-robin, partial sums combined with shuffles): SPLIT = 1 streams the
// large levels, SPLIT = 8 and 32 shorten the dependent load chain on smaller
// levels where too few wavefronts exist to hide memory latency.
template <int DIM, int KIND, int CLS, typename WT, int SPLIT>
__device__ __forceinline__ void rav_apply_body(const GridDev* __restrict__ G, const BlockTask t) {
  typedef typename WTraits<WT>::acc_t acc_t;
  typedef typename WTraits<WT>::vec_t vec_t;
  constexpr int V = WTraits<WT>::V;
  constexpr int NPAD = patch_npad(DIM, KIND);
  constexpr int NOWN = bucket_nown(DIM, KIND, CLS);
  constexpr int GC = V / gcd_c(NOWN, V);      // columns per group
  constexpr int CPG = GC * NOWN / V;          // 16-byte chunks per group
  constexpr int NG = NPAD / GC;               // full groups
  constexpr int TAIL = NPAD - NG * GC;        // leftover columns
  constexpr int TAIL_E = TAIL * NOWN;
  constexpr int TAIL_CH = (TAIL_E + V - 1) / V;
  if (t.grid < 0) return;
  const GridDev& gd = G[t.grid];
  if (grid_idle(gd)) return;
  const Bucket& bk = gd.bk[t.part];
  const int sl = SPLIT > 1 ? (int)(threadIdx.x % SPLIT) : 0;
  const long long p = t.start + threadIdx.x / SPLIT;
  if (p >= bk.count) return;   // whole groups of SPLIT lanes leave together
  const Geo& g = gd.g;
  int k[3] = {0, 0, 0};
  bucket_anchor(g, KIND, CLS, p, k);
  const ColMap cm{(unsigned)g.nn, (unsigned)g.nV, (unsigned)g.np1, 2u * (unsigned)g.N, g.dmask};
  gcdouble* __restrict__ r = (gcdouble*)gd.r;
  typedef __attribute__((address_space(1))) const vec_t gcvec;
  gcvec* __restrict__ W = (gcvec*)bk.W + w_vec(bk, p, 0);
  const long long cs = bk.count_pad;   // chunk stride in vectors (chunk-major layout)
  // Patches with few owned rows read their x entries and weight up front: no
  // other patch writes them, and the update at the end then waits on nothing.
  constexpr bool XPRE = NOWN <= 12;
  gdouble* __restrict__ x = (gdouble*)gd.x;
  int xi[XPRE ? NOWN : 1];   // level vectors hold fewer than 2^28 entries
  double xo[XPRE ? NOWN : 1];
  double om = 0.0;
  if constexpr (XPRE) {
#pragma unroll
    for (int j = 0; j < NOWN; ++j) {
      xi[j] = (int)own_index<DIM, KIND>(cm, k, bucket_own_local(DIM, KIND, CLS, j));
      xo[j] = (xi[j] >= 0 && (SPLIT == 1 || (j % SPLIT) == sl)) ? x[xi[j]] : 0.0;
    }
    om = gd.omega_patch ? (double)gd.omega_patch[patch_lin(g, KIND, k)] : gd.omega;
  }
  acc_t acc[NOWN];
#pragma unroll
  for (int j = 0; j < NOWN; ++j) acc[j] = acc_t(0);
#pragma unroll 1
  for (int gi = sl; gi < NG; gi += SPLIT) {
    vec_t w[CPG];
#pragma unroll
    for (int i = 0; i < CPG; ++i) w[i] = __builtin_nontemporal_load(W + (long long)(gi * CPG + i) * cs);
    acc_t rv[GC];
#pragma unroll
    for (int q = 0; q < GC; ++q) rv[q] = acc_t(ldr(r, col_index<DIM, KIND>(cm, k, gi * GC + q)));
#pragma unroll
    for (int i = 0; i < CPG; ++i) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int el = i * V + v;
        acc[el % NOWN] += vec_elem<WT>(w[i], v) * rv[el / NOWN];
      }
    }
  }
  if constexpr (TAIL > 0) {
    if (sl == SPLIT - 1) {
      vec_t w[TAIL_CH];
#pragma unroll
      for (int i = 0; i < TAIL_CH; ++i) w[i] = __builtin_nontemporal_load(W + (long long)(NG * CPG + i) * cs);
      acc_t rv[TAIL];
#pragma unroll
      for (int q = 0; q < TAIL; ++q) rv[q] = acc_t(ldr(r, col_index<DIM, KIND>(cm, k, NG * GC + q)));
#pragma unroll
      for (int el = 0; el < TAIL_E; ++el) acc[el % NOWN] += vec_elem<WT>(w[el / V], el % V) * rv[el / NOWN];
    }
  }
  if constexpr (SPLIT > 1) {
#pragma unroll
    for (int j = 0; j < NOWN; ++j) {
#pragma unroll
      for (int o = SPLIT / 2; o > 0; o >>= 1) acc[j] += __shfl_xor(acc[j], o, SPLIT);
    }
  }
  if constexpr (XPRE) {
#pragma unroll
    for (int j = 0; j < NOWN; ++j) {
      if (SPLIT > 1 && (j % SPLIT) != sl) continue;
      if (xi[j] >= 0) x[xi[j]] = xo[j] + om * (double)acc[j];
    }
  } else {
    om = gd.omega_patch ? (double)gd.omega_patch[patch_lin(g, KIND, k)] : gd.omega;
#pragma unroll
    for (int j = 0; j < NOWN; ++j) {
      if (SPLIT > 1 && (j % SPLIT) != sl) continue;
      const long long gi = own_index<DIM, KIND>(cm, k, bucket_own_local(DIM, KIND, CLS, j));
      if (gi >= 0) x[gi] += om * (double)acc[j];
    }
  }
}

template <int DIM, int KIND, int CLS, typename WT, int SPLIT>
__global__ __launch_bounds__(APPLY_BLOCK_MAX) void k_rav_apply(const GridDev* __restrict__ G,
                                                      const BlockTask* __restrict__ tasks) {
  rav_apply_body<DIM, KIND, CLS, WT, SPLIT>(G, tasks[blockIdx.x]);
}

// ---- RAV apply from the factored inverse (vertex patches) --------------------
// With A_i = I_d (x) K and one pressure (k_factor's block structure) the owned
// rows of L_i^{-1} applied to r_i are
//   u = S^{-1} (z^T r_u - r_p),   y_c[a] = sum_j K^{-1}[a][j] r_c[j] + z_c[a] u,   y_p = -u
// for the owned nodes a, with z = K^{-1} B.  Stored per patch, node-major (see
// fact_nvals): 151 values for a 2D vertex patch instead of the 459 of its
// owned rows, 1,376 for a 3D one instead of 9,400, so the stream of W, which
// bounds the sweep, is 3x (2D) to 7x (3D) shorter.  Nodes are processed in
// groups that start on a 16-byte chunk boundary, as the columns of the
// row-format kernel; SPLIT lanes share a patch the same way.
template <typename WT>
__device__ __forceinline__ typename WTraits<WT>::acc_t fact_elem(
    const __attribute__((address_space(1))) typename WTraits<WT>::vec_t* __restrict__ W, long long cs, int e) {
  constexpr int V = WTraits<WT>::V;
  return vec_elem<WT>(__builtin_nontemporal_load(W + (long long)(e / V) * cs), e % V);
}

template <int DIM, typename WT, int SPLIT>
__device__ __forceinline__ void rav_apply_fact_body(const GridDev* __restrict__ G, const BlockTask t) {
  typedef typename WTraits<WT>::acc_t acc_t;
  typedef typename WTraits<WT>::vec_t vec_t;
  constexpr int KIND = KIND_VERTEX;
  constexpr int V = WTraits<WT>::V;
  constexpr int NN = fact_nn(DIM);
  constexpr int NO = fact_nown_nodes(DIM);    // owned nodes
  constexpr int GV = fact_per_node(DIM);      // values per node
  constexpr int GN = V / gcd_c(GV, V);        // nodes per group
  constexpr int CPG = GN * GV / V;            // 16-byte chunks per group
  constexpr int NG = NN / GN;
  constexpr int TAILN = NN - NG * GN;
  constexpr int TAIL_E = TAILN * GV;
  constexpr int TAIL_CH = (TAIL_E + V - 1) / V;
  constexpr int SINV = NN * GV;               // element index of S^{-1}
  if (t.grid < 0) return;
  const GridDev& gd = G[t.grid];
  if (grid_idle(gd)) return;
  const Bucket& bk = gd.bk[t.part];
  const int sl = SPLIT > 1 ? (int)(threadIdx.x % SPLIT) : 0;
  const long long p = t.start + threadIdx.x / SPLIT;
  if (p >= bk.count) return;   // whole groups of SPLIT lanes leave together
  const Geo& g = gd.g;
  int k[3] = {0, 0, 0};
  bucket_anchor(g, KIND, 0, p, k);
  const ColMap cm{(unsigned)g.nn, (unsigned)g.nV, (unsigned)g.np1, 2u * (unsigned)g.N, g.dmask};
  gcdouble* __restrict__ r = (gcdouble*)gd.r;
  typedef __attribute__((address_space(1))) const vec_t gcvec;
  gcvec* __restrict__ W = (gcvec*)bk.W + w_vec(bk, p, 0);
  const long long cs = bk.count_pad;
  acc_t y[DIM][NO], tz = acc_t(0);
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int a = 0; a < NO; ++a) y[c][a] = acc_t(0);
#pragma unroll 1
  for (int gi = sl; gi < NG; gi += SPLIT) {
    vec_t w[CPG];
#pragma unroll
    for (int i = 0; i < CPG; ++i) w[i] = __builtin_nontemporal_load(W + (long long)(gi * CPG + i) * cs);
    acc_t rv[GN][DIM];
#pragma unroll
    for (int i = 0; i < GN; ++i)
#pragma unroll
      for (int c = 0; c < DIM; ++c) rv[i][c] = acc_t(ldr(r, col_index<DIM, KIND>(cm, k, c * NN + gi * GN + i)));
#pragma unroll
    for (int el = 0; el < GN * GV; ++el) {
      const int i = el / GV, q = el % GV;
      const acc_t v = vec_elem<WT>(w[el / V], el % V);
      if (q < NO) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) y[c][q] += v * rv[i][c];
      } else {
        tz += v * rv[i][q - NO];
      }
    }
  }
  if constexpr (TAILN > 0) {
    if (sl == SPLIT - 1) {
      vec_t w[TAIL_CH];
#pragma unroll
      for (int i = 0; i < TAIL_CH; ++i) w[i] = __builtin_nontemporal_load(W + (long long)(NG * CPG + i) * cs);
      acc_t rv[TAILN][DIM];
#pragma unroll
      for (int i = 0; i < TAILN; ++i)
#pragma unroll
        for (int c = 0; c < DIM; ++c) rv[i][c] = acc_t(ldr(r, col_index<DIM, KIND>(cm, k, c * NN + NG * GN + i)));
#pragma unroll
      for (int el = 0; el < TAIL_E; ++el) {
        const int i = el / GV, q = el % GV;
        const acc_t v = vec_elem<WT>(w[el / V], el % V);
        if (q < NO) {
#pragma unroll
          for (int c = 0; c < DIM; ++c) y[c][q] += v * rv[i][c];
        } else {
          tz += v * rv[i][q - NO];
        }
      }
    }
  }
  if constexpr (SPLIT > 1) {
#pragma unroll
    for (int o = SPLIT / 2; o > 0; o >>= 1) {
      tz += __shfl_xor(tz, o, SPLIT);
#pragma unroll
      for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int a = 0; a < NO; ++a) y[c][a] += __shfl_xor(y[c][a], o, SPLIT);
    }
  }
  // u = S^{-1} (z^T r_u - r_p); then the owned rows get z_c[a] u
  const acc_t u = fact_elem<WT>(W, cs, SINV) * (tz - acc_t(ldr(r, col_index<DIM, KIND>(cm, k, DIM * NN))));
  const double om = gd.omega_patch ? (double)gd.omega_patch[patch_lin(g, KIND, k)] : gd.omega;
  gdouble* __restrict__ x = (gdouble*)gd.x;
#pragma unroll
  for (int j = 0; j <= DIM * NO; ++j) {
    if (SPLIT > 1 && (j % SPLIT) != sl) continue;
    const int l = bucket_own_local(DIM, KIND, 0, j);
    acc_t val;
    if (j < DIM * NO) {
      const int c = j / NO, a = j % NO;
      const int node = bucket_own_local(DIM, KIND, 0, a);   // component 0: local index = node
      val = y[c][a] + fact_elem<WT>(W, cs, node * GV + NO + c) * u;
    } else {
      val = -u;
    }
    const long long gi = own_index<DIM, KIND>(cm, k, l);
    if (gi >= 0) x[gi] += om * (double)val;
  }
}

template <int DIM, typename WT, int SPLIT>
__global__ __launch_bounds__(APPLY_BLOCK_MAX) void k_rav_apply_fact(const GridDev* __restrict__ G,
                                                                   const BlockTask* __restrict__ tasks) {
  rav_apply_fact_body<DIM, WT, SPLIT>(G, tasks[blockIdx.x]);
}

// Row-parallel RAV apply for tiny buckets: one wavefront per patch, lane j
// accumulates owned rows j and j + 64 over the patch columns.  The column loop
// is wave-uniform (the r value of a column is one broadcast load), so the
// per-lane state is two accumulators however many rows the bucket owns.
// Arithmetic as in the column-group kernel: FP64 for FP64 rows, FP32 products
// and accumulation (r rounded to FP32) for FP32 and BF16 rows.
template <typename WT> __device__ __forceinline__ typename WTraits<WT>::acc_t w_elem(const WT* W, long long i);
template <> __device__ __forceinline__ double w_elem<double>(const double* W, long long i) {
  return ((gcdouble*)W)[i];
}
template <> __device__ __forceinline__ float w_elem<float>(const float* W, long long i) {
  return ((__attribute__((address_space(1))) const float*)W)[i];
}
template <> __device__ __forceinline__ float w_elem<bf16_t>(const bf16_t* W, long long i) {
  const unsigned short u = ((__attribute__((address_space(1))) const unsigned short*)W)[i];
  return __uint_as_float((unsigned)u << 16);
}

template <int DIM, int KIND, typename WT>
__device__ __forceinline__ void rav_apply_rows_body(const GridDev* __restrict__ G, const BlockTask t) {
  constexpr int NPAD = patch_npad(DIM, KIND);
  constexpr int V = WTraits<WT>::V;
  if (t.grid < 0) return;
  const GridDev& gd = G[t.grid];
  if (grid_idle(gd)) return;
  const Bucket& bk = gd.bk[t.part];
  const long long p = t.start + (threadIdx.x >> 6);
  if (p >= bk.count) return;   // whole wavefronts leave together
  const int j = threadIdx.x & 63;
  const Geo& g = gd.g;
  int k[3] = {0, 0, 0};
  bucket_anchor(g, KIND, bk.cls, p, k);
  const ColMap cm{(unsigned)g.nn, (unsigned)g.nV, (unsigned)g.np1, 2u * (unsigned)g.N, g.dmask};
  gcdouble* __restrict__ r = (gcdouble*)gd.r;
  const WT* __restrict__ W = reinterpret_cast<const WT*>(bk.W);
  const int nown = bk.nown;
  const long long cp = bk.count_pad;
  typedef typename WTraits<WT>::acc_t acc_t;
  acc_t acc[2] = {acc_t(0), acc_t(0)};
#pragma unroll 16
  for (int c = 0; c < NPAD; ++c) {
    const acc_t rv = acc_t(ldr(r, col_index<DIM, KIND>(cm, k, c)));
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      // unconditional load at a clamped row (no branch, so the unrolled loads stay in flight)
      const int jj = j + 64 * h;
      const long long e = (long long)c * nown + min(jj, nown - 1);
      const acc_t w = w_elem<WT>(W, ((e / V) * cp + p) * V + e % V);
      acc[h] += jj < nown ? w * rv : acc_t(0);
    }
  }
  const double om = gd.omega_patch ? (double)gd.omega_patch[patch_lin(g, KIND, k)] : gd.omega;
  gdouble* __restrict__ x = (gdouble*)gd.x;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int jj = j + 64 * h;
    if (jj >= nown) continue;
    const long long gi = own_index<DIM, KIND>(cm, k, bucket_own_local(DIM, KIND, bk.cls, jj));
    if (gi >= 0) x[gi] += om * (double)acc[h];
  }
}

template <int DIM, int KIND, typename WT>
__global__ __launch_bounds__(APPLY_BLOCK_MAX) void k_rav_apply_rows(const GridDev* __restrict__ G,
                                                                   const BlockTask* __restrict__ tasks) {
  rav_apply_rows_body<DIM, KIND, WT>(G, tasks[blockIdx.x]);
}

// The boundary buckets of a level in one launch of 256-thread blocks: each
// block runs the variant its task names (pad = 4 or APPLY_SPLIT lanes per
// patch, or APPLY_ROWS) for its bucket's class.  Separate launches of these small, latency-bound buckets
// ran one after another with a launch gap each.
// EDGES = false leaves out the column-group bodies of the 3D edge and corner
// classes (3, 5, 6, 7: up to 28 owned rows), whose registers would set the
// whole launch's occupancy; the host then sends no column-group task of those
// classes (their buckets, at most N - 1 patches, go row-parallel up to N = 65).
template <int DIM, int KIND, typename WT, int SPLIT, bool EDGES>
__device__ __forceinline__ void multi_body(const GridDev* __restrict__ G, const BlockTask t) {
  const int cls = G[t.grid].bk[t.part].cls;
  if constexpr (DIM == 3 && KIND == KIND_ELEMENT) {
    switch (cls) {
      case 0: rav_apply_body<3, KIND_ELEMENT, 0, WT, SPLIT>(G, t); break;
      case 1: rav_apply_body<3, KIND_ELEMENT, 1, WT, SPLIT>(G, t); break;
      case 2: rav_apply_body<3, KIND_ELEMENT, 2, WT, SPLIT>(G, t); break;
      case 4: rav_apply_body<3, KIND_ELEMENT, 4, WT, SPLIT>(G, t); break;
      default:
        if constexpr (EDGES) {
          switch (cls) {
            case 3: rav_apply_body<3, KIND_ELEMENT, 3, WT, SPLIT>(G, t); break;
            case 5: rav_apply_body<3, KIND_ELEMENT, 5, WT, SPLIT>(G, t); break;
            case 6: rav_apply_body<3, KIND_ELEMENT, 6, WT, SPLIT>(G, t); break;
            default: rav_apply_body<3, KIND_ELEMENT, 7, WT, SPLIT>(G, t); break;
          }
        }
        break;
    }
  } else if constexpr (KIND == KIND_ELEMENT) {
    switch (cls) {
      case 0: rav_apply_body<2, KIND_ELEMENT, 0, WT, SPLIT>(G, t); break;
      case 1: rav_apply_body<2, KIND_ELEMENT, 1, WT, SPLIT>(G, t); break;
      case 2: rav_apply_body<2, KIND_ELEMENT, 2, WT, SPLIT>(G, t); break;
      default: rav_apply_body<2, KIND_ELEMENT, 3, WT, SPLIT>(G, t); break;
    }
  } else {
    rav_apply_body<DIM, KIND, 0, WT, SPLIT>(G, t);
  }
}

template <int DIM, int KIND, typename WT, bool EDGES>
__global__ __launch_bounds__(APPLY_BLOCK_MAX) void k_rav_apply_multi(const GridDev* __restrict__ G,
                                                                    const BlockTask* __restrict__ tasks) {
  const BlockTask t = tasks[blockIdx.x];
  if (t.grid < 0) return;
  if (t.pad == APPLY_ROWS) {
    rav_apply_rows_body<DIM, KIND, WT>(G, t);
    return;
  }
  if (t.pad == 4) multi_body<DIM, KIND, WT, 4, EDGES>(G, t);
  else multi_body<DIM, KIND, WT, APPLY_SPLIT, EDGES>(G, t);
}

void launch_rav_apply_multi(int dim, int kind, int prec, bool edges, const GridDev* G, const BlockTask* tasks,
                            int ntasks, hipStream_t s) {
#define RAV_MULTI(D, K, E)                                                                                   \
  do {                                                                                                       \
    if (prec == P_FP64)                                                                                      \
      hipLaunchKernelGGL((k_rav_apply_multi<D, K, double, E>), dim3(ntasks), dim3(APPLY_BLOCK_MAX), 0, s, G, tasks); \
    else if (prec == P_FP32)                                                                                 \
      hipLaunchKernelGGL((k_rav_apply_multi<D, K, float, E>), dim3(ntasks), dim3(APPLY_BLOCK_MAX), 0, s, G, tasks);  \
    else                                                                                                     \
      hipLaunchKernelGGL((k_rav_apply_multi<D, K, bf16_t, E>), dim3(ntasks), dim3(APPLY_BLOCK_MAX), 0, s, G, tasks); \
  } while (0)
  if (dim == 2 && kind == KIND_VERTEX) RAV_MULTI(2, KIND_VERTEX, true);
  else if (dim == 2) RAV_MULTI(2, KIND_ELEMENT, true);
  else if (kind == KIND_VERTEX) RAV_MULTI(3, KIND_VERTEX, true);
  else if (edges) RAV_MULTI(3, KIND_ELEMENT, true);
  else RAV_MULTI(3, KIND_ELEMENT, false);
#undef RAV_MULTI
}

template <int DIM, int KIND>
static void launch_apply_rows(int prec, const GridDev* G, const BlockTask* tasks, int ntasks, hipStream_t s) {
  if (prec == P_FP64)
    hipLaunchKernelGGL((k_rav_apply_rows<DIM, KIND, double>), dim3(ntasks), dim3(APPLY_BLOCK_MAX), 0, s, G, tasks);
  else if (prec == P_FP32)
    hipLaunchKernelGGL((k_rav_apply_rows<DIM, KIND, float>), dim3(ntasks), dim3(APPLY_BLOCK_MAX), 0, s, G, tasks);
  else
    hipLaunchKernelGGL((k_rav_apply_rows<DIM, KIND, bf16_t>), dim3(ntasks), dim3(APPLY_BLOCK_MAX), 0, s, G, tasks);
}

template <int DIM, int KIND, typename WT, int SPLIT>
static void launch_apply_t(int cls, const GridDev* G, const BlockTask* tasks, int ntasks, hipStream_t s) {
#define RAV_APPLY_CASE(C)                                                                                 \
  case C:                                                                                                \
    hipLaunchKernelGGL((k_rav_apply<DIM, KIND, C, WT, SPLIT>), dim3(ntasks), dim3(apply_block(SPLIT)), 0, s, G, tasks); \
    break;
  if constexpr (KIND == KIND_VERTEX) {
    hipLaunchKernelGGL((k_rav_apply<DIM, KIND, 0, WT, SPLIT>), dim3(ntasks), dim3(apply_block(SPLIT)), 0, s, G, tasks);
  } else if constexpr (DIM == 2) {
    switch (cls) {
      RAV_APPLY_CASE(0)
      RAV_APPLY_CASE(1)
      RAV_APPLY_CASE(2)
      RAV_APPLY_CASE(3)
      default: break;
    }
  } else {
    switch (cls) {
      RAV_APPLY_CASE(0)
      RAV_APPLY_CASE(1)
      RAV_APPLY_CASE(2)
      RAV_APPLY_CASE(3)
      RAV_APPLY_CASE(4)
      RAV_APPLY_CASE(5)
      RAV_APPLY_CASE(6)
      RAV_APPLY_CASE(7)
      default: break;
    }
  }
#undef RAV_APPLY_CASE
}

template <int DIM, int KIND, int SPLIT>
static void launch_apply_k(int cls, int prec, const GridDev* G, const BlockTask* tasks, int ntasks, hipStream_t s) {
  if (prec == P_FP64) launch_apply_t<DIM, KIND, double, SPLIT>(cls, G, tasks, ntasks, s);
  else if (prec == P_FP32) launch_apply_t<DIM, KIND, float, SPLIT>(cls, G, tasks, ntasks, s);
  else launch_apply_t<DIM, KIND, bf16_t, SPLIT>(cls, G, tasks, ntasks, s);
}

template <int SPLIT>
static void launch_apply_s(int dim, int kind, int cls, int prec, const GridDev* G, const BlockTask* tasks,
                           int ntasks, hipStream_t s) {
  if (dim == 2 && kind == KIND_VERTEX) launch_apply_k<2, KIND_VERTEX, SPLIT>(cls, prec, G, tasks, ntasks, s);
  else if (dim == 2) launch_apply_k<2, KIND_ELEMENT, SPLIT>(cls, prec, G, tasks, ntasks, s);
  else if (kind == KIND_VERTEX) launch_apply_k<3, KIND_VERTEX, SPLIT>(cls, prec, G, tasks, ntasks, s);
  else launch_apply_k<3, KIND_ELEMENT, SPLIT>(cls, prec, G, tasks, ntasks, s);
}

template <int DIM, int SPLIT>
static void launch_fact_k(int prec, const GridDev* G, const BlockTask* tasks, int ntasks, hipStream_t s) {
  const dim3 grid(ntasks), blk(apply_block(SPLIT));
  if (prec == P_FP64) hipLaunchKernelGGL((k_rav_apply_fact<DIM, double, SPLIT>), grid, blk, 0, s, G, tasks);
  else if (prec == P_FP32) hipLaunchKernelGGL((k_rav_apply_fact<DIM, float, SPLIT>), grid, blk, 0, s, G, tasks);
  else hipLaunchKernelGGL((k_rav_apply_fact<DIM, bf16_t, SPLIT>), grid, blk, 0, s, G, tasks);
}

template <int SPLIT>
static void launch_fact_s(int dim, int prec, const GridDev* G, const BlockTask* tasks, int ntasks, hipStream_t s) {
  if (dim == 2) launch_fact_k<2, SPLIT>(prec, G, tasks, ntasks, s);
  else launch_fact_k<3, SPLIT>(prec, G, tasks, ntasks, s);
}

void launch_rav_apply(int dim, int kind, int cls, int prec, int split, const GridDev* G, const BlockTask* tasks,
                      int ntasks, hipStream_t s, int factored) {
  if (factored) {   // vertex patches; tiny buckets take the widest split (no row-parallel variant)
    if (split == APPLY_SPLIT_SMALL || split == APPLY_ROWS) launch_fact_s<APPLY_SPLIT_SMALL>(dim, prec, G, tasks, ntasks, s);
    else if (split == 4) launch_fact_s<4>(dim, prec, G, tasks, ntasks, s);
    else if (split > 1) launch_fact_s<APPLY_SPLIT>(dim, prec, G, tasks, ntasks, s);
    else launch_fact_s<1>(dim, prec, G, tasks, ntasks, s);
    return;
  }
  if (split == APPLY_ROWS) {
    if (dim == 2 && kind == KIND_VERTEX) launch_apply_rows<2, KIND_VERTEX>(prec, G, tasks, ntasks, s);
    else if (dim == 2) launch_apply_rows<2, KIND_ELEMENT>(prec, G, tasks, ntasks, s);
    else if (kind == KIND_VERTEX) launch_apply_rows<3, KIND_VERTEX>(prec, G, tasks, ntasks, s);
    else launch_apply_rows<3, KIND_ELEMENT>(prec, G, tasks, ntasks, s);
    return;
  }
  if (split == APPLY_SPLIT_SMALL) launch_apply_s<APPLY_SPLIT_SMALL>(dim, kind, cls, prec, G, tasks, ntasks, s);
  else if (split == 4) launch_apply_s<4>(dim, kind, cls, prec, G, tasks, ntasks, s);
  else if (split > 1) launch_apply_s<APPLY_SPLIT>(dim, kind, cls, prec, G, tasks, ntasks, s);
  else launch_apply_s<1>(dim, kind, cls, prec, G, tasks, ntasks, s);
}

// ---- AV ---------------------------------------------------------------------
// One wavefront per patch; lane l owns local rows l and l + 64.  The patch's
// residual entries are loaded once, in parallel, into LDS; the column loop
// then streams the inverse (one coalesced column per step) against them.
template <int DIM, int KIND>
__global__ __launch_bounds__(64) void k_av_apply(const GridDev* __restrict__ G, long long npatch) {
  constexpr int NPAD = patch_npad(DIM, KIND);
  __shared__ double rs[NPAD];
  const long long p = blockIdx.x;
  if (p >= npatch) return;
  const GridDev& gd = *G;
  const Geo& g = gd.g;
  int k[3] = {0, 0, 0};
  patch_anchor(g, KIND, p, k);
  const double* __restrict__ Wi = gd.Winv + p * (long long)NPAD * NPAD;
  const int lane = threadIdx.x;
  for (int l = lane; l < NPAD; l += 64) {
    const long long gi = patch_col<DIM, KIND>(g, k, l);
    rs[l] = gi >= 0 ? gd.r[gi] : 0.0;
  }
  __syncthreads();
  double y0 = 0.0, y1 = 0.0;
#pragma unroll 4
  for (int c = 0; c < NPAD; ++c) {
    const double rc = rs[c];
    if (lane < NPAD) y0 += Wi[c * NPAD + lane] * rc;
    if (lane + 64 < NPAD) y1 += Wi[c * NPAD + lane + 64] * rc;
  }
  const double om = gd.omega_patch ? (double)gd.omega_patch[p] : gd.omega;
  if (lane < NPAD) gd.Y[p * NPAD + lane] = om * y0;
  if (lane + 64 < NPAD) gd.Y[p * NPAD + lane + 64] = om * y1;
}

// x[i] += sum over patches q containing DoF i of Y[q][local index of i in q].
template <int DIM, int KIND>
__global__ __launch_bounds__(256) void k_av_gather(const GridDev* __restrict__ G, long long n) {
  constexpr int NPAD = patch_npad(DIM, KIND);
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const GridDev& gd = *G;
  const Geo& g = gd.g;
  int a[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  int comp;
  if (i < DIM * g.nV) {
    long long nl_;
    comp = split_vel(g, i, &nl_);
    node_of(g, nl_, a);
    if (node_dirichlet(g, a)) return;
    for (int d = 0; d < DIM; ++d) {
      if (KIND == KIND_VERTEX) {   // 2k - 2 <= a <= 2k + 2
        lo[d] = max((a[d] - 1) >> 1, 0);
        hi[d] = min((a[d] + 2) >> 1, g.N);
      } else {                     // 2e <= a <= 2e + 2
        lo[d] = max((a[d] - 1) >> 1, 0);
        hi[d] = min(a[d] >> 1, g.N - 1);
      }
    }
  } else {
    comp = DIM;
    vert_of(g, i - DIM * g.nV, a);
    for (int d = 0; d < DIM; ++d) {
      if (KIND == KIND_VERTEX) { lo[d] = a[d]; hi[d] = a[d]; }
      else { lo[d] = max(a[d] - 1, 0); hi[d] = min(a[d], g.N - 1); }
    }
  }
  double s = 0.0;
  for (int qz = (DIM == 3 ? lo[2] : 0); qz <= (DIM == 3 ? hi[2] : 0); ++qz)
    for (int qy = lo[1]; qy <= hi[1]; ++qy)
      for (int qx = lo[0]; qx <= hi[0]; ++qx) {
        int q[3] = {qx, qy, qz};
        int l = 0, st = 1;
        if (comp < DIM) {
          const int base = KIND == KIND_VERTEX ? 5 : 3;
          for (int d = 0; d < DIM; ++d) {
            l += (KIND == KIND_VERTEX ? a[d] - 2 * q[d] + 2 : a[d] - 2 * q[d]) * st;
            st *= base;
          }
          l += comp * ipow(base, DIM);
        } else if (KIND == KIND_VERTEX) {
          l = DIM * ipow(5, DIM);
        } else {
          for (int d = 0; d < DIM; ++d) { l += (a[d] - q[d]) * st; st *= 2; }
          l += DIM * ipow(3, DIM);
        }
        s += gd.Y[patch_lin(g, KIND, q) * NPAD + l];
      }
  gd.x[i] += s;
}

void launch_av_apply(int dim, int kind, const GridDev* G, long long npatch, hipStream_t s) {
  if (dim == 2 && kind == KIND_VERTEX) hipLaunchKernelGGL((k_av_apply<2, KIND_VERTEX>), dim3(npatch), dim3(64), 0, s, G, npatch);
  else if (dim == 2) hipLaunchKernelGGL((k_av_apply<2, KIND_ELEMENT>), dim3(npatch), dim3(64), 0, s, G, npatch);
  else hipLaunchKernelGGL((k_av_apply<3, KIND_ELEMENT>), dim3(npatch), dim3(64), 0, s, G, npatch);
}

void launch_av_gather(int dim, int kind, const GridDev* G, long long n, hipStream_t s) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (dim == 2 && kind == KIND_VERTEX) hipLaunchKernelGGL((k_av_gather<2, KIND_VERTEX>), dim3(nb), dim3(256), 0, s, G, n);
  else if (dim == 2) hipLaunchKernelGGL((k_av_gather<2, KIND_ELEMENT>), dim3(nb), dim3(256), 0, s, G, n);
  else hipLaunchKernelGGL((k_av_gather<3, KIND_ELEMENT>), dim3(nb), dim3(256), 0, s, G, n);
}


}  // namespace rav
