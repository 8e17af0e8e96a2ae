// Kernels of the stabilized Q1-Q1 levels on adaptive quadtree grids (Sec. 2,
// eqs. 5-8, Fig. 2) and of their Vanka smoothers (Sec. 3, eqs. 11-13).  The
// operator and the patch lists are stored as described in rav_adapt.h.
//
// Every kernel gathers: a thread (or a lane group) owns what it writes, so no
// atomics are needed and results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <climits>

#include "rav_adapt.h"

namespace rav {

namespace {

inline unsigned nblk(long long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Entry e of the row of vertex i: column j and tuple id.
template <bool WIDE>
__device__ __forceinline__ void entry(const AdDev& a, int i, long long e, int& j, int& id) {
  const unsigned w = a.ent[e];
  if (WIDE) {
    j = a.col[e];
    id = (int)w;
  } else {
    j = i + ((int)w >> a.id_bits);   // arithmetic shift keeps the offset's sign
    id = (int)(w & ((1u << a.id_bits) - 1u));
  }
}

// Patch vertex k of patch i (slot e).
template <bool WIDE>
__device__ __forceinline__ int patch_vertex(const AdDev& a, int, long long e) {
  return a.pv[e];
}

// Value of field p at (row vertex v, column vertex j); 0 if j is not in the row.
template <bool WIDE>
__device__ double lookup(const AdDev& a, int v, int j, int p) {
  const int e0 = a.soff[v >> 6], w = (a.soff[(v >> 6) + 1] - e0) >> 6;
  const int t = v & 63;
  double out = 0.0;
  for (int k = 0; k < w; ++k) {
    int jj, id;
    entry<WIDE>(a, v, e0 + 64LL * k + t, jj, id);
    if (jj == j) out += a.vtab[8 * id + p];   // one entry per column; padding entries hold zeros
  }
  return out;
}

// ---- patch factorization: one 64-lane block per configuration ----------------
// Gauss-Jordan elimination without pivoting on [K | b_x b_y | I] (K SPD,
// padded to AD_NFMAX with identity rows), giving z_c = K^{-1} b_c and K^{-1};
// then S = c - b_x.z_x - b_y.z_y (negative: c < 0 and K^{-1} SPD).  The
// matrix is read from the operator at the configuration's representative.
constexpr int NF = AD_NFMAX;
constexpr int NCOL = 2 * NF + 2;
constexpr int KI = NF + 2;

template <bool WIDE>
__global__ __launch_bounds__(64) void k_ad_factor(AdDev a, int mode, const int* __restrict__ rep, AdFactors f,
                                                  int* __restrict__ status) {
  __shared__ int verts[NF];
  __shared__ double M[NF][NCOL];
  __shared__ double bsave[2][NF];
  __shared__ double fac[NF];
  __shared__ double cii;
  const int c = blockIdx.x;
  const int i = rep[c];
  const int lane = threadIdx.x;
  const int sl = i >> 6, t = i & 63;
  const int p0 = a.poff[sl];
  const int nf = a.cnf[c];
  if (lane < NF) verts[lane] = lane < nf ? patch_vertex<WIDE>(a, i, p0 + 64LL * lane + t) : -1;
  __syncthreads();
  for (int idx = lane; idx < NF * NCOL; idx += 64) {
    const int row = idx / NCOL, col = idx % NCOL;
    const int vr = verts[row];
    double v;
    if (col >= KI) {
      v = (col - KI == row) ? 1.0 : 0.0;
    } else if (vr < 0) {
      v = (col == row) ? 1.0 : 0.0;
    } else if (col < NF) {
      const int vc = verts[col];
      v = vc < 0 ? 0.0 : lookup<WIDE>(a, vr, vc, AD_A);
    } else {
      v = lookup<WIDE>(a, vr, i, col == NF ? AD_BTX : AD_BTY);
    }
    if (col == NF || col == NF + 1) bsave[col - NF][row] = v;
    M[row][col] = v;
  }
  if (lane == 0) cii = lookup<WIDE>(a, i, i, AD_C);
  __syncthreads();
  bool bad = false;
  for (int p = 0; p < NF; ++p) {
    const double piv = M[p][p];
    if (!(piv > 0.0)) bad = true;
    const double inv = 1.0 / piv;
    __syncthreads();
    for (int j = lane; j < NCOL; j += 64) M[p][j] *= inv;
    for (int r = lane; r < NF; r += 64) fac[r] = M[r][p];
    __syncthreads();
    for (int idx = lane; idx < NF * NCOL; idx += 64) {
      const int r = idx / NCOL, j = idx % NCOL;
      if (r != p) M[r][j] -= fac[r] * M[p][j];
    }
    __syncthreads();
  }
  double part = 0.0;
  for (int idx = lane; idx < 2 * NF; idx += 64) {
    const int cc = idx / NF, m = idx % NF;
    part += bsave[cc][m] * M[m][NF + cc];
  }
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  const double S = cii - part;
  const double sinv = 1.0 / S;
  if (!(S < 0.0) || !isfinite(sinv)) bad = true;
  if (bad && lane == 0) atomicMin(status, i);
  if (lane < NF) {
    f.zx[c * NF + lane] = M[lane][NF];
    f.zy[c * NF + lane] = M[lane][NF + 1];
  }
  if (lane == 0) f.invS[c] = sinv;
  if (mode == AD_RAV) {
    const int ao = a.cown[c];
    if (lane < NF) f.kr[c * NF + lane] = ao >= 0 ? M[ao][KI + lane] : 0.0;
  } else {
    for (int idx = lane; idx < NF * NF; idx += 64) f.kfull[(long long)c * NF * NF + idx] = M[idx / NF][KI + idx % NF];
  }
}

// ---- per-vertex and per-patch bodies -------------------------------------------

// r = b - L x on the three rows of vertex i (masked velocity rows 0); returns
// the sum of their squares.
template <bool WIDE, bool LDS = false>
__device__ __forceinline__ double residual_vertex(const AdDev& a, int i, const double* __restrict__ x,
                                                  const double* __restrict__ b, double* __restrict__ r,
                                                  const double2* tab = nullptr) {
  const int nV = a.nV;
  const int e0 = a.soff[i >> 6], w = (a.soff[(i >> 6) + 1] - e0) >> 6;
  const int t = i & 63;
  double su = 0.0, sv = 0.0, sp = 0.0;
#pragma unroll 2
  for (int k = 0; k < w; ++k) {
    int j, id;
    entry<WIDE>(a, i, e0 + 64LL * k + t, j, id);
    const double2* vt = LDS ? tab + 3 * id : reinterpret_cast<const double2*>(a.vtab + 8 * id);
    const double2 v01 = vt[0], v23 = vt[1], v45 = vt[2];   // (A, BTx), (BTy, Bx), (By, C)
    const double uj = x[j], vj = x[nV + j], pj = x[2 * nV + j];
    su += v01.x * uj + v01.y * pj;
    sv += v01.x * vj + v23.x * pj;
    sp += v23.y * uj + v45.x * vj + v45.y * pj;
  }
  const bool vm = a.vmask[i] != 0;
  const double ru = vm ? 0.0 : b[i] - su;
  const double rv = vm ? 0.0 : b[nV + i] - sv;
  const double rp = b[2 * nV + i] - sp;
  r[i] = ru;
  r[nV + i] = rv;
  r[2 * nV + i] = rp;
  return ru * ru + rv * rv + rp * rp;
}

// RAV on patch i from the factored form: y_p = (r_p - z_x.r_x - z_y.r_y) / S,
// u_c,i = (K^{-1} r_c)_i - z_c,i y_p (eq. 13: only the owned p_i and u_i are written).
template <bool WIDE>
__device__ __forceinline__ void rav_patch(const AdDev& a, const AdFactors& f, int i, const double* __restrict__ r,
                                          double* __restrict__ x, double omega) {
  const int nV = a.nV;
  const int p0 = a.poff[i >> 6];
  const int t = i & 63;
  const int c = a.pcfg[i];
  const int nf = a.cnf[c], ao = a.cown[c];
  const double* zxc = f.zx + c * NF;
  const double* zyc = f.zy + c * NF;
  const double* krc = f.kr + c * NF;
  double tz = 0.0, ku = 0.0, kv = 0.0;
#pragma unroll 2   // two patch vertices' loads in flight (measured 39.7 -> 30.4 us per Omega^10 launch)
  for (int k = 0; k < nf; ++k) {
    const int v = patch_vertex<WIDE>(a, i, p0 + 64LL * k + t);
    const double rx = r[v], ry = r[nV + v];
    const double zx = zxc[k], zy = zyc[k], kr = krc[k];
    tz += zx * rx + zy * ry;
    ku += kr * rx;
    kv += kr * ry;
  }
  const double yp = (r[2 * nV + i] - tz) * f.invS[c];
  x[2 * nV + i] += omega * yp;
  if (ao >= 0) {
    x[i] += omega * (ku - zxc[ao] * yp);
    x[nV + i] += omega * (kv - zyc[ao] * yp);
  }
}

// AV / MV on a group of AD_NFMAX lanes per patch.  Lane k holds patch vertex
// k: r_x, r_y of that vertex (AV: read from r; MV: recomputed from b and the
// current x, eq. 15), y_c,k = (K^{-1} r_c)_k - z_c,k y_p.  AV writes the
// corrections per patch slot; MV adds them to x at once.  Stage 1 loads the
// patch residual into the group's row of shared memory (srx, sry); stage 2,
// after a barrier, solves and writes.
constexpr int GRP = AD_NFMAX;

struct GroupState {
  int i, v, c, nf;
  long long e;
  double rx, ry, rp;
  bool live;
};

template <bool MV, bool WIDE, bool LDS>
__device__ __forceinline__ GroupState group_load(const AdDev& a, bool live, int i, int k,
                                                 const double* __restrict__ rb, const double* __restrict__ x,
                                                 double* srx, double* sry, const double2* tab) {
  GroupState g;
  g.live = live;
  g.i = live ? i : 0;
  const int nV = a.nV;
  const int sl = g.i >> 6, t = g.i & 63;
  g.c = live ? a.pcfg[g.i] : 0;
  g.nf = live ? a.cnf[g.c] : 0;
  g.e = a.poff[sl] + 64LL * k + t;
  g.v = k < g.nf ? patch_vertex<WIDE>(a, g.i, g.e) : -1;
  g.rx = 0.0;
  g.ry = 0.0;
  if (g.v >= 0) {
    const int v = g.v;
    if (MV) {
      const int e0 = a.soff[v >> 6], vw = (a.soff[(v >> 6) + 1] - e0) >> 6;
      const int vt = v & 63;
      double su = 0.0, sv = 0.0;
      for (int m = 0; m < vw; ++m) {
        int j, id;
        entry<WIDE>(a, v, e0 + 64LL * m + vt, j, id);
        const double2* vt = LDS ? tab + 3 * id : reinterpret_cast<const double2*>(a.vtab + 8 * id);
        const double2 v01 = vt[0], v23 = vt[1];   // (A, BTx), (BTy, Bx)
        const double pj = x[2 * nV + j];
        su += v01.x * x[j] + v01.y * pj;
        sv += v01.x * x[nV + j] + v23.x * pj;
      }
      g.rx = rb[v] - su;
      g.ry = rb[nV + v] - sv;
    } else {
      g.rx = rb[v];
      g.ry = rb[nV + v];
    }
  }
  srx[k] = g.rx;
  sry[k] = g.ry;
  g.rp = 0.0;
  if (live && k == 0) {
    if (MV) {
      const int e0 = a.soff[sl], iw = (a.soff[sl + 1] - e0) >> 6;
      double sp = 0.0;
      for (int m = 0; m < iw; ++m) {
        int j, id;
        entry<WIDE>(a, g.i, e0 + 64LL * m + t, j, id);
        const double2* vt = LDS ? tab + 3 * id : reinterpret_cast<const double2*>(a.vtab + 8 * id);
        const double2 v23 = vt[1], v45 = vt[2];   // (BTy, Bx), (By, C)
        sp += v23.y * x[j] + v45.x * x[nV + j] + v45.y * x[2 * nV + j];
      }
      g.rp = rb[2 * nV + g.i] - sp;
    } else {
      g.rp = rb[2 * nV + g.i];
    }
  }
  return g;
}

// All lanes of the wavefront call this (the group reduction uses shuffles).
template <bool MV>
__device__ __forceinline__ void group_solve(const AdFactors& f, const GroupState& g, int k, int nV,
                                            const double* srx, const double* sry, double* __restrict__ x,
                                            double* __restrict__ yx, double* __restrict__ yy,
                                            double* __restrict__ yp_out, double omega) {
  double zx = 0.0, zy = 0.0, kx = 0.0, ky = 0.0;
  if (g.v >= 0) {
    zx = f.zx[g.c * NF + k];
    zy = f.zy[g.c * NF + k];
    const double* krow = f.kfull + (long long)g.c * NF * NF + k * NF;
    for (int m = 0; m < g.nf; ++m) {
      const double kv = krow[m];
      kx += kv * srx[m];
      ky += kv * sry[m];
    }
  }
  double tz = zx * g.rx + zy * g.ry;
  for (int o = GRP / 2; o > 0; o >>= 1) tz += __shfl_xor(tz, o, GRP);
  const double rp = __shfl(g.rp, 0, GRP);
  const double yp = g.live ? (rp - tz) * f.invS[g.c] : 0.0;
  const double ux = kx - zx * yp, uy = ky - zy * yp;
  if (MV) {
    if (g.v >= 0) {
      x[g.v] += omega * ux;
      x[nV + g.v] += omega * uy;
    }
    if (g.live && k == 0) x[2 * nV + g.i] += omega * yp;
  } else {
    if (g.v >= 0) {
      yx[g.e] = ux;
      yy[g.e] = uy;
    }
    if (g.live && k == 0) yp_out[g.i] = yp;
  }
}

// AV gather: vertex v adds the corrections of the patches that hold it.
__device__ __forceinline__ void av_gather_vertex(const AdDev& a, const int* __restrict__ tsoff,
                                                 const int* __restrict__ tpos, const double* __restrict__ yx,
                                                 const double* __restrict__ yy, const double* __restrict__ yp,
                                                 double* __restrict__ x, double omega, int v) {
  const int nV = a.nV;
  const int e0 = tsoff[v >> 6], w = (tsoff[(v >> 6) + 1] - e0) >> 6;
  const int t = v & 63;
  double su = 0.0, sv = 0.0;
  for (int k = 0; k < w; ++k) {
    const int s = tpos[e0 + 64 * k + t];
    if (s < 0) break;
    su += yx[s];
    sv += yy[s];
  }
  if (a.vmask[v] == 0) {
    x[v] += omega * su;
    x[nV + v] += omega * sv;
  }
  x[2 * nV + v] += omega * yp[v];
}

// xf += P xc on the three rows of fine vertex i.
__device__ __forceinline__ void prolong_vertex(const AdDev& f, const AdDev& c, const int* __restrict__ ptr,
                                               const int* __restrict__ idx, const double* __restrict__ w,
                                               const double* __restrict__ xc, double* __restrict__ xf, int i) {
  double su = 0.0, sv = 0.0, sp = 0.0;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
    const int j = idx[k];
    const double wk = w[k];
    const double fm = c.vmask[j] ? 0.0 : wk;
    su += fm * xc[j];
    sv += fm * xc[c.nV + j];
    sp += wk * xc[2 * c.nV + j];
  }
  if (f.vmask[i] == 0) {
    xf[i] += su;
    xf[f.nV + i] += sv;
  }
  xf[2 * f.nV + i] += sp;
}

// bc = P^T rf on coarse vertex j; xc = 0 and (rc != NULL) rc = bc, the residual of xc = 0.
__device__ __forceinline__ void restrict_vertex(const AdDev& f, const AdDev& c, const int* __restrict__ ptr,
                                                const int* __restrict__ idx, const double* __restrict__ w,
                                                const double* __restrict__ rf, double* __restrict__ bc,
                                                double* __restrict__ xc, double* __restrict__ rc, int j) {
  double su = 0.0, sv = 0.0, sp = 0.0;
  for (int k = ptr[j]; k < ptr[j + 1]; ++k) {
    const int i = idx[k];
    const double wk = w[k];
    const double fm = f.vmask[i] ? 0.0 : wk;
    su += fm * rf[i];
    sv += fm * rf[f.nV + i];
    sp += wk * rf[2 * f.nV + i];
  }
  if (c.vmask[j]) { su = 0.0; sv = 0.0; }
  const int n = c.nV;
  bc[j] = su; bc[n + j] = sv; bc[2 * n + j] = sp;
  xc[j] = 0.0; xc[n + j] = 0.0; xc[2 * n + j] = 0.0;
  if (rc) { rc[j] = su; rc[n + j] = sv; rc[2 * n + j] = sp; }
}

// ---- grid-wide kernels -----------------------------------------------------------
// The value table is read three times per operator entry; when it fits and
// the grid is large, each 1024-thread block stages it in LDS first (48 KB for
// 1024 tuples), which takes those reads off the vector-memory path (Omega^10:
// 40.8 -> 31.1 us).  Below AD_RES_LDS_MIN_VERTICES the 256-thread kernel with
// the table in global memory gives more blocks to a launch-bound grid.
constexpr int LDS_TUPLES = AD_LDS_TUPLES;
constexpr int RB_LDS = 1024;   // block of the LDS variant
constexpr int RB = 256;        // block of the plain variant

// Copies the six values of every tuple (the first three double2 of its row of
// vtab) into tab; every thread of the block calls it.
template <int BLOCK>
__device__ __forceinline__ void stage_table(const AdDev& a, double2* tab) {
  for (int q = threadIdx.x; q < a.ntuple * 3; q += BLOCK)
    tab[q] = reinterpret_cast<const double2*>(a.vtab)[(q / 3) * 4 + q % 3];
  __syncthreads();
}

template <bool WIDE, bool LDS, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_ad_residual(AdDev a, const double* __restrict__ x,
                                                       const double* __restrict__ b, double* __restrict__ r,
                                                       double* __restrict__ partials) {
  __shared__ double2 tab[LDS ? LDS_TUPLES * 3 : 1];
  __shared__ double red[BLOCK];
  if (LDS) stage_table<BLOCK>(a, tab);
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  const double sq = i < a.nV ? residual_vertex<WIDE, LDS>(a, i, x, b, r, tab) : 0.0;
  if (!partials) return;
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

template <bool WIDE>
__global__ __launch_bounds__(256) void k_ad_rav(AdDev a, AdFactors f, const double* __restrict__ r,
                                                double* __restrict__ x, double omega) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < a.nV) rav_patch<WIDE>(a, f, i, r, x, omega);
}

// BLOCK / GRP patches per block.  AV reads no operator values (64-lane
// blocks); MV recomputes residual rows and, when the table fits, stages it in
// LDS with 512-thread blocks (Omega^10 finest MV sweep: 1.52 -> 1.32 ms).
constexpr int GB = 64;
constexpr int GB_LDS = 512;

template <bool MV, bool WIDE, bool LDS, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_ad_group(AdDev a, AdFactors f, const int* __restrict__ order, int first,
                                                    int count, const double* __restrict__ rb, double* __restrict__ x,
                                                    double* __restrict__ yx, double* __restrict__ yy,
                                                    double* __restrict__ yp_out, double omega) {
  __shared__ double2 tab[LDS ? LDS_TUPLES * 3 : 1];
  __shared__ double srx[BLOCK / GRP][GRP], sry[BLOCK / GRP][GRP];
  if (LDS) stage_table<BLOCK>(a, tab);
  const int g = threadIdx.x / GRP, k = threadIdx.x % GRP;
  const int q = blockIdx.x * (BLOCK / GRP) + g;
  const bool live = q < count;
  const int i = live ? (order ? order[first + q] : first + q) : 0;
  const GroupState st = group_load<MV, WIDE, LDS>(a, live, i, k, rb, x, srx[g], sry[g], tab);
  __syncthreads();
  group_solve<MV>(f, st, k, a.nV, srx[g], sry[g], x, yx, yy, yp_out, omega);
}

__global__ __launch_bounds__(256) void k_ad_av_gather(AdDev a, const int* __restrict__ tsoff,
                                                      const int* __restrict__ tpos, const double* __restrict__ yx,
                                                      const double* __restrict__ yy, const double* __restrict__ yp,
                                                      double* __restrict__ x, double omega) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v < a.nV) av_gather_vertex(a, tsoff, tpos, yx, yy, yp, x, omega, v);
}

__global__ __launch_bounds__(256) void k_ad_prolong(AdDev f, AdDev c, const int* __restrict__ ptr,
                                                    const int* __restrict__ idx, const double* __restrict__ w,
                                                    const double* __restrict__ xc, double* __restrict__ xf) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < f.nV) prolong_vertex(f, c, ptr, idx, w, xc, xf, i);
}

__global__ __launch_bounds__(256) void k_ad_restrict(AdDev f, AdDev c, const int* __restrict__ ptr,
                                                     const int* __restrict__ idx, const double* __restrict__ w,
                                                     const double* __restrict__ rf, double* __restrict__ bc,
                                                     double* __restrict__ xc, double* __restrict__ rc) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < c.nV) restrict_vertex(f, c, ptr, idx, w, rf, bc, xc, rc, j);
}

__global__ __launch_bounds__(256) void k_ad_scale(const double* __restrict__ src, double alpha,
                                                  double* __restrict__ dst, long long n) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i < n) dst[i] = alpha * src[i];
}

__global__ __launch_bounds__(256) void k_ad_owner(AdDev a, int* __restrict__ owner) {
  const long long d = blockIdx.x * 256LL + threadIdx.x;
  if (d >= 3LL * a.nV) return;
  const int v = (int)(d % a.nV);
  const int field = (int)(d / a.nV);
  const int masked = (int)(field < 2) & (int)(a.vmask[v] != 0);
  owner[d] = v - masked * (v + 1);   // -1 for masked velocity, else the vertex's patch
}

}  // namespace

int ad_residual_blocks(const AdDev& a) {
  return (int)(a.res_lds ? nblk(a.nV, RB_LDS) : nblk(a.nV, RB));
}

#define AD_WIDE(a, K, ...)                                                              \
  do {                                                                                  \
    if ((a).wide) hipLaunchKernelGGL(K<true>, __VA_ARGS__);                             \
    else hipLaunchKernelGGL(K<false>, __VA_ARGS__);                                     \
  } while (0)

void ad_launch_residual(const AdDev& a, const double* x, const double* b, double* r, double* partials,
                        hipStream_t s) {
  const bool lds = a.res_lds != 0;
  const dim3 g(lds ? nblk(a.nV, RB_LDS) : nblk(a.nV, RB)), blk(lds ? RB_LDS : RB);
  if (a.wide) {
    if (lds) hipLaunchKernelGGL((k_ad_residual<true, true, RB_LDS>), g, blk, 0, s, a, x, b, r, partials);
    else hipLaunchKernelGGL((k_ad_residual<true, false, RB>), g, blk, 0, s, a, x, b, r, partials);
  } else {
    if (lds) hipLaunchKernelGGL((k_ad_residual<false, true, RB_LDS>), g, blk, 0, s, a, x, b, r, partials);
    else hipLaunchKernelGGL((k_ad_residual<false, false, RB>), g, blk, 0, s, a, x, b, r, partials);
  }
}

void ad_launch_factor(const AdDev& a, int mode, const int* rep, int ncfg, AdFactors f, int* status, hipStream_t s) {
  if (ncfg <= 0) return;
  AD_WIDE(a, k_ad_factor, dim3((unsigned)ncfg), dim3(64), 0, s, a, mode, rep, f, status);
}

void ad_launch_rav(const AdDev& a, AdFactors f, const double* r, double* x, double omega, hipStream_t s) {
  AD_WIDE(a, k_ad_rav, dim3(nblk(a.nV)), dim3(256), 0, s, a, f, r, x, omega);
}

void ad_launch_av(const AdDev& a, AdFactors f, const int* tsoff, const int* tpos, const double* r, double* yx,
                  double* yy, double* yp, double* x, double omega, hipStream_t s) {
  const dim3 g(nblk(a.nV, GB / GRP)), blk(GB);
  if (a.wide)
    hipLaunchKernelGGL((k_ad_group<false, true, false, GB>), g, blk, 0, s, a, f, (const int*)nullptr, 0, a.nV, r,
                       (double*)nullptr, yx, yy, yp, omega);
  else
    hipLaunchKernelGGL((k_ad_group<false, false, false, GB>), g, blk, 0, s, a, f, (const int*)nullptr, 0, a.nV, r,
                       (double*)nullptr, yx, yy, yp, omega);
  hipLaunchKernelGGL(k_ad_av_gather, dim3(nblk(a.nV)), dim3(256), 0, s, a, tsoff, tpos, yx, yy, yp, x, omega);
}

void ad_launch_mv(const AdDev& a, AdFactors f, const int* order, int first, int count, const double* b, double* x,
                  double omega, hipStream_t s) {
  if (count <= 0) return;
  double* const none = nullptr;
  if (a.table_lds) {
    const dim3 g(nblk(count, GB_LDS / GRP)), blk(GB_LDS);
    if (a.wide)
      hipLaunchKernelGGL((k_ad_group<true, true, true, GB_LDS>), g, blk, 0, s, a, f, order, first, count, b, x, none,
                         none, none, omega);
    else
      hipLaunchKernelGGL((k_ad_group<true, false, true, GB_LDS>), g, blk, 0, s, a, f, order, first, count, b, x,
                         none, none, none, omega);
    return;
  }
  const dim3 g(nblk(count, GB / GRP)), blk(GB);
  if (a.wide)
    hipLaunchKernelGGL((k_ad_group<true, true, false, GB>), g, blk, 0, s, a, f, order, first, count, b, x, none,
                       none, none, omega);
  else
    hipLaunchKernelGGL((k_ad_group<true, false, false, GB>), g, blk, 0, s, a, f, order, first, count, b, x, none,
                       none, none, omega);
}

void ad_launch_prolong(const AdDev& f, const AdDev& c, const int* ptr, const int* idx, const double* w,
                       const double* xc, double* xf, hipStream_t s) {
  hipLaunchKernelGGL(k_ad_prolong, dim3(nblk(f.nV)), dim3(256), 0, s, f, c, ptr, idx, w, xc, xf);
}

void ad_launch_restrict(const AdDev& f, const AdDev& c, const int* ptr, const int* idx, const double* w,
                        const double* rf, double* bc, double* xc, double* rc, hipStream_t s) {
  hipLaunchKernelGGL(k_ad_restrict, dim3(nblk(c.nV)), dim3(256), 0, s, f, c, ptr, idx, w, rf, bc, xc, rc);
}

void ad_launch_scale(const double* src, double alpha, double* dst, long long n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_ad_scale, dim3(nblk(n)), dim3(256), 0, s, src, alpha, dst, n);
}

void ad_launch_owner(const AdDev& a, int* owner, hipStream_t s) {
  hipLaunchKernelGGL(k_ad_owner, dim3(nblk(3LL * a.nV)), dim3(256), 0, s, a, owner);
}

}  // namespace rav
