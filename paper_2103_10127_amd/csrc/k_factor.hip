// Local patch systems and the rows of their inverses (Sec. 3; Sec. 4.3).
//
// The local matrix of a patch is the principal submatrix
//   L_i = [[A_i, B_i], [B_i^T, 0]]
// of the Stokes operator (eqs. 6-7).  Its velocity block couples no two
// components and is the same scalar viscous block K_i for every component:
// the form (eta grad v, grad u) of eq. 5 acts componentwise and a Dirichlet
// mask removes a node for all components.  So A_i = I_d (x) K_i with K_i
// symmetric positive definite, B_i = [B_1; ...; B_d] stacks one block per
// component, and the inverse follows by block elimination:
//   Z_c = K^{-1} B_c,   S = -sum_c B_c^T Z_c   (Schur complement, negative definite)
//   L^{-1} = [[A^{-1} + Z S^{-1} Z^T, -Z S^{-1}], [-S^{-1} Z^T, S^{-1}]],  Z = [Z_1; ...; Z_d].
// One Gauss-Jordan inversion of K (3^d or 5^d nodes) with the d*np columns
// of B carried along replaces elimination on the whole d*n + np system:
// 2D vertex patches invert 25 instead of 51 unknowns (8x fewer flops), 3D
// element patches 27 instead of 89 (36x), 3D vertex patches 125 instead of
// 376.  K (positive definite) and S (negative definite) need no pivoting.
//
// Padding (local DoFs outside the grid or on a masked side) enters K as unit
// rows and columns and B as zero rows, so the inverse restricted to the real
// DoFs is unchanged and the padding rows and columns of L^{-1} are unit
// vectors (the apply kernel relies on exact zeros there).
//
// One block per patch: the gather of K and B from the ELL operator, the
// elimination (two barriers per pivot), S and S^{-1}, Z S^{-1}, then the
// needed entries of L^{-1}:
//   RAV: the owned rows, cast to the storage precision, in the
//        chunk-interleaved bucket layout read by the apply kernel;
//   AV/MV: the full inverse, column-major per patch.
// A non-positive pivot of K or a zero pivot of S records the patch index in
// *status (atomicMin).
#include <hip/hip_runtime.h>

#include "rav_internal.h"

namespace rav {

struct bf16s { unsigned short u; };

__device__ __forceinline__ void store_w(double* W, long long i, double v) { W[i] = v; }
__device__ __forceinline__ void store_w(float* W, long long i, double v) { W[i] = (float)v; }
__device__ __forceinline__ void store_w(bf16s* W, long long i, double v) {
  // float64 -> float32 (round to nearest even) -> bfloat16 (round to nearest even)
  const float f = (float)v;
  unsigned bits = __float_as_uint(f);
  bits += 0x7fffu + ((bits >> 16) & 1u);
  W[i].u = (unsigned short)(bits >> 16);
}

// Operator entry in the row of (component cr, node a): velocity column (same
// component, node b) when cc < DIM, pressure column at vertex b when cc == DIM.
template <int DIM>
__device__ double op_entry(const GridDev& gd, int cr, const int* a, int cc, const int* b) {
  const Geo& g = gd.g;
  const int t = node_type(g, a);
  const int s = cr * (1 << DIM) + t;
  const int slot = cc < DIM ? aslot(g, t, a, b) : bslot(g, t, a, b);
  if (slot < 0) return 0.0;
  return gd.vals[gd.seg_off[s] + (long long)slot * gd.seg_rows[s] + vel_seg_row(g, t, a)];
}

template <int DIM, int KIND>
struct FactorShape {
  static constexpr int NN = KIND == KIND_VERTEX ? ipow(5, DIM) : ipow(3, DIM);   // velocity nodes
  static constexpr int NPR = KIND == KIND_VERTEX ? 1 : ipow(2, DIM);             // pressures
  static constexpr int NB = DIM * NPR;                                            // columns of B
  static constexpr int WID = NN + NB;                                             // [K | B_1 .. B_d]
  static constexpr int LD = WID + 1;
  static constexpr int NPAD = DIM * NN + NPR;
  static constexpr int NT = (KIND == KIND_VERTEX && DIM == 3) ? 256 : 64;         // threads per patch
};

template <int DIM, int KIND, typename WT>
__global__ __launch_bounds__((FactorShape<DIM, KIND>::NT)) void k_factor(const GridDev* __restrict__ G, int bucket,
                                                                        int cls, int full, long long count,
                                                                        int* __restrict__ status) {
  typedef FactorShape<DIM, KIND> F;
  constexpr int NN = F::NN, NPR = F::NPR, NB = F::NB, WID = F::WID, LD = F::LD, NPAD = F::NPAD, NT = F::NT;
  __shared__ double M[NN * LD];      // [K | B] -> [K^{-1} | Z]
  __shared__ double Bs[NN * NB];     // B, kept for S
  __shared__ double ZS[NN * NB];     // Z_c S^{-1}
  __shared__ double Sm[NPR * NPR];   // S, then S^{-1}
  __shared__ double prow[WID];
  __shared__ double fcol[NN];
  __shared__ int nd[NN][3];
  __shared__ int pv[NPR][3];
  __shared__ int pad[NN];
  __shared__ int bad;
  const long long p = blockIdx.x;
  if (p >= count) return;
  const GridDev& gd = *G;
  const Geo& g = gd.g;
  const int tid = threadIdx.x;
  int k[3] = {0, 0, 0};
  if (full) patch_anchor(g, KIND, p, k);
  else bucket_anchor(g, KIND, cls, p, k);
  // local velocity nodes (component 0 part of the local numbering) and pressures
  for (int l = tid; l < NN + NPR; l += NT) {
    int comp, node[3] = {0, 0, 0};
    const int loc = l < NN ? l : DIM * NN + (l - NN);
    const long long gi = patch_local_dof(g, KIND, k, loc, &comp, node);
    if (l < NN) {
      pad[l] = gi < 0 ? 1 : 0;
      nd[l][0] = node[0]; nd[l][1] = node[1]; nd[l][2] = node[2];
    } else {
      pv[l - NN][0] = node[0]; pv[l - NN][1] = node[1]; pv[l - NN][2] = node[2];
    }
  }
  if (tid == 0) bad = 0;
  __syncthreads();
#pragma unroll 1
  for (int e = tid; e < NN * WID; e += NT) {
    const int r = e / WID, c = e - r * WID;
    double v;
    if (c < NN) {
      v = (pad[r] || pad[c]) ? (r == c ? 1.0 : 0.0) : op_entry<DIM>(gd, 0, nd[r], 0, nd[c]);
    } else {
      const int cb = c - NN, comp = cb / NPR, q = cb - comp * NPR;
      v = pad[r] ? 0.0 : op_entry<DIM>(gd, comp, nd[r], DIM, pv[q]);
      Bs[r * NB + cb] = v;
    }
    M[r * LD + c] = v;
  }
  // In-place Gauss-Jordan on K, applied to the B columns as right-hand sides.
#pragma unroll 1
  for (int kk = 0; kk < NN; ++kk) {
    __syncthreads();
    const double pivot = M[kk * LD + kk];
    if (!(pivot > 0.0)) {   // K must be positive definite
      if (tid == 0) atomicMin(status, (int)patch_lin(g, KIND, k));
      return;
    }
    const double ipv = 1.0 / pivot;
    for (int j = tid; j < WID; j += NT) prow[j] = j == kk ? ipv : M[kk * LD + j] * ipv;
    for (int i = tid; i < NN; i += NT) fcol[i] = M[i * LD + kk];
    __syncthreads();
    for (int e = tid; e < NN * WID; e += NT) {
      const int i = e / WID, j = e - i * WID;
      double& m = M[i * LD + j];
      if (i == kk) m = prow[j];
      else if (j == kk) m = -fcol[i] * ipv;
      else m -= fcol[i] * prow[j];
    }
  }
  __syncthreads();
  // S = -sum_c B_c^T Z_c
  for (int e = tid; e < NPR * NPR; e += NT) {
    const int q = e / NPR, q2 = e - q * NPR;
    double s = 0.0;
    for (int c = 0; c < DIM; ++c)
      for (int a = 0; a < NN; ++a) s += Bs[a * NB + c * NPR + q] * M[a * LD + NN + c * NPR + q2];
    Sm[e] = -s;
  }
  __syncthreads();
  if (tid == 0) {   // S^{-1} in place (negative definite: no pivoting)
    for (int kk = 0; kk < NPR; ++kk) {
      const double pivot = Sm[kk * NPR + kk];
      if (!(pivot < 0.0)) { bad = 1; break; }
      const double ipv = 1.0 / pivot;
      for (int j = 0; j < NPR; ++j) Sm[kk * NPR + j] = j == kk ? ipv : Sm[kk * NPR + j] * ipv;
      for (int i = 0; i < NPR; ++i) {
        if (i == kk) continue;
        const double f = Sm[i * NPR + kk];
        for (int j = 0; j < NPR; ++j)
          Sm[i * NPR + j] = j == kk ? -f * ipv : Sm[i * NPR + j] - f * Sm[kk * NPR + j];
      }
    }
    if (bad) atomicMin(status, (int)patch_lin(g, KIND, k));
  }
  __syncthreads();
  if (bad) return;
  // ZS_c = Z_c S^{-1}
  for (int e = tid; e < NN * NB; e += NT) {
    const int a = e / NB, cb = e - a * NB, c = cb / NPR, q = cb - c * NPR;
    double s = 0.0;
    for (int q2 = 0; q2 < NPR; ++q2) s += M[a * LD + NN + c * NPR + q2] * Sm[q2 * NPR + q];
    ZS[e] = s;
  }
  __syncthreads();
  // entry (row l, column m) of the padded L^{-1}
  auto inv_entry = [&](int l, int m) -> double {
    const bool lv = l < DIM * NN, mv = m < DIM * NN;
    if (lv && mv) {
      const int cr = l / NN, a = l - cr * NN, cc = m / NN, b = m - cc * NN;
      double s = cr == cc ? M[a * LD + b] : 0.0;
      for (int q = 0; q < NPR; ++q) s += ZS[a * NB + cr * NPR + q] * M[b * LD + NN + cc * NPR + q];
      return s;
    }
    if (lv) {
      const int cr = l / NN, a = l - cr * NN;
      return -ZS[a * NB + cr * NPR + (m - DIM * NN)];
    }
    if (mv) {
      const int cc = m / NN, b = m - cc * NN;
      return -ZS[b * NB + cc * NPR + (l - DIM * NN)];
    }
    return Sm[(l - DIM * NN) * NPR + (m - DIM * NN)];
  };
  if (full) {
    double* out = gd.Winv + p * (long long)NPAD * NPAD;
#pragma unroll 1
    for (int e = tid; e < NPAD * NPAD; e += NT) {
      const int c = e / NPAD, l = e - c * NPAD;
      out[e] = inv_entry(l, c);
    }
    return;
  }
  const Bucket& bk = gd.bk[bucket];
  constexpr int V = 16 / (int)sizeof(WT);
  WT* W = reinterpret_cast<WT*>(bk.W);
  if constexpr (KIND == KIND_VERTEX) {
    if (bk.factored) {   // owned rows of K^{-1}, z = K^{-1} B and S^{-1} (layout of fact_nvals)
      constexpr int NO = fact_nown_nodes(DIM), GV = fact_per_node(DIM);
#pragma unroll 1
      for (int e = tid; e < fact_nvals(DIM); e += NT) {
        double v;
        if (e < NN * GV) {
          const int j = e / GV, q = e - j * GV;
          v = q < NO ? M[bucket_own_local(DIM, KIND, 0, q) * LD + j] : M[j * LD + NN + (q - NO)];
        } else {
          v = Sm[0];
        }
        store_w(W, w_vec(bk, p, e / V) * V + e % V, v);
      }
      return;
    }
  }
  const int nown = bk.nown;
#pragma unroll 1
  for (int e = tid; e < NPAD * nown; e += NT) {
    const int c = e / nown, j = e - c * nown;
    store_w(W, w_vec(bk, p, e / V) * V + e % V, inv_entry(bucket_own_local(DIM, KIND, cls, j), c));
  }
}

template <int DIM, int KIND>
static void launch_factor_k(int cls, int prec, int full, const GridDev* G, long long count, int bucket,
                            int* status, hipStream_t s) {
  if (count <= 0) return;
  const dim3 grid((unsigned)count), blk(FactorShape<DIM, KIND>::NT);
  if (full || prec == P_FP64)
    hipLaunchKernelGGL((k_factor<DIM, KIND, double>), grid, blk, 0, s, G, bucket, cls, full, count, status);
  else if (prec == P_FP32)
    hipLaunchKernelGGL((k_factor<DIM, KIND, float>), grid, blk, 0, s, G, bucket, cls, full, count, status);
  else
    hipLaunchKernelGGL((k_factor<DIM, KIND, bf16s>), grid, blk, 0, s, G, bucket, cls, full, count, status);
}

void launch_factor(int dim, int kind, int cls, int prec, int full, const GridDev* G, long long count, int bucket,
                   int* status, hipStream_t s) {
  if (dim == 2 && kind == KIND_VERTEX) launch_factor_k<2, KIND_VERTEX>(cls, prec, full, G, count, bucket, status, s);
  else if (dim == 2) launch_factor_k<2, KIND_ELEMENT>(cls, prec, full, G, count, bucket, status, s);
  else if (kind == KIND_VERTEX) launch_factor_k<3, KIND_VERTEX>(cls, prec, full, G, count, bucket, status, s);
  else launch_factor_k<3, KIND_ELEMENT>(cls, prec, full, G, count, bucket, status, s);
}

}  // namespace rav
