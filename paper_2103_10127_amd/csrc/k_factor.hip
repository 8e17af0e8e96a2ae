// Local patch systems and their inverses (Sec. 3; Sec. 4.3).
//
// One wavefront per patch.  The padded local matrix L_i = R_i L R_i^T is
// gathered from the ELL operator into LDS (padding DoFs become identity rows
// and columns), inverted in place by Gauss-Jordan elimination with partial
// pivoting (row interchanges undone as column interchanges at the end), and
// the needed rows are written out:
//   RAV: the owned rows of L_i^{-1}, cast to the storage precision, in the
//        chunk-interleaved bucket layout read by the apply kernel;
//   AV/MV: the full inverse, column-major per patch.
// A zero pivot records the patch index in *status (atomicMin).
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

template <int DIM, int KIND>
__device__ double local_entry(const GridDev& gd, long long R, int cr, const int* a, long long C, int cc,
                              const int* b) {
  const Geo& g = gd.g;
  if (cr < DIM) {
    const int t = node_type(g, a);
    const int s = cr * (1 << DIM) + t;
    int slot;
    if (cc < DIM) {
      if (cc != cr) return 0.0;
      slot = aslot(g, t, a, b);
    } else {
      slot = bslot(g, t, a, b);
    }
    if (slot < 0) return 0.0;
    return gd.vals[gd.seg_off[s] + (long long)slot * gd.seg_rows[s] + vel_seg_row(g, t, a)];
  }
  if (cc >= DIM) return 0.0;
  const int s = pressure_segment(DIM);
  const int slot = pslot(g, a, cc, b);
  if (slot < 0) return 0.0;
  return gd.vals[gd.seg_off[s] + (long long)slot * gd.seg_rows[s] + vert_lin(g, a)];
}

template <int DIM, int KIND, typename WT>
__global__ __launch_bounds__(64) void k_factor(const GridDev* __restrict__ G, int bucket, int cls, int full,
                                                long long count, int* __restrict__ status) {
  constexpr int NPAD = patch_npad(DIM, KIND);
  constexpr int LD = NPAD + 1;
  __shared__ double A[NPAD * LD];
  __shared__ long long glob[NPAD];
  __shared__ int cmp[NPAD];
  __shared__ int nd[NPAD][3];
  __shared__ int piv[NPAD];
  const long long p = blockIdx.x;
  if (p >= count) return;
  const GridDev& gd = *G;
  const Geo& g = gd.g;
  const int lane = threadIdx.x;
  int k[3] = {0, 0, 0};
  if (full) patch_anchor(g, KIND, p, k);
  else bucket_anchor(g, KIND, cls, p, k);
  for (int l = lane; l < NPAD; l += 64) {
    int comp, node[3] = {0, 0, 0};
    glob[l] = patch_local_dof(g, KIND, k, l, &comp, node);
    cmp[l] = comp;
    nd[l][0] = node[0]; nd[l][1] = node[1]; nd[l][2] = node[2];
  }
  __syncthreads();
  for (int r = lane; r < NPAD; r += 64) {
    for (int c = 0; c < NPAD; ++c) {
      double v;
      if (glob[r] < 0 || glob[c] < 0) v = (r == c) ? 1.0 : 0.0;
      else v = local_entry<DIM, KIND>(gd, glob[r], cmp[r], nd[r], glob[c], cmp[c], nd[c]);
      A[r * LD + c] = v;
    }
  }
  __syncthreads();
  // In-place Gauss-Jordan inversion with partial pivoting; lanes own columns.
  for (int kk = 0; kk < NPAD; ++kk) {
    double best = -1.0;
    int bi = kk;
    for (int i = kk + lane; i < NPAD; i += 64) {
      const double v = fabs(A[i * LD + kk]);
      if (v > best) { best = v; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (best <= 0.0) {
      if (lane == 0) {
        const long long gp = patch_lin(g, KIND, k);
        atomicMin(status, (int)gp);
      }
      return;
    }
    if (lane == 0) piv[kk] = bi;
    if (bi != kk) {
      for (int j = lane; j < NPAD; j += 64) {
        const double tmp = A[kk * LD + j];
        A[kk * LD + j] = A[bi * LD + j];
        A[bi * LD + j] = tmp;
      }
    }
    __syncthreads();
    const double pv = A[kk * LD + kk];
    const double ipv = 1.0 / pv;
    __syncthreads();
    for (int j = lane; j < NPAD; j += 64) A[kk * LD + j] = (j == kk) ? ipv : A[kk * LD + j] * ipv;
    __syncthreads();
    for (int i = 0; i < NPAD; ++i) {
      if (i == kk) continue;
      const double f = A[i * LD + kk];
      __syncthreads();
      for (int j = lane; j < NPAD; j += 64)
        A[i * LD + j] = (j == kk) ? -f * ipv : A[i * LD + j] - f * A[kk * LD + j];
    }
    __syncthreads();
  }
  for (int kk = NPAD - 1; kk >= 0; --kk) {
    const int q = piv[kk];
    if (q != kk) {
      for (int i = lane; i < NPAD; i += 64) {
        const double tmp = A[i * LD + kk];
        A[i * LD + kk] = A[i * LD + q];
        A[i * LD + q] = tmp;
      }
    }
    __syncthreads();
  }
  if (full) {
    double* out = gd.Winv + p * (long long)NPAD * NPAD;
    for (int c = 0; c < NPAD; ++c)
      for (int l = lane; l < NPAD; l += 64) out[c * NPAD + l] = A[l * LD + c];
    return;
  }
  const Bucket& bk = gd.bk[bucket];
  constexpr int V = 16 / (int)sizeof(WT);
  WT* W = reinterpret_cast<WT*>(bk.W);
  const int nown = bk.nown;
  for (int j = 0; j < nown; ++j) {
    const int l = bucket_own_local(DIM, KIND, cls, j);
    for (int c = lane; c < NPAD; c += 64) {
      const long long e = (long long)c * nown + j;
      store_w(W, w_vec(bk, p, e / V) * V + e % V, A[l * LD + c]);
    }
  }
}

template <int DIM, int KIND>
static void launch_factor_k(int cls, int prec, int full, const GridDev* G, long long count, int bucket,
                            int* status, hipStream_t s) {
  if (count <= 0) return;
  const dim3 grid((unsigned)count), blk(64);
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
  else launch_factor_k<3, KIND_ELEMENT>(cls, prec, full, G, count, bucket, status, s);
}

}  // namespace rav
