// Learned per-patch damping: features, network forward/backward, Adam, and
// the adjoint pieces of the RAV sweep used to differentiate a two-grid cycle
// with respect to every patch weight omega_i (the per-patch form of the
// diagonal weighting of eq. 11).
//
// Network: 16 -> 64 -> 64 -> 1, ReLU, omega = 0.2 + sigmoid(z), FP32
// parameters; gradients are accumulated in FP64.  Parameters are flat:
// W1 (64x16), b1 (64), W2 (64x64), b2 (64), w3 (64), b3 (1).
#include <hip/hip_runtime.h>

#include "rav_internal.h"

namespace rav {

constexpr int NF = 16, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NF, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;
static_assert(NPARAM == 5313, "parameter layout");

// ---- features of 2D vertex patches -----------------------------------------
__global__ __launch_bounds__(256) void k_features(const GridDev* __restrict__ G, const double* __restrict__ incl,
                                                   int n_incl, double eta_out, double eta_in,
                                                   float* __restrict__ F) {
#pragma clang fp contract(off)
  const GridDev& gd = *G;
  const Geo& g = gd.g;
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= g.nP) return;
  int k[3] = {0, 0, 0};
  patch_anchor(g, KIND_VERTEX, p, k);
  const double h = gd.h;
  float f[9];
  float mn = 1e30f, mx = -1e30f, sum = 0.f;
  int q = 0;
  for (int b = -1; b <= 1; ++b)
    for (int a = -1; a <= 1; ++a, ++q) {
      double x = ((double)k[0] + 0.5 * a) * h, y = ((double)k[1] + 0.5 * b) * h;
      x = fmin(fmax(x, 0.0), 1.0);
      y = fmin(fmax(y, 0.0), 1.0);
      bool inside = false;
      for (int i = 0; i < n_incl; ++i) {
        const double* ic = incl + 4 * i;
        const double dx = x - ic[0], dy = y - ic[1];
        const double d2 = dx * dx + dy * dy;
        inside = inside || (d2 <= ic[3] * ic[3]);
      }
      const double eta = inside ? eta_in : eta_out;
      f[q] = (float)(log10(eta / eta_out) / 4.0);
      mn = fminf(mn, f[q]);
      mx = fmaxf(mx, f[q]);
      sum += f[q];
    }
  float* out = F + p * NF;
  for (int i = 0; i < 9; ++i) out[i] = f[i];
  out[9] = mn;
  out[10] = mx;
  out[11] = sum / 9.0f;
  out[12] = (k[0] == 0 || k[0] == g.N) ? 1.f : 0.f;
  out[13] = (k[1] == 0 || k[1] == g.N) ? 1.f : 0.f;
  out[14] = (float)(log2((double)g.N) / 10.0);
  out[15] = 1.f;
}

__device__ __forceinline__ float sigmoidf(float z) { return 1.f / (1.f + expf(-z)); }

// ---- forward: omega per patch ----------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ theta, const float* __restrict__ F,
                                                      long long n, float* __restrict__ omega) {
  __shared__ float th[NPARAM];
  for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) th[i] = theta[i];
  __syncthreads();
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= n) return;
  float f[NF], h1[NH];
  for (int i = 0; i < NF; ++i) f[i] = F[p * NF + i];
#pragma unroll 4
  for (int j = 0; j < NH; ++j) {
    float z = th[OFF_B1 + j];
#pragma unroll
    for (int i = 0; i < NF; ++i) z += th[OFF_W1 + j * NF + i] * f[i];
    h1[j] = fmaxf(z, 0.f);
  }
  float z3 = th[OFF_B3];
  for (int j = 0; j < NH; ++j) {
    float z = th[OFF_B2 + j];
#pragma unroll
    for (int i = 0; i < NH; ++i) z += th[OFF_W2 + j * NH + i] * h1[i];
    z3 += th[OFF_W3 + j] * fmaxf(z, 0.f);
  }
  omega[p] = 0.2f + sigmoidf(z3);
}

// ---- backward: d(sum_p g_p omega_p)/d theta, per-block FP64 partial sums ----
__global__ __launch_bounds__(256) void k_mlp_backward(const float* __restrict__ theta, const float* __restrict__ F,
                                                       const double* __restrict__ gom, long long n,
                                                       double* __restrict__ partial) {
  __shared__ float th[NPARAM];
  __shared__ double acc[NPARAM];
  for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) { th[i] = theta[i]; acc[i] = 0.0; }
  __syncthreads();
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p < n) {
    float f[NF], h1[NH];
    for (int i = 0; i < NF; ++i) f[i] = F[p * NF + i];
    for (int j = 0; j < NH; ++j) {
      float z = th[OFF_B1 + j];
      for (int i = 0; i < NF; ++i) z += th[OFF_W1 + j * NF + i] * f[i];
      h1[j] = fmaxf(z, 0.f);
    }
    float z3 = th[OFF_B3];
    unsigned long long act2 = 0ull;
    for (int j = 0; j < NH; ++j) {
      float z = th[OFF_B2 + j];
      for (int i = 0; i < NH; ++i) z += th[OFF_W2 + j * NH + i] * h1[i];
      if (z > 0.f) { act2 |= 1ull << j; z3 += th[OFF_W3 + j] * z; }
    }
    const float s = sigmoidf(z3);
    const double d3 = gom[p] * (double)s * (1.0 - (double)s);
    atomicAdd(&acc[OFF_B3], d3);
    double d1[NH];
    for (int i = 0; i < NH; ++i) d1[i] = 0.0;
    for (int j = 0; j < NH; ++j) {
      if (!((act2 >> j) & 1ull)) continue;
      // recompute h2_j
      float z = th[OFF_B2 + j];
      for (int i = 0; i < NH; ++i) z += th[OFF_W2 + j * NH + i] * h1[i];
      atomicAdd(&acc[OFF_W3 + j], d3 * (double)z);
      const double d2 = d3 * (double)th[OFF_W3 + j];
      atomicAdd(&acc[OFF_B2 + j], d2);
      for (int i = 0; i < NH; ++i) {
        if (h1[i] != 0.f) atomicAdd(&acc[OFF_W2 + j * NH + i], d2 * (double)h1[i]);
        d1[i] += (double)th[OFF_W2 + j * NH + i] * d2;
      }
    }
    for (int i = 0; i < NH; ++i) {
      if (!(h1[i] > 0.f)) continue;
      atomicAdd(&acc[OFF_B1 + i], d1[i]);
      for (int m = 0; m < NF; ++m)
        if (f[m] != 0.f) atomicAdd(&acc[OFF_W1 + i * NF + m], d1[i] * (double)f[m]);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) partial[(long long)blockIdx.x * NPARAM + i] = acc[i];
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partial, int nblk,
                                                       double* __restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(long long)b * NPARAM + i];
  grad[i] = s;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ theta, double* __restrict__ m,
                                               double* __restrict__ v, const double* __restrict__ grad, double lr,
                                               double b1, double b2, double eps, int t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  const double g = grad[i];
  m[i] = b1 * m[i] + (1.0 - b1) * g;
  v[i] = b2 * v[i] + (1.0 - b2) * g * g;
  const double mh = m[i] / (1.0 - pow(b1, (double)t));
  const double vh = v[i] / (1.0 - pow(b2, (double)t));
  theta[i] = (float)((double)theta[i] - lr * mh / (sqrt(vh) + eps));
}

// ---- adjoint pieces of the RAV sweep (2D vertex patches, FP64 rows) ---------
// Owned-row entry e of patch p in the tile-major FP64 layout (V = 2).
__device__ __forceinline__ double wrow(const Bucket& bk, long long p, int e) {
  const double* W = reinterpret_cast<const double*>(bk.W);
  return W[w_vec(bk, p, e >> 1) * 2 + (e & 1)];
}

__device__ __forceinline__ long long vcol(const Geo& g, const int* k, int c) {
  if (c < 50) {
    const int comp = c / 25, r = c % 25;
    int a[3] = {2 * k[0] + (r % 5) - 2, 2 * k[1] + (r / 5) - 2, 0};
    if (a[0] < 0 || a[0] > 2 * g.N || a[1] < 0 || a[1] > 2 * g.N) return -1;
    return comp * g.nV + node_lin(g, a);
  }
  return 2 * g.nV + vert_lin(g, k);
}

// g[p] += sum_j lam[owned_j(p)] * (W_p r[I_p])_j
__global__ __launch_bounds__(256) void k_rav_grad(const GridDev* __restrict__ G, const double* __restrict__ r,
                                                   const double* __restrict__ lam, double* __restrict__ gom) {
  const GridDev& gd = *G;
  const Geo& g = gd.g;
  const Bucket& bk = gd.bk[0];
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= bk.count) return;
  int k[3] = {0, 0, 0};
  patch_anchor(g, KIND_VERTEX, p, k);
  double acc[9];
  for (int j = 0; j < 9; ++j) acc[j] = 0.0;
  for (int c = 0; c < 51; ++c) {
    const long long col = vcol(g, k, c);
    const double rc = col >= 0 ? r[col] : 0.0;
    for (int j = 0; j < 9; ++j) acc[j] += wrow(bk, p, c * 9 + j) * rc;
  }
  double s = 0.0;
  for (int j = 0; j < 9; ++j) {
    int comp, node[3];
    const long long gi = patch_local_dof(g, KIND_VERTEX, k, bucket_own_local(2, KIND_VERTEX, 0, j), &comp, node);
    if (gi >= 0) s += lam[gi] * acc[j];
  }
  gom[p] += s;
}

// Y[p][c] = sum_j W_p[j][c] * omega_p * lam[owned_j(p)]  (transpose of the restricted apply)
__global__ __launch_bounds__(256) void k_rav_transpose(const GridDev* __restrict__ G, const double* __restrict__ lam,
                                                        const float* __restrict__ omega, double* __restrict__ Y) {
  const GridDev& gd = *G;
  const Geo& g = gd.g;
  const Bucket& bk = gd.bk[0];
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= bk.count) return;
  int k[3] = {0, 0, 0};
  patch_anchor(g, KIND_VERTEX, p, k);
  const double w = omega ? (double)omega[p] : gd.omega;
  double lo[9];
  for (int j = 0; j < 9; ++j) {
    int comp, node[3];
    const long long gi = patch_local_dof(g, KIND_VERTEX, k, bucket_own_local(2, KIND_VERTEX, 0, j), &comp, node);
    lo[j] = gi >= 0 ? w * lam[gi] : 0.0;
  }
  for (int c = 0; c < 51; ++c) {
    double s = 0.0;
    for (int j = 0; j < 9; ++j) s += wrow(bk, p, c * 9 + j) * lo[j];
    Y[p * 51 + c] = s;
  }
}

// z[i] = sum over vertex patches q containing DoF i of Y[q][local(i)]; masked DoFs 0.
__global__ __launch_bounds__(256) void k_patch_gather(const GridDev* __restrict__ G, const double* __restrict__ Y,
                                                       double* __restrict__ z) {
  const GridDev& gd = *G;
  const Geo& g = gd.g;
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  double s = 0.0;
  if (i < 2 * g.nV) {
    long long nl;
    const int comp = split_vel(g, i, &nl);
    int a[3] = {0, 0, 0};
    node_of(g, nl, a);
    if (!node_dirichlet(g, a)) {
      const int x0 = max((a[0] - 1) >> 1, 0), x1 = min((a[0] + 2) >> 1, g.N);
      const int y0 = max((a[1] - 1) >> 1, 0), y1 = min((a[1] + 2) >> 1, g.N);
      for (int qy = y0; qy <= y1; ++qy)
        for (int qx = x0; qx <= x1; ++qx) {
          const int l = comp * 25 + (a[1] - 2 * qy + 2) * 5 + (a[0] - 2 * qx + 2);
          s += Y[((long long)qy * g.np1 + qx) * 51 + l];
        }
    }
  } else {
    s = Y[(i - 2 * g.nV) * 51 + 50];
  }
  z[i] = s;
}

// y = a * x + b * y
// y = a x + b y; with b == 0 the old y is not read (it may be uninitialised).
__global__ __launch_bounds__(256) void k_axpby(double a, const double* __restrict__ x, double b, double* __restrict__ y,
                                                long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}

static inline unsigned nb256(long long n) { return (unsigned)((n + 255) / 256); }

void launch_features(const GridDev* G, long long npatch, const double* incl, int n_incl, double eta_out,
                     double eta_in, float* F, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3(nb256(npatch)), dim3(256), 0, s, G, incl, n_incl, eta_out, eta_in, F);
}
void launch_mlp_forward(const float* theta, const float* F, long long n, float* omega, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_forward, dim3(nb256(n)), dim3(256), 0, s, theta, F, n, omega);
}
int mlp_backward_blocks(long long n) { return (int)nb256(n); }
void launch_mlp_backward(const float* theta, const float* F, const double* gom, long long n, double* partial,
                         double* grad, hipStream_t s) {
  const int nblk = (int)nb256(n);
  hipLaunchKernelGGL(k_mlp_backward, dim3(nblk), dim3(256), 0, s, theta, F, gom, n, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(nb256(NPARAM)), dim3(256), 0, s, partial, nblk, grad);
}
void launch_adam(float* theta, double* m, double* v, const double* grad, double lr, int t, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(nb256(NPARAM)), dim3(256), 0, s, theta, m, v, grad, lr, 0.9, 0.999, 1e-8, t);
}
void launch_rav_grad(const GridDev* G, long long npatch, const double* r, const double* lam, double* gom,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_rav_grad, dim3(nb256(npatch)), dim3(256), 0, s, G, r, lam, gom);
}
void launch_rav_transpose(const GridDev* G, long long npatch, const double* lam, const float* omega, double* Y,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_rav_transpose, dim3(nb256(npatch)), dim3(256), 0, s, G, lam, omega, Y);
}
void launch_patch_gather(const GridDev* G, long long n, const double* Y, double* z, hipStream_t s) {
  hipLaunchKernelGGL(k_patch_gather, dim3(nb256(n)), dim3(256), 0, s, G, Y, z);
}
void launch_axpby(double a, const double* x, double b, double* y, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(nb256(n)), dim3(256), 0, s, a, x, b, y, n);
}

}  // namespace rav
