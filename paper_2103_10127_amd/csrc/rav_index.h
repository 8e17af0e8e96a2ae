// Index math of the uniform Q2/Q1 hierarchy, shared by host and device code.
//
// Numbering (eq. 6 ordering [u; p]): velocity component c at half-grid node
// a in [0,2N]^d -> c*nV + lin(a), pressure at vertex k in [0,N]^d ->
// d*nV + lin(k), both lexicographic with x fastest.
//
// Operator storage ("ELL by node type", implicit columns).  Rows are split
// into segments: one per (velocity component c, node parity type t) with
// t = sum_d (a_d & 1) << d, plus one pressure segment.  Inside a segment rows
// are ordered lexicographically over i_d = a_d >> 1, and values are stored
// slot-major: vals[seg_off + slot * seg_rows + row], so consecutive threads
// read consecutive addresses.  Columns are implied by the slot:
//   velocity row at node a, type t:  A-slots: same-component nodes a + o with
//     |o_d| <= w_d (w_d = 2 if a_d even, 1 if odd), lexicographic in o;
//     B-slots: pressure vertices k with k_d in [lo_d, lo_d + m_d),
//     lo_d = (a_d >> 1) - 1 + (a_d & 1), m_d = 3 - (a_d & 1).
//   pressure row at vertex k: B^T-slots over components c and nodes 2k + o,
//     o in [-2,2]^d: slot = c*5^d + lex(o + 2).
// Slots whose column lies outside the grid or on a masked node hold 0.
//
// Patch local numbering (Sec. 3): component-major, then lexicographic nodes,
// then pressure, padded to a fixed size per patch kind:
//   vertex patch k : nodes 2k + o, o in [-2,2]^d, then p_k        (2D: 51)
//   element patch e: nodes 2e + i, i in [0,2]^d, then p_{e+j}, j in {0,1}^d (3D: 89)
// Local DoFs outside the grid or masked are padding: identity rows/columns
// of the local matrix, which leaves the inverse on the real DoFs unchanged.
// Ownership (restricted prolongation of eq. 13, floor rule): vertex patches
// own velocity nodes 2k + {0,1}^d and p_k; element patches own nodes 2e + i
// with i_d in {0,1}, plus i_d = 2 where e_d = N-1, and pressures e + j with
// j_d = 0, plus j_d = 1 where e_d = N-1.  Element patches are bucketed by the
// class mask m (bit d set when e_d = N-1), which fixes the owned pattern.
#pragma once
#include <hip/hip_runtime.h>

#define RAV_HD __host__ __device__ __forceinline__
#define RAV_HDC __host__ __device__ constexpr

namespace rav {

enum { KIND_VERTEX = 0, KIND_ELEMENT = 1 };

struct Geo {
  int dim, N;
  unsigned dmask;
  long long nn, np1, nV, nP, n;
};

RAV_HD Geo make_geo(int dim, int N, unsigned dmask) {
  Geo g;
  g.dim = dim; g.N = N; g.dmask = dmask;
  g.nn = 2LL * N + 1; g.np1 = N + 1LL;
  g.nV = g.nn * g.nn * (dim == 3 ? g.nn : 1);
  g.nP = g.np1 * g.np1 * (dim == 3 ? g.np1 : 1);
  g.n = dim * g.nV + g.nP;
  return g;
}

RAV_HDC int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

RAV_HD bool coord_dirichlet(const Geo& g, int d, int ad) {
  return (((g.dmask >> (2 * d)) & 1u) && ad == 0) || (((g.dmask >> (2 * d + 1)) & 1u) && ad == 2 * g.N);
}
RAV_HD bool node_dirichlet(const Geo& g, const int* a) {
  bool r = false;
  for (int d = 0; d < g.dim; ++d) r = r || coord_dirichlet(g, d, a[d]);
  return r;
}
RAV_HD bool node_inside(const Geo& g, const int* a) {
  bool r = true;
  for (int d = 0; d < g.dim; ++d) r = r && a[d] >= 0 && a[d] <= 2 * g.N;
  return r;
}
RAV_HD long long node_lin(const Geo& g, const int* a) {
  long long i = a[g.dim - 1];
  for (int d = g.dim - 2; d >= 0; --d) i = i * g.nn + a[d];
  return i;
}
RAV_HD long long vert_lin(const Geo& g, const int* k) {
  long long i = k[g.dim - 1];
  for (int d = g.dim - 2; d >= 0; --d) i = i * g.np1 + k[d];
  return i;
}
// Level sizes stay below 2^31, so index decoding uses 32-bit unsigned
// division (64-bit division is a long software sequence on the GPU).
RAV_HD void node_of(const Geo& g, long long lin, int* a) {
  unsigned u = (unsigned)lin;
  const unsigned nn = (unsigned)g.nn;
  for (int d = 0; d < g.dim; ++d) { a[d] = (int)(u % nn); u /= nn; }
}
RAV_HD void vert_of(const Geo& g, long long lin, int* k) {
  unsigned u = (unsigned)lin;
  const unsigned np1 = (unsigned)g.np1;
  for (int d = 0; d < g.dim; ++d) { k[d] = (int)(u % np1); u /= np1; }
}
// Split a global velocity index into component and node (32-bit division).
RAV_HD int split_vel(const Geo& g, long long i, long long* node_lin_out) {
  const unsigned u = (unsigned)i, nv = (unsigned)g.nV;
  *node_lin_out = (long long)(u % nv);
  return (int)(u / nv);
}

// ---- ELL segments -------------------------------------------------------
RAV_HDC int n_segments(int dim) { return dim * (1 << dim) + 1; }
RAV_HDC int pressure_segment(int dim) { return dim * (1 << dim); }
RAV_HDC int a_halfwidth(int t, int d) { return ((t >> d) & 1) ? 1 : 2; }
RAV_HDC int n_aslots(int dim, int t) {
  int s = 1;
  for (int d = 0; d < dim; ++d) s *= 2 * a_halfwidth(t, d) + 1;
  return s;
}
RAV_HDC int n_bslots(int dim, int t) {
  int s = 1;
  for (int d = 0; d < dim; ++d) s *= 3 - ((t >> d) & 1);
  return s;
}
RAV_HDC int seg_slots(int dim, int s) {
  if (s == pressure_segment(dim)) return dim * ipow(5, dim);
  int t = s & ((1 << dim) - 1);
  return n_aslots(dim, t) + n_bslots(dim, t);
}
RAV_HD long long type_count(const Geo& g, int t, int d) { return ((t >> d) & 1) ? g.N : g.N + 1LL; }
RAV_HD long long seg_rows(const Geo& g, int s) {
  if (s == pressure_segment(g.dim)) return g.nP;
  int t = s & ((1 << g.dim) - 1);
  long long r = 1;
  for (int d = 0; d < g.dim; ++d) r *= type_count(g, t, d);
  return r;
}
RAV_HD int node_type(const Geo& g, const int* a) {
  int t = 0;
  for (int d = 0; d < g.dim; ++d) t |= (a[d] & 1) << d;
  return t;
}
RAV_HD long long vel_seg_row(const Geo& g, int t, const int* a) {
  long long r = a[g.dim - 1] >> 1;
  for (int d = g.dim - 2; d >= 0; --d) r = r * type_count(g, t, d) + (a[d] >> 1);
  return r;
}
RAV_HD void vel_row_node(const Geo& g, int t, long long row, int* a) {
  unsigned u = (unsigned)row;
  for (int d = 0; d < g.dim; ++d) {
    const unsigned c = (unsigned)type_count(g, t, d);
    a[d] = 2 * (int)(u % c) + ((t >> d) & 1);
    u /= c;
  }
}
// Slot of velocity column node b in the row of node a (same component), or -1.
RAV_HD int aslot(const Geo& g, int t, const int* a, const int* b) {
  int s = 0, stride = 1;
  for (int d = 0; d < g.dim; ++d) {
    int w = a_halfwidth(t, d), o = b[d] - a[d];
    if (o < -w || o > w) return -1;
    s += (o + w) * stride;
    stride *= 2 * w + 1;
  }
  return s;
}
// Slot of pressure column vertex k in the row of velocity node a, or -1.
RAV_HD int bslot(const Geo& g, int t, const int* a, const int* k) {
  int s = 0, stride = 1;
  for (int d = 0; d < g.dim; ++d) {
    int px = (t >> d) & 1, lo = (a[d] >> 1) - 1 + px, m = 3 - px, j = k[d] - lo;
    if (j < 0 || j >= m) return -1;
    s += j * stride;
    stride *= m;
  }
  return n_aslots(g.dim, t) + s;
}
// Slot of velocity column (component c, node b) in the pressure row of vertex k, or -1.
RAV_HD int pslot(const Geo& g, const int* k, int c, const int* b) {
  int s = 0, stride = 1;
  for (int d = 0; d < g.dim; ++d) {
    int o = b[d] - 2 * k[d];
    if (o < -2 || o > 2) return -1;
    s += (o + 2) * stride;
    stride *= 5;
  }
  return c * ipow(5, g.dim) + s;
}

// ---- patches ------------------------------------------------------------
RAV_HDC int patch_npad(int dim, int kind) {
  return kind == KIND_VERTEX ? dim * ipow(5, dim) + 1 : dim * ipow(3, dim) + ipow(2, dim);
}
RAV_HD long long n_patches(const Geo& g, int kind) {
  return kind == KIND_VERTEX ? g.nP : (long long)g.N * g.N * (g.dim == 3 ? g.N : 1);
}
RAV_HD long long patch_lin(const Geo& g, int kind, const int* k) {
  long long base = kind == KIND_VERTEX ? g.np1 : g.N;
  long long i = k[g.dim - 1];
  for (int d = g.dim - 2; d >= 0; --d) i = i * base + k[d];
  return i;
}
RAV_HD void patch_anchor(const Geo& g, int kind, long long p, int* k) {
  const unsigned base = (unsigned)(kind == KIND_VERTEX ? g.np1 : g.N);
  unsigned u = (unsigned)p;
  for (int d = 0; d < g.dim; ++d) { k[d] = (int)(u % base); u /= base; }
}

// Local DoF `l` of the patch anchored at k: returns -1 for padding (outside
// the grid or masked), else the global index; *comp = component or dim for pressure.
RAV_HD long long patch_local_dof(const Geo& g, int kind, const int* k, int l, int* comp, int* node) {
  const int dim = g.dim;
  if (kind == KIND_VERTEX) {
    const int nv = ipow(5, dim);
    if (l < dim * nv) {
      int c = l / nv, r = l % nv;
      for (int d = 0; d < dim; ++d) { node[d] = 2 * k[d] + (r % 5) - 2; r /= 5; }
      *comp = c;
      if (!node_inside(g, node) || node_dirichlet(g, node)) return -1;
      return c * g.nV + node_lin(g, node);
    }
    for (int d = 0; d < dim; ++d) node[d] = k[d];
    *comp = dim;
    return dim * g.nV + vert_lin(g, node);
  }
  const int nv = ipow(3, dim);
  if (l < dim * nv) {
    int c = l / nv, r = l % nv;
    for (int d = 0; d < dim; ++d) { node[d] = 2 * k[d] + (r % 3); r /= 3; }
    *comp = c;
    if (node_dirichlet(g, node)) return -1;
    return c * g.nV + node_lin(g, node);
  }
  int r = l - dim * nv;
  for (int d = 0; d < dim; ++d) { node[d] = k[d] + (r & 1); r >>= 1; }
  *comp = dim;
  return dim * g.nV + vert_lin(g, node);
}

// Element class mask of element e (bit d set when e_d = N-1).
RAV_HD int element_class(const Geo& g, const int* e) {
  int m = 0;
  for (int d = 0; d < g.dim; ++d) m |= (e[d] == g.N - 1 ? 1 : 0) << d;
  return m;
}
// Number of owned local rows of a bucket (class mask m; vertex patches use m = 0).
RAV_HDC int bucket_nown(int dim, int kind, int m) {
  if (kind == KIND_VERTEX) return dim * ipow(2, dim) + 1;
  int nv = 1, np = 1;
  for (int d = 0; d < dim; ++d) { int top = (m >> d) & 1; nv *= 2 + top; np *= 1 + top; }
  return dim * nv + np;
}
// j-th owned local index (ascending local order) of a bucket.
RAV_HDC int bucket_own_local(int dim, int kind, int m, int j) {
  if (kind == KIND_VERTEX) {
    const int per = ipow(2, dim), nv = ipow(5, dim);
    if (j >= dim * per) return dim * nv;
    int c = j / per, r = j % per, l = 0, stride = 1;
    for (int d = 0; d < dim; ++d) { l += ((r & 1) + 2) * stride; r >>= 1; stride *= 5; }
    return c * nv + l;
  }
  int cnt[3] = {0, 0, 0}, per = 1;
  for (int d = 0; d < dim; ++d) { cnt[d] = 2 + ((m >> d) & 1); per *= cnt[d]; }
  const int nv = ipow(3, dim);
  if (j < dim * per) {
    int c = j / per, r = j % per, l = 0, stride = 1;
    for (int d = 0; d < dim; ++d) { l += (r % cnt[d]) * stride; r /= cnt[d]; stride *= 3; }
    return c * nv + l;
  }
  int r = j - dim * per, l = 0, stride = 1;
  for (int d = 0; d < dim; ++d) {
    int pc = 1 + ((m >> d) & 1);
    l += (r % pc) * stride; r /= pc; stride *= 2;
  }
  return dim * nv + l;
}
// Factored storage of a vertex patch's owned inverse rows (RAV_FACTORED):
// with the local velocity block I_d (x) K and one pressure, the owned rows of
// L_i^{-1} are determined by the owned rows of K^{-1} (2^d owned nodes x 5^d
// nodes), Z = K^{-1} B (d x 5^d) and the scalar S^{-1}.  Values per node j:
// [K^{-1}[own_0][j] .. K^{-1}[own_{2^d-1}][j], Z_0[j] .. Z_{d-1}[j]], then S^{-1}.
RAV_HDC int fact_nn(int dim) { return ipow(5, dim); }
RAV_HDC int fact_nown_nodes(int dim) { return ipow(2, dim); }
RAV_HDC int fact_per_node(int dim) { return fact_nown_nodes(dim) + dim; }
RAV_HDC int fact_nvals(int dim) { return fact_nn(dim) * fact_per_node(dim) + 1; }

// Elements of bucket m: e_d = N-1 where bit d is set, e_d in [0, N-2] elsewhere.
RAV_HD long long bucket_count(const Geo& g, int kind, int m) {
  if (kind == KIND_VERTEX) return g.nP;
  long long c = 1;
  for (int d = 0; d < g.dim; ++d) c *= ((m >> d) & 1) ? 1 : (g.N - 1);
  return c;
}
RAV_HD void bucket_anchor(const Geo& g, int kind, int m, long long p, int* k) {
  if (kind == KIND_VERTEX) { patch_anchor(g, kind, p, k); return; }
  unsigned u = (unsigned)p;
  for (int d = 0; d < g.dim; ++d) {
    if ((m >> d) & 1) { k[d] = g.N - 1; }
    else { const unsigned ext = (unsigned)(g.N - 1); k[d] = (int)(u % ext); u /= ext; }
  }
}
// Position of an element inside its bucket.
RAV_HD long long bucket_pos(const Geo& g, int m, const int* e) {
  long long p = 0, stride = 1;
  for (int d = 0; d < g.dim; ++d) {
    if ((m >> d) & 1) continue;
    p += e[d] * stride;
    stride *= g.N - 1;
  }
  return p;
}
RAV_HDC int n_buckets(int dim, int kind) { return kind == KIND_VERTEX ? 1 : (1 << dim); }

// Owner patch (global patch index) of a free DoF (floor rule).
RAV_HD long long owner_of(const Geo& g, int kind, long long dof) {
  int a[3], k[3];
  if (dof < g.dim * g.nV) {
    long long nl;
    split_vel(g, dof, &nl);
    node_of(g, nl, a);
    for (int d = 0; d < g.dim; ++d) {
      int o = a[d] >> 1;
      k[d] = (kind == KIND_ELEMENT && o > g.N - 1) ? g.N - 1 : o;
    }
  } else {
    vert_of(g, dof - g.dim * g.nV, a);
    for (int d = 0; d < g.dim; ++d) k[d] = (kind == KIND_ELEMENT && a[d] > g.N - 1) ? g.N - 1 : a[d];
  }
  return patch_lin(g, kind, k);
}

// MV colours: vertex patches (k_d mod 4), element patches (e_d mod 3).
RAV_HDC int colour_modulus(int kind) { return kind == KIND_VERTEX ? 4 : 3; }

}  // namespace rav
