// Host driver of stabilized Q1-Q1 on adaptively refined quadtree grids with
// hanging nodes (Sec. 2, eqs. 5-8 and Fig. 2; Sec. 4.1, Table 1): the grid
// topology, the hanging-node constraints, the conforming operator of every
// grid (assembled once on the host), the Vanka patches, the grid transfers and
// the coarse direct solve are set up here; smoothing (RAV, AV, MV), residuals,
// transfers and V-cycles run in the kernels of k_adapt.hip.  The public entry
// points of rav.h route here for contexts made by rav_create_adaptive.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "rav_adapt.h"
#include "rav_ctx.h"
#include "rav_q1_unit.h"

using namespace rav;

struct rav_ad_state {
  struct Level {
    AdDev dev{};
    int nV = 0;
    long long nfree = 0;
    unsigned char* vmask = nullptr;
    int *soff = nullptr, *col = nullptr;
    unsigned* ent = nullptr;
    double* vtab = nullptr;
    int *poff = nullptr, *pv = nullptr, *pcfg = nullptr, *cnf = nullptr, *cown = nullptr, *rep = nullptr;
    int ncfg = 0, ntuple = 0;
    AdFactors fac{};
    int *tsoff = nullptr, *tpos = nullptr;
    double *yx = nullptr, *yy = nullptr, *yp = nullptr;
    int* order = nullptr;               // MV: patches colour-major
    std::vector<int> cstart;            // MV: colour c is order[cstart[c] .. cstart[c+1])
    int *pptr = nullptr, *pidx = nullptr;   // prolongation from the next coarser grid (rows: this grid)
    double* pw = nullptr;
    int *rptr = nullptr, *ridx = nullptr;   // restriction to the next coarser grid (rows: that grid)
    double* rw = nullptr;
    double *x = nullptr, *b = nullptr, *r = nullptr, *partials = nullptr;
    int nres = 0;
    long long pnnz = 0;
    long long nnz_true = 0, pnnz_true = 0;   // entries without the slice padding
    // host copies for the patch getters
    std::vector<int> h_poff, h_pv, h_pcfg, h_cnf, h_cown;
  };
  std::vector<Level> lv;
  double* Minv = nullptr;
  long long nb = 0;
  double* blid = nullptr;   // finest grid: lid lifting for a lid velocity of 1 (null without a Dirichlet top)
  // finest grid, host: velocity Dirichlet flag per vertex and the couplings of
  // L_all to masked columns (row, column, A, B_x, B_y) for general lifting
  std::vector<unsigned char> fine_mask;
  std::vector<int> dc_row, dc_col;
  std::vector<double> dc_val;
  int mode = AD_RAV;
  bool have_factors = false;
};

#define ACK(expr)                                                                    \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                  \
      return e_ == hipErrorOutOfMemory ? RAV_ENOMEM : RAV_EDEVICE;                   \
    }                                                                                \
  } while (0)

namespace {

using Level = rav_ad_state::Level;

struct Wt {
  int v;
  double w;
};

// f(0) .. f(n-1) on the host's cores (set-up only).
template <class F>
void parallel_for(int n, F f) {
  const int nt = std::max(1, std::min(n, (int)std::thread::hardware_concurrency()));
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&] {
      for (int i = next++; i < n; i = next++) f(i);
    });
  for (auto& t : th) t.join();
}

// ---- host set-up ---------------------------------------------------------------
// Grid topology: regular vertices, hanging nodes and the regular-vertex weights
// of every leaf corner (a hanging node is the mean of the two endpoints of the
// coarse edge whose midpoint it is, applied recursively).
struct Topo {
  long long Mx = 0, My = 0;    // the domain lies in [0, Mx] x [0, My] (lattice units)
  const int* leaf = nullptr;   // (x0, y0, s) per leaf
  long long nl = 0;
  std::vector<long long> reg, hang, ha, hb;
  std::vector<int> cw_ptr;     // 4 nl + 1
  std::vector<Wt> cw;
  std::vector<std::vector<Wt>> hmemo;
  std::vector<char> hstate;
  std::string err;

  long long key(long long x, long long y) const { return y * (Mx + 1) + x; }
  long long kx(long long k) const { return k % (Mx + 1); }
  long long ky(long long k) const { return k / (Mx + 1); }
  int nV() const { return (int)reg.size(); }
  int find_reg(long long k) const {
    auto it = std::lower_bound(reg.begin(), reg.end(), k);
    return (it != reg.end() && *it == k) ? (int)(it - reg.begin()) : -1;
  }
  int find_hang(long long k) const {
    auto it = std::lower_bound(hang.begin(), hang.end(), k);
    return (it != hang.end() && *it == k) ? (int)(it - hang.begin()) : -1;
  }
  static void merge_half(const std::vector<Wt>& a, const std::vector<Wt>& b, std::vector<Wt>& out) {
    out.clear();
    size_t i = 0, j = 0;
    while (i < a.size() || j < b.size()) {
      if (j == b.size() || (i < a.size() && a[i].v < b[j].v)) { out.push_back({a[i].v, 0.5 * a[i].w}); ++i; }
      else if (i == a.size() || b[j].v < a[i].v) { out.push_back({b[j].v, 0.5 * b[j].w}); ++j; }
      else { out.push_back({a[i].v, 0.5 * a[i].w + 0.5 * b[j].w}); ++i; ++j; }
    }
  }
  bool weights(long long k, std::vector<Wt>& out, int depth = 0) {
    const int r = find_reg(k);
    if (r >= 0) { out.assign(1, Wt{r, 1.0}); return true; }
    const int h = find_hang(k);
    if (h < 0 || depth > 64) { err = "a leaf corner is neither a vertex nor a hanging node"; return false; }
    if (hstate[h] == 2) { out = hmemo[h]; return true; }
    if (hstate[h] == 1) { err = "cyclic hanging-node constraints"; return false; }
    hstate[h] = 1;
    std::vector<Wt> wa, wb;
    if (!weights(ha[h], wa, depth + 1) || !weights(hb[h], wb, depth + 1)) return false;
    merge_half(wa, wb, out);
    hmemo[h] = out;
    hstate[h] = 2;
    return true;
  }

  bool build(const int* leaves, long long n, long long Mlx, long long Mly) {
    leaf = leaves;
    nl = n;
    Mx = Mlx;
    My = Mly;
    std::vector<long long> corners(4 * nl), mids(4 * nl);
    for (long long e = 0; e < nl; ++e) {
      const long long x0 = leaf[3 * e], y0 = leaf[3 * e + 1], s = leaf[3 * e + 2], h = s / 2;
      for (int a = 0; a < 4; ++a) corners[4 * e + a] = key(x0 + (a & 1) * s, y0 + (a >> 1) * s);
      mids[4 * e + 0] = key(x0 + h, y0);
      mids[4 * e + 1] = key(x0 + h, y0 + s);
      mids[4 * e + 2] = key(x0, y0 + h);
      mids[4 * e + 3] = key(x0 + s, y0 + h);
    }
    std::vector<long long> cs = corners, ms = mids;
    std::sort(cs.begin(), cs.end());
    cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
    std::sort(ms.begin(), ms.end());
    ms.erase(std::unique(ms.begin(), ms.end()), ms.end());
    std::set_intersection(cs.begin(), cs.end(), ms.begin(), ms.end(), std::back_inserter(hang));
    std::set_difference(cs.begin(), cs.end(), hang.begin(), hang.end(), std::back_inserter(reg));
    // 2:1 balance: no corner lies at a quarter point of a leaf edge
    for (long long e = 0; e < nl; ++e) {
      const long long x0 = leaf[3 * e], y0 = leaf[3 * e + 1], s = leaf[3 * e + 2];
      if (s < 4) continue;
      for (int f = 1; f <= 3; f += 2) {
        const long long q = s * f / 4;
        const long long pts[4] = {key(x0 + q, y0), key(x0 + q, y0 + s), key(x0, y0 + q), key(x0 + s, y0 + q)};
        for (long long p : pts)
          if (std::binary_search(cs.begin(), cs.end(), p)) { err = "grid is not 2:1 balanced"; return false; }
      }
    }
    ha.assign(hang.size(), -1);
    hb.assign(hang.size(), -1);
    for (long long e = 0; e < nl; ++e) {
      const long long x0 = leaf[3 * e], y0 = leaf[3 * e + 1], s = leaf[3 * e + 2];
      const long long ends[4][2] = {{key(x0, y0), key(x0 + s, y0)},
                                    {key(x0, y0 + s), key(x0 + s, y0 + s)},
                                    {key(x0, y0), key(x0, y0 + s)},
                                    {key(x0 + s, y0), key(x0 + s, y0 + s)}};
      for (int m = 0; m < 4; ++m) {
        const int h = find_hang(mids[4 * e + m]);
        if (h >= 0) { ha[h] = ends[m][0]; hb[h] = ends[m][1]; }
      }
    }
    hmemo.assign(hang.size(), {});
    hstate.assign(hang.size(), 0);
    cw_ptr.assign(4 * nl + 1, 0);
    cw.clear();
    std::vector<Wt> tmp;
    for (long long c = 0; c < 4 * nl; ++c) {
      if (!weights(corners[c], tmp)) return false;
      cw.insert(cw.end(), tmp.begin(), tmp.end());
      cw_ptr[c + 1] = (int)cw.size();
    }
    return true;
  }
  void leaf_verts(long long e, std::vector<int>& out) const {
    out.clear();
    for (int c = cw_ptr[4 * e]; c < cw_ptr[4 * e + 4]; ++c) out.push_back(cw[c].v);
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
  }
};

// Rows of small integer lists, filled in two passes (count, then fill) by a
// generator that emits (row, value) pairs; rows optionally sorted and made
// unique.
struct Csr {
  std::vector<long long> ptr;
  std::vector<int> idx;
  int len(int i) const { return (int)(ptr[i + 1] - ptr[i]); }
  const int* begin(int i) const { return idx.data() + ptr[i]; }
  const int* end(int i) const { return idx.data() + ptr[i + 1]; }
};

template <class Gen>
Csr build_csr(int nrows, Gen gen, bool sort_unique) {
  Csr c;
  c.ptr.assign(nrows + 1, 0);
  gen([&](int r, int) { ++c.ptr[r + 1]; });
  for (int i = 0; i < nrows; ++i) c.ptr[i + 1] += c.ptr[i];
  c.idx.resize(c.ptr.back());
  std::vector<long long> pos(c.ptr.begin(), c.ptr.end() - 1);
  gen([&](int r, int v) { c.idx[pos[r]++] = v; });
  if (!sort_unique) return c;
  long long w = 0, a = c.ptr[0];
  for (int i = 0; i < nrows; ++i) {
    const long long b = c.ptr[i + 1];
    std::sort(c.idx.begin() + a, c.idx.begin() + b);
    const long long e = std::unique(c.idx.begin() + a, c.idx.begin() + b) - c.idx.begin();
    c.ptr[i] = w;
    for (long long k = a; k < e; ++k) c.idx[w++] = c.idx[k];
    a = b;
  }
  c.ptr[nrows] = w;
  c.idx.resize(w);
  return c;
}

// Host image of one level, uploaded as a whole.
struct HostLevel {
  int nV = 0;
  std::vector<unsigned char> vmask;
  Csr nbr;                             // structural columns of every vertex row
  std::vector<int> soff, col;
  std::vector<double> val;             // 6 planes (host only: coarse matrix, exports)
  long long nnz = 0;
  std::vector<int> vid;                // tuple id of every stored entry
  std::vector<double> vtab;            // 8 doubles per distinct tuple
  std::vector<double> blid;            // lid lifting (finest grid; empty without a Dirichlet top side)
  // finest grid: the entries (row vertex, masked column vertex) of L_all with
  // A, B_x, B_y, for the lifting of any Dirichlet data
  std::vector<int> dc_row, dc_col;
  std::vector<double> dc_val;
  // patches
  Csr pall;                            // all vertices of patch i (MV colouring)
  std::vector<int> poff, pv;
  long long pnnz = 0;
  std::vector<int> pcfg, cnf, cown, rep;   // configuration of every patch; per configuration nf, owned, representative
  // device encoding
  bool wide = false;
  int id_bits = 1;
  std::vector<unsigned> ent;
  std::vector<int> tsoff, tpos, order, cstart;
  // prolongation from the next coarser grid
  std::vector<int> pptr, pidx, rptr, ridx;
  std::vector<double> pwt, rwt;
};

std::vector<int> sell_offsets(int n, const std::vector<int>& len) {
  const int ns = (n + AD_SLICE - 1) / AD_SLICE;
  std::vector<int> off(ns + 1, 0);
  for (int s = 0; s < ns; ++s) {
    int w = 0;
    for (int t = 0; t < AD_SLICE && s * AD_SLICE + t < n; ++t) w = std::max(w, len[s * AD_SLICE + t]);
    off[s + 1] = off[s] + AD_SLICE * w;
  }
  return off;
}

long long sell_slot(const std::vector<int>& off, int v, int k) {
  return off[v / AD_SLICE] + (long long)AD_SLICE * k + (v % AD_SLICE);
}

// Velocity Dirichlet vertices: a regular vertex is on the boundary when one of
// the four quadrants around it holds no leaf.  It is Dirichlet when such a
// quadrant lies inside the rectangle (a hole: obstacles are no-slip) or across
// a side of the rectangle whose bit is set in dmask (bit 0: x = 0, 1: x = Mx,
// 2: y = 0, 3: y = My); across open sides only, it keeps its velocity unknowns
// (natural outflow condition).
std::vector<unsigned char> dirichlet_vertices(const Topo& g, unsigned dmask) {
  const int nV = g.nV();
  std::vector<unsigned char> cover(nV, 0), mask(nV, 0);
  for (long long e = 0; e < g.nl; ++e) {
    const long long x0 = g.leaf[3 * e], y0 = g.leaf[3 * e + 1], s = g.leaf[3 * e + 2];
    for (int a = 0; a < 4; ++a) {
      const int v = g.find_reg(g.key(x0 + (a & 1) * s, y0 + (a >> 1) * s));
      if (v >= 0) cover[v] |= (unsigned char)(1u << ((1 - (a & 1)) | (2 - (a & 2))));   // quadrant: +x bit 0, +y bit 1
    }
  }
  for (int v = 0; v < nV; ++v) {
    const long long x = g.kx(g.reg[v]), y = g.ky(g.reg[v]);
    for (int q = 0; q < 4 && !mask[v]; ++q) {
      if (cover[v] >> q & 1) continue;
      const bool px = q & 1, py = q & 2;
      unsigned sides = 0;
      if (!px && x == 0) sides |= 1u;
      if (px && x == g.Mx) sides |= 2u;
      if (!py && y == 0) sides |= 4u;
      if (py && y == g.My) sides |= 8u;
      mask[v] = (sides == 0 || (sides & dmask)) ? 1 : 0;
    }
  }
  return mask;
}

// Conforming operator L = T^T L_corners T of one grid (rows and columns of
// masked velocity zero); on the finest grid also the couplings of L_all to the
// masked velocity columns (any Dirichlet data's lifting b = -L_all[:, masked]
// u_D) and, with a Dirichlet top side, that lifting for the lid velocity
// u_x = 1 on the top side strictly between the corners.  Lengths are in units
// of the domain height: a leaf of s lattice units has size s / My.
bool assemble(const Topo& g, double beta, double eta, unsigned dmask, bool finest, HostLevel& H,
              std::string& err) {
  const int nV = g.nV();
  H.nV = nV;
  H.vmask = dirichlet_vertices(g, dmask);
  const bool lid = finest && (dmask & 8u);
  std::vector<unsigned char> is_lid(nV, 0);
  for (int v = 0; v < nV; ++v) {
    const long long x = g.kx(g.reg[v]), y = g.ky(g.reg[v]);
    is_lid[v] = (y == g.My && x > 0 && x < g.Mx) ? 1 : 0;
  }
  std::vector<int> ve;
  H.nbr = build_csr(nV, [&](auto&& emit) {
    for (long long e = 0; e < g.nl; ++e) {
      g.leaf_verts(e, ve);
      for (int i : ve)
        for (int j : ve) emit(i, j);
    }
  }, true);
  std::vector<int> len(nV);
  for (int v = 0; v < nV; ++v) len[v] = H.nbr.len(v);
  H.soff = sell_offsets(nV, len);
  if ((long long)H.soff.back() >= (long long)INT_MAX / 2) { err = "grid too large"; return false; }
  H.nnz = H.soff.back();
  H.col.assign(H.nnz, 0);
  H.val.assign(6 * H.nnz, 0.0);
  for (int v = 0; v < nV; ++v) {
    const int w = (H.soff[v / AD_SLICE + 1] - H.soff[v / AD_SLICE]) / AD_SLICE;
    for (int k = 0; k < w; ++k) H.col[sell_slot(H.soff, v, k)] = k < len[v] ? H.nbr.begin(v)[k] : v;
  }
  double Ar[4][4], Br[2][4][4], Cr[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      Ar[a][b] = q1unit::kunit<2>(a, b);
      Cr[a][b] = q1unit::kunit<2>(a, b);
      for (int c = 0; c < 2; ++c) Br[c][a][b] = q1unit::bunit<2>(c, a, b);
    }
  const long long P = H.nnz;
  for (long long e = 0; e < g.nl; ++e) {
    const double h = (double)g.leaf[3 * e + 2] / (double)g.My;
    const double sB = -h, sC = -beta * 2.0 * h * h;
    for (int a = 0; a < 4; ++a)
      for (int ca = g.cw_ptr[4 * e + a]; ca < g.cw_ptr[4 * e + a + 1]; ++ca) {
        const int i = g.cw[ca].v;
        const double wi = g.cw[ca].w;
        const int* row = H.nbr.begin(i);
        const int* rend = H.nbr.end(i);
        for (int b = 0; b < 4; ++b)
          for (int cb = g.cw_ptr[4 * e + b]; cb < g.cw_ptr[4 * e + b + 1]; ++cb) {
            const int j = g.cw[cb].v;
            const double ww = wi * g.cw[cb].w;
            const int k = (int)(std::lower_bound(row, rend, j) - row);
            const long long s = sell_slot(H.soff, i, k);
            H.val[AD_A * P + s] += ww * eta * Ar[a][b];
            H.val[AD_BTX * P + s] += ww * sB * Br[0][a][b];
            H.val[AD_BTY * P + s] += ww * sB * Br[1][a][b];
            H.val[AD_BX * P + s] += ww * sB * Br[0][b][a];
            H.val[AD_BY * P + s] += ww * sB * Br[1][b][a];
            H.val[AD_C * P + s] += ww * sC * Cr[a][b];
          }
      }
  }
  if (lid) {
    H.blid.assign(3LL * nV, 0.0);
    for (int i = 0; i < nV; ++i)
      for (int k = 0; k < len[i]; ++k) {
        const int j = H.nbr.begin(i)[k];
        if (!is_lid[j]) continue;
        const long long s = sell_slot(H.soff, i, k);
        if (!H.vmask[i]) H.blid[i] -= H.val[AD_A * P + s];
        H.blid[2LL * nV + i] -= H.val[AD_BX * P + s];
      }
  }
  if (finest)
    for (int i = 0; i < nV; ++i)
      for (int k = 0; k < len[i]; ++k) {
        const int j = H.nbr.begin(i)[k];
        if (!H.vmask[j]) continue;
        const long long s = sell_slot(H.soff, i, k);
        H.dc_row.push_back(i);
        H.dc_col.push_back(j);
        H.dc_val.insert(H.dc_val.end(), {H.val[AD_A * P + s], H.val[AD_BX * P + s], H.val[AD_BY * P + s]});
      }
  for (int i = 0; i < nV; ++i)
    for (int k = 0; k < len[i]; ++k) {
      const int j = H.nbr.begin(i)[k];
      const long long s = sell_slot(H.soff, i, k);
      if (H.vmask[i]) { H.val[AD_A * P + s] = 0.0; H.val[AD_BTX * P + s] = 0.0; H.val[AD_BTY * P + s] = 0.0; }
      if (H.vmask[j]) { H.val[AD_A * P + s] = 0.0; H.val[AD_BX * P + s] = 0.0; H.val[AD_BY * P + s] = 0.0; }
    }
  // distinct value tuples (by bit pattern, so the kernels see the same values)
  struct TupleHash {
    size_t operator()(const std::array<uint64_t, 6>& t) const {
      uint64_t h = 1469598103934665603ull;
      for (uint64_t v : t) h = (h ^ (v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2))) * 1099511628211ull;
      return (size_t)h;
    }
  };
  std::unordered_map<std::array<uint64_t, 6>, int, TupleHash> ids;
  H.vid.assign(H.nnz, 0);
  std::array<uint64_t, 6> zero{};
  ids.emplace(zero, 0);
  H.vtab.assign(8, 0.0);
  for (long long e = 0; e < H.nnz; ++e) {
    std::array<uint64_t, 6> t;
    for (int p = 0; p < 6; ++p) std::memcpy(&t[p], &H.val[p * P + e], 8);
    auto it = ids.find(t);
    if (it == ids.end()) {
      it = ids.emplace(t, (int)ids.size()).first;
      for (int p = 0; p < 8; ++p) H.vtab.push_back(p < 6 ? H.val[p * P + e] : 0.0);
    }
    H.vid[e] = it->second;
  }
  return true;
}

// Vanka patches (Sec. 3): patch i holds p_i and the free velocity at the
// vertices of the leaves around vertex i (hanging corners through their
// constraining vertices); RAV owns p_i and the velocity at i.  MV order: greedy
// colouring in patch order, a patch taking the smallest colour of no earlier
// patch whose vertex set meets the row pattern of its own vertices.
bool build_patches(const Topo& g, HostLevel& H, std::string& err) {
  const int nV = H.nV;
  // vertices of patch i: the vertices the corners of the leaves around i depend on
  H.pall = build_csr(nV, [&](auto&& emit) {
    for (long long e = 0; e < g.nl; ++e) {
      const long long x0 = g.leaf[3 * e], y0 = g.leaf[3 * e + 1], s = g.leaf[3 * e + 2];
      for (int a = 0; a < 4; ++a) {
        const int r = g.find_reg(g.key(x0 + (a & 1) * s, y0 + (a >> 1) * s));
        if (r < 0) continue;
        for (int c = g.cw_ptr[4 * e]; c < g.cw_ptr[4 * e + 4]; ++c) emit(r, g.cw[c].v);
      }
    }
  }, true);
  Csr pfree = build_csr(nV, [&](auto&& emit) {
    for (int i = 0; i < nV; ++i)
      for (const int* v = H.pall.begin(i); v != H.pall.end(i); ++v)
        if (!H.vmask[*v]) emit(i, *v);
  }, false);
  std::vector<int> len(nV);
  for (int i = 0; i < nV; ++i) {
    len[i] = pfree.len(i);
    if (len[i] > AD_NFMAX) { err = "a patch has more than 16 free velocity vertices"; return false; }
  }
  H.poff = sell_offsets(nV, len);
  H.pnnz = H.poff.back();
  H.pv.assign(H.pnnz, -1);
  std::vector<int> own(nV, -1);
  for (int i = 0; i < nV; ++i)
    for (int k = 0; k < len[i]; ++k) {
      const int v = pfree.begin(i)[k];
      H.pv[sell_slot(H.poff, i, k)] = v;
      if (v == i) own[i] = k;
    }
  // configurations: patches whose matrices have the same tuple ids (and owned position)
  auto tuple_at = [&](int row, int colv) -> int {
    const int* b = H.nbr.begin(row);
    const int* e = H.nbr.end(row);
    const int* f = std::lower_bound(b, e, colv);
    return (f != e && *f == colv) ? H.vid[sell_slot(H.soff, row, (int)(f - b))] : -1;
  };
  struct VecHash {
    size_t operator()(const std::vector<int>& v) const {
      uint64_t h = 1469598103934665603ull;
      for (int x : v) h = (h ^ (uint64_t)(uint32_t)x) * 1099511628211ull;
      return (size_t)h;
    }
  };
  std::unordered_map<std::vector<int>, int, VecHash> cfgs;
  H.pcfg.assign(nV, 0);
  H.cnf.clear();
  H.cown.clear();
  H.rep.clear();
  std::vector<int> sig;
  for (int i = 0; i < nV; ++i) {
    const int nf = len[i];
    const int* F = pfree.begin(i);
    sig.assign({nf, own[i], tuple_at(i, i)});
    for (int a = 0; a < nf; ++a) {
      sig.push_back(tuple_at(F[a], i));
      for (int b = 0; b < nf; ++b) sig.push_back(tuple_at(F[a], F[b]));
    }
    auto it = cfgs.find(sig);
    if (it == cfgs.end()) {
      it = cfgs.emplace(sig, (int)H.rep.size()).first;
      H.cnf.push_back(nf);
      H.cown.push_back(own[i]);
      H.rep.push_back(i);
    }
    H.pcfg[i] = it->second;
  }
  // AV gather lists: the slots that hold vertex v, in patch order
  Csr tslots = build_csr(nV, [&](auto&& emit) {
    for (int i = 0; i < nV; ++i)
      for (int k = 0; k < len[i]; ++k) emit(pfree.begin(i)[k], (int)sell_slot(H.poff, i, k));
  }, false);
  std::vector<int> tl(nV);
  for (int v = 0; v < nV; ++v) tl[v] = tslots.len(v);
  H.tsoff = sell_offsets(nV, tl);
  H.tpos.assign(H.tsoff.back(), -1);
  for (int v = 0; v < nV; ++v)
    for (int k = 0; k < tl[v]; ++k) H.tpos[sell_slot(H.tsoff, v, k)] = tslots.begin(v)[k];
  // MV colouring
  Csr holders = build_csr(nV, [&](auto&& emit) {   // patches whose vertex set holds v
    for (int i = 0; i < nV; ++i)
      for (const int* v = H.pall.begin(i); v != H.pall.end(i); ++v) emit(*v, i);
  }, false);
  std::vector<int> colour(nV, -1), stamp(nV, -1);
  int ncol = 0;
  for (int i = 0; i < nV; ++i) {
    uint64_t banned = 0;
    for (const int* v = H.pall.begin(i); v != H.pall.end(i); ++v)
      for (const int* u = H.nbr.begin(*v); u != H.nbr.end(*v); ++u) {
        if (stamp[*u] == i) continue;
        stamp[*u] = i;
        for (const int* q = holders.begin(*u); q != holders.end(*u); ++q)
          if (*q < i) banned |= 1ull << colour[*q];
      }
    int c = 0;
    while (c < 64 && ((banned >> c) & 1ull)) ++c;
    if (c >= 64) { err = "MV colouring needs more than 64 colours"; return false; }
    colour[i] = c;
    ncol = std::max(ncol, c + 1);
  }
  H.cstart.assign(ncol + 1, 0);
  for (int i = 0; i < nV; ++i) ++H.cstart[colour[i] + 1];
  for (int c = 0; c < ncol; ++c) H.cstart[c + 1] += H.cstart[c];
  H.order.assign(nV, 0);
  std::vector<int> fill(H.cstart.begin(), H.cstart.end() - 1);
  for (int i = 0; i < nV; ++i) H.order[fill[colour[i]]++] = i;
  return true;
}

// Transfer from the coarse grid: the coarse function at the fine vertices
// (bilinear on a coarse leaf that contains the vertex, hanging coarse corners
// through their constraints), and its transpose.
bool build_transfer(const Topo& fine, const Topo& coarse, HostLevel& H, int nVc, std::string& err) {
  const long long Mx = fine.Mx, My = fine.My, M = std::max(Mx, My);
  std::unordered_map<long long, int> cells;
  cells.reserve((size_t)coarse.nl * 2);
  int smin = INT_MAX;
  auto ckey = [&](long long x0, long long y0, long long s) { return ((y0 * (Mx + 1)) + x0) * 64 + __builtin_ctzll(s); };
  for (long long e = 0; e < coarse.nl; ++e) {
    cells[ckey(coarse.leaf[3 * e], coarse.leaf[3 * e + 1], coarse.leaf[3 * e + 2])] = (int)e;
    smin = std::min(smin, coarse.leaf[3 * e + 2]);
  }
  // nesting: every fine leaf lies in a coarse leaf at least as large
  for (long long e = 0; e < fine.nl; ++e) {
    const long long x0 = fine.leaf[3 * e], y0 = fine.leaf[3 * e + 1], s = fine.leaf[3 * e + 2];
    bool found = false;
    for (long long sc = s; sc <= M && !found; sc *= 2)
      found = cells.count(ckey(x0 / sc * sc, y0 / sc * sc, sc)) > 0;
    if (!found) { err = "grids are not nested (each grid must refine the previous one)"; return false; }
  }
  const int nV = fine.nV();
  H.pptr.assign(nV + 1, 0);
  H.pidx.clear();
  H.pwt.clear();
  std::vector<Wt> row;
  for (int i = 0; i < nV; ++i) {
    const long long px = fine.kx(fine.reg[i]), py = fine.ky(fine.reg[i]);
    int li = -1;
    long long x0 = 0, y0 = 0, sc = smin;
    // the coarse leaf that holds the vertex: of the cells of size sc that touch
    // it (one to four), the first that is a leaf
    for (; sc <= M && li < 0; sc *= 2)
      for (int c = 0; c < 4 && li < 0; ++c) {
        const long long cx = px / sc * sc - ((c & 1) && px % sc == 0 ? sc : 0);
        const long long cy = py / sc * sc - ((c & 2) && py % sc == 0 ? sc : 0);
        if (cx < 0 || cy < 0 || cx + sc > Mx || cy + sc > My) continue;
        auto it = cells.find(ckey(cx, cy, sc));
        if (it != cells.end()) { li = it->second; x0 = cx; y0 = cy; }
      }
    sc = li >= 0 ? coarse.leaf[3 * li + 2] : sc;
    if (li < 0) { err = "a fine vertex lies in no coarse leaf"; return false; }
    const double tx = (double)(px - x0) / (double)sc, ty = (double)(py - y0) / (double)sc;
    row.clear();
    for (int a = 0; a < 4; ++a) {
      const double w = ((a & 1) ? tx : 1.0 - tx) * ((a >> 1) ? ty : 1.0 - ty);
      if (w == 0.0) continue;
      for (int c = coarse.cw_ptr[4 * li + a]; c < coarse.cw_ptr[4 * li + a + 1]; ++c) {
        const int j = coarse.cw[c].v;
        auto it = std::find_if(row.begin(), row.end(), [&](const Wt& t) { return t.v == j; });
        if (it == row.end()) row.push_back({j, w * coarse.cw[c].w});
        else it->w += w * coarse.cw[c].w;
      }
    }
    std::sort(row.begin(), row.end(), [](const Wt& p, const Wt& q) { return p.v < q.v; });
    for (const Wt& t : row) { H.pidx.push_back(t.v); H.pwt.push_back(t.w); }
    H.pptr[i + 1] = (int)H.pidx.size();
  }
  H.rptr.assign(nVc + 1, 0);
  for (int j : H.pidx) ++H.rptr[j + 1];
  for (int j = 0; j < nVc; ++j) H.rptr[j + 1] += H.rptr[j];
  H.ridx.assign(H.pidx.size(), 0);
  H.rwt.assign(H.pidx.size(), 0.0);
  std::vector<int> fill(H.rptr.begin(), H.rptr.end() - 1);
  for (int i = 0; i < nV; ++i)
    for (int k = H.pptr[i]; k < H.pptr[i + 1]; ++k) {
      const int j = H.pidx[k];
      H.ridx[fill[j]] = i;
      H.rwt[fill[j]] = H.pwt[k];
      ++fill[j];
    }
  return true;
}

// Leaves of one grid: aligned power-of-two cells (s >= 2) inside the
// rectangle, pairwise disjoint; `area` receives their total area (every grid
// must cover the coarsest grid's region, which nesting then makes the same).
bool check_leaves(const int* lv, long long n, long long Mx, long long My, long long& area, std::string& err) {
  std::unordered_set<long long> seen;
  seen.reserve((size_t)n * 2);
  area = 0;
  const long long M = std::max(Mx, My);
  auto k3 = [&](long long x0, long long y0, long long s) { return ((y0 * (Mx + 1)) + x0) * 64 + __builtin_ctzll(s); };
  for (long long e = 0; e < n; ++e) {
    const long long x0 = lv[3 * e], y0 = lv[3 * e + 1], s = lv[3 * e + 2];
    if (s < 2 || (s & (s - 1)) || x0 < 0 || y0 < 0 || x0 % s || y0 % s || x0 + s > Mx || y0 + s > My) {
      err = "leaf " + std::to_string(e) + " is not an aligned cell of even power-of-two size inside the rectangle";
      return false;
    }
    if (!seen.insert(k3(x0, y0, s)).second) { err = "duplicate leaf " + std::to_string(e); return false; }
    area += s * s;
  }
  for (long long e = 0; e < n; ++e) {   // no leaf inside another
    const long long x0 = lv[3 * e], y0 = lv[3 * e + 1], s = lv[3 * e + 2];
    for (long long sc = 2 * s; sc <= M; sc *= 2)
      if (seen.count(k3(x0 / sc * sc, y0 / sc * sc, sc))) { err = "overlapping leaves"; return false; }
  }
  return true;
}

template <class T>
hipError_t upload(T** d, const std::vector<T>& h) {
  *d = nullptr;
  if (h.empty()) return hipSuccess;
  hipError_t e = rav_dmalloc((void**)d, sizeof(T) * h.size());
  if (e == hipSuccess) e = hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice);
  return e;
}

rav_ad_state* st(const rav_ctx* ctx) { return ctx->ad; }

rav_status check_lv(const rav_ctx* ctx, int level, bool smoothed) {
  if (level < 0 || level >= (int)st(ctx)->lv.size()) return RAV_EINVAL;
  if (smoothed && level == 0) return RAV_EINVAL;
  return RAV_OK;
}

// ---- cycle -------------------------------------------------------------------
void residual(rav_ctx* ctx, int l, bool with_norm) {
  Level& L = st(ctx)->lv[l];
  ad_launch_residual(L.dev, L.x, L.b, L.r, with_norm ? L.partials : nullptr, ctx->stream);
  if (with_norm) launch_norm_finalize(L.partials, 0, L.nres, ctx->d_norm, ctx->h_norm_dev, ctx->stream);
}

void apply(rav_ctx* ctx, int l) {
  Level& L = st(ctx)->lv[l];
  const rav_problem_desc& D = ctx->desc;
  if (D.smoother == RAV_SMOOTHER_AV)
    ad_launch_av(L.dev, L.fac, L.tsoff, L.tpos, L.r, L.yx, L.yy, L.yp, L.x, D.omega, ctx->stream);
  else
    ad_launch_rav(L.dev, L.fac, L.r, L.x, D.omega, ctx->stream);
}

// RAV (eq. 13) and AV (eq. 12) from one residual each sweep (r_valid: L.r
// already holds b - L x); MV (eq. 11) colour by colour, each patch recomputing
// its residual rows (eq. 15).
void smooth(rav_ctx* ctx, int l, int sweeps, bool r_valid) {
  Level& L = st(ctx)->lv[l];
  const rav_problem_desc& D = ctx->desc;
  for (int k = 0; k < sweeps; ++k) {
    if (D.smoother == RAV_SMOOTHER_MV) {
      for (size_t c = 0; c + 1 < L.cstart.size(); ++c)
        ad_launch_mv(L.dev, L.fac, L.order, L.cstart[c], L.cstart[c + 1] - L.cstart[c], L.b, L.x, D.omega,
                     ctx->stream);
      continue;
    }
    if (!(k == 0 && r_valid)) residual(ctx, l, false);
    apply(ctx, l);
  }
}

void coarse_solve(rav_ctx* ctx) {
  rav_ad_state* S = st(ctx);
  Level& L0 = S->lv[0];
  launch_coarse_gemv(S->Minv, S->nb, 3LL * L0.nV, L0.b, L0.x, ctx->stream);
}

void restrict_to(rav_ctx* ctx, int l, double* rc) {
  Level& L = st(ctx)->lv[l];
  Level& C = st(ctx)->lv[l - 1];
  ad_launch_restrict(L.dev, C.dev, L.rptr, L.ridx, L.rw, L.r, C.b, C.x, rc, ctx->stream);
}

void prolong(rav_ctx* ctx, int l) {
  Level& L = st(ctx)->lv[l];
  Level& C = st(ctx)->lv[l - 1];
  ad_launch_prolong(L.dev, C.dev, L.pptr, L.pidx, L.pw, C.x, L.x, ctx->stream);
}

// V-cycle on level l (Sec. 2, Fig. 1); r_valid: L.r holds the residual of
// the current x (coarse levels: restriction writes r_c = b_c for x_c = 0).
void vcycle(rav_ctx* ctx, int l, bool r_valid) {
  if (l == 0) {
    coarse_solve(ctx);
    return;
  }
  smooth(ctx, l, ctx->desc.nu_pre, r_valid);
  if (ctx->desc.nu_pre > 0 || !r_valid) residual(ctx, l, false);
  restrict_to(ctx, l, l - 1 > 0 ? st(ctx)->lv[l - 1].r : nullptr);
  vcycle(ctx, l - 1, true);
  prolong(ctx, l);
  smooth(ctx, l, ctx->desc.nu_post, false);
}

void issue_cycle(rav_ctx* ctx) {
  const int lf = (int)st(ctx)->lv.size() - 1;
  vcycle(ctx, lf, true);
  residual(ctx, lf, true);
}

rav_status need_factors(rav_ctx* ctx) {
  if (!st(ctx)->have_factors) return rav_set_error(ctx, RAV_EINVAL, "rav_factor_patches has not been called");
  return RAV_OK;
}

// Dense coarse matrix (masked rows and columns replaced by the identity),
// inverted once on the device.  With Dirichlet velocity on the whole boundary
// the pressure is fixed only up to a constant: the matrix is then bordered by
// the zero-mean pressure constraint.
rav_status build_coarse(rav_ctx* ctx, const HostLevel& H) {
  rav_ad_state* S = st(ctx);
  const bool border = ctx->desc.bc_dirichlet_mask == 0xFu;
  const long long n0 = 3LL * H.nV, nb = n0 + (border ? 1 : 0), nV = H.nV, P = H.nnz;
  S->nb = nb;
  std::vector<double> M((size_t)(nb * nb), 0.0);
  for (int i = 0; i < H.nV; ++i) {
    const int w = H.nbr.len(i);
    for (int k = 0; k < w; ++k) {
      const int j = H.nbr.begin(i)[k];
      const long long s = sell_slot(H.soff, i, k);
      M[(size_t)(i * nb + j)] += H.val[AD_A * P + s];
      M[(size_t)((nV + i) * nb + nV + j)] += H.val[AD_A * P + s];
      M[(size_t)(i * nb + 2 * nV + j)] += H.val[AD_BTX * P + s];
      M[(size_t)((nV + i) * nb + 2 * nV + j)] += H.val[AD_BTY * P + s];
      M[(size_t)((2 * nV + i) * nb + j)] += H.val[AD_BX * P + s];
      M[(size_t)((2 * nV + i) * nb + nV + j)] += H.val[AD_BY * P + s];
      M[(size_t)((2 * nV + i) * nb + 2 * nV + j)] += H.val[AD_C * P + s];
    }
    if (H.vmask[i]) {
      M[(size_t)(i * nb + i)] = 1.0;
      M[(size_t)((nV + i) * nb + nV + i)] = 1.0;
    }
  }
  for (long long j = 2 * nV; j < n0 && border; ++j) {
    M[(size_t)(n0 * nb + j)] = 1.0;
    M[(size_t)(j * nb + n0)] = 1.0;
  }
  ACK(rav_dmalloc((void**)&S->Minv, sizeof(double) * nb * nb));
  ACK(hipMemcpy(S->Minv, M.data(), sizeof(double) * nb * nb, hipMemcpyHostToDevice));
  double** dM = nullptr;
  int *piv = nullptr, *perm = nullptr, *pst = nullptr;
  double *colk = nullptr, *Rs = nullptr;
  const int big = INT_MAX;
  ACK(rav_dmalloc((void**)&dM, sizeof(double*)));
  ACK(rav_dmalloc((void**)&piv, sizeof(int) * nb));
  ACK(rav_dmalloc((void**)&perm, sizeof(int) * nb));
  ACK(rav_dmalloc((void**)&pst, sizeof(int)));
  ACK(rav_dmalloc((void**)&colk, sizeof(double) * nb));
  ACK(rav_dmalloc((void**)&Rs, sizeof(double) * GJ_PANEL * nb));
  ACK(hipMemcpy(dM, &S->Minv, sizeof(double*), hipMemcpyHostToDevice));
  ACK(hipMemcpy(pst, &big, sizeof(int), hipMemcpyHostToDevice));
  launch_bgj_invert(dM, nb, 1, piv, colk, Rs, perm, pst, ctx->stream);
  ACK(hipGetLastError());
  int status = 0;
  ACK(hipMemcpyAsync(&status, pst, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  ACK(hipStreamSynchronize(ctx->stream));
  (void)rav_dfree(dM); (void)rav_dfree(piv); (void)rav_dfree(perm); (void)rav_dfree(pst); (void)rav_dfree(colk);
  (void)rav_dfree(Rs);
  if (status != INT_MAX)
    return rav_set_error(ctx, RAV_ESINGULAR, "zero pivot in the coarse matrix at column " + std::to_string(status));
  return RAV_OK;
}

// Device encoding of the operator entries: packed (column offset and tuple id
// in one 32-bit word, id_bits = bits the ids need) when every offset fits the
// remaining bits, else wide.
void encode(HostLevel& H) {
  const int nV = H.nV;
  const long long ntuple = (long long)(H.vtab.size() / 8);
  int id_bits = 1;
  while ((1LL << id_bits) < ntuple) ++id_bits;
  const long long lim = 1LL << (31 - id_bits);   // offsets in [-lim, lim)
  bool fit = id_bits <= 24;
  for (int i = 0; i < nV && fit; ++i) {
    const int w = (H.soff[i / AD_SLICE + 1] - H.soff[i / AD_SLICE]) / AD_SLICE;
    for (int k = 0; k < w; ++k) {
      const long long d = (long long)H.col[sell_slot(H.soff, i, k)] - i;
      fit = fit && d >= -lim && d < lim;
    }
  }
  H.wide = !fit;
  H.id_bits = id_bits;
  H.ent.assign(H.nnz, 0u);
  for (int i = 0; i < nV; ++i) {
    const int w = (H.soff[i / AD_SLICE + 1] - H.soff[i / AD_SLICE]) / AD_SLICE;
    for (int k = 0; k < w; ++k) {
      const long long e = sell_slot(H.soff, i, k);
      const unsigned id = (unsigned)H.vid[e];
      H.ent[e] = H.wide ? id : (((unsigned)(H.col[e] - i) << id_bits) | id);
    }
  }
}

rav_status upload_level(rav_ctx* ctx, Level& L, const HostLevel& H, bool smoothed, bool has_transfer) {
  L.nV = H.nV;
  long long masked = 0;
  for (unsigned char m : H.vmask) masked += m;
  L.nfree = 3LL * H.nV - 2 * masked;
  L.nnz_true = (long long)H.nbr.idx.size();
  for (int v : H.pv) L.pnnz_true += v >= 0;
  L.ntuple = (int)(H.vtab.size() / 8);
  ACK(upload(&L.vmask, H.vmask));
  ACK(upload(&L.soff, H.soff));
  ACK(upload(&L.ent, H.ent));
  if (H.wide) ACK(upload(&L.col, H.col));
  ACK(upload(&L.vtab, H.vtab));
  const long long n = 3LL * H.nV;
  ACK(rav_dmalloc((void**)&L.x, sizeof(double) * n));
  ACK(rav_dmalloc((void**)&L.b, sizeof(double) * n));
  ACK(rav_dmalloc((void**)&L.r, sizeof(double) * n));
  ACK(hipMemset(L.x, 0, sizeof(double) * n));
  ACK(hipMemset(L.b, 0, sizeof(double) * n));
  ACK(hipMemset(L.r, 0, sizeof(double) * n));
  AdDev& a = L.dev;
  a.nV = H.nV;
  a.nslice = (int)H.soff.size() - 1;
  a.wide = H.wide ? 1 : 0;
  a.id_bits = H.id_bits;
  a.ntuple = L.ntuple;
  {   // RAV_AD_TABLE_LDS=0 keeps the table in global memory (the path of larger tables),
      // =1 stages it for the residual on every grid size
    const char* e = std::getenv("RAV_AD_TABLE_LDS");
    const bool off = e && std::string(e) == "0", all = e && std::string(e) == "1";
    a.table_lds = (L.ntuple <= AD_LDS_TUPLES && !off) ? 1 : 0;
    a.res_lds = (a.table_lds && (all || L.nV >= AD_RES_LDS_MIN_VERTICES)) ? 1 : 0;
  }
  a.nnz = H.nnz;
  a.vmask = L.vmask;
  a.soff = L.soff;
  a.ent = L.ent;
  a.col = L.col;
  a.vtab = L.vtab;
  L.nres = ad_residual_blocks(a);
  ACK(rav_dmalloc((void**)&L.partials, sizeof(double) * L.nres));
  if (smoothed) {
    ACK(upload(&L.poff, H.poff));
    ACK(upload(&L.pv, H.pv));
    ACK(upload(&L.pcfg, H.pcfg));
    ACK(upload(&L.cnf, H.cnf));
    ACK(upload(&L.cown, H.cown));
    ACK(upload(&L.rep, H.rep));
    ACK(upload(&L.tsoff, H.tsoff));
    ACK(upload(&L.tpos, H.tpos));
    ACK(upload(&L.order, H.order));
    L.cstart = H.cstart;
    L.pnnz = H.pnnz;
    L.ncfg = (int)H.rep.size();
    L.h_poff = H.poff;
    L.h_pv = H.pv;
    L.h_pcfg = H.pcfg;
    L.h_cnf = H.cnf;
    L.h_cown = H.cown;
    a.pnnz = H.pnnz;
    a.poff = L.poff;
    a.pv = L.pv;
    a.pcfg = L.pcfg;
    a.cnf = L.cnf;
    a.cown = L.cown;
  }
  if (has_transfer) {
    ACK(upload(&L.pptr, H.pptr));
    ACK(upload(&L.pidx, H.pidx));
    ACK(upload(&L.pw, H.pwt));
    ACK(upload(&L.rptr, H.rptr));
    ACK(upload(&L.ridx, H.ridx));
    ACK(upload(&L.rw, H.rwt));
  }
  return RAV_OK;
}

rav_status check_desc(const rav_problem_desc* d, long lattice_x, long lattice_y) {
  if (d->discretization != RAV_Q1Q1_ADAPTIVE)
    return rav_set_error(nullptr, RAV_EINVAL, "rav_create_adaptive needs discretization RAV_Q1Q1_ADAPTIVE");
  if (d->dim != 2) return rav_set_error(nullptr, RAV_EUNSUPPORTED, "adaptive grids are provided in 2D");
  if (d->n_levels < 2 || d->n_levels > 24) return rav_set_error(nullptr, RAV_EINVAL, "n_levels must be in [2, 24]");
  if (lattice_x < 2 || lattice_x > (1L << 24) || lattice_y < 2 || lattice_y > (1L << 24))
    return rav_set_error(nullptr, RAV_EINVAL, "lattice sizes must be in [2, 2^24]");
  if (d->bc_dirichlet_mask > 0xFu)
    return rav_set_error(nullptr, RAV_EINVAL, "bc_dirichlet_mask has bits beyond the four sides");
  if (!(d->beta > 0.0)) return rav_set_error(nullptr, RAV_EINVAL, "the stabilization constant beta must be > 0");
  if (!(d->eta_out > 0.0)) return rav_set_error(nullptr, RAV_EINVAL, "viscosity must be > 0");
  if (d->n_incl != 0) return rav_set_error(nullptr, RAV_EUNSUPPORTED, "adaptive grids use a constant viscosity");
  if (!(d->omega > 0.0) || d->nu_pre < 0 || d->nu_post < 0)
    return rav_set_error(nullptr, RAV_EINVAL, "omega must be > 0 and smoothing steps >= 0");
  if (d->smoother < RAV_SMOOTHER_RAV || d->smoother > RAV_SMOOTHER_MV)
    return rav_set_error(nullptr, RAV_EINVAL, "bad smoother");
  if (d->patch != RAV_PATCH_VERTEX || d->inv_precision != RAV_FP64 || d->coarse_galerkin != 0)
    return rav_set_error(nullptr, RAV_EUNSUPPORTED,
                         "adaptive grids are provided with vertex patches, FP64 inverses and rediscretised levels");
  if (d->inv_format != RAV_ROWS && d->inv_format != RAV_FACTORED)
    return rav_set_error(nullptr, RAV_EINVAL, "bad inverse format");
  return RAV_OK;
}

// Validates every grid and builds its topology.
bool build_topos(const rav_problem_desc* d, const int* leaves, const long* n_leaves, long lattice_x,
                 long lattice_y, std::vector<Topo>& topo, std::string& err) {
  const int nl = d->n_levels;
  std::vector<long long> first(nl + 1, 0);
  for (int l = 0; l < nl; ++l) {
    if (n_leaves[l] <= 0) { err = "every grid needs leaves"; return false; }
    first[l + 1] = first[l] + n_leaves[l];
  }
  topo.assign(nl, Topo());
  std::vector<std::string> errs(nl);
  std::vector<long long> area(nl, 0);
  parallel_for(nl, [&](int t) {
    const int l = nl - 1 - t;   // largest grids first
    const int* lv = leaves + 3 * first[l];
    std::string e2;
    if (!check_leaves(lv, n_leaves[l], lattice_x, lattice_y, area[l], e2) ||
        !topo[l].build(lv, n_leaves[l], lattice_x, lattice_y))
      errs[l] = "grid " + std::to_string(l) + ": " + (e2.empty() ? topo[l].err : e2);
  });
  for (int l = 0; l < nl; ++l)
    if (!errs[l].empty()) {
      err = errs[l];
      return false;
    }
  for (int l = 1; l < nl; ++l)
    if (area[l] != area[0]) {
      err = "grid " + std::to_string(l) + ": leaves do not cover the region of the coarsest grid";
      return false;
    }
  if (3LL * topo[0].nV() + 1 > MAX_COARSE) {
    err = "coarsest grid too large for the dense direct solve";
    return false;
  }
  return true;
}

}  // namespace

// ============================================================================
rav_status rav_ad_create(const rav_problem_desc* d, const int* leaves, const long* n_leaves, long lattice_x,
                         long lattice_y, void* hip_stream, rav_ctx** out) {
  if (!d || !leaves || !n_leaves || !out) return rav_set_error(nullptr, RAV_EINVAL, "null argument");
  rav_status s0 = check_desc(d, lattice_x, lattice_y);
  if (s0 != RAV_OK) return s0;
  const int nl = d->n_levels;
  std::vector<Topo> topo;
  std::string err;
  if (!build_topos(d, leaves, n_leaves, lattice_x, lattice_y, topo, err))
    return rav_set_error(nullptr, RAV_EINVAL, err);

  rav_ctx* ctx = new rav_ctx();
  ctx->desc = *d;
  ctx->desc.incl = nullptr;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->prec = P_FP64;
  ctx->ad = new rav_ad_state();
  auto fail = [&](rav_status s) {
    rav_set_error(nullptr, s, ctx->err);
    rav_destroy(ctx);
    return s;
  };
  rav_status s = rav_init_common(ctx, d);
  if (s != RAV_OK) return fail(s);
  rav_ad_state* S = ctx->ad;
  S->mode = d->smoother == RAV_SMOOTHER_RAV ? AD_RAV : AD_FULL;
  S->lv.resize(nl);
  std::vector<HostLevel> hosts(nl);
  std::vector<std::string> errs(nl);
  parallel_for(nl, [&](int t) {
    const int l = nl - 1 - t;
    HostLevel& H = hosts[l];
    std::string e2;
    if (!assemble(topo[l], d->beta, d->eta_out, d->bc_dirichlet_mask, l == nl - 1, H, e2) ||
        (l > 0 && (!build_patches(topo[l], H, e2) || !build_transfer(topo[l], topo[l - 1], H, topo[l - 1].nV(), e2))))
      errs[l] = "grid " + std::to_string(l) + ": " + e2;
  });
  for (int l = 0; l < nl; ++l)
    if (!errs[l].empty()) {
      ctx->err = errs[l];
      return fail(errs[l].find("more than") != std::string::npos ? RAV_EUNSUPPORTED : RAV_EINVAL);
    }
  parallel_for(nl, [&](int l) { encode(hosts[l]); });
  for (int l = 0; l < nl; ++l) {
    HostLevel& H = hosts[l];
    if ((s = upload_level(ctx, S->lv[l], H, l > 0, l > 0)) != RAV_OK) return fail(s);
    if (l == nl - 1) {
      hipError_t e = upload(&S->blid, H.blid);
      if (e != hipSuccess) { ctx->err = hipGetErrorString(e); return fail(RAV_EDEVICE); }
      S->fine_mask = H.vmask;
      S->dc_row = std::move(H.dc_row);
      S->dc_col = std::move(H.dc_col);
      S->dc_val = std::move(H.dc_val);
    }
    if (l == 0 && (s = build_coarse(ctx, H)) != RAV_OK) return fail(s);
    H = HostLevel();
  }
  *out = ctx;
  return RAV_OK;
}

void rav_ad_free(rav_ctx* ctx) {
  rav_ad_state* S = ctx->ad;
  if (!S) return;
  for (Level& L : S->lv) {
    void* ptrs[] = {L.vmask, L.soff, L.col, L.ent, L.vtab, L.poff, L.pv, L.pcfg, L.cnf, L.cown, L.rep,
                    L.fac.zx, L.fac.zy, L.fac.invS,
                    L.fac.kr, L.fac.kfull, L.tsoff, L.tpos, L.yx, L.yy, L.yp, L.order, L.pptr, L.pidx, L.pw,
                    L.rptr, L.ridx, L.rw, L.x, L.b, L.r, L.partials};
    for (void* p : ptrs) (void)rav_dfree(p);
  }
  (void)rav_dfree(S->Minv);
  (void)rav_dfree(S->blid);
  delete S;
  ctx->ad = nullptr;
}

rav_status rav_ad_factor(rav_ctx* ctx) {
  rav_ad_state* S = st(ctx);
  const int big = INT_MAX;
  for (size_t l = 1; l < S->lv.size(); ++l) {
    Level& L = S->lv[l];
    if (!L.fac.zx) {
      const long long nc = std::max(L.ncfg, 1);
      ACK(rav_dmalloc((void**)&L.fac.zx, sizeof(double) * nc * AD_NFMAX));
      ACK(rav_dmalloc((void**)&L.fac.zy, sizeof(double) * nc * AD_NFMAX));
      ACK(rav_dmalloc((void**)&L.fac.invS, sizeof(double) * nc));
      if (S->mode == AD_RAV) {
        ACK(rav_dmalloc((void**)&L.fac.kr, sizeof(double) * nc * AD_NFMAX));
      } else {
        ACK(rav_dmalloc((void**)&L.fac.kfull, sizeof(double) * nc * AD_NFMAX * AD_NFMAX));
        ACK(rav_dmalloc((void**)&L.yx, sizeof(double) * L.pnnz));
        ACK(rav_dmalloc((void**)&L.yy, sizeof(double) * L.pnnz));
        ACK(rav_dmalloc((void**)&L.yp, sizeof(double) * L.nV));
      }
    }
    ACK(hipMemcpy(ctx->d_status, &big, sizeof(int), hipMemcpyHostToDevice));
    ad_launch_factor(L.dev, S->mode, L.rep, L.ncfg, L.fac, ctx->d_status, ctx->stream);
    ACK(hipGetLastError());
    int stv = 0;
    ACK(hipMemcpyAsync(&stv, ctx->d_status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    ACK(hipStreamSynchronize(ctx->stream));
    if (stv != INT_MAX)
      return rav_set_error(ctx, RAV_ESINGULAR,
                           "singular local system in patch " + std::to_string(stv) + " on level " + std::to_string(l));
  }
  rav_drop_graph(ctx);
  S->have_factors = true;
  ctx->factored = 1;
  return RAV_OK;
}

rav_status rav_ad_dofs(const rav_ctx* ctx, int level, long* n_total, long* n_free) {
  if (check_lv(ctx, level, false) != RAV_OK) return RAV_EINVAL;
  const Level& L = st(ctx)->lv[level];
  if (n_total) *n_total = 3L * L.nV;
  if (n_free) *n_free = (long)L.nfree;
  return RAV_OK;
}

int rav_ad_n_levels(const rav_ctx* ctx) { return (int)st(ctx)->lv.size(); }

rav_status rav_ad_n_patches(const rav_ctx* ctx, int level, long* n) {
  if (check_lv(ctx, level, false) != RAV_OK || !n) return RAV_EINVAL;
  *n = (long)st(ctx)->lv[level].nV;
  return RAV_OK;
}

rav_status rav_ad_assemble_rhs_lid(rav_ctx* ctx, double lid_u, double* b_dev) {
  const Level& L = st(ctx)->lv.back();
  if (!st(ctx)->blid) return rav_set_error(ctx, RAV_EINVAL, "the lid needs Dirichlet velocity on the top side");
  ad_launch_scale(st(ctx)->blid, lid_u, b_dev, 3LL * L.nV, ctx->stream);
  ACK(hipGetLastError());
  ACK(hipStreamSynchronize(ctx->stream));
  return RAV_OK;
}

// b = -L_all[:, masked] u_D on the finest grid, masked rows zero (host sums
// over the stored couplings, then one copy).
rav_status rav_ad_assemble_rhs_dirichlet(rav_ctx* ctx, const double* ud, double* b_dev) {
  const rav_ad_state* S = st(ctx);
  const long long nV = S->lv.back().nV;
  std::vector<double> b(3 * nV, 0.0);
  for (size_t q = 0; q < S->dc_row.size(); ++q) {
    const int i = S->dc_row[q], j = S->dc_col[q];
    const double a = S->dc_val[3 * q], bx = S->dc_val[3 * q + 1], by = S->dc_val[3 * q + 2];
    const double ux = ud[j], uy = ud[nV + j];
    if (!S->fine_mask[i]) {
      b[i] -= a * ux;
      b[nV + i] -= a * uy;
    }
    b[2 * nV + i] -= bx * ux + by * uy;
  }
  ACK(hipMemcpyAsync(b_dev, b.data(), sizeof(double) * b.size(), hipMemcpyHostToDevice, ctx->stream));
  ACK(hipStreamSynchronize(ctx->stream));
  return RAV_OK;
}

rav_status rav_ad_residual(rav_ctx* ctx, int level, const double* x, const double* b, double* r, double* norm) {
  if (check_lv(ctx, level, false) != RAV_OK) return RAV_EINVAL;
  Level& L = st(ctx)->lv[level];
  const long long n = 3LL * L.nV;
  launch_copy(L.x, x, n, ctx->stream);
  launch_copy(L.b, b, n, ctx->stream);
  residual(ctx, level, norm != nullptr);
  launch_copy(r, L.r, n, ctx->stream);
  ACK(hipGetLastError());
  if (norm) return rav_read_norm(ctx, norm);
  return RAV_OK;
}

rav_status rav_ad_smooth(rav_ctx* ctx, int level, int sweeps, double* x, const double* b) {
  if (check_lv(ctx, level, true) != RAV_OK) return RAV_EINVAL;
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  Level& L = st(ctx)->lv[level];
  const long long n = 3LL * L.nV;
  launch_copy(L.x, x, n, ctx->stream);
  launch_copy(L.b, b, n, ctx->stream);
  smooth(ctx, level, sweeps, false);
  launch_copy(x, L.x, n, ctx->stream);
  ACK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_ad_restrict(rav_ctx* ctx, int level, const double* rf, double* bc) {
  if (check_lv(ctx, level, true) != RAV_OK) return RAV_EINVAL;
  Level& L = st(ctx)->lv[level];
  Level& C = st(ctx)->lv[level - 1];
  launch_copy(L.r, rf, 3LL * L.nV, ctx->stream);
  restrict_to(ctx, level, nullptr);
  launch_copy(bc, C.b, 3LL * C.nV, ctx->stream);
  ACK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_ad_prolong_add(rav_ctx* ctx, int level, const double* xc, double* xf) {
  if (check_lv(ctx, level, true) != RAV_OK) return RAV_EINVAL;
  Level& L = st(ctx)->lv[level];
  Level& C = st(ctx)->lv[level - 1];
  launch_copy(C.x, xc, 3LL * C.nV, ctx->stream);
  launch_copy(L.x, xf, 3LL * L.nV, ctx->stream);
  prolong(ctx, level);
  launch_copy(xf, L.x, 3LL * L.nV, ctx->stream);
  ACK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_ad_coarse_solve(rav_ctx* ctx, const double* b0, double* x0) {
  rav_ad_state* S = st(ctx);
  launch_coarse_gemv(S->Minv, S->nb, 3LL * S->lv[0].nV, b0, x0, ctx->stream);
  ACK(hipGetLastError());
  return RAV_OK;
}

// FGMRES hooks (rav_krylov.hip): the finest level's vectors, its residual
// (norm into the context's norm slot) and one V-cycle in place on them.
RavFinest rav_ad_finest(rav_ctx* ctx) {
  Level& L = st(ctx)->lv.back();
  return RavFinest{3LL * L.nV, L.x, L.b, L.r, st(ctx)->have_factors};
}
void rav_ad_residual_finest(rav_ctx* ctx, bool with_norm) { residual(ctx, (int)st(ctx)->lv.size() - 1, with_norm); }
void rav_ad_vcycle_finest(rav_ctx* ctx) { vcycle(ctx, (int)st(ctx)->lv.size() - 1, false); }

rav_status rav_ad_vcycle(rav_ctx* ctx, double* x, const double* b) {
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  const int lf = (int)st(ctx)->lv.size() - 1;
  Level& L = st(ctx)->lv[lf];
  const long long n = 3LL * L.nV;
  launch_copy(L.x, x, n, ctx->stream);
  launch_copy(L.b, b, n, ctx->stream);
  vcycle(ctx, lf, false);
  launch_copy(x, L.x, n, ctx->stream);
  ACK(hipGetLastError());
  return RAV_OK;
}

rav_status rav_ad_solve(rav_ctx* ctx, double* x, const double* b, double rtol, int maxit, int* iters,
                        double* rel_res) {
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  const int lf = (int)st(ctx)->lv.size() - 1;
  Level& L = st(ctx)->lv[lf];
  const long long n = 3LL * L.nV;
  launch_copy(L.x, x, n, ctx->stream);
  launch_copy(L.b, b, n, ctx->stream);
  residual(ctx, lf, true);
  double r0 = 0.0;
  rav_status s = rav_read_norm(ctx, &r0);
  if (s != RAV_OK) return s;
  if (iters) *iters = 0;
  if (rel_res) *rel_res = r0 > 0.0 ? 1.0 : 0.0;
  if (!std::isfinite(r0)) return rav_set_error(ctx, RAV_EDIVERGED, "initial residual is not finite");
  rav_status result = r0 == 0.0 ? RAV_OK : RAV_NOT_CONVERGED;
  int k = 0;
  double rk = r0;
  while (result == RAV_NOT_CONVERGED && k < maxit) {
    rav_graph_cycle(ctx, issue_cycle);   // the finest residual is current from the norm evaluation
    if ((s = rav_read_norm(ctx, &rk)) != RAV_OK) return s;
    ++k;
    if (!std::isfinite(rk) || rk > 1e3 * r0) {
      result = RAV_EDIVERGED;
      ctx->err = "residual diverged at cycle " + std::to_string(k);
    } else if (rk <= rtol * r0) {
      result = RAV_OK;
    }
  }
  if (iters) *iters = k;
  if (rel_res) *rel_res = r0 > 0.0 ? rk / r0 : 0.0;
  launch_copy(x, L.x, n, ctx->stream);
  ACK(hipGetLastError());
  ACK(hipStreamSynchronize(ctx->stream));
  return result;
}

// Patch DoFs in local order: u_x of the free patch vertices (ascending), u_y of
// the same vertices, p_i; owned: u_x,i, u_y,i (if free) and p_i.
static int ad_patch_list(const Level& L, long long i, int* dofs, int* owned) {
  const int nV = L.nV;
  const long long sl = i / AD_SLICE, t = i % AD_SLICE;
  const int w = (L.h_poff[sl + 1] - L.h_poff[sl]) / AD_SLICE;
  std::vector<int> vs;
  for (int k = 0; k < w; ++k) {
    const int v = L.h_pv[L.h_poff[sl] + AD_SLICE * k + t];
    if (v >= 0) vs.push_back(v);
  }
  int n = 0;
  for (int c = 0; c < 2; ++c)
    for (int v : vs) {
      dofs[n] = c * nV + v;
      if (owned) owned[n] = v == (int)i;
      ++n;
    }
  dofs[n] = 2 * nV + (int)i;
  if (owned) owned[n] = 1;
  return n + 1;
}

rav_status rav_ad_get_owner(rav_ctx* ctx, int level, int* owner_dev) {
  if (check_lv(ctx, level, false) != RAV_OK) return RAV_EINVAL;
  ad_launch_owner(st(ctx)->lv[level].dev, owner_dev, ctx->stream);
  ACK(hipGetLastError());
  ACK(hipStreamSynchronize(ctx->stream));
  return RAV_OK;
}

rav_status rav_ad_get_patch_map(const rav_ctx* ctx, int level, long patch, int* dofs, int* n, int* owned) {
  if (check_lv(ctx, level, true) != RAV_OK || !dofs || !n) return RAV_EINVAL;
  const Level& L = st(ctx)->lv[level];
  if (patch < 0 || patch >= L.nV) return RAV_EINVAL;
  *n = ad_patch_list(L, patch, dofs, owned);
  return RAV_OK;
}

// Owned rows (RAV) or every row (AV, MV) of L_i^{-1} over the patch DoFs,
// rebuilt from the factored values: with z_c = K^{-1} b_c and S,
// L_i^{-1} = [[K^{-1} + z z^T / S, -z / S], [-z^T / S, 1 / S]] per component.
rav_status rav_ad_get_patch_inverse(rav_ctx* ctx, int level, long patch, double* out, int* rows, int* cols) {
  if (check_lv(ctx, level, true) != RAV_OK) return RAV_EINVAL;
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  rav_ad_state* S = st(ctx);
  const Level& L = S->lv[level];
  if (patch < 0 || patch >= L.nV) return RAV_EINVAL;
  ACK(hipStreamSynchronize(ctx->stream));
  const int c = L.h_pcfg[patch];
  const int nf = L.h_cnf[c], ao = L.h_cown[c];
  std::vector<double> zx(AD_NFMAX), zy(AD_NFMAX), kin((size_t)AD_NFMAX * AD_NFMAX, 0.0);
  double sinv = 0.0;
  ACK(hipMemcpy(zx.data(), L.fac.zx + (long long)c * AD_NFMAX, sizeof(double) * AD_NFMAX, hipMemcpyDeviceToHost));
  ACK(hipMemcpy(zy.data(), L.fac.zy + (long long)c * AD_NFMAX, sizeof(double) * AD_NFMAX, hipMemcpyDeviceToHost));
  ACK(hipMemcpy(&sinv, L.fac.invS + c, sizeof(double), hipMemcpyDeviceToHost));
  if (S->mode == AD_RAV) {
    if (ao >= 0)
      ACK(hipMemcpy(&kin[(size_t)ao * AD_NFMAX], L.fac.kr + (long long)c * AD_NFMAX, sizeof(double) * AD_NFMAX,
                    hipMemcpyDeviceToHost));
  } else {
    ACK(hipMemcpy(kin.data(), L.fac.kfull + (long long)c * AD_NFMAX * AD_NFMAX,
                  sizeof(double) * AD_NFMAX * AD_NFMAX, hipMemcpyDeviceToHost));
  }
  const int n = 2 * nf + 1;
  // entry of L_i^{-1} at local (row, col): velocity (c, m) = c nf + m, pressure 2 nf
  auto entry = [&](int r, int c) -> double {
    const bool rv = r < 2 * nf, cv = c < 2 * nf;
    const int c1 = r < nf ? 0 : 1, m1 = r - c1 * nf, c2 = c < nf ? 0 : 1, m2 = c - c2 * nf;
    const std::vector<double>& zr = c1 == 0 ? zx : zy;
    const std::vector<double>& zc = c2 == 0 ? zx : zy;
    if (rv && cv) return (c1 == c2 ? kin[(size_t)m1 * AD_NFMAX + m2] : 0.0) + zr[m1] * sinv * zc[m2];
    if (rv) return -zr[m1] * sinv;
    if (cv) return -sinv * zc[m2];
    return sinv;
  };
  int nr = 0;
  for (int r = 0; r < n; ++r) {
    const bool own = r == 2 * nf || (ao >= 0 && (r == ao || r == nf + ao));
    if (S->mode == AD_RAV && !own) continue;
    for (int c = 0; c < n; ++c) out[(size_t)nr * n + c] = entry(r, c);
    ++nr;
  }
  *rows = nr;
  *cols = n;
  return RAV_OK;
}

rav_status rav_ad_time_sweep(rav_ctx* ctx, int level, int reps, double* x, const double* b, float* ms_res,
                             float* ms_apply) {
  if (check_lv(ctx, level, true) != RAV_OK) return RAV_EINVAL;
  if (need_factors(ctx) != RAV_OK) return RAV_EINVAL;
  Level& L = st(ctx)->lv[level];
  const long long n = 3LL * L.nV;
  launch_copy(L.x, x, n, ctx->stream);
  launch_copy(L.b, b, n, ctx->stream);
  std::vector<hipEvent_t> ev(3 * reps);
  for (auto& e : ev) ACK(hipEventCreate(&e));
  const bool mv = ctx->desc.smoother == RAV_SMOOTHER_MV;
  for (int i = 0; i < reps; ++i) {
    ACK(hipEventRecord(ev[3 * i], ctx->stream));
    if (!mv) residual(ctx, level, false);
    ACK(hipEventRecord(ev[3 * i + 1], ctx->stream));
    if (mv) smooth(ctx, level, 1, false);
    else apply(ctx, level);
    ACK(hipEventRecord(ev[3 * i + 2], ctx->stream));
  }
  ACK(hipEventSynchronize(ev.back()));
  double tr = 0.0, ta = 0.0;
  for (int i = 0; i < reps; ++i) {
    float a = 0.f, c = 0.f;
    ACK(hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]));
    ACK(hipEventElapsedTime(&c, ev[3 * i + 1], ev[3 * i + 2]));
    tr += a;
    ta += c;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (ms_res) *ms_res = (float)(tr / reps);
  if (ms_apply) *ms_apply = (float)(ta / reps);
  launch_copy(x, L.x, n, ctx->stream);
  ACK(hipStreamSynchronize(ctx->stream));
  return RAV_OK;
}

// Grid statistics for the host: vertices, operator and patch entries (padded), MV colours, the
// operator and patch entries without padding, distinct value tuples, patch configurations and
// the entry format (0 packed, 1 wide).
rav_status rav_ad_level_info(const rav_ctx* ctx, int level, long* info) {
  if (check_lv(ctx, level, false) != RAV_OK || !info) return RAV_EINVAL;
  const Level& L = st(ctx)->lv[level];
  info[0] = L.nV;
  info[1] = (long)L.dev.nnz;
  info[2] = (long)L.pnnz;
  info[3] = L.cstart.empty() ? 0 : (long)L.cstart.size() - 1;
  info[4] = (long)L.nnz_true;
  info[5] = (long)L.pnnz_true;
  info[6] = L.ntuple;
  info[7] = L.ncfg;
  info[8] = L.dev.wide;
  return RAV_OK;
}

// Host-only set-up of one grid, for checks without a device.
rav_status rav_ad_host_export(const rav_problem_desc* d, const int* leaves, const long* n_leaves, long lattice_x,
                              long lattice_y, int level, int what, double* out, long* rows, long* cols) {
  if (!d || !leaves || !n_leaves || !rows || !cols) return rav_set_error(nullptr, RAV_EINVAL, "null argument");
  rav_status s0 = check_desc(d, lattice_x, lattice_y);
  if (s0 != RAV_OK) return s0;
  if (level < 0 || level >= d->n_levels || what < 0 || what > 4 || (level == 0 && (what == 1 || what == 3)))
    return rav_set_error(nullptr, RAV_EINVAL, "bad level or export kind");
  if (what == 2 && !(d->bc_dirichlet_mask & 8u))
    return rav_set_error(nullptr, RAV_EINVAL, "the lid needs Dirichlet velocity on the top side");
  std::vector<Topo> topo;
  std::string err;
  if (!build_topos(d, leaves, n_leaves, lattice_x, lattice_y, topo, err))
    return rav_set_error(nullptr, RAV_EINVAL, err);
  HostLevel H;
  if (!assemble(topo[level], d->beta, d->eta_out, d->bc_dirichlet_mask, what == 2, H, err))
    return rav_set_error(nullptr, RAV_EINVAL, err);
  const long long nV = H.nV, n = 3 * nV, P = H.nnz;
  if (what == 4) {
    *rows = (long)nV;
    *cols = 3;
    if (!out) return RAV_OK;
    for (long long v = 0; v < nV; ++v) {
      out[3 * v] = (double)topo[level].kx(topo[level].reg[v]);
      out[3 * v + 1] = (double)topo[level].ky(topo[level].reg[v]);
      out[3 * v + 2] = (double)H.vmask[v];
    }
    return RAV_OK;
  }
  if (what == 0) {
    *rows = (long)n;
    *cols = (long)n;
    if (!out) return RAV_OK;
    std::fill(out, out + n * n, 0.0);
    for (long long i = 0; i < nV; ++i)
      for (int k = 0; k < H.nbr.len((int)i); ++k) {
        const long long j = H.nbr.begin((int)i)[k];
        const long long sl = sell_slot(H.soff, (int)i, (int)k);
        out[i * n + j] += H.val[AD_A * P + sl];
        out[(nV + i) * n + nV + j] += H.val[AD_A * P + sl];
        out[i * n + 2 * nV + j] += H.val[AD_BTX * P + sl];
        out[(nV + i) * n + 2 * nV + j] += H.val[AD_BTY * P + sl];
        out[(2 * nV + i) * n + j] += H.val[AD_BX * P + sl];
        out[(2 * nV + i) * n + nV + j] += H.val[AD_BY * P + sl];
        out[(2 * nV + i) * n + 2 * nV + j] += H.val[AD_C * P + sl];
      }
    return RAV_OK;
  }
  if (what == 2) {
    *rows = (long)n;
    *cols = 1;
    if (out) std::copy(H.blid.begin(), H.blid.end(), out);
    return RAV_OK;
  }
  if (what == 3) {
    if (!build_patches(topo[level], H, err)) return rav_set_error(nullptr, RAV_EUNSUPPORTED, err);
    *rows = (long)nV;
    *cols = 1;
    if (!out) return RAV_OK;
    for (size_t c = 0; c + 1 < H.cstart.size(); ++c)
      for (int q = H.cstart[c]; q < H.cstart[c + 1]; ++q) out[H.order[q]] = (double)c;
    return RAV_OK;
  }
  // what == 1: prolongation from grid level-1, all three fields, masked rows and columns zero
  const long long nVc = topo[level - 1].nV(), nc = 3 * nVc;
  if (!build_transfer(topo[level], topo[level - 1], H, (int)nVc, err)) return rav_set_error(nullptr, RAV_EINVAL, err);
  *rows = (long)n;
  *cols = (long)nc;
  if (!out) return RAV_OK;
  HostLevel Hc;
  if (!assemble(topo[level - 1], d->beta, d->eta_out, d->bc_dirichlet_mask, false, Hc, err))
    return rav_set_error(nullptr, RAV_EINVAL, err);
  std::fill(out, out + n * nc, 0.0);
  for (long long i = 0; i < nV; ++i)
    for (int k = H.pptr[i]; k < H.pptr[i + 1]; ++k) {
      const long long j = H.pidx[k];
      const double w = H.pwt[k];
      if (!H.vmask[i] && !Hc.vmask[j]) {
        out[i * nc + j] += w;
        out[(nV + i) * nc + nVc + j] += w;
      }
      out[(2 * nV + i) * nc + 2 * nVc + j] += w;
    }
  return RAV_OK;
}
