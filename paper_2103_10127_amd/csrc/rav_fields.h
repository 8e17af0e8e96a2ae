// Point-wise fields shared by the assembly kernels of both discretizations:
// the viscosity of the inclusion model and the manufactured forcing.
#pragma once
#include <hip/hip_runtime.h>

namespace rav {

// Viscosity at a point: eta_in inside any inclusion (closed disc/ball), else eta_out.
template <int DIM>
__device__ __forceinline__ double eta_at(const double* x, const double* incl, int n_incl, double eta_out,
                                         double eta_in) {
#pragma clang fp contract(off)
  bool inside = false;
  for (int i = 0; i < n_incl; ++i) {
    const double* ic = incl + 4 * i;
    double d2 = 0.0;
    for (int d = 0; d < DIM; ++d) { double dd = x[d] - ic[d]; d2 = d2 + dd * dd; }
    double rad = ic[3];
    inside = inside || (d2 <= rad * rad);
  }
  return inside ? eta_in : eta_out;
}

// ---- manufactured right-hand side (eq. 5 with f = -eta Lap u + grad p) ------
__device__ __forceinline__ double sfun(int order, double t, double m) {
  const double w = m * M_PI;
  switch (order) {
    case 0: { double s = sin(w * t); return s * s; }
    case 1: return w * sin(2.0 * w * t);
    case 2: return 2.0 * w * w * cos(2.0 * w * t);
    default: return -4.0 * w * w * w * sin(2.0 * w * t);
  }
}

template <int DIM>
__device__ double prod_term(const double* x, const double* w, const int* ord) {
  double p = 1.0;
  for (int d = 0; d < DIM; ++d) p *= sfun(ord[d], x[d], w[d]);
  return p;
}
template <int DIM>
__device__ double lap_prod(const double* x, const double* w, const int* ord) {
  double s = 0.0;
  for (int d = 0; d < DIM; ++d) {
    int o[3] = {ord[0], ord[1], DIM == 3 ? ord[2] : 0};
    o[d] += 2;
    s += prod_term<DIM>(x, w, o);
  }
  return s;
}

template <int DIM>
__device__ void forcing(const double* P, const double* x, double* f) {
  const double eta = P[0];
  double lap[3] = {0, 0, 0}, gp[3] = {0, 0, 0};
  if (DIM == 2) {
    const double *a = P + 1, *m = P + 5, *n = P + 9, *c = P + 13, *r = P + 17, *s = P + 21;
    for (int k = 0; k < 4; ++k) {
      double w[2] = {m[k], n[k]};
      int o01[2] = {0, 1}, o10[2] = {1, 0};
      lap[0] += a[k] * lap_prod<2>(x, w, o01);
      lap[1] -= a[k] * lap_prod<2>(x, w, o10);
      double wr = r[k] * M_PI, ws = s[k] * M_PI;
      gp[0] += c[k] * (-wr * sin(wr * x[0])) * cos(ws * x[1]);
      gp[1] += c[k] * cos(wr * x[0]) * (-ws * sin(ws * x[1]));
    }
  } else {
    for (int i = 0; i < 3; ++i) {
      int j = (i + 1) % 3, kk = (i + 2) % 3;
      const double* Pk = P + 1 + 16 * kk;
      const double* Pj = P + 1 + 16 * j;
      for (int m = 0; m < 4; ++m) {
        int oj[3] = {0, 0, 0}, ok[3] = {0, 0, 0};
        oj[j] = 1; ok[kk] = 1;
        double wk[3] = {Pk[4 + m], Pk[8 + m], Pk[12 + m]};
        double wj[3] = {Pj[4 + m], Pj[8 + m], Pj[12 + m]};
        lap[i] += Pk[m] * lap_prod<3>(x, wk, oj);
        lap[i] -= Pj[m] * lap_prod<3>(x, wj, ok);
      }
    }
    const double *c = P + 49, *r = P + 53, *s = P + 57, *t = P + 61;
    for (int k = 0; k < 4; ++k) {
      double w[3] = {r[k] * M_PI, s[k] * M_PI, t[k] * M_PI};
      for (int cc = 0; cc < 3; ++cc) {
        double term = c[k];
        for (int d = 0; d < 3; ++d) term *= (d == cc) ? -w[d] * sin(w[d] * x[d]) : cos(w[d] * x[d]);
        gp[cc] += term;
      }
    }
  }
  for (int d = 0; d < DIM; ++d) f[d] = -eta * lap[d] + gp[d];
}

}  // namespace rav
