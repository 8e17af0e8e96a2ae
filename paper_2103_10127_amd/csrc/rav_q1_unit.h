// Closed-form integrals of the Q1 basis over the unit cell [0,1]^d (tensor
// products of the 1D mass, stiffness and derivative-mass entries), from which
// the element matrices of eqs. 5-8 follow by scaling with the cell size h:
// viscous block h^(d-2) eta kunit, divergence block -h^(d-1) bunit, and
// stabilization -beta d h^2 h^(d-2) kunit.  Basis index a has bit d set when
// the vertex sits at x_d = 1.
#pragma once

namespace rav {
namespace q1unit {

__host__ __device__ constexpr int bit(int a, int d) { return (a >> d) & 1; }
__host__ __device__ constexpr double m1(int a, int b) { return a == b ? 1.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double s1(int a, int b) { return a == b ? 1.0 : -1.0; }
__host__ __device__ constexpr double d1(int a) { return a == 0 ? -0.5 : 0.5; }

// int grad phi_a . grad phi_b over the unit cell
template <int DIM>
__host__ __device__ constexpr double kunit(int a, int b) {
  double s = 0.0;
  for (int c = 0; c < DIM; ++c) {
    double t = s1(bit(a, c), bit(b, c));
    for (int d = 0; d < DIM; ++d)
      if (d != c) t *= m1(bit(a, d), bit(b, d));
    s += t;
  }
  return s;
}

// int d_c phi_a psi_k over the unit cell
template <int DIM>
__host__ __device__ constexpr double bunit(int c, int a, int k) {
  double t = d1(bit(a, c));
  for (int d = 0; d < DIM; ++d)
    if (d != c) t *= m1(bit(a, d), bit(k, d));
  return t;
}

}  // namespace q1unit
}  // namespace rav
