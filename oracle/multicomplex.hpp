// Bicomplex numbers for exact second derivatives -- TEST INFRASTRUCTURE ONLY.
//
// Multicomplex-step differentiation (Lantoine, Russell & Dargent, "Using
// multicomplex variables for automatic computation of high-order derivatives",
// ACM TOMS 38(3), 2012): with two commuting imaginary units i1, i2
// (i1^2 = i2^2 = -1, i1 i2 = i2 i1), a real-analytic f satisfies
//   f(x + i1 h d1 + i2 h d2) = f(x) + i1 h Df d1 + i2 h Df d2 + i1 i2 h^2 d1^T D^2f d2 + O(h^2) (real part),
// and the i1 i2 coefficient holds d1^T D^2f d2 with no difference of nearly
// equal numbers, so with h = 1e-20 it is exact to rounding, as complex step is
// for first derivatives.
//
// A bicomplex number is stored as z = a + b i2 with a, b complex in i1. Every
// operation the oracle's recursions use is written out from that form:
//   (a + b i2)(c + d i2) = (ac - bd) + (ad + bc) i2
//   (a + b i2) / (c + d i2) = ((ac + bd) + (bc - ad) i2) / (c^2 + d^2)
//   sin(a + b i2) = sin a cosh b + i2 cos a sinh b
//   cos(a + b i2) = cos a cosh b - i2 sin a sinh b
// (the last two from cos(i2 b) = cosh b and sin(i2 b) = i2 sinh b).
#pragma once

#include <cmath>
#include <complex>
#include <vector>

#include "oracle.hpp"

namespace oracle {

struct Bicomplex {
  std::complex<double> a, b;  // a + b i2
  Bicomplex(double x = 0.0) : a(x), b(0.0) {}
  Bicomplex(std::complex<double> a_, std::complex<double> b_) : a(a_), b(b_) {}
  Bicomplex& operator+=(const Bicomplex& o) { a += o.a; b += o.b; return *this; }
  Bicomplex& operator-=(const Bicomplex& o) { a -= o.a; b -= o.b; return *this; }
};

inline Bicomplex operator+(const Bicomplex& x, const Bicomplex& y) { return {x.a + y.a, x.b + y.b}; }
inline Bicomplex operator-(const Bicomplex& x, const Bicomplex& y) { return {x.a - y.a, x.b - y.b}; }
inline Bicomplex operator-(const Bicomplex& x) { return {-x.a, -x.b}; }
inline Bicomplex operator*(const Bicomplex& x, const Bicomplex& y) {
  return {x.a * y.a - x.b * y.b, x.a * y.b + x.b * y.a};
}
inline Bicomplex operator/(const Bicomplex& x, const Bicomplex& y) {
  const std::complex<double> den = y.a * y.a + y.b * y.b;
  return {(x.a * y.a + x.b * y.b) / den, (x.b * y.a - x.a * y.b) / den};
}
inline Bicomplex sin(const Bicomplex& z) {
  return {std::sin(z.a) * std::cosh(z.b), std::cos(z.a) * std::sinh(z.b)};
}
inline Bicomplex cos(const Bicomplex& z) {
  return {std::cos(z.a) * std::cosh(z.b), -(std::sin(z.a) * std::sinh(z.b))};
}
// Principal square root: w = c + d i2 with w^2 = z, i.e. c^2 - d^2 = a and
// 2 c d = b, solved as c^2 = (a + sqrt(a^2 + b^2)) / 2, d = b / (2 c).
inline Bicomplex sqrt(const Bicomplex& z) {
  const std::complex<double> c = std::sqrt((z.a + std::sqrt(z.a * z.a + z.b * z.b)) * 0.5);
  return {c, z.b / (2.0 * c)};
}

// The i1 i2 coefficient.
inline double im12(const Bicomplex& z) { return z.b.imag(); }

// Second derivatives of the inverse dynamics (the Hessians the paper lists as
// future work in Sec. VI), one block at a time:
//   H[i][j][k] = d^2 tau_i / (dx_j dy_k),   tau = ID(q, qd, qdd) of eqs. (1)-(3),
// with (x, y) = (q, q), (q, qd), (qd, qd) or (q, qdd) for block 0, 1, 2, 3
// (tau is linear in qdd, so the other blocks vanish). Each entry is one
// bicomplex evaluation of rnea with x_j + i1 h and y_k + i2 h. H is [n][n][n].
inline void rnea_hessian_block(const Chain<double>& ch, const double* q, const double* qd,
                               const double* qdd, const double V0[6], const double dV0[6],
                               const double* Ftip, int block, double* H) {
  const int n = ch.n;
  const double h = 1e-20;
  const int xv = (block == 2) ? 1 : 0;                              // 0: q, 1: qd, 2: qdd
  const int yv = (block == 0) ? 0 : (block == 1 || block == 2) ? 1 : 2;
  std::vector<Bicomplex> pl(ch.placement, ch.placement + 7 * n), tw(ch.twist, ch.twist + 6 * n),
      in(ch.inertia, ch.inertia + 10 * n);
  const Chain<Bicomplex> cb{n, pl.data(), tw.data(), in.data()};
  Bicomplex v0[6], dv0[6], ft[6];
  for (int k = 0; k < 6; ++k) { v0[k] = V0[k]; dv0[k] = dV0[k]; ft[k] = Ftip ? Ftip[k] : 0.0; }
  std::vector<Bicomplex> x[3], tau(n);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k) {
      x[0].assign(q, q + n);
      x[1].assign(qd, qd + n);
      x[2].assign(qdd, qdd + n);
      x[xv][j] += Bicomplex(std::complex<double>(0.0, h), 0.0);
      x[yv][k] += Bicomplex(0.0, h);
      rnea(cb, x[0].data(), x[1].data(), x[2].data(), v0, dv0, ft, tau.data());
      for (int i = 0; i < n; ++i) H[((size_t)i * n + j) * n + k] = im12(tau[i]) / (h * h);
    }
}

}  // namespace oracle
