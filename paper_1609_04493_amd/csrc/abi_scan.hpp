// The articulated-body inertia recursion (eq. (7), Sec. II-B) as a prefix scan.
//
// Sec. II-B keeps eq. (7) serial because its step is not linear in Jhat_{i+1}.
// It is a Riccati map, though: the projected inertia
//   P - P S (S^T P S)^-1 S^T P
// is the limit of P (I + r S S^T P)^-1 as r -> infinity, so each link's step is
//   Jhat_i = E_i(Jhat_{i+1}),  E(P) = Q + A^T P (I + C P)^-1 A,
// with (A, C, Q) = (X_{i+1}, infinity * S_{i+1} S_{i+1}^T, J_i) and, for the tip
// link, (I, 0, J_n). Maps of this form are closed under composition. Writing
// E as the two-port z = A v - C y, f = Q v + A^T y (y = P z the response beyond
// the tip end) and eliminating the inner port gives, for E_1 o E_2 (E_2 applied
// first) and W = (I + C_1 Q_2)^-1:
//   A = A_2 W A_1,   C = C_2 + A_2 W C_1 A_2^T,   Q = Q_1 + A_1^T Q_2 W A_1.
// An element keeps C as a finite part plus at most one infinite direction u.
// With B = I + C_1f Q_2 and kappa = u_1^T Q_2 B^-1 u_1 (> 0 whenever the inner
// element holds a link) the limits are
//   W = B^-1 - B^-1 u_1 u_1^T Q_2 B^-1 / kappa,   W C_1 = W C_1f + B^-1 u_1 u_1^T / kappa,
// and the composite keeps the inner element's direction u_2. The composite of
// links i..n evaluated at P = 0 (nothing beyond the tip) is its Q: Jhat_i.
//
// B^-1 is formed without pivoting through the Cholesky factor Q_2 = L L^T and
// the Woodbury identity, B^-1 = I - C_1f L K^-1 L^T with K = I + L^T C_1f L
// symmetric positive definite (eigenvalues >= 1): Q_2 is an articulated inertia
// (positive definite), C_1f a sum of rank-one compliances (positive
// semidefinite).
//
// The scan runs on a team of P lanes per state, as the other segmented scans
// (team.hpp): each lane folds the elements of its consecutive segment of links
// (the step with a single-link outer element reduces to the serial step on Q
// plus rank-one updates of A and C), the team combines the aggregates with a
// Kogge-Stone suffix scan (base-side lanes compose with tip-side ones), and each
// lane runs the serial recursion over its segment again from the Jhat that the
// scan gives at its tip end. Everything after the joint angles' (sin, cos) is
// double.
#pragma once

#include "jsiia.hpp"
#include "team.hpp"

namespace pdyn {

// General 6x6, row-major.
struct M6 {
  double m[36];
};

PD_HD M6 m6_identity() {
  M6 r;
#pragma unroll
  for (int k = 0; k < 36; ++k) r.m[k] = (k % 7 == 0) ? 1.0 : 0.0;
  return r;
}
PD_HD M6 m6_mul(const M6& a, const M6& b) {
  M6 r;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) s += a.m[6 * i + k] * b.m[6 * k + j];
      r.m[6 * i + j] = s;
    }
  return r;
}
// a^T b
PD_HD M6 m6_tmul(const M6& a, const M6& b) {
  M6 r;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) s += a.m[6 * k + i] * b.m[6 * k + j];
      r.m[6 * i + j] = s;
    }
  return r;
}
// a b^T
PD_HD M6 m6_mult(const M6& a, const M6& b) {
  M6 r;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) s += a.m[6 * i + k] * b.m[6 * j + k];
      r.m[6 * i + j] = s;
    }
  return r;
}
PD_HD void sp_to(const Sp<double>& x, double* v) {
  v[0] = x.a.x; v[1] = x.a.y; v[2] = x.a.z; v[3] = x.b.x; v[4] = x.b.y; v[5] = x.b.z;
}
PD_HD Sp<double> sp_of(const double* v) { return {v3(v[0], v[1], v[2]), v3(v[3], v[4], v[5])}; }
PD_HD Sp<double> m6_apply(const M6& a, const Sp<double>& x) {
  double v[6], r[6];
  sp_to(x, v);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) s += a.m[6 * i + k] * v[k];
    r[i] = s;
  }
  return sp_of(r);
}
PD_HD Sp<double> m6_apply_t(const M6& a, const Sp<double>& x) {  // a^T x
  double v[6], r[6];
  sp_to(x, v);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) s += a.m[6 * k + i] * v[k];
    r[i] = s;
  }
  return sp_of(r);
}

// The symmetric [[A, B], [B^T, C]] written out, and back (the mean of the two triangles).
PD_HD M6 m6_of(const Sym6<double>& s) {
  M6 r;
  const double A[9] = {s.A.xx, s.A.xy, s.A.xz, s.A.xy, s.A.yy, s.A.yz, s.A.xz, s.A.yz, s.A.zz};
  const double C[9] = {s.C.xx, s.C.xy, s.C.xz, s.C.xy, s.C.yy, s.C.yz, s.C.xz, s.C.yz, s.C.zz};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      r.m[6 * i + j] = A[3 * i + j];
      r.m[6 * i + 3 + j] = s.B.m[3 * i + j];
      r.m[6 * (3 + i) + j] = s.B.m[3 * j + i];
      r.m[6 * (3 + i) + 3 + j] = C[3 * i + j];
    }
  return r;
}
PD_HD Sym6<double> sym6_of(const M6& a) {
  auto e = [&](int i, int j) { return 0.5 * (a.m[6 * i + j] + a.m[6 * j + i]); };
  Sym6<double> s;
  s.A = {e(0, 0), e(1, 1), e(2, 2), e(0, 1), e(0, 2), e(1, 2)};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) s.B.m[3 * i + j] = e(i, 3 + j);
  s.C = {e(3, 3), e(4, 4), e(5, 5), e(3, 4), e(3, 5), e(4, 5)};
  return s;
}

// Lower Cholesky factor of a symmetric positive definite 6x6 (upper triangle of
// the result zero). Returns false if a pivot is not positive.
PD_HD bool m6_cholesky(const M6& s, M6* L) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 36; ++k) L->m[k] = 0.0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double d = s.m[6 * j + j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L->m[6 * j + k] * L->m[6 * j + k];
    ok = ok && d > 0.0;
    const double ljj = sqrt(d > 0.0 ? d : 0.0), inv = 1.0 / ljj;
    L->m[6 * j + j] = ljj;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double t = s.m[6 * i + j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= L->m[6 * i + k] * L->m[6 * j + k];
      L->m[6 * i + j] = t * inv;
    }
  }
  return ok;
}

// K^-1 R for K = Lk Lk^T (each column of R by a forward and a backward substitution).
PD_HD M6 m6_chol_solve(const M6& Lk, const M6& R) {
  M6 X;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double y[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double t = R.m[6 * i + c];
#pragma unroll
      for (int k = 0; k < i; ++k) t -= Lk.m[6 * i + k] * y[k];
      y[i] = t / Lk.m[6 * i + i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
      double t = y[i];
#pragma unroll
      for (int k = i + 1; k < 6; ++k) t -= Lk.m[6 * k + i] * X.m[6 * k + c];
      X.m[6 * i + c] = t / Lk.m[6 * i + i];
    }
  }
  return X;
}

// An element E(P) = Q + A^T P (I + C P)^-1 A, C = Cf + infinity * u u^T when has_u.
struct AbiEl {
  M6 A;
  Sym6<double> Cf, Q;
  Sp<double> u;
  bool has_u, ident;
};

PD_HD AbiEl abi_identity() {
  AbiEl e;
  e.A = m6_identity();
  e.Cf = sym6_of(M6{});
  e.Q = e.Cf;
  e.u = sp_zero<double>();
  e.has_u = false;
  e.ident = true;
  return e;
}

// X = Ad_{g^-1} as a matrix: column c is X applied to the c-th unit twist.
PD_HD M6 m6_of_X(const Pose<double>& g) {
  M6 r;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double e[6] = {0, 0, 0, 0, 0, 0};
    e[c] = 1.0;
    double col[6];
    sp_to(X_twist(g, sp_of(e)), col);
#pragma unroll
    for (int i = 0; i < 6; ++i) r.m[6 * i + c] = col[i];
  }
  return r;
}

// M X for X = Ad_{g^-1}: row r of the product is X^T applied to row r of M.
PD_HD M6 m6_mul_X(const M6& M, const Pose<double>& g) {
  M6 r;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double row[6];
    sp_to(XT_wrench(g, sp_of(M.m + 6 * i)), row);
#pragma unroll
    for (int c = 0; c < 6; ++c) r.m[6 * i + c] = row[c];
  }
  return r;
}

// Element of link i (0-based) of an n-link chain: (X_{i+1}, infinity S_{i+1} S_{i+1}^T, J_i),
// or (I, 0, J_{n-1}) for the tip link. g_next = f_{i,i+1}, S_next = S_{i+1} (unused for the tip).
PD_HD AbiEl abi_link(bool tip, const Sym6<double>& J, const Pose<double>& g_next, const Sp<double>& S_next) {
  AbiEl e;
  e.A = tip ? m6_identity() : m6_of_X(g_next);
  e.Cf = sym6_of(M6{});
  e.Q = J;
  e.u = tip ? sp_zero<double>() : S_next;
  e.has_u = !tip;
  e.ident = false;
  return e;
}

// e_i o agg, e_i the (non-tip) element of one link given by (g_next, S_next, J): the fold step,
// with B = I. *pivot_ok turns false if kappa = S^T Q S is not positive.
PD_HD AbiEl abi_fold_link(const Sym6<double>& J, const Pose<double>& g_next, const Sp<double>& S_next,
                          const AbiEl& agg, bool* pivot_ok) {
  const Sp<double> y = mul(agg.Q, S_next);  // Q_2 u_1
  const double kappa = dot(S_next, y);
  *pivot_ok = *pivot_ok && kappa > 0.0;
  const double inv = 1.0 / kappa;
  const Sp<double> Au = m6_apply(agg.A, S_next);  // A_2 u_1
  double au[6], yy[6];
  sp_to(Au, au);
  sp_to(y, yy);
  M6 M = agg.A;  // A_2 W = A_2 - (A_2 u_1) y^T / kappa
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) M.m[6 * i + j] -= au[i] * yy[j] * inv;
  AbiEl r;
  r.A = m6_mul_X(M, g_next);
  r.Cf = sym6_minus_outer(agg.Cf, Au, -inv);  // C_2 + (A_2 u_1)(A_2 u_1)^T / kappa
  r.Q = sym6_add(J, congruence_to_parent(g_next, sym6_minus_outer(agg.Q, y, inv)));
  r.u = agg.u;
  r.has_u = agg.has_u;
  r.ident = false;
  return r;
}

// outer o inner (inner applied first), both general elements, read through views
// (AbiView below: each part is loaded where it is used, so that neither element
// has to stay in registers whole).
template <class O, class I> PD_HD AbiEl abi_compose(const O& o, const I& in, bool* pivot_ok);

// An element in a word-major store: word w of slot l at p[w * stride + l].
constexpr int kAbiElWords = 36 + 21 + 21 + 6 + 1;
PD_HD void sym6_words(const Sym6<double>& s, double* w) {
  w[0] = s.A.xx; w[1] = s.A.yy; w[2] = s.A.zz; w[3] = s.A.xy; w[4] = s.A.xz; w[5] = s.A.yz;
#pragma unroll
  for (int k = 0; k < 9; ++k) w[6 + k] = s.B.m[k];
  w[15] = s.C.xx; w[16] = s.C.yy; w[17] = s.C.zz; w[18] = s.C.xy; w[19] = s.C.xz; w[20] = s.C.yz;
}
PD_HD Sym6<double> sym6_from_words(const double* w) {
  Sym6<double> s;
  s.A = {w[0], w[1], w[2], w[3], w[4], w[5]};
#pragma unroll
  for (int k = 0; k < 9; ++k) s.B.m[k] = w[6 + k];
  s.C = {w[15], w[16], w[17], w[18], w[19], w[20]};
  return s;
}
template <class P> PD_HD void abi_store(P p, int stride, int l, const AbiEl& e) {
  double w[kAbiElWords];
#pragma unroll
  for (int k = 0; k < 36; ++k) w[k] = e.A.m[k];
  sym6_words(e.Cf, w + 36);
  sym6_words(e.Q, w + 57);
  sp_to(e.u, w + 78);
  w[84] = (e.ident ? 2.0 : 0.0) + (e.has_u ? 1.0 : 0.0);
#pragma unroll
  for (int k = 0; k < kAbiElWords; ++k) p[k * stride + l] = w[k];
}

// Slot l of a word-major store, part by part.
struct AbiView {
  const double* p;
  int stride, l;
  PD_HD double w(int k) const { return p[k * stride + l]; }
  PD_HD bool ident() const { return w(84) >= 2.0; }
  PD_HD bool has_u() const { const double f = w(84); return f == 1.0 || f == 3.0; }
  PD_HD M6 A() const {
    M6 a;
#pragma unroll
    for (int k = 0; k < 36; ++k) a.m[k] = w(k);
    return a;
  }
  PD_HD Sym6<double> sym(int at) const {
    double v[21];
#pragma unroll
    for (int k = 0; k < 21; ++k) v[k] = w(at + k);
    return sym6_from_words(v);
  }
  PD_HD Sym6<double> Cf() const { return sym(36); }
  PD_HD Sym6<double> Q() const { return sym(57); }
  PD_HD Sp<double> u() const { return {v3(w(78), w(79), w(80)), v3(w(81), w(82), w(83))}; }
  PD_HD AbiEl load() const {
    AbiEl e;
    e.A = A();
    e.Cf = Cf();
    e.Q = Q();
    e.u = u();
    e.ident = ident();
    e.has_u = has_u();
    return e;
  }
};

template <class O, class I> PD_HD AbiEl abi_compose(const O& o, const I& in, bool* pivot_ok) {
  if (in.ident()) return o.load();
  if (o.ident()) return in.load();
  // W0 = (I + C1 Q2)^-1 = I - C1 L K^-1 L^T,  Q2 = L L^T,  K = I + L^T C1 L
  M6 L, Lk, W;
  bool ok = m6_cholesky(m6_of(in.Q()), &L);
  {
    const M6 Z = m6_mul(m6_of(o.Cf()), L);
    M6 K = m6_tmul(L, Z);
#pragma unroll
    for (int k = 0; k < 6; ++k) K.m[7 * k] += 1.0;
    ok = m6_cholesky(K, &Lk) && ok;  // reads the lower triangle only
    M6 Lt;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 6; ++j) Lt.m[6 * i + j] = L.m[6 * j + i];
    W = m6_mul(Z, m6_chol_solve(Lk, Lt));
#pragma unroll
    for (int k = 0; k < 36; ++k) W.m[k] = (k % 7 == 0 ? 1.0 : 0.0) - W.m[k];
  }
  double bu[6], uu[6], inv = 0.0;
  const bool hu = o.has_u();
  if (hu) {
    const Sp<double> u1 = o.u();
    const Sp<double> Bu = m6_apply(W, u1);
    const Sp<double> y = mul(in.Q(), u1);   // Q2 u1
    const Sp<double> r = m6_apply_t(W, y);  // (u1^T Q2 W0)^T
    const double kappa = dot(y, Bu);
    ok = ok && kappa > 0.0;
    inv = 1.0 / kappa;
    double rr[6];
    sp_to(Bu, bu);
    sp_to(r, rr);
    sp_to(u1, uu);
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 6; ++j) W.m[6 * i + j] -= bu[i] * rr[j] * inv;
  }
  *pivot_ok = *pivot_ok && ok;
  AbiEl r;
  {
    M6 WC1 = m6_mul(W, m6_of(o.Cf()));
    if (hu) {
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) WC1.m[6 * i + j] += bu[i] * uu[j] * inv;
    }
    const M6 A2 = in.A();
    r.Cf = sym6_add(in.Cf(), sym6_of(m6_mult(m6_mul(A2, WC1), A2)));
  }
  const M6 A1 = o.A();
  r.A = m6_mul(m6_mul(in.A(), W), A1);
  r.Q = sym6_add(o.Q(), sym6_of(m6_tmul(A1, m6_mul(m6_mul(m6_of(in.Q()), W), A1))));
  r.u = in.u();
  r.has_u = in.has_u();
  r.ident = false;
  return r;
}

// f_{i-1,i} of link i (0-based) in double from the (sin, cos) of its joint angle in T.
template <class T, class Tab, class WTab>
PD_HD Pose<double> abi_pose(Tab table, WTab wtable, const T* q, int i) {
  const Link<T> Lt = link_at(table, i);
  const Link<double> Lw = link_at(wtable, i);
  T sn, cs;
  joint_sincos(Lt, q[i], &sn, &cs);
  return joint_transform_wide_sc(Lw, q[i], sn, cs);
}

// The aggregate e_a o ... o e_{b-1} of links [a, b) of an n-link chain (identity if a == b), folded
// from the tip end of the segment. pose(i) gives f_{i-1,i} in double.
template <class WTab, class PoseOf>
PD_HD AbiEl abi_fold_segment(int n, int a, int b, WTab wtable, const PoseOf& pose, bool* pivot_ok) {
  if (a >= b) return abi_identity();
  const int last = b - 1;
  Pose<double> g_next;
  Sp<double> S_next = sp_zero<double>();
  if (last < n - 1) {
    g_next = pose(last + 1);
    S_next = link_at(wtable, last + 1).S;
  }
  AbiEl agg = abi_link(last == n - 1, sym6_from_inertia(inertia_of(link_at(wtable, last))), g_next, S_next);
  for (int i = last - 1; i >= a; --i) {
    g_next = pose(i + 1);
    S_next = link_at(wtable, i + 1).S;
    agg = abi_fold_link(sym6_from_inertia(inertia_of(link_at(wtable, i))), g_next, S_next, agg, pivot_ok);
  }
  return agg;
}

// The serial recursion (7) over links [a, b), tip end first, from carry = Jhat_b (used when b < n):
// out(i, Jhat_i) for i = b-1 .. a.
template <class WTab, class PoseOf, class Out>
PD_HD void abi_serial_segment(int n, int a, int b, WTab wtable, const PoseOf& pose, const Sym6<double>& carry,
                              const Out& out, bool* pivot_ok) {
  Sym6<double> Jh = carry;
  for (int i = b - 1; i >= a; --i) {
    const Sym6<double> Ji = sym6_from_inertia(inertia_of(link_at(wtable, i)));
    if (i == n - 1) {
      Jh = Ji;
    } else {
      const Sp<double> S = link_at(wtable, i + 1).S;
      const Sp<double> U = mul(Jh, S);
      const double D = dot(S, U);
      *pivot_ok = *pivot_ok && D > 0.0;
      Jh = sym6_add(Ji, congruence_to_parent(pose(i + 1), sym6_minus_outer(Jh, U, 1.0 / D)));
    }
    out(i, Jh);
  }
}

// Link transforms formed from the joint angles wherever they are asked for.
template <class T, class Tab, class WTab> struct AbiPoses {
  Tab table;
  WTab wtable;
  const T* q;
  PD_HD Pose<double> operator()(int i) const { return abi_pose<T>(table, wtable, q, i); }
};

}  // namespace pdyn
