// Second derivatives of the inverse dynamics (the Hessians that Sec. VI names
// as future work), by hyper-dual numbers (Fike & Alonso, "The development of
// hyper-dual numbers for exact second-derivative calculations", AIAA 2011-886):
// x = a + b e1 + c e2 + d e1e2 with e1^2 = e2^2 = 0 and e1e2 != 0. Running the
// recursions of eqs. (1)-(2) on such numbers, with e1 seeded on one input x_j
// and e2 on one input y_k, leaves d^2 tau_i / dx_j dy_k in the e1e2 part of
// every tau_i, exactly (no step size, no cancellation).
//
// One thread per (state, block, j, k). The link records are plain (T); only
// the joint variables and what depends on them carry the hyper-dual parts, so
// the products with the records cost 4 multiplies instead of 9.
//
// The backward sweep needs V_i and dV_i again. Rather than keeping 2 x 24
// numbers per link, it runs the forward recursion backwards: with
// X V_{i-1} = V_i - S_i qd_i it recovers
//   V_{i-1}  = Ad_{f_i} (V_i - S_i qd_i)
//   dV_{i-1} = Ad_{f_i} (dV_i - S_i qdd_i + ad_{S_i qd_i} (V_i - S_i qd_i)),
// so the thread holds a constant number of values whatever the chain length.
#pragma once

#include "sweeps.hpp"

namespace pdyn {

template <class T> struct HD {
  T a, b, c, d;
  HD() = default;
  PD_HD constexpr HD(T x) : a(x), b(T(0)), c(T(0)), d(T(0)) {}
  PD_HD constexpr HD(T a_, T b_, T c_, T d_) : a(a_), b(b_), c(c_), d(d_) {}
};

template <class T> PD_HD HD<T> operator+(const HD<T>& x, const HD<T>& y) {
  return {x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d};
}
template <class T> PD_HD HD<T> operator-(const HD<T>& x, const HD<T>& y) {
  return {x.a - y.a, x.b - y.b, x.c - y.c, x.d - y.d};
}
template <class T> PD_HD HD<T> operator-(const HD<T>& x) { return {-x.a, -x.b, -x.c, -x.d}; }
// (a + b e1 + c e2 + d e1e2)(a' + b' e1 + c' e2 + d' e1e2)
template <class T> PD_HD HD<T> operator*(const HD<T>& x, const HD<T>& y) {
  return {x.a * y.a, x.a * y.b + x.b * y.a, x.a * y.c + x.c * y.a, x.a * y.d + x.b * y.c + x.c * y.b + x.d * y.a};
}
template <class T> PD_HD HD<T> operator*(T s, const HD<T>& y) { return {s * y.a, s * y.b, s * y.c, s * y.d}; }
template <class T> PD_HD HD<T> operator*(const HD<T>& y, T s) { return s * y; }
template <class T> PD_HD HD<T> operator+(const HD<T>& x, T s) { return {x.a + s, x.b, x.c, x.d}; }

// sin and cos of a hyper-dual: f(x) = f(a) + f'(a) (b e1 + c e2 + d e1e2) + f''(a) b c e1e2.
template <class T> PD_HD void hd_sincos(const HD<T>& x, HD<T>* s, HD<T>* c) {
  T s0, c0;
  sin_cos(x.a, &s0, &c0);
  const T bc = x.b * x.c;
  *s = {s0, c0 * x.b, c0 * x.c, c0 * x.d - s0 * bc};
  *c = {c0, -s0 * x.b, -s0 * x.c, -s0 * x.d - c0 * bc};
}

// ---- products of plain records with hyper-dual vectors

template <class T> PD_HD V3<HD<T>> lift(const V3<T>& v) { return {HD<T>(v.x), HD<T>(v.y), HD<T>(v.z)}; }
template <class T> PD_HD Sp<HD<T>> lift(const Sp<T>& v) { return {lift(v.a), lift(v.b)}; }
template <class T> PD_HD V3<HD<T>> scale(const HD<T>& s, const V3<T>& v) { return {s * v.x, s * v.y, s * v.z}; }
template <class T> PD_HD Sp<HD<T>> scale(const HD<T>& s, const Sp<T>& v) { return {scale(s, v.a), scale(s, v.b)}; }
template <class T> PD_HD V3<HD<T>> scale(T s, const V3<HD<T>>& v) { return {s * v.x, s * v.y, s * v.z}; }
template <class T> PD_HD V3<HD<T>> cross(const V3<T>& a, const V3<HD<T>>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> PD_HD V3<HD<T>> mul(const M3<T>& A, const V3<HD<T>>& x) {
  return {A.m[0] * x.x + A.m[1] * x.y + A.m[2] * x.z, A.m[3] * x.x + A.m[4] * x.y + A.m[5] * x.z,
          A.m[6] * x.x + A.m[7] * x.y + A.m[8] * x.z};
}
template <class T> PD_HD M3<HD<T>> mul(const M3<T>& A, const M3<HD<T>>& B) {
  M3<HD<T>> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      r.m[3 * i + j] = A.m[3 * i] * B.m[j] + A.m[3 * i + 1] * B.m[3 + j] + A.m[3 * i + 2] * B.m[6 + j];
  return r;
}
template <class T> PD_HD V3<HD<T>> mul(const S3<T>& S, const V3<HD<T>>& x) {
  return {S.xx * x.x + S.xy * x.y + S.xz * x.z, S.xy * x.x + S.yy * x.y + S.yz * x.z,
          S.xz * x.x + S.yz * x.y + S.zz * x.z};
}
template <class T> PD_HD Sp<HD<T>> mul(const Inertia<T>& J, const Sp<HD<T>>& V) {
  return {scale(J.m, V.a) - cross(J.h, V.b), cross(J.h, V.a) + mul(J.Io, V.b)};
}
template <class T> PD_HD HD<T> dot(const Sp<T>& S, const Sp<HD<T>>& F) {
  return S.a.x * F.a.x + S.a.y * F.a.y + S.a.z * F.a.z + S.b.x * F.b.x + S.b.y * F.b.y + S.b.z * F.b.z;
}
// Ad_g V = (R v + p x (R w), R w): the inverse of X_twist.
template <class T> PD_HD Sp<T> Ad_twist(const Pose<T>& g, const Sp<T>& V) {
  const V3<T> Rw = mul(g.R, V.b);
  return {mul(g.R, V.a) + cross(g.p, Rw), Rw};
}

// f_{i-1,i} = M_i exp(S_i q_i) with a hyper-dual joint angle (the closed form
// of joint_transform_sc, with the record's constants kept plain).
template <class T> PD_HD Pose<HD<T>> hd_joint_transform(const Link<T>& L, const HD<T>& q) {
  const HD<T> th = L.k * q;
  HD<T> s, c;
  hd_sincos(th, &s, &c);
  const HD<T> a = L.ik * s;
  const HD<T> b = L.ik2 * (HD<T>(T(1)) - c);
  const HD<T> e = L.pc * (th - s);
  const V3<T> w = L.S.b, v = L.S.a, wv = cross(w, v);
  M3<HD<T>> Re;
  Re.m[0] = c + (w.x * w.x) * b;
  Re.m[1] = (w.x * w.y) * b - w.z * a;
  Re.m[2] = (w.x * w.z) * b + w.y * a;
  Re.m[3] = (w.x * w.y) * b + w.z * a;
  Re.m[4] = c + (w.y * w.y) * b;
  Re.m[5] = (w.y * w.z) * b - w.x * a;
  Re.m[6] = (w.x * w.z) * b - w.y * a;
  Re.m[7] = (w.y * w.z) * b + w.x * a;
  Re.m[8] = c + (w.z * w.z) * b;
  const V3<HD<T>> pe = scale(a, v) + scale(b, wv) + scale(e, w);
  Pose<HD<T>> g;
  g.R = mul(L.RM, Re);
  const V3<HD<T>> Rp = mul(L.RM, pe);
  g.p = {Rp.x + L.pM.x, Rp.y + L.pM.y, Rp.z + L.pM.z};
  return g;
}

// Blocks of the output: H[i][j][k] = d^2 tau_i / dx_j dy_k with (x, y) =
// (q, q), (q, qd), (qd, qd), (q, qdd). Input codes: 0 q, 1 qd, 2 qdd.
PD_HD int hess_x(int block) { return block == 2 ? 1 : 0; }
PD_HD int hess_y(int block) { return block == 0 ? 0 : (block == 3 ? 2 : 1); }

template <class T> PD_HD HD<T> seeded(T v, int var, int i, int xv, int j, int yv, int k) {
  return {v, T(var == xv && i == j ? 1 : 0), T(var == yv && i == k ? 1 : 0), T(0)};
}

// The e1e2 parts of tau_0..tau_{n-1} for one (block, j, k), written as out(i, value).
// Ftip may be null (no tip wrench).
template <class T, class Tab, class Out>
PD_HD void id_hessian_one(int n, Tab table, const T* q, const T* qd, const T* qdd, const Sp<T>& V0,
                          const Sp<T>& dV0, const Sp<T>* Ftip, int block, int j, int k, const Out& out) {
  const int xv = hess_x(block), yv = hess_y(block);
  Sp<HD<T>> V = lift(V0), A = lift(dV0);
  for (int i = 0; i < n; ++i) {
    const Link<T> L = link_at(table, i);
    const Pose<HD<T>> g = hd_joint_transform(L, seeded(q[i], 0, i, xv, j, yv, k));
    const Sp<HD<T>> XV = X_twist(g, V);
    const Sp<HD<T>> Sqd = scale(seeded(qd[i], 1, i, xv, j, yv, k), L.S);
    V = XV + Sqd;
    A = X_twist(g, A) + scale(seeded(qdd[i], 2, i, xv, j, yv, k), L.S) - ad_twist(Sqd, XV);
  }
  Sp<HD<T>> F = Ftip ? lift(*Ftip) : lift(sp_zero<T>());
  Pose<HD<T>> gnext;
  for (int i = n - 1; i >= 0; --i) {
    const Link<T> L = link_at(table, i);
    if (i < n - 1) F = XT_wrench(gnext, F);
    F = F + mul(L.J, A) - adT_wrench(V, mul(L.J, V));
    out(i, dot(L.S, F).d);
    if (i == 0) break;
    gnext = hd_joint_transform(L, seeded(q[i], 0, i, xv, j, yv, k));
    const Sp<HD<T>> Sqd = scale(seeded(qd[i], 1, i, xv, j, yv, k), L.S);
    const Sp<HD<T>> XV = V - Sqd;
    V = Ad_twist(gnext, XV);
    A = Ad_twist(gnext, A - scale(seeded(qdd[i], 2, i, xv, j, yv, k), L.S) + ad_twist(Sqd, XV));
  }
}

}  // namespace pdyn
